// Horner step by blocks: w_l = theta_l + T w_{l+1} for cell-based fields that
// span every axis they have (Section 2.2: T is the tensor product of the 1-D
// cell-based interpolation).
//
// A thread owns one coarse cell J and writes the 2 x 2 (x 2) fine cells it
// covers.  Along each axis the two fine cells 2J, 2J+1 need the coarse cells
// J-1, J, J+1 (interior: 1/4, 3/4 and 3/4, 1/4; the end cells extrapolate with
// 5/4, -1/4).  Along x the neighbours come from the adjacent lanes by
// shuffles, so a thread loads one value of each of the 3 (or 9) coarse rows
// around it; theta and the result move as pairs along x.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"
#include "multigrid.h"

namespace modil {

template <typename T> struct PPair;
template <> struct PPair<float> { using type = float2; };
template <> struct PPair<double> { using type = double2; };

struct ProlongPlan {
  int W, wshift, groups, nseg;  // lanes per coarse row, rows per wave, 64-lane segments
  long n_rows;                  // coarse rows over instances, fields and planes
};

// weights of coarse cells J-1, J, J+1 for the fine cells 2J (e = 0), 2J+1 (e = 1)
template <typename T>
__device__ inline void pair_weights(int J, int n, T (&w)[2][3]) {
  if (J >= 1) { w[0][0] = T(0.25); w[0][1] = T(0.75); w[0][2] = T(0); }
  else { w[0][0] = T(0); w[0][1] = T(1.25); w[0][2] = T(-0.25); }
  if (J <= n - 2) { w[1][0] = T(0); w[1][1] = T(0.75); w[1][2] = T(0.25); }
  else { w[1][0] = T(-0.25); w[1][1] = T(1.25); w[1][2] = T(0); }
}

template <typename T, bool SPANZ, bool SEG>
__global__ __launch_bounds__(256) void prolong_block_kernel(Levels G, int l, const T *__restrict__ theta,
                                                            const T *__restrict__ csrc,
                                                            T *__restrict__ dst, ProlongPlan P) {
  using P2 = typename PPair<T>::type;
  const int lane = threadIdx.x & 63;
  const long wave = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int W = P.W, grp = lane >> P.wshift, gl = lane & (W - 1);
  long row = wave * P.groups + grp;  // coarse row index over (inst, f, cz, cy) and segments
  const int seg = (int)(row % P.nseg);
  row /= P.nseg;
  const bool active = row < P.n_rows;  // whole row groups leave together
  if (!active) row = 0;                // keep the addresses valid for the shuffles
  const int nz = G.n[l][0][0], ny = G.n[l][0][1], nx = G.n[l][0][2];
  const int cnz = G.n[l + 1][0][0], cny = G.n[l + 1][0][1], cnx = G.n[l + 1][0][2];
  const int cy = (int)(row % cny);
  long r2 = row / cny;
  const int cz = SPANZ ? (int)(r2 % cnz) : 0;
  r2 = SPANZ ? r2 / cnz : r2;
  const int f = (int)(r2 % G.nf), inst = (int)(r2 / G.nf);
  const int cx = seg * 64 + gl;

  const T *cb = csrc + inst * G.stride[l + 1] + G.foff[l + 1][f];
  const long fbase = (long)inst * G.stride[l] + G.foff[l][f];

  T wx[2][3], wy[2][3], wz[2][3];
  pair_weights(cx, cnx, wx);
  pair_weights(cy, cny, wy);
  if (SPANZ) pair_weights(cz, cnz, wz);
  const int ym = cy > 0 ? cy - 1 : 0, yp = cy < cny - 1 ? cy + 1 : cny - 1;
  const int zm = cz > 0 ? cz - 1 : 0, zp = cz < cnz - 1 ? cz + 1 : cnz - 1;
  const int ys[3] = {ym, cy, yp}, zs[3] = {zm, cz, zp};
  const int lo = (SEG && gl == 0 && cx > 0) ? cx - 1 : cx;
  const int hi = (SEG && gl == W - 1 && cx < cnx - 1) ? cx + 1 : cx;

  // theta of the fine cells written, loaded with the coarse rows (an
  // inactive lane reads row 0's, which exist) and taken before the shuffles:
  // all loads go out in one round, and none is waited for after a store
  constexpr int NEZ = SPANZ ? 2 : 1;
  P2 th[NEZ][2];
#pragma unroll
  for (int ez = 0; ez < NEZ; ++ez)
#pragma unroll
    for (int ey = 0; ey < 2; ++ey) {
      const int z = SPANZ ? 2 * cz + ez : cz, y = 2 * cy + ey;
      th[ez][ey] = *reinterpret_cast<const P2 *>(theta + fbase + ((long)z * ny + y) * nx + 2 * cx);
    }

  // x-interpolated coarse rows: X[dz][dy][e] for the fine x cells 2cx + e
  constexpr int NZ = SPANZ ? 3 : 1;
  T c[NZ][3], el[NZ][3], eh[NZ][3];
#pragma unroll
  for (int a = 0; a < NZ; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const T *r = cb + ((long)(SPANZ ? zs[a] : cz) * cny + ys[b]) * cnx;
      c[a][b] = r[cx];
      el[a][b] = SEG ? r[lo] : T(0);
      eh[a][b] = SEG ? r[hi] : T(0);
    }
#pragma unroll
  for (int ez = 0; ez < NEZ; ++ez)
#pragma unroll
    for (int ey = 0; ey < 2; ++ey) {
      settle(th[ez][ey].x);
      settle(th[ez][ey].y);
    }
  T X[NZ][3][2];
#pragma unroll
  for (int a = 0; a < NZ; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      T left = __shfl_up(c[a][b], 1, W);
      T right = __shfl_down(c[a][b], 1, W);
      if (SEG && gl == 0) left = el[a][b];
      if (SEG && gl == W - 1) right = eh[a][b];
      if (cx == 0) left = c[a][b];          // weight 0 there; keep it finite
      if (cx == cnx - 1) right = c[a][b];
#pragma unroll
      for (int e = 0; e < 2; ++e)
        X[a][b][e] = wx[e][0] * left + wx[e][1] * c[a][b] + wx[e][2] * right;
    }
  if (!active) return;
#pragma unroll
  for (int ez = 0; ez < NEZ; ++ez)
#pragma unroll
    for (int ey = 0; ey < 2; ++ey) {
      T v[2];
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        T acc = T(0);
#pragma unroll
        for (int a = 0; a < NZ; ++a) {
          const T yv = wy[ey][0] * X[a][0][e] + wy[ey][1] * X[a][1][e] + wy[ey][2] * X[a][2][e];
          acc += (SPANZ ? wz[ez][a] : T(1)) * yv;
        }
        v[e] = acc;
      }
      const int z = SPANZ ? 2 * cz + ez : cz, y = 2 * cy + ey;
      const long o = fbase + ((long)z * ny + y) * nx + 2 * cx;
      P2 out;
      out.x = th[ez][ey].x + v[0];
      out.y = th[ez][ey].y + v[1];
      *reinterpret_cast<P2 *>(dst + o) = out;
    }
  (void)nz;
}

// Two Horner steps in one launch, for cell-based fields spanning z, y and x:
// w_l = theta_l + T (theta_{l+1} + T w_{l+2}).  The level-(l+1) values are
// formed in LDS where a block needs them and are never written.  A block
// takes rows [y0, y0 + kP2Rows) of plane Jz of level l+1 of one field of one
// instance: it stages the level-(l+2) planes that level-(l+1) planes Jz-1 ..
// Jz+1 interpolate from, forms those planes on the rows y0-1 .. y0+kP2Rows
// (theta_{l+1} plus the eight-tap T), and writes the level-l cells the owned
// cells cover, one level-(l+1) cell per thread with the three-tap weights of
// pair_weights along each axis (the same arithmetic as prolong_block_kernel).
// All its global reads are issued when it starts.
constexpr int kP2Threads = 512;

template <typename T>
__global__ __launch_bounds__(kP2Threads) void prolong2_kernel(Levels G, int l, int rows,
                                                              const T *__restrict__ th_l,
                                                              const T *__restrict__ th_m,
                                                              const T *__restrict__ csrc,
                                                              T *__restrict__ dst) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *const Cs = reinterpret_cast<T *>(smem_raw);
  const int ny = G.n[l][0][1], nx = G.n[l][0][2];
  const int mz = G.n[l + 1][0][0], my = G.n[l + 1][0][1], mx = G.n[l + 1][0][2];
  const int cz = G.n[l + 2][0][0], cy = G.n[l + 2][0][1], cx = G.n[l + 2][0][2];
  const int nyb = (my + rows - 1) / rows;  // row blocks per plane
  int b = blockIdx.x;
  const int yb = b % nyb;
  b /= nyb;
  const int Jz = b % mz, fi = b / mz;
  const int f = fi % G.nf, inst = fi / G.nf;
  const int tid = threadIdx.x;
  const int y0 = yb * rows, y1 = y0 + rows < my ? y0 + rows : my;
  // level-(l+1) planes m_lo .. m_hi on rows r_lo .. r_hi - 1, and the
  // level-(l+2) planes they read (whole)
  const int m_lo = Jz > 0 ? Jz - 1 : 0, m_hi = Jz < mz - 1 ? Jz + 1 : mz - 1;
  const int r_lo = y0 > 0 ? y0 - 1 : 0, r_hi = y1 < my ? y1 + 1 : my;
  int c_lo = (m_lo >> 1) - 1, c_hi = (m_hi >> 1) + 1;
  c_lo = c_lo < 0 ? 0 : c_lo;
  c_hi = c_hi > cz - 1 ? cz - 1 : c_hi;
  const int cplane = cy * cx, mrows = r_hi - r_lo, mslab = mrows * mx;
  const int ncs = (c_hi - c_lo + 1) * cplane, nms = (m_hi - m_lo + 1) * mslab;
  T *const Ms = Cs + ncs;
  const T *cb = csrc + (long)inst * G.stride[l + 2] + G.foff[l + 2][f] + (long)c_lo * cplane;
  const T *mb = th_m + (long)inst * G.stride[l + 1] + G.foff[l + 1][f];
  const long fb = (long)inst * G.stride[l] + G.foff[l][f];
  const float rs = 1.0f / (float)mslab, rx = 1.0f / (float)mx;
  // the loads: coarse planes (kC per thread), theta_{l+1} of the mid slab
  // (kM), theta_l of the eight cells the thread's level-(l+1) cell covers
  constexpr int kC = 2, kM = 4;
  T cv[kC], mv[kM];
#pragma unroll
  for (int u = 0; u < kC; ++u) {
    const int e = tid + u * kP2Threads;
    cv[u] = e < ncs ? cb[e] : T(0);
  }
#pragma unroll
  for (int u = 0; u < kM; ++u) {
    const int e = tid + u * kP2Threads;
    mv[u] = T(0);
    if (e < nms) {
      const int k = small_div(e, mslab, rs), rem = e - k * mslab, j = small_div(rem, mx, rx);
      mv[u] = mb[((long)(m_lo + k) * my + r_lo + j) * mx + (rem - j * mx)];
    }
  }
  const bool own = tid < (y1 - y0) * mx;
  const int Jy = own ? y0 + small_div(tid, mx, rx) : y0, Jx = own ? tid - (Jy - y0) * mx : 0;
  using P2 = typename PPair<T>::type;
  T tf[2][2][2];
#pragma unroll
  for (int ez = 0; ez < 2; ++ez)
#pragma unroll
    for (int ey = 0; ey < 2; ++ey) {
      const long o = fb + ((long)(2 * Jz + ez) * ny + (2 * Jy + ey)) * nx + 2 * Jx;
      P2 t2;
      t2.x = t2.y = T(0);
      if (own) t2 = *reinterpret_cast<const P2 *>(th_l + o);  // 2 Jx: pair-aligned
      tf[ez][ey][0] = t2.x;
      tf[ez][ey][1] = t2.y;
    }
  // every load above is issued before the first is waited for: the level-l
  // values are taken here, with the coarse planes, in one round trip
#pragma unroll
  for (int ez = 0; ez < 2; ++ez)
#pragma unroll
    for (int ey = 0; ey < 2; ++ey) {
      settle(tf[ez][ey][0]);
      settle(tf[ez][ey][1]);
    }
#pragma unroll
  for (int u = 0; u < kC; ++u) {
    const int e = tid + u * kP2Threads;
    if (e < ncs) Cs[e] = cv[u];
  }
  lds_barrier();
  // level-(l+1) slab: theta_{l+1} + T w_{l+2}
#pragma unroll
  for (int u = 0; u < kM; ++u) {
    const int e = tid + u * kP2Threads;
    if (e >= nms) continue;
    const int kk = small_div(e, mslab, rs), rem = e - kk * mslab, jj = small_div(rem, mx, rx);
    const int k = m_lo + kk, j = r_lo + jj, i = rem - jj * mx;
    int iz[2], iy[2], ix[2];
    T wz[2], wy[2], wx[2];
    prolong_taps(k, cz, iz, wz);
    prolong_taps(j, cy, iy, wy);
    prolong_taps(i, cx, ix, wx);
    T acc = T(0);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int bb = 0; bb < 2; ++bb) {
        const T *r = Cs + (iz[a] - c_lo) * cplane + iy[bb] * cx;
        acc += wz[a] * wy[bb] * (wx[0] * r[ix[0]] + wx[1] * r[ix[1]]);
      }
    Ms[e] = mv[u] + acc;
  }
  lds_barrier();
  if (!own) return;
  // the eight level-l cells of level-(l+1) cell (Jz, Jy, Jx)
  T wz[2][3], wy[2][3], wx[2][3];
  pair_weights(Jz, mz, wz);
  pair_weights(Jy, my, wy);
  pair_weights(Jx, mx, wx);
  const int ks[3] = {Jz > 0 ? Jz - 1 : Jz, Jz, Jz < mz - 1 ? Jz + 1 : Jz};
  const int js[3] = {Jy > 0 ? Jy - 1 : Jy, Jy, Jy < my - 1 ? Jy + 1 : Jy};
  const int is[3] = {Jx > 0 ? Jx - 1 : Jx, Jx, Jx < mx - 1 ? Jx + 1 : Jx};
  T X[3][3][2];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int bb = 0; bb < 3; ++bb) {
      const T *r = Ms + (ks[a] - m_lo) * mslab + (js[bb] - r_lo) * mx;
      const T v0 = r[is[0]], v1 = r[is[1]], v2 = r[is[2]];
#pragma unroll
      for (int e = 0; e < 2; ++e) X[a][bb][e] = wx[e][0] * v0 + wx[e][1] * v1 + wx[e][2] * v2;
    }
#pragma unroll
  for (int ez = 0; ez < 2; ++ez)
#pragma unroll
    for (int ey = 0; ey < 2; ++ey) {
      T v[2];
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        T acc = T(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const T yv = wy[ey][0] * X[a][0][e] + wy[ey][1] * X[a][1][e] + wy[ey][2] * X[a][2][e];
          acc += wz[ez][a] * yv;
        }
        v[e] = tf[ez][ey][e] + acc;
      }
      const long o = fb + ((long)(2 * Jz + ez) * ny + (2 * Jy + ey)) * nx + 2 * Jx;
      P2 out;
      out.x = v[0];
      out.y = v[1];
      *reinterpret_cast<P2 *>(dst + o) = out;
    }
}

// Launch the two-step Horner kernel for levels l + 2 -> l (w_l into dst;
// th_l, th_m and dst are the level-l and level-(l+1) bases of theta and the
// level-l base of the output, csrc the level-(l+2) base) if the levels admit
// it: cell-based, every field the same 3-D shape halving along every axis,
// and the per-thread load counts and LDS within the kernel's.  A block takes
// kP2Threads / mx rows of a level-(l+1) plane.  False if nothing launched.
template <typename T>
bool launch_prolong2(const Levels &G, int l, const T *th_l, const T *th_m, const T *csrc, T *dst,
                     hipStream_t s) {
  if (G.node || l + 2 >= G.L) return false;
  // level l is read and written in pairs of x-neighbours (fields and
  // instances start at even offsets: nx is even)
  if (reinterpret_cast<uintptr_t>(th_l) % (2 * sizeof(T)) || reinterpret_cast<uintptr_t>(dst) % (2 * sizeof(T)))
    return false;
  for (int j = l; j <= l + 2; ++j)
    for (int f = 1; f < G.nf; ++f)
      for (int a = 0; a < 3; ++a)
        if (G.n[j][f][a] != G.n[j][0][a]) return false;
  for (int j = l; j < l + 2; ++j)
    for (int a = 0; a < 3; ++a)
      if (G.n[j][0][a] != 2 * G.n[j + 1][0][a] || G.n[j + 1][0][a] < 2) return false;
  const int mz = G.n[l + 1][0][0], my = G.n[l + 1][0][1], mx = G.n[l + 1][0][2];
  const int cy = G.n[l + 2][0][1], cx = G.n[l + 2][0][2];
  if (mx > kP2Threads) return false;
  const int rows = std::min(my, kP2Threads / mx);  // owned rows per block
  const long mslab = (long)(rows + 2) * mx;
  // the loads per thread the kernel holds: coarse planes (2), mid slab (4)
  if (4L * cy * cx > 2L * kP2Threads || 3 * mslab > 4L * kP2Threads) return false;
  const size_t lds = (size_t)(4L * cy * cx + 3 * mslab) * sizeof(T);
  if (lds > 64 * 1024) return false;
  const long blocks = (long)G.batch * G.nf * mz * ((my + rows - 1) / rows);
  if (blocks > (1L << 30)) return false;
  prolong2_kernel<T><<<(unsigned)blocks, kP2Threads, lds, s>>>(G, l, rows, th_l, th_m, csrc, dst);
  return true;
}

template bool launch_prolong2<float>(const Levels &, int, const float *, const float *, const float *,
                                     float *, hipStream_t);
template bool launch_prolong2<double>(const Levels &, int, const double *, const double *,
                                      const double *, double *, hipStream_t);

// Launch the block Horner step of level l (w_l into dst; theta and dst are
// level-l bases in the pack layout, csrc the level-(l+1) base) if the level
// admits it; returns false (nothing launched) otherwise.
template <typename T>
bool launch_prolong_block(const Levels &G, int l, const T *theta, const T *csrc, T *dst,
                          hipStream_t s) {
  if (G.node || l + 1 >= G.L) return false;
  const uintptr_t al = 2 * sizeof(T);
  if (reinterpret_cast<uintptr_t>(theta) % al || reinterpret_cast<uintptr_t>(dst) % al)
    return false;
  for (int f = 1; f < G.nf; ++f)
    for (int a = 0; a < 3; ++a)
      if (G.n[l][f][a] != G.n[l][0][a] || G.n[l + 1][f][a] != G.n[l + 1][0][a]) return false;
  const int nz = G.n[l][0][0], ny = G.n[l][0][1], nx = G.n[l][0][2];
  const int cnz = G.n[l + 1][0][0], cny = G.n[l + 1][0][1], cnx = G.n[l + 1][0][2];
  if (nx != 2 * cnx || ny != 2 * cny || cnx < 2 || cny < 2) return false;
  const bool spanz = nz > 1;
  if (spanz ? (nz != 2 * cnz || cnz < 2) : cnz != 1) return false;
  ProlongPlan P{};
  if (cnx % 64 == 0) {
    P.W = 64;
    P.nseg = cnx / 64;
  } else if (cnx < 64 && (cnx & (cnx - 1)) == 0) {
    P.W = cnx;
    P.nseg = 1;
  } else {
    return false;
  }
  P.wshift = 0;
  while ((1 << P.wshift) < P.W) ++P.wshift;
  P.groups = 64 / P.W;
  P.n_rows = (long)G.batch * G.nf * (spanz ? cnz : 1) * cny;
  const long waves = (P.n_rows * P.nseg + P.groups - 1) / P.groups;
  const unsigned blocks = (unsigned)((waves + 3) / 4);
  const bool seg = P.nseg > 1;
  if (spanz) {
    if (seg) prolong_block_kernel<T, true, true><<<blocks, 256, 0, s>>>(G, l, theta, csrc, dst, P);
    else prolong_block_kernel<T, true, false><<<blocks, 256, 0, s>>>(G, l, theta, csrc, dst, P);
  } else {
    if (seg) prolong_block_kernel<T, false, true><<<blocks, 256, 0, s>>>(G, l, theta, csrc, dst, P);
    else prolong_block_kernel<T, false, false><<<blocks, 256, 0, s>>>(G, l, theta, csrc, dst, P);
  }
  return true;
}

// Horner step for node-based fields of one shape that span all three axes
// (Section 2.2: T is the tensor product of the 1-D node interpolation; an even
// fine node takes the coarse node it sits on, an odd one the mean of its two
// coarse neighbours).  One thread per fine node, x fastest; the (instance,
// field, z, y) of a node comes from divisions by block-uniform sizes.  Same
// taps and order of operations as the generic per-value kernel.
template <typename T>
__global__ __launch_bounds__(256) void prolong_node_kernel(Levels G, int l, const T *__restrict__ theta,
                                                           const T *__restrict__ csrc,
                                                           T *__restrict__ dst, int total) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const int nz = G.n[l][0][0], ny = G.n[l][0][1], nx = G.n[l][0][2];
  const int cny = G.n[l + 1][0][1], cnx = G.n[l + 1][0][2];
  const int cells = nz * ny * nx;
  // below 2^22 the float-reciprocal division (exact there) replaces the
  // integer divisions, which take tens of instructions each
  const bool small = total < (1 << 22);
  const int q = small ? small_div(e, cells, 1.0f / (float)cells) : e / cells;
  const int r = e - q * cells;  // q = instance * fields + field
  const int inst = small ? small_div(q, G.nf, 1.0f / (float)G.nf) : q / G.nf, f = q - inst * G.nf;
  const int zy = small ? small_div(r, nx, 1.0f / (float)nx) : r / nx, x = r - zy * nx;
  const int z = small ? small_div(zy, ny, 1.0f / (float)ny) : zy / ny, y = zy - z * ny;
  int ix[2], iy[2], iz[2];
  T wx[2], wy[2], wz[2];
  prolong_taps_node(x, ix, wx);
  prolong_taps_node(y, iy, wy);
  prolong_taps_node(z, iz, wz);
  const T *cb = csrc + (long)inst * G.stride[l + 1] + G.foff[l + 1][f];
  T acc = T(0);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const T *rw = cb + ((long)iz[a] * cny + iy[b]) * cnx;
      acc += wz[a] * wy[b] * (wx[0] * rw[ix[0]] + wx[1] * rw[ix[1]]);
    }
  const long k = (long)inst * G.stride[l] + G.foff[l][f] + r;
  dst[k] = theta[k] + acc;
}

template <typename T>
bool launch_prolong_node(const Levels &G, int l, const T *theta, const T *csrc, T *dst,
                         hipStream_t s) {
  if (!G.node || l + 1 >= G.L) return false;
  for (int f = 0; f < G.nf; ++f)
    for (int a = 0; a < 3; ++a) {
      if (G.n[l][f][a] != G.n[l][0][a] || G.n[l + 1][f][a] != G.n[l + 1][0][a]) return false;
      // nodes of a spanned axis: 2 (coarse cells) + 1
      if (G.n[l + 1][0][a] < 2 || G.n[l][0][a] != 2 * (G.n[l + 1][0][a] - 1) + 1) return false;
    }
  // one instance's level is contiguous: fields at foff = f * cells
  const long cells = (long)G.n[l][0][0] * G.n[l][0][1] * G.n[l][0][2];
  for (int f = 0; f < G.nf; ++f)
    if (G.foff[l][f] != f * cells) return false;
  const long total = (long)G.batch * G.nf * cells;
  if (total >= (1L << 31) - 256) return false;
  prolong_node_kernel<T><<<(unsigned)((total + 255) / 256), 256, 0, s>>>(G, l, theta, csrc, dst,
                                                                         (int)total);
  return true;
}

template bool launch_prolong_node<float>(const Levels &, int, const float *, const float *, float *,
                                         hipStream_t);
template bool launch_prolong_node<double>(const Levels &, int, const double *, const double *,
                                          double *, hipStream_t);

template bool launch_prolong_block<float>(const Levels &, int, const float *, const float *, float *,
                                          hipStream_t);
template bool launch_prolong_block<double>(const Levels &, int, const double *, const double *,
                                           double *, hipStream_t);

}  // namespace modil
