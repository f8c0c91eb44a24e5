// Kernels of one mODIL iteration on gfx950.
//
//   prolong_level   w_l = theta_l + T w_{l+1}          (Horner step, Section 2.2)
//   restrict_level  g_{l+1} = T^T g_l                  (exact transpose of T)
//   fine_kernel     residuals, FP64 loss partials and the gathered adjoint
//                   g(c) = sum_o s_o(c - o) of every equation whose stencil
//                   touches c (Section 2.1 loss, adjoint by hand)
//   data_kernel     measurement misfits and their adjoint
//   colsum_kernel   column sums of the contributions of a field that spans x only
//   reduce_kernel   fixed-order reduction of the FP64 partials per instance
//   adam_kernel     elementwise Adam over a pack
//
// Every reduction is deterministic: wave shuffles in a fixed pattern, LDS
// across the waves of a block, and one block per instance for the final sum.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "internal.h"
#include "multigrid.h"
#include "ops.h"

namespace modil {

// ---------------------------------------------------------------- geometry
// 32-bit geometry of every level (pack sizes are validated to fit in int32).
__device__ inline void locate(const Levels &G, int l, int e, int &inst, int &f, int (&i)[3]) {
  // below 2^22 the float-reciprocal division (exact there) replaces the
  // integer divisions, which take tens of instructions each
  const bool small = G.stride[l] * G.batch < (1 << 22);
  inst = small ? small_div(e, G.stride[l], 1.0f / (float)G.stride[l]) : e / G.stride[l];
  int rem = e - inst * G.stride[l];
  f = 0;
  for (int k = 1; k < G.nf; ++k)
    if (rem >= G.foff[l][k]) f = k;
  int cell = rem - G.foff[l][f];
  const int nx = G.n[l][f][2], ny = G.n[l][f][1];
  if (small) {
    small_index(cell, ny, nx, 1.0f / (float)ny, 1.0f / (float)nx, i);
  } else {
    i[2] = cell % nx;
    cell /= nx;
    i[1] = cell % ny;
    i[0] = cell / ny;
  }
}

// (T w)(i) of field f at fine level l from the level-(l+1) array base cb
template <typename T>
__device__ inline T prolong_value_at(const Levels &G, int l, int f, const int (&i)[3],
                                     const T *__restrict__ cb);

template <typename T>
__device__ inline T prolong_value(const Levels &G, int l, int inst, int f, const int (&i)[3],
                                  const T *__restrict__ cbase) {
  return prolong_value_at(G, l, f, i, cbase + inst * G.stride[l + 1] + G.foff[l + 1][f]);
}

// (T w)(i) from cb, the level-(l+1) array of field f of one instance
template <typename T>
__device__ inline T prolong_value_at(const Levels &G, int l, int f, const int (&i)[3],
                                     const T *__restrict__ cb) {
  if (G.node) {
    const int cnx = G.n[l + 1][f][2], cny = G.n[l + 1][f][1];
    const bool sz_ = G.n[l][f][0] != G.n[l + 1][f][0], sy_ = G.n[l][f][1] != cny;
    int ix[2], iy[2], iz[2];
    T wx[2], wy[2], wz[2];
    prolong_taps_node(i[2], ix, wx);
    if (sy_) prolong_taps_node(i[1], iy, wy); else { iy[0] = iy[1] = i[1]; wy[0] = T(1); wy[1] = T(0); }
    if (sz_) prolong_taps_node(i[0], iz, wz); else { iz[0] = iz[1] = i[0]; wz[0] = T(1); wz[1] = T(0); }
    T acc = T(0);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const T *r = cb + ((long)iz[a] * cny + iy[b]) * cnx;
        acc += wz[a] * wy[b] * (wx[0] * r[ix[0]] + wx[1] * r[ix[1]]);
      }
    return acc;
  }
  const int cnx = G.n[l + 1][f][2], cny = G.n[l + 1][f][1];
  const int sy = cnx, sz = cny * cnx;
  const bool span_z = G.n[l][f][0] != G.n[l + 1][f][0];
  const bool span_y = G.n[l][f][1] != cny;
  int ix[2], iy[2], iz[2];
  T wx[2], wy[2], wz[2];
  prolong_taps(i[2], cnx, ix, wx);
  if (span_y) prolong_taps(i[1], cny, iy, wy);
  if (span_z) prolong_taps(i[0], G.n[l + 1][f][0], iz, wz);
  if (span_z && span_y) {  // 3-D: eight taps
    T acc = T(0);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc += wz[a] * wy[b] * (wx[0] * cb[iz[a] * sz + iy[b] * sy + ix[0]] +
                                wx[1] * cb[iz[a] * sz + iy[b] * sy + ix[1]]);
    return acc;
  }
  const int zoff = i[0] * sz;  // unspanned z keeps the index
  if (span_y) {
    return wy[0] * (wx[0] * cb[zoff + iy[0] * sy + ix[0]] + wx[1] * cb[zoff + iy[0] * sy + ix[1]]) +
           wy[1] * (wx[0] * cb[zoff + iy[1] * sy + ix[0]] + wx[1] * cb[zoff + iy[1] * sy + ix[1]]);
  }
  const int yoff = zoff + i[1] * sy;
  return wx[0] * cb[yoff + ix[0]] + wx[1] * cb[yoff + ix[1]];
}

// (T^T g)(I) of field f at coarse level l+1 from the level-l array base fb.
// Column J of T is a window of four contiguous fine cells plus, for coarse
// cells next to a wall, the extrapolated end cells (restrict_taps6, six
// slots with zero weights where unused).  Along x, which varies across a
// wave, all six slots are loaded unconditionally; the 4 x 4 window rows in
// y and z are summed unconditionally too, so a thread issues all its loads
// before it waits.  The end-cell rows in y and z sit in one branch that is
// uniform across a wave running along x.
template <typename T>
__device__ inline T restrict_value_at(const Levels &G, int l, int f, const int (&I)[3],
                                      const T *__restrict__ fb);

template <typename T>
__device__ inline T restrict_value(const Levels &G, int l, int inst, int f, const int (&I)[3],
                                   const T *__restrict__ fbase) {
  return restrict_value_at(G, l, f, I, fbase + inst * G.stride[l] + G.foff[l][f]);
}

// (T^T g)(I) from fb, the level-l array of field f of one instance
template <typename T>
__device__ inline T restrict_value_at(const Levels &G, int l, int f, const int (&I)[3],
                                      const T *__restrict__ fb) {
  if (G.node) {
    const int nx = G.n[l][f][2], ny = G.n[l][f][1], nz = G.n[l][f][0];
    const bool sz_ = nz != G.n[l + 1][f][0], sy_ = ny != G.n[l + 1][f][1];
    int ix[3], iy[3], iz[3];
    T wx[3], wy[3], wz[3];
    restrict_taps_node(I[2], nx, ix, wx);
    if (sy_) restrict_taps_node(I[1], ny, iy, wy);
    else { iy[0] = iy[1] = iy[2] = I[1]; wy[0] = wy[2] = T(0); wy[1] = T(1); }
    if (sz_) restrict_taps_node(I[0], nz, iz, wz);
    else { iz[0] = iz[1] = iz[2] = I[0]; wz[0] = wz[2] = T(0); wz[1] = T(1); }
    T acc = T(0);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const T *r = fb + (iz[a] * ny + iy[b]) * nx;  // level offsets are int
        acc += wz[a] * wy[b] * (wx[0] * r[ix[0]] + wx[1] * r[ix[1]] + wx[2] * r[ix[2]]);
      }
    return acc;
  }
  const int sy = G.n[l][f][2], sz = G.n[l][f][1] * sy;
  const bool span_z = G.n[l][f][0] != G.n[l + 1][f][0];
  const bool span_y = G.n[l][f][1] != G.n[l + 1][f][1];
  int iz[6], iy[6], ix[6];
  T wz[6], wy[6], wx[6];
  if (span_z) {
    restrict_taps6(I[0], G.n[l + 1][f][0], iz, wz);
  } else {
    for (int k = 0; k < 6; ++k) { iz[k] = I[0]; wz[k] = T(k == 0); }
  }
  if (span_y) {
    restrict_taps6(I[1], G.n[l + 1][f][1], iy, wy);
  } else {
    for (int k = 0; k < 6; ++k) { iy[k] = I[1]; wy[k] = T(k == 0); }
  }
  restrict_taps6(I[2], G.n[l + 1][f][2], ix, wx);
  auto row6 = [&](int zz, int yy) {
    const T *r = fb + zz * sz + yy * sy;
    return wx[0] * r[ix[0]] + wx[1] * r[ix[1]] + wx[2] * r[ix[2]] + wx[3] * r[ix[3]] +
           wx[4] * r[ix[4]] + wx[5] * r[ix[5]];
  };
  T acc = T(0);
  if (span_z) {
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      T pl = T(0);
#pragma unroll
      for (int b = 0; b < 4; ++b) pl += wy[b] * row6(iz[a], iy[b]);
      acc += wz[a] * pl;
    }
    if (wy[4] != T(0) || wy[5] != T(0) || wz[4] != T(0) || wz[5] != T(0)) {
#pragma unroll
      for (int a = 0; a < 6; ++a)
#pragma unroll
        for (int b = 0; b < 6; ++b)
          if (a >= 4 || b >= 4) acc += wz[a] * wy[b] * row6(iz[a], iy[b]);
    }
  } else if (span_y) {
#pragma unroll
    for (int b = 0; b < 4; ++b) acc += wy[b] * row6(iz[0], iy[b]);
    if (wy[4] != T(0) || wy[5] != T(0)) acc += wy[4] * row6(iz[0], iy[4]) + wy[5] * row6(iz[0], iy[5]);
  } else {
    acc = row6(iz[0], iy[0]);
  }
  return acc;
}

template <typename T>
__device__ inline void adam_elem(const AdamArgs<T> &A, int e, T g) {
  const T mm = A.b1 * A.m[e] + (T(1) - A.b1) * g;
  const T vv = A.b2 * A.v[e] + (T(1) - A.b2) * g * g;
  A.m[e] = mm;
  A.v[e] = vv;
  A.th_out[e] = adam_theta(A.th_in[e], mm, vv, A.step, A.isb2, A.eps);
}

// Adam with the old state already loaded (lets the loads overlap the gather)
template <typename T>
__device__ inline void adam_elem_loaded(const AdamArgs<T> &A, int e, T g, T th, T m, T v) {
  const T mm = A.b1 * m + (T(1) - A.b1) * g;
  const T vv = A.b2 * v + (T(1) - A.b2) * g * g;
  A.m[e] = mm;
  A.v[e] = vv;
  A.th_out[e] = adam_theta(th, mm, vv, A.step, A.isb2, A.eps);
}

// ------------------------------------------------------------- prolongation
// w_l = theta_l + T w_{l+1}; csrc points at the level-(l+1) source array
template <typename T>
__global__ __launch_bounds__(kBlock) void prolong_kernel(Levels G, int l, const T *__restrict__ theta,
                                                         const T *__restrict__ csrc, T *__restrict__ dst) {
  const int total = G.stride[l] * G.batch;
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= total) return;
  const T th = theta[G.off[l] + e];
  int inst, f, i[3];
  locate(G, l, e, inst, f, i);
  dst[e] = th + prolong_value(G, l, inst, f, i, csrc);
}

// cells of field f on level l and the 3-D index of cell e of it
__device__ inline int field_cells(const Levels &G, int l, int f) {
  return G.n[l][f][0] * G.n[l][f][1] * G.n[l][f][2];
}
__device__ inline void field_index(const Levels &G, int l, int f, int e, int (&i)[3]) {
  const int nx = G.n[l][f][2], ny = G.n[l][f][1];
  small_index(e, ny, nx, 1.0f / (float)ny, 1.0f / (float)nx, i);
}

// dst[e] = src[e] for lo <= e < hi, global -> LDS, up to eight values in
// flight per thread.  A round takes K = 1, 2, 4 or 8 slots, chosen per wave
// (enough for its first lane, whose elements are the wave's smallest), and a
// lane past hi loads and stores element hi - 1 (the same value to the same
// place): each round is straight-line code whose K loads are all issued
// before the first is waited for.
template <int K, typename T>
__device__ inline void tail_copy_round(T *dst, const T *__restrict__ src, int e0, int bd, int hi) {
  T v[K];
#pragma unroll
  for (int u = 0; u < K; ++u) v[u] = src[min(e0 + u * bd, hi - 1)];
#pragma unroll
  for (int u = 0; u < K; ++u) dst[min(e0 + u * bd, hi - 1)] = v[u];
}

template <typename T>
__device__ inline void tail_copy_in(T *dst, const T *__restrict__ src, int lo, int hi) {
  const int bd = (int)blockDim.x;
  const int lane0 = __builtin_amdgcn_readfirstlane((int)threadIdx.x);  // the wave's first lane
  for (int r = 0; lo + lane0 + r < hi; r += 8 * bd) {
    const int e0 = lo + (int)threadIdx.x + r;
    const int need = (hi - (lo + lane0 + r) + bd - 1) / bd;  // slots of the first lane
    if (need > 4) tail_copy_round<8>(dst, src, e0, bd, hi);
    else if (need > 2) tail_copy_round<4>(dst, src, e0, bd, hi);
    else if (need > 1) tail_copy_round<2>(dst, src, e0, bd, hi);
    else tail_copy_round<1>(dst, src, e0, bd, hi);
  }
}

// The Horner tail of the small coarse levels, one field of one instance per
// `parts` blocks: w_{L-1} = theta_{L-1}, then w_l = theta_l + T w_{l+1} for
// l = L-2 .. l_stop, every w_l below L-1 written to w (pack layout).  The last
// (largest) level l_stop is split over the parts; every part computes the
// levels above it (part 0 writes them).  Levels above l_stop alternate between
// two LDS buffers of level l_stop + 1's size, level l in buffer
// (l - l_stop - 1) & 1.  The restriction tail carries the same steps with the
// same function for the updated theta, so both give the same bits.
template <typename T>
__global__ __launch_bounds__(1024) void horner_tail_kernel(Levels G, int l_stop, int parts,
                                                           const T *__restrict__ theta, T *w) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *const sm = reinterpret_cast<T *>(smem_raw);
  constexpr int kPf = 4;  // theta values of the part's slice per thread, loaded first
  const int part = blockIdx.x % parts, fi = blockIdx.x / parts;
  const int inst = fi / G.nf, f = fi % G.nf;
  const bool lead = part == 0;
  const int bd = blockDim.x, tid = threadIdx.x;
  const int n_stop = field_cells(G, l_stop, f);
  const int h_lo = (int)((long)n_stop * part / parts), h_hi = (int)((long)n_stop * (part + 1) / parts);
  const int bstop = G.off[l_stop] + inst * G.stride[l_stop] + G.foff[l_stop][f];
  T pth[kPf];
#pragma unroll
  for (int u = 0; u < kPf; ++u) {
    const int e = h_lo + tid + u * bd;
    pth[u] = e < h_hi ? theta[bstop + e] : T(0);
  }
  // the two LDS buffers, chosen by a select (not an indexed array) so that
  // the compiler keeps their accesses as LDS instructions; a generic (flat)
  // access would wait on global stores as well
  T *const hb0 = sm, *const hb1 = sm + field_cells(G, l_stop + 1, f);
  {
    const int l = G.L - 1;
    const T *src = theta + G.off[l] + inst * G.stride[l] + G.foff[l][f];
    tail_copy_in(((l - l_stop - 1) & 1) ? hb1 : hb0, src, 0, field_cells(G, l, f));
  }
  lds_barrier();
  for (int l = G.L - 2; l >= l_stop; --l) {
    const bool last = l == l_stop;
    T *dst = ((l - l_stop - 1) & 1) ? hb1 : hb0;
    const T *cs = ((l - l_stop) & 1) ? hb1 : hb0;
    const int base = G.off[l] + inst * G.stride[l] + G.foff[l][f];
    const int n1 = G.n[l][f][1], n2 = G.n[l][f][2];
    const float r1 = 1.0f / (float)n1, r2 = 1.0f / (float)n2;
    if (last) {
#pragma unroll
      for (int u = 0; u < kPf; ++u) {
        const int e = h_lo + tid + u * bd;
        if (e < h_hi) {
          int i[3];
          small_index(e, n1, n2, r1, r2, i);
          w[base + e] = pth[u] + prolong_value_at(G, l, f, i, cs);
        }
      }
      for (int e = h_lo + tid + kPf * bd; e < h_hi; e += bd) {
        int i[3];
        small_index(e, n1, n2, r1, r2, i);
        w[base + e] = theta[base + e] + prolong_value_at(G, l, f, i, cs);
      }
      break;
    }
    const int n = field_cells(G, l, f);
    for (int e = tid; e < n; e += bd) {
      int i[3];
      small_index(e, n1, n2, r1, r2, i);
      const T val = theta[base + e] + prolong_value_at(G, l, f, i, cs);
      dst[e] = val;
      if (lead) w[base + e] = val;
    }
    lds_barrier();
  }
}

// --------------------------------------------------------------- restriction
// g_{l+1} = T^T g_l (pack layout in g); with ADAM also Adam on level l+1
template <typename T, bool ADAM>
__global__ __launch_bounds__(kBlock) void restrict_kernel(Levels G, int l, T *g, AdamArgs<T> A) {
  const int total = G.stride[l + 1] * G.batch;
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= total) return;
  const int k = G.off[l + 1] + e;
  T th = T(0), m = T(0), v = T(0);
  if (ADAM) {  // issued before the gather so both latencies overlap
    th = A.th_in[k];
    m = A.m[k];
    v = A.v[k];
  }
  int inst, f, I[3];
  locate(G, l + 1, e, inst, f, I);
  const T val = restrict_value(G, l, inst, f, I, g + G.off[l]);
  g[k] = val;
  if (ADAM) adam_elem_loaded(A, k, val, th, m, v);
}

// One pass of the cell-based T^T along axis a (0 z, 1 y, 2 x) over an array
// in LDS: src has dims n (z, y, x), dst the same dims with n[a] replaced by
// the coarse extent c.  T^T gathers fine 2J-1 .. 2J+2 with 1/4, 3/4, 3/4,
// 1/4 and the end rows' 5/4, -1/4.  Applied once per spanned axis it is the
// tensor-product T^T of one level.  All six slots are read at once, at
// indices clamped into the row, and a slot that does not apply adds zero
// times its value: the sum takes the same terms in the same order as the
// conditional form, with one LDS wait instead of up to five.  The index
// split uses the hardware reciprocal (within one ulp, which small_index
// allows).
template <typename T>
__device__ inline void tail_restrict_pass(const T *__restrict__ src, T *__restrict__ dst,
                                          const int (&n)[3], int a, int c) {
  int m[3] = {n[0], n[1], n[2]};
  m[a] = c;
  const int total = m[0] * m[1] * m[2];
  if ((int)threadIdx.x >= total) return;
  const float r1 = __builtin_amdgcn_rcpf((float)m[1]), r2 = __builtin_amdgcn_rcpf((float)m[2]);
  const int sa = a == 2 ? 1 : (a == 1 ? n[2] : n[1] * n[2]);  // stride of axis a in src
  const int nf = n[a];
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    int i[3];
    small_index(e, m[1], m[2], r1, r2, i);
    const int J = i[a];
    i[a] = 0;
    const T *s = src + (i[0] * n[1] + i[1]) * n[2] + i[2];
    const T x0 = s[2 * J * sa], x1 = s[(2 * J + 1) * sa];
    const T xm = s[max(2 * J - 1, 0) * sa], xp = s[min(2 * J + 2, nf - 1) * sa];
    const T xa = s[0], xb = s[(nf - 1) * sa];
    T acc = (J == 0 ? T(1.25) : T(0.75)) * x0 + (J == c - 1 ? T(1.25) : T(0.75)) * x1;
    acc += (J >= 1 ? T(0.25) : T(0)) * xm;
    acc += (J <= c - 2 ? T(0.25) : T(0)) * xp;
    acc += (J == 1 ? T(-0.25) : T(0)) * xa;
    acc += (J == c - 2 ? T(-0.25) : T(0)) * xb;
    dst[e] = acc;
  }
}

// g_{l+1} = T^T g_l for l = l_lo .. L-2 of one field of one instance per
// block, in LDS, with Adam on every level produced; level l_lo is read from g,
// every level produced is written back to g.  The levels alternate between
// two LDS regions of cap0 elements each; cell-based T^T is applied one axis
// at a time, node-based T^T (three taps per axis) to all axes at once.
// With H.w set (and Adam), the blocks then do the Horner tail of their field
// for the updated theta, w_{L-1} = theta'_{L-1}, w_l = theta'_l + T w_{l+1}
// down to level H.l_stop, so the next iteration starts from it.  The last
// (largest) level l_stop is split over H.parts blocks per field: every part
// does the restriction and the Horner levels above l_stop identically (part 0
// alone writes what they share) and its slice of level l_stop.  Levels above
// l_stop alternate between two LDS buffers of level l_stop + 1's size.  The
// updated theta is kept in LDS at element H.toff: the part's slice of level
// l_stop, then the levels above it in turn; the levels this block produces
// are stored there by their Adam update, the others (final before the
// launch) are loaded there at the start.  Every read of global memory is
// issued at the start: level l_lo of g, the carried theta and the Adam state
// of every level produced.  l_lo is l_big for fields f < nf_big and l_small
// <= l_big for the others: small fields beside larger ones (the heat
// problem's 1-D q beside its 2-D u) can start here at a finer level while
// the marching kernel restricts the larger fields alone.
// With gq set, the block of field f (which starts at level 0) first forms
// that field's level-0 gradient from gq, the tile rows' sums of its per-cell
// contributions (rows x cells per instance), adding the rows in order, and
// applies Adam to level 0 (the x-only field of the heat problem, whose
// column sums would otherwise take a launch of their own).
template <typename T>
struct ColFold {
  const T *gq = nullptr;
  int rows = 0, f = -1;
};

template <typename T>
struct CarryTail {
  T *w = nullptr;
  int l_stop = 0, toff = 0, parts = 1;
};

constexpr int kTailThreads = 1024;
constexpr int kTailR = 2;  // restricted values per thread per level (cap / kTailThreads)

__device__ inline int field_base(const Levels &G, int l, int inst, int f) {
  return G.off[l] + inst * G.stride[l] + G.foff[l][f];
}

template <typename T, bool ADAM>
__global__ __launch_bounds__(kTailThreads) void restrict_tail_kernel(Levels G, int l_big, int l_small,
                                                                     int nf_big, int cap0, T *g,
                                                                     AdamArgs<T> A, TermSum S,
                                                                     CarryTail<T> H, ColFold<T> Q) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *const sm = reinterpret_cast<T *>(smem_raw);
  // blocks past the (instance, field) ones sum the loss partials of an
  // earlier kernel, one instance each
  const int nfb = G.batch * G.nf * H.parts;
  if ((int)blockIdx.x >= nfb) {
    const int i = blockIdx.x - nfb;
    final_terms(S.partials + (long)i * S.n_part_blocks * kTerms, S.n_a, S.off_b, S.n_b,
                S.terms + (long)i * kTerms, S.flag);
    return;
  }
  const int part = blockIdx.x % H.parts, fi = blockIdx.x / H.parts;
  const int inst = fi / G.nf, f = fi % G.nf;
  const int l_lo = f < nf_big ? l_big : l_small;
  const bool lead = part == 0;  // writes what the parts share
  const int bd = blockDim.x, tid = threadIdx.x;
  const bool carry = ADAM && H.w != nullptr;
  T *const tl = sm + H.toff;  // updated theta of levels l_stop .. L-1 (carry)
  // this field's extents (z, y, x), cell count and pack offset on every level,
  // read once into LDS: the level loops index them by a run-time level, which
  // from the kernel arguments takes a chain of scalar loads per level
  __shared__ int geo[kMaxL][5];
  if (tid < G.L * 5) {
    const int gl = tid / 5, gk = tid - 5 * gl;
    geo[gl][gk] = gk < 3 ? G.n[gl][f][gk] : (gk == 3 ? field_cells(G, gl, f) : field_base(G, gl, inst, f));
  }
  // this part's slice of the largest Horner level
  const int n_stop = carry ? field_cells(G, H.l_stop, f) : 0;
  const int h_lo = (int)((long)n_stop * part / H.parts);
  const int h_hi = (int)((long)n_stop * (part + 1) / H.parts);

  // The levels produced, l_lo+1 .. L-1, hold at most kTailR * blockDim.x
  // values together (the host's choice of l_lo); a thread owns the values
  // tid + u * blockDim.x of their concatenation, and the Adam state of all of
  // them is loaded here, before the block stores anything: a wait for a load
  // issued after a store would also wait for the store.
  T th[kTailR], mo[kTailR], vo[kTailR];
#pragma unroll
  for (int u = 0; u < kTailR; ++u) {
    th[u] = mo[u] = vo[u] = T(0);
    if (!ADAM) continue;
    int e = tid + u * bd;
    for (int j = l_lo + 1; j < G.L; ++j) {
      const int n = field_cells(G, j, f);
      if (e < n) {
        const int k = field_base(G, j, inst, f) + e;
        th[u] = A.th_in[k];
        mo[u] = A.m[k];
        vo[u] = A.v[k];
        break;
      }
      e -= n;
    }
  }
  // level l_lo of g (or its column sums), and the theta of the carried
  // levels l_stop .. l_lo
  const bool fold = Q.gq != nullptr && f == Q.f;
  const int n0 = fold ? field_cells(G, 0, f) : 0, base0 = field_base(G, 0, inst, f);
  T s0 = T(0), th0 = T(0), m0 = T(0), v0 = T(0);
  if (fold) {
    if (tid < n0) {
      if (ADAM) {
        th0 = A.th_in[base0 + tid];
        m0 = A.m[base0 + tid];
        v0 = A.v[base0 + tid];
      }
      const T *src = Q.gq + (long)inst * Q.rows * n0 + tid;
#pragma unroll 8
      for (int r = 0; r < Q.rows; ++r) s0 += src[(long)r * n0];
      sm[tid] = s0;
    }
  } else {
    tail_copy_in(sm, g + field_base(G, l_lo, inst, f), 0, field_cells(G, l_lo, f));
  }
  const int slice = h_hi - h_lo;
  int toff = 0;  // offset in tl of the next level
  if (carry)
    for (int j = H.l_stop; j <= l_lo && j < G.L; ++j) {
      const T *src = A.th_out + field_base(G, j, inst, f);
      if (j == H.l_stop) {
        tail_copy_in(tl, src + h_lo, 0, slice);
        toff = slice;
      } else {
        const int n = field_cells(G, j, f);
        tail_copy_in(tl + toff, src, 0, n);
        toff += n;
      }
    }
  lds_barrier();
  // every load above has returned (vmcnt 0; the other counters left at their
  // maximum), so no wait inside the level loop includes the stores it issues
  __builtin_amdgcn_s_waitcnt(0x0F70);
  if (fold && lead && tid < n0) {
    g[base0 + tid] = s0;
    if (ADAM) adam_elem_loaded(A, base0 + tid, s0, th0, m0, v0);
  }
  T *cur = sm, *oth = sm + cap0;
  int cat = 0;  // offset of level l + 1 in the concatenation
  for (int l = l_lo; l + 1 < G.L; ++l) {
    if (!G.node) {
      // cell-based: T^T one axis at a time (4-6 taps per output and pass)
      int n[3] = {geo[l][0], geo[l][1], geo[l][2]};
      for (int a = 2; a >= 0; --a) {
        const int c = geo[l + 1][a];
        if (c == n[a]) continue;  // the field does not span this axis
        tail_restrict_pass(cur, oth, n, a, c);
        n[a] = c;
        T *t = cur;
        cur = oth;
        oth = t;
        lds_barrier();
      }
    } else {
      // node-based: T^T of every spanned axis at once (3 taps per axis), one
      // LDS phase per level; measured faster than one pass per axis here,
      // while for cell-based fields (up to 6 taps per axis) the passes are
      const int c1 = G.n[l + 1][f][1], c2 = G.n[l + 1][f][2];
      const int total = G.n[l + 1][f][0] * c1 * c2;
      const float r1 = 1.0f / (float)c1, r2 = 1.0f / (float)c2;
      for (int e = tid; e < total; e += bd) {
        int I[3];
        small_index(e, c1, c2, r1, r2, I);
        oth[e] = restrict_value_at(G, l, f, I, cur);
      }
      T *t = cur;
      cur = oth;
      oth = t;
      lds_barrier();
    }
    // cur holds g_{l+1}
    const int base = geo[l + 1][4], nl = geo[l + 1][3];
    const bool keep = carry && l + 1 > H.l_stop, keep_slice = carry && l + 1 == H.l_stop;
#pragma unroll
    for (int u = 0; u < kTailR; ++u) {
      const int e = tid + u * bd - cat;
      if (e < 0 || e >= nl) continue;
      const T val = cur[e];
      if (lead) g[base + e] = val;
      if (ADAM) {
        const T mm = A.b1 * mo[u] + (T(1) - A.b1) * val;
        const T vv = A.b2 * vo[u] + (T(1) - A.b2) * val * val;
        const T tn = adam_theta(th[u], mm, vv, A.step, A.isb2, A.eps);
        if (lead) {
          A.m[base + e] = mm;
          A.v[base + e] = vv;
          A.th_out[base + e] = tn;
        }
        if (keep) tl[toff + e] = tn;
        if (keep_slice && e >= h_lo && e < h_hi) tl[e - h_lo] = tn;
      }
    }
    cat += nl;
    if (keep) toff += nl;
    if (keep_slice) toff = slice;
    // the next level's first pass writes oth, which no thread reads any more
  }
  if (!carry) return;
  lds_barrier();
  // Horner tail; level l > l_stop sits in LDS buffer (l - l_stop - 1) & 1 at
  // the start of the LDS, the restriction's regions being free
  T *const hb0 = sm, *const hb1 = sm + field_cells(G, H.l_stop + 1, f);
  for (int l = G.L - 1; l >= H.l_stop; --l) {
    const bool last = l == H.l_stop;
    const int n = geo[l][3];
    if (!last) toff -= n;  // now the offset of level l in tl
    T *dst = ((l - H.l_stop - 1) & 1) ? hb1 : hb0;  // selects keep them LDS accesses
    const T *cs = ((l - H.l_stop) & 1) ? hb1 : hb0;
    const int base = geo[l][4];
    const bool top = l == G.L - 1;
    const int n1 = geo[l][1], n2 = geo[l][2];
    const float r1 = 1.0f / (float)n1, r2 = 1.0f / (float)n2;
    for (int e = tid + (last ? h_lo : 0); e < (last ? h_hi : n); e += bd) {
      T val = last ? tl[e - h_lo] : tl[toff + e];
      if (!top) {
        int i[3];
        small_index(e, n1, n2, r1, r2, i);
        val += prolong_value_at(G, l, f, i, cs);
        if (last || lead) H.w[base + e] = val;
      }
      if (!last) dst[e] = val;
    }
    if (last) break;
    lds_barrier();
  }
}

// ---------------------------------------------------------------------- Adam
template <typename T>
__global__ __launch_bounds__(kBlock) void adam_kernel(const T *__restrict__ th_in,
                                                      T *__restrict__ th_out, T *__restrict__ m,
                                                      T *__restrict__ v, const T *__restrict__ g,
                                                      long n, T b1, T b2, T step, T inv_sqrt_bc2,
                                                      T eps) {
  const long e = (long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n) return;
  // the same update, in the same form, as Adam fused into the other kernels
  const AdamArgs<T> A{th_in, th_out, m, v, b1, b2, step, inv_sqrt_bc2, eps};
  adam_elem(A, (int)e, g[e]);
}

// ------------------------------------------------------- block-sum of terms
__device__ inline void block_terms(double (&t)[kTerms], double *out) {
  __shared__ double sh[kBlock / 64][kTerms];
  for (int k = 0; k < kTerms; ++k) t[k] = wave_sum(t[k]);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 63)
    for (int k = 0; k < kTerms; ++k) sh[wave][k] = t[k];
  __syncthreads();
  if (threadIdx.x < kTerms) {
    double s = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) s += sh[w][threadIdx.x];
    out[threadIdx.x] = s;
  }
}

// ------------------------------------------------------------ stencil engine
template <typename T>
struct FineArgs {
  OpParams p;
  FineFields ff;
  const T *u;          // [inst][field][cells]
  T *g;                // gradient at the finest level, same layout
  T *gq;               // [inst][grid cells] contributions of the x-only field
  const T *forcing[4]; // [inst][grid cells] or null
  const T *chi;        // [inst][grid cells] or null
  double *partials;    // [inst][n_part_blocks][kTerms]
  long n_part_blocks;
  long ncell;          // cells of the full grid
  int want_grad;
  int xonly_field;     // index of the field spanning x only, or -1
  // prolongation fused into the 2-D tile kernel's staging: with w1 given, u
  // holds theta (level 0 of the pack) and the kernel stages u = theta_0 +
  // T w_1, w1 being level 1 of the prolonged levels (pack layout)
  const T *w1;
  long w1_inst;          // level-1 elements of one instance
  int w1_off[kMaxF];     // field offsets on level 1
  int w1_n[kMaxF][2];    // level-1 values along y and x of each field
  int node;              // node-based T, else cell-based
};

// (T w_1) at fine cell (y, x) of field f of one instance (2-D tiled engine),
// in two steps so that a caller can issue the loads of many cells before it
// uses any: tile_prolong_load fetches the (up to) four coarse values, and
// tile_prolong_sum forms the same taps in the same order as the generic step
// on a grid without z.
template <typename T>
__device__ inline void tile_prolong_taps(const FineArgs<T> &A, int f, int y, int x, int (&ix)[2],
                                         int (&iy)[2], T (&wx)[2], T (&wy)[2]) {
  const bool sy = A.ff.stride[f][1] != 0;  // the field spans y
  iy[0] = iy[1] = 0;
  wy[0] = wy[1] = T(0);
  if (A.node) {
    prolong_taps_node(x, ix, wx);
    if (sy) prolong_taps_node(y, iy, wy);
  } else {
    prolong_taps(x, A.w1_n[f][1], ix, wx);
    if (sy) prolong_taps(y, A.w1_n[f][0], iy, wy);
  }
}

template <typename T>
__device__ inline void tile_prolong_load(const FineArgs<T> &A, int f, int inst, int y, int x,
                                         T (&cv)[4]) {
  const T *c = A.w1 + inst * A.w1_inst + A.w1_off[f];
  const int cnx = A.w1_n[f][1];
  int ix[2], iy[2];
  T wx[2], wy[2];
  tile_prolong_taps(A, f, y, x, ix, iy, wx, wy);
  cv[0] = c[iy[0] * cnx + ix[0]];
  cv[1] = c[iy[0] * cnx + ix[1]];
  if (A.ff.stride[f][1] != 0) {
    cv[2] = c[iy[1] * cnx + ix[0]];
    cv[3] = c[iy[1] * cnx + ix[1]];
  }
}

template <typename T>
__device__ inline T tile_prolong_sum(const FineArgs<T> &A, int f, int y, int x, const T (&cv)[4]) {
  int ix[2], iy[2];
  T wx[2], wy[2];
  tile_prolong_taps(A, f, y, x, ix, iy, wx, wy);
  if (A.ff.stride[f][1] == 0) return wx[0] * cv[0] + wx[1] * cv[1];
  return wy[0] * (wx[0] * cv[0] + wx[1] * cv[1]) + wy[1] * (wx[0] * cv[2] + wx[1] * cv[3]);
}

// ND: the grid's dimension when known at compile time (3 for the 3-D
// kernels, whose slot indices then stay in registers), else 0 (p.ndim)
template <class Op, int ND = 0, typename T>
__device__ inline void load_star(const OpParams &p, const FineFields &ff, const T *ub,
                                 const int (&i)[3], T (&U)[Op::NF][7]) {
  const int a0 = ND ? 3 - ND : 3 - p.ndim;
#pragma unroll
  for (int f = 0; f < Op::NF; ++f) {
    const T *base = ub + ff.off[f];
    const long lin = i[0] * ff.stride[f][0] + i[1] * ff.stride[f][1] + i[2] * ff.stride[f][2];
    const T c = base[lin];
    for (int s = 0; s < 7; ++s) U[f][s] = c;
    if (!Op::needs_nb(f)) continue;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (a < a0) continue;
      const long st = ff.stride[f][a];
      if (st == 0) continue;
      if (i[a] > 0) {
        U[f][slot_m(a)] = base[lin - st];
      } else {
        const GhostRule gr = Op::ghost(p, f, a, 0);
        U[f][slot_m(a)] = T(gr.b2) + T(gr.c0) * c + T(gr.c1) * base[lin + st];
      }
      if (i[a] < p.n[a] - 1) {
        U[f][slot_p(a)] = base[lin + st];
      } else {
        const GhostRule gr = Op::ghost(p, f, a, 1);
        U[f][slot_p(a)] = T(gr.b2) + T(gr.c0) * c + T(gr.c1) * base[lin - st];
      }
    }
  }
}

template <class Op, int ND = 0, typename T>
__device__ inline void fold_ghosts(const OpParams &p, const FineFields &ff, const int (&i)[3],
                                   T (&s)[Op::NF][7]) {
  const int a0 = ND ? 3 - ND : 3 - p.ndim;
#pragma unroll
  for (int f = 0; f < Op::NF; ++f) {
    if (!Op::needs_nb(f)) continue;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (a < a0) continue;
      if (ff.stride[f][a] == 0) continue;
      if (i[a] == 0) {
        const GhostRule gr = Op::ghost(p, f, a, 0);
        const T v = s[f][slot_m(a)];
        s[f][S_C] += T(gr.c0) * v;
        s[f][slot_p(a)] += T(gr.c1) * v;
        s[f][slot_m(a)] = T(0);
      }
      if (i[a] == p.n[a] - 1) {
        const GhostRule gr = Op::ghost(p, f, a, 1);
        const T v = s[f][slot_p(a)];
        s[f][S_C] += T(gr.c0) * v;
        s[f][slot_m(a)] += T(gr.c1) * v;
        s[f][slot_p(a)] = T(0);
      }
    }
  }
}

// residuals (forcing subtracted) and weights at cell j of instance inst
template <class Op, int ND = 0, typename T>
__device__ inline void cell_residual(const FineArgs<T> &A, int inst, const int (&j)[3],
                                     T (&U)[Op::NF][7], T &chi, T (&r)[Op::NE], T (&wv)[Op::NE],
                                     int (&term)[Op::NE]) {
  const long lin = ((long)j[0] * A.p.n[1] + j[1]) * A.p.n[2] + j[2];
  load_star<Op, ND>(A.p, A.ff, A.u + (long)inst * A.ff.inst_stride, j, U);
  chi = A.chi ? A.chi[(long)inst * A.ncell + lin] : T(0);
  Op::eval(A.p, j, inst, U, chi, r, wv, term);
  for (int e = 0; e < Op::NE && e < 4; ++e)
    if (A.forcing[e] && wv[e] != T(0) && (!Op::kForcePdeOnly || term[e] == MODIL_TERM_PDE))
      r[e] -= A.forcing[e][(long)inst * A.ncell + lin];
}

template <class Op, typename T>
__global__ __launch_bounds__(kBlock) void fine_kernel(FineArgs<T> A) {
  const int inst = blockIdx.y;
  const long c = (long)blockIdx.x * kBlock + threadIdx.x;
  double part[kTerms] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (c < A.ncell) {
    int i[3];
    i[2] = (int)(c % A.p.n[2]);
    i[1] = (int)((c / A.p.n[2]) % A.p.n[1]);
    i[0] = (int)(c / ((long)A.p.n[1] * A.p.n[2]));
    T U[Op::NF][7], r[Op::NE], wv[Op::NE], chi;
    int term[Op::NE];
    cell_residual<Op>(A, inst, i, U, chi, r, wv, term);
    for (int e = 0; e < Op::NE; ++e) part[term[e]] += (double)wv[e] * (double)r[e] * (double)r[e];
    if (A.want_grad) {
      T gacc[Op::NF];
      for (int f = 0; f < Op::NF; ++f) gacc[f] = T(0);
      for (int o = 0; o < 7; ++o) {
        int j[3] = {i[0], i[1], i[2]};
        if (o > 0) {
          const int a = (o - 1) >> 1;
          if (a < 3 - A.p.ndim) continue;
          // slot o of cell j refers to c: j = c - offset(o)
          j[a] += (o & 1) ? 1 : -1;
          if (j[a] < 0 || j[a] >= A.p.n[a]) continue;
        }
        T Uj[Op::NF][7], rj[Op::NE], wj[Op::NE], chij, aj[Op::NE];
        int tj[Op::NE];
        cell_residual<Op>(A, inst, j, Uj, chij, rj, wj, tj);
        for (int e = 0; e < Op::NE; ++e) aj[e] = T(2) * wj[e] * rj[e];
        T s[Op::NF][7];
        for (int f = 0; f < Op::NF; ++f)
          for (int q = 0; q < 7; ++q) s[f][q] = T(0);
        Op::vjp(A.p, j, inst, Uj, chij, aj, s);
        fold_ghosts<Op>(A.p, A.ff, j, s);
        for (int f = 0; f < Op::NF; ++f) gacc[f] += s[f][o];
      }
      for (int f = 0; f < Op::NF; ++f) {
        if (f == A.xonly_field)
          A.gq[(long)inst * A.ncell + c] = gacc[f];
        else
          A.g[(long)inst * A.ff.inst_stride + A.ff.off[f] + c] = gacc[f];
      }
    }
  }
  block_terms(part, A.partials + ((long)inst * A.n_part_blocks + blockIdx.x) * kTerms);
}

// ------------------------------------------------ 3-D adjoint in two passes
// fine_kernel forms the residuals of all seven cells of a star for every
// cell, which costs seven times the work of the residuals.  In 3-D the
// adjoint runs in two streaming passes instead:
//   fine_sens_kernel    every cell forms its residuals once (loss partials),
//                       the sensitivities of its weighted residual to the 7
//                       slots of its star (ghost slots folded back), writes the
//                       centre slot to the gradient and the six face slots of
//                       the first nnb fields (those whose neighbours enter the
//                       stencil) to S[face slot - 1][field][inst][cell];
//   fine_gather_kernel  every cell adds the face slots of its six neighbours
//                       that refer to it.
// Same sum as fine_kernel, in another order.
template <class Op, typename T>
__global__ __launch_bounds__(kBlock) void fine_sens_kernel(FineArgs<T> A, T *S, int nnb, int batch) {
  const int inst = blockIdx.y;
  const long c = (long)blockIdx.x * kBlock + threadIdx.x;
  double part[kTerms] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (c < A.ncell) {
    int i[3];
    i[2] = (int)(c % A.p.n[2]);
    i[1] = (int)((c / A.p.n[2]) % A.p.n[1]);
    i[0] = (int)(c / ((long)A.p.n[1] * A.p.n[2]));
    T U[Op::NF][7], r[Op::NE], wv[Op::NE], chi, a[Op::NE];
    int term[Op::NE];
    cell_residual<Op, 3>(A, inst, i, U, chi, r, wv, term);
    for (int e = 0; e < Op::NE; ++e) {
      part[term[e]] += (double)wv[e] * (double)r[e] * (double)r[e];
      a[e] = T(2) * wv[e] * r[e];
    }
    T s[Op::NF][7];
    for (int f = 0; f < Op::NF; ++f)
      for (int q = 0; q < 7; ++q) s[f][q] = T(0);
    Op::vjp(A.p, i, inst, U, chi, a, s);
    fold_ghosts<Op, 3>(A.p, A.ff, i, s);
    const long plane = (long)batch * A.ncell;
    for (int f = 0; f < Op::NF; ++f) {
      A.g[(long)inst * A.ff.inst_stride + A.ff.off[f] + c] = s[f][S_C];
      if (f < nnb)
        for (int o = 1; o < 7; ++o)
          S[((long)(o - 1) * nnb + f) * plane + (long)inst * A.ncell + c] = s[f][o];
    }
  }
  block_terms(part, A.partials + ((long)inst * A.n_part_blocks + blockIdx.x) * kTerms);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void fine_gather_kernel(FineArgs<T> A, const T *S, int nnb,
                                                             int batch) {
  const int inst = blockIdx.y;
  const long c = (long)blockIdx.x * kBlock + threadIdx.x;
  if (c >= A.ncell) return;
  int i[3];
  i[2] = (int)(c % A.p.n[2]);
  i[1] = (int)((c / A.p.n[2]) % A.p.n[1]);
  i[0] = (int)(c / ((long)A.p.n[1] * A.p.n[2]));
  const long st[3] = {(long)A.p.n[1] * A.p.n[2], (long)A.p.n[2], 1};
  const long plane = (long)batch * A.ncell;
  const T *Si = S + (long)inst * A.ncell + c;
  for (int f = 0; f < nnb; ++f) {
    T *gp = A.g + (long)inst * A.ff.inst_stride + A.ff.off[f] + c;
    T acc = *gp;
    for (int ax = 0; ax < 3; ++ax) {
      // slot_m of the cell above refers to c, slot_p of the cell below too
      if (i[ax] + 1 < A.p.n[ax]) acc += Si[((long)(slot_m(ax) - 1) * nnb + f) * plane + st[ax]];
      if (i[ax] > 0) acc += Si[((long)(slot_p(ax) - 1) * nnb + f) * plane - st[ax]];
    }
    *gp = acc;
  }
}

template <class Op, typename T>
static void launch_fine_3d(modil_ctx *c, const FineArgs<T> &A, dim3 grid) {
  const int nnb = sens_fields(c->prob);
  if (!A.want_grad || nnb == 0 || !c->sens_buf || !c->two_pass_enabled) {
    fine_kernel<Op, T><<<grid, kBlock, 0, c->stream>>>(A);
    return;
  }
  T *S = (T *)c->sens_buf;
  fine_sens_kernel<Op, T><<<grid, kBlock, 0, c->stream>>>(A, S, nnb, c->prob.batch);
  fine_gather_kernel<T><<<grid, kBlock, 0, c->stream>>>(A, S, nnb, c->prob.batch);
}

// ------------------------------------------------ 2-D stencil engine by tiles
// A block owns TX x TY cells of one instance.  It stages the fields of its tile
// with a 2-cell halo in LDS; every cell of the tile plus a 1-cell halo forms
// its residuals once (loss partials from the owned cells) and writes the
// sensitivities of its weighted residual to the 7 slots of its star, ghost
// slots folded back, to LDS; every owned cell then sums the slots that refer
// to it.  Same adjoint as fine_kernel (which forms each neighbour's residuals
// again per cell), without atomics.
template <int TX, int TY>
struct FineTile {
  static constexpr int UX = TX + 4, UY = TY + 4;  // staged fields
  static constexpr int SX = TX + 2, SY = TY + 2;  // cells forming residuals
};

// block sum of the loss partials for a block of NT threads (a whole number of waves)
template <int NT>
__device__ inline void block_terms_n(double (&t)[kTerms], double *out) {
  static_assert(NT % 64 == 0 && NT <= 1024, "whole waves");
  __shared__ double sh[NT / 64][kTerms];
  for (int k = 0; k < kTerms; ++k) t[k] = wave_sum(t[k]);
  if ((threadIdx.x & 63) == 63)
    for (int k = 0; k < kTerms; ++k) sh[threadIdx.x >> 6][k] = t[k];
  __syncthreads();
  if (threadIdx.x < kTerms) {
    double sum = 0.0;
    for (int w = 0; w < NT / 64; ++w) sum += sh[w][threadIdx.x];
    out[threadIdx.x] = sum;
  }
}

// star of cell i (2-D) from the staged tile ut ([field][UY][UX], cell at X, Y),
// ghost values at the domain edges as load_star forms them
template <class Op, typename T, int UX, int UY>
__device__ inline void star_from_tile(const OpParams &p, const FineFields &ff, const int (&i)[3],
                                      const T *ut, int X, int Y, T (&U)[Op::NF][7]) {
  for (int f = 0; f < Op::NF; ++f) {
    const T *b = ut + f * UX * UY;
    const T c = b[Y * UX + X];
    for (int q = 0; q < 7; ++q) U[f][q] = c;
    if (!Op::needs_nb(f)) continue;
    for (int a = 1; a < 3; ++a) {
      if (ff.stride[f][a] == 0) continue;
      const int d = a == 2 ? 1 : UX;  // neighbour offset in the tile
      const int k = Y * UX + X;
      if (i[a] > 0) {
        U[f][slot_m(a)] = b[k - d];
      } else {
        const GhostRule gr = Op::ghost(p, f, a, 0);
        U[f][slot_m(a)] = T(gr.b2) + T(gr.c0) * c + T(gr.c1) * b[k + d];
      }
      if (i[a] < p.n[a] - 1) {
        U[f][slot_p(a)] = b[k + d];
      } else {
        const GhostRule gr = Op::ghost(p, f, a, 1);
        U[f][slot_p(a)] = T(gr.b2) + T(gr.c0) * c + T(gr.c1) * b[k - d];
      }
    }
  }
}

// measurements bucketed per (instance, tile): ptr[key] .. ptr[key + 1] index
// rec; lx, ly are the cell's position among the tile's owned cells
struct TileMeas {
  const int32_t *ptr;
  const FusedMeas *rec;
};

// ADAM: also Adam on level 0 of every field spanning the grid (A0: level-0
// pointers of theta_in / theta_out / m / v, the pack layout).  NT threads
// (at least TX * TY): the first TX * TY own one cell each for the gather.
template <class Op, typename T, int TX, int TY, int NT, bool ADAM>
__global__ __launch_bounds__(NT) void fine_tile_kernel(FineArgs<T> A, int tiles_x, TileMeas M,
                                                       AdamArgs<T> A0) {
  using FT = FineTile<TX, TY>;
  constexpr int NF = Op::NF, NE = Op::NE;
  static_assert(NT >= TX * TY, "a thread per owned cell");
  __shared__ T Ut[NF][FT::UY][FT::UX];
  __shared__ T St[NF][7][FT::SY][FT::SX];
  __shared__ T Dt[NF][TY][TX];  // gradient of the data terms at the owned cells
  const int inst = blockIdx.y, tid = threadIdx.x;
  const int x0 = (blockIdx.x % tiles_x) * TX, y0 = (blockIdx.x / tiles_x) * TY;
  const int ny = A.p.n[1], nx = A.p.n[2];
  const T *ub = A.u + (long)inst * A.ff.inst_stride;
  const bool owner = tid < TX * TY;
  const int cx = tid % TX, cy = tid / TX, ox = x0 + cx, oy = y0 + cy;
  const bool own_cell = owner && ox < nx && oy < ny;
  if (owner)
    for (int f = 0; f < NF; ++f) Dt[f][cy][cx] = T(0);
  // Adam state of the owned cell, loaded first so its latency overlaps the
  // residuals
  T ath[NF], am[NF], av[NF];
  for (int f = 0; f < NF; ++f) {
    ath[f] = am[f] = av[f] = T(0);
    if (ADAM && A.want_grad && own_cell && f != A.xonly_field) {
      const long k = (long)inst * A.ff.inst_stride + A.ff.off[f] + (long)oy * nx + ox;
      ath[f] = A0.th_in[k];
      am[f] = A0.m[k];
      av[f] = A0.v[k];
    }
  }
  // Staging: the thread's staged values (and their level-1 taps) are all
  // loaded before any is used, from coordinates clamped into the grid so
  // that every load is in bounds; cells outside the grid then stage zero.
  constexpr int KS = (FT::UX * FT::UY + NT - 1) / NT;
  T sv[KS][NF], cv[KS][NF][4];
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int k = tid + s * NT;
    const int xc = min(max(x0 - 2 + k % FT::UX, 0), nx - 1);
    const int yc = min(max(y0 - 2 + k / FT::UX, 0), ny - 1);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      sv[s][f] = ub[A.ff.off[f] + yc * A.ff.stride[f][1] + xc * A.ff.stride[f][2]];
      if (A.w1) tile_prolong_load(A, f, inst, A.ff.stride[f][1] ? yc : 0, xc, cv[s][f]);
    }
  }
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int k = tid + s * NT;
    if (KS * NT > FT::UX * FT::UY && k >= FT::UX * FT::UY) break;
    const int X = k % FT::UX, Y = k / FT::UX, x = x0 - 2 + X, y = y0 - 2 + Y;
    const bool in = x >= 0 && x < nx && y >= 0 && y < ny;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      T val = T(0);
      if (in) {
        val = sv[s][f];
        if (A.w1) val += tile_prolong_sum(A, f, A.ff.stride[f][1] ? y : 0, x, cv[s][f]);
      }
      Ut[f][Y][X] = val;
    }
  }
  __syncthreads();
  double part[kTerms] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int k = tid; k < FT::SX * FT::SY; k += NT) {
    const int X = k % FT::SX, Y = k / FT::SX, x = x0 - 1 + X, y = y0 - 1 + Y;
    T s[NF][7];
    for (int f = 0; f < NF; ++f)
      for (int q = 0; q < 7; ++q) s[f][q] = T(0);
    if (x >= 0 && x < nx && y >= 0 && y < ny) {
      const int i[3] = {0, y, x};
      T U[NF][7];
      star_from_tile<Op, T, FT::UX, FT::UY>(A.p, A.ff, i, &Ut[0][0][0], X + 1, Y + 1, U);
      const long lin = (long)y * nx + x;
      const T chi = A.chi ? A.chi[(long)inst * A.ncell + lin] : T(0);
      T r[NE], wv[NE];
      int term[NE];
      Op::eval(A.p, i, inst, U, chi, r, wv, term);
      for (int e = 0; e < NE && e < 4; ++e)
        if (A.forcing[e] && wv[e] != T(0) && (!Op::kForcePdeOnly || term[e] == MODIL_TERM_PDE))
          r[e] -= A.forcing[e][(long)inst * A.ncell + lin];
      if (X >= 1 && X <= TX && Y >= 1 && Y <= TY)
        for (int e = 0; e < NE; ++e) part[term[e]] += (double)wv[e] * (double)r[e] * (double)r[e];
      if (A.want_grad) {
        T a[NE];
        for (int e = 0; e < NE; ++e) a[e] = T(2) * wv[e] * r[e];
        Op::vjp(A.p, i, inst, U, chi, a, s);
        fold_ghosts<Op, 2>(A.p, A.ff, i, s);
      }
    }
    if (A.want_grad)
      for (int f = 0; f < NF; ++f)
        for (int q = 0; q < 7; ++q) St[f][q][Y][X] = s[f][q];
  }
  // measurement misfits of the tile's cells (entries of one (field, cell) are
  // adjacent; the first of a run writes their summed gradient)
  {
    const long key = (long)inst * gridDim.x + blockIdx.x;
    const int e0 = M.ptr[key], e1 = M.ptr[key + 1];
    for (int e = e0 + tid; e < e1; e += NT) {
      const FusedMeas me = M.rec[e];
      const T uv = Ut[me.field][me.ly + 2][me.lx + 2];
      const double r = (double)uv - me.val;
      part[me.term] += me.w * r * r;
      if (A.want_grad &&
          (e == e0 || M.rec[e - 1].field != me.field || M.rec[e - 1].cell != me.cell)) {
        double gs = 0.0;
        for (int j = e; j < e1 && M.rec[j].field == me.field && M.rec[j].cell == me.cell; ++j)
          gs += 2.0 * M.rec[j].w * ((double)uv - M.rec[j].val);
        Dt[me.field][me.ly][me.lx] = T(gs);
      }
    }
  }
  if (A.want_grad) {
    __syncthreads();
    const int x = ox, y = oy;
    if (own_cell) {
      T gacc[NF];
      for (int f = 0; f < NF; ++f) gacc[f] = T(0);
      for (int o = 0; o < 7; ++o) {
        int X = cx + 1, Y = cy + 1, jx = x, jy = y;
        if (o > 0) {
          // slot o of cell j refers to this cell: j = this cell - offset(o)
          const int a = (o - 1) >> 1, d = (o & 1) ? 1 : -1;
          if (a == 0) continue;
          if (a == 1) { jy += d; Y += d; } else { jx += d; X += d; }
          if (jy < 0 || jy >= ny || jx < 0 || jx >= nx) continue;
        }
        for (int f = 0; f < NF; ++f) gacc[f] += St[f][o][Y][X];
      }
      const long c = (long)y * nx + x;
      for (int f = 0; f < NF; ++f) {
        const T gf = gacc[f] + Dt[f][cy][cx];
        if (f == A.xonly_field) {
          Dt[f][cy][cx] = gf;  // the cell's own slot, summed over the tile's rows below
        } else {
          const long k = (long)inst * A.ff.inst_stride + A.ff.off[f] + c;
          A.g[k] = gf;
          if (ADAM) adam_elem_loaded(A0, (int)k, gf, ath[f], am[f], av[f]);
        }
      }
    }
    if (A.xonly_field >= 0) {
      // the x-only field's contributions summed over the tile's rows in row
      // order (rows past the grid hold zero): one row of gq per row of tiles,
      // which the restriction tail (or the column-sum kernel) adds up
      __syncthreads();
      if (tid < TX && x0 + tid < nx) {
        T s = T(0);
        for (int r = 0; r < TY; ++r) s += Dt[A.xonly_field][r][tid];
        const int trow = blockIdx.x / tiles_x, trows = gridDim.x / tiles_x;
        A.gq[((long)inst * trows + trow) * nx + x0 + tid] = s;
      }
    }
  }
  block_terms_n<NT>(part, A.partials + ((long)inst * A.n_part_blocks + blockIdx.x) * kTerms);
}

// Column sums of the x-only field's contributions, nt rows of nx (the grid's
// rows of cells, or the tile kernel's sums over each row of tiles): a block
// takes 64 columns of one instance; 16 row groups sum every 16th row, then the
// group sums are added in group order (fixed order: deterministic).
constexpr int kColX = 64, kColY = 16;

template <typename T, bool ADAM>
__global__ __launch_bounds__(kColX * kColY) void colsum_kernel(const T *__restrict__ gq,
                                                               T *__restrict__ g, long inst_stride,
                                                               long foff, int nt, int nx,
                                                               AdamArgs<T> A0) {
  __shared__ T sh[kColY][kColX];
  const int inst = blockIdx.y;
  const int ix = blockIdx.x * kColX + threadIdx.x;
  const long e = (long)inst * inst_stride + foff + ix;
  // the Adam state is loaded with the columns, so both latencies overlap
  T th = T(0), m = T(0), v = T(0);
  if (ADAM && threadIdx.y == 0 && ix < nx) {
    th = A0.th_in[e];
    m = A0.m[e];
    v = A0.v[e];
  }
  T acc = T(0);
  if (ix < nx) {
    const T *src = gq + (long)inst * nt * nx + ix;
#pragma unroll 4
    for (int it = threadIdx.y; it < nt; it += kColY) acc += src[(long)it * nx];
  }
  sh[threadIdx.y][threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.y == 0 && ix < nx) {
    T s = T(0);
    for (int k = 0; k < kColY; ++k) s += sh[k][threadIdx.x];
    g[e] = s;
    if (ADAM) adam_elem_loaded(A0, (int)e, s, th, m, v);  // level 0 of the x-only field
  }
}

// measurement misfits; entries sorted by (instance, field, index, term)
template <typename T>
__global__ __launch_bounds__(kBlock) void data_kernel(
    const T *__restrict__ u, T *__restrict__ g, FineFields ff, const int32_t *__restrict__ ptr,
    const int32_t *__restrict__ fld, const int32_t *__restrict__ idx, const int32_t *__restrict__ trm,
    const double *__restrict__ val, const double *__restrict__ wt, double *partials,
    long n_part_blocks, long first_block, int want_grad, long n_fine, double *terms,
    int32_t *flag) {
  const int inst = blockIdx.y;
  const long b0 = ptr[inst], b1 = ptr[inst + 1];
  const long e = b0 + (long)blockIdx.x * kBlock + threadIdx.x;
  double part[kTerms] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (e < b1) {
    const T *ub = u + (long)inst * ff.inst_stride;
    const int f = fld[e];
    const long k = idx[e];
    const double r = (double)ub[ff.off[f] + k] - val[e];
    part[trm[e]] += wt[e] * r * r;
    const bool first = (e == b0) || fld[e - 1] != f || idx[e - 1] != k;
    if (want_grad && first) {
      double gs = 0.0;
      for (long q = e; q < b1 && fld[q] == f && idx[q] == k; ++q)
        gs += 2.0 * wt[q] * ((double)ub[ff.off[f] + k] - val[q]);
      T *gp = g + (long)inst * ff.inst_stride + ff.off[f] + k;
      *gp = *gp + T(gs);
    }
  }
  double *src = partials + (long)inst * n_part_blocks * kTerms;
  block_terms(part, src + (first_block + blockIdx.x) * kTerms);
  // with one data block per instance (terms given), the block also sums the
  // fine kernel's partials [0, n_fine) (an earlier launch) and its own
  if (terms) {
    __syncthreads();
    final_terms(src, n_fine, first_block, 1, terms + (long)inst * kTerms, flag);
  }
}

// fixed-order sum of the partial blocks [0, n_a) and [off_b, off_b + n_b) of one instance
__global__ __launch_bounds__(kBlock) void reduce_kernel(const double *__restrict__ partials,
                                                        long n_part_blocks, long n_a, long off_b,
                                                        long n_b, double *terms, int32_t *flag) {
  final_terms(partials + (long)blockIdx.x * n_part_blocks * kTerms, n_a, off_b, n_b,
              terms + (long)blockIdx.x * kTerms, flag);
}

__global__ void metric_kernel(const double *terms, double *r, int batch, double scale) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < batch) r[b] = sqrt(fmax(terms[(long)b * kTerms + MODIL_TERM_PDE], 0.0) * scale);
}

// -------------------------------------------------------------- launchers
static inline unsigned nblk(long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

Levels levels_of(const modil_ctx *c) {
  Levels G{};
  G.L = c->prob.n_levels;
  G.nf = c->lay.n_fields;
  G.batch = c->prob.batch;
  G.node = c->prob.centering == MODIL_NODE ? 1 : 0;
  for (int l = 0; l < G.L; ++l) {
    G.off[l] = (int)c->lay.level_offset[l];
    G.stride[l] = (int)c->lay.level_stride[l];
    for (int f = 0; f < G.nf; ++f) {
      G.foff[l][f] = (int)c->lay.field_offset[l][f];
      for (int a = 0; a < 3; ++a) G.n[l][f][a] = c->lay.field_dims[l][f][a];
    }
  }
  return G;
}

static long field_size(const Levels &G, int l, int f) {
  return (long)G.n[l][f][0] * G.n[l][f][1] * G.n[l][f][2];
}

// Largest per-field cell count of level l
static long max_field(const Levels &G, int l) {
  long m = 0;
  for (int f = 0; f < G.nf; ++f) m = std::max(m, field_size(G, l, f));
  return m;
}

// The restriction tail gives the small coarse levels one block per field and
// instance.  tail_level returns the smallest level l >= lo whose two LDS
// regions (level l's size each, for the one-axis passes) fit the budget and
// below which a block produces at most `cap` values, L - 1 if there is none.
static int tail_level(const Levels &G, int lo, size_t elem, size_t budget, long cap) {
  for (int l = lo; l + 1 < G.L; ++l) {
    long work = 0;
    for (int f = 0; f < G.nf; ++f) {
      long wf = 0;
      for (int j = l + 1; j < G.L; ++j) wf += field_size(G, j, f);
      work = std::max(work, wf);
    }
    if ((size_t)2 * max_field(G, l) * elem <= budget && work <= cap) return l;
  }
  return G.L - 1;
}

constexpr long kTailCapRestrict = (long)kTailR * kTailThreads;  // values one block restricts

template <typename K>
static bool lds_ready(K kernel, size_t bytes) {
  if (bytes <= 64 * 1024) return true;
  return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess;
}

// The Horner tail of the small levels (horner_tail_kernel, or carried by the
// restriction tail): levels L-1 .. l_stop, the largest split over `parts`
// blocks per field.  The lowest level l_stop >= 1 (below L - 1) whose part
// holds at most kCarrySlice values, with at most kCarryAbove values in the
// levels above it (every part computes those), whose two LDS buffers of level
// l_stop + 1 fit.  Both uses take the same plan, so they compute every level
// with the same function.
struct HornerPlan {
  int l_stop = 0, parts = 1;
  long slice = 0, above = 0;  // per part: values of level l_stop; values above it
  size_t hbytes = 0;          // LDS of the two buffers
};
constexpr long kCarrySlice = 4096;
constexpr long kCarryAbove = 2048;  // measured: a full 16^3 level in every part costs more than a launch
constexpr int kCarryParts = 16;

static bool horner_plan(const modil_ctx *c, const Levels &G, size_t elem, HornerPlan &P) {
  if (!c->tail_enabled) return false;
  for (int l = 1; l <= G.L - 2; ++l) {
    const long n_stop = max_field(G, l);
    const int parts = (int)std::min<long>(kCarryParts, std::max<long>(1, (n_stop + 511) / 512));
    const long slice = (n_stop + parts - 1) / parts;
    long above = 0;
    for (int f = 0; f < G.nf; ++f) {
      long n = 0;
      for (int j = l + 1; j < G.L; ++j) n += field_size(G, j, f);
      above = std::max(above, n);
    }
    const size_t hbytes = (size_t)2 * max_field(G, l + 1) * elem;
    if (slice > kCarrySlice || above > kCarryAbove || hbytes + 1024 > c->lds_budget) continue;
    P.l_stop = l;
    P.parts = parts;
    P.slice = slice;
    P.above = above;
    P.hbytes = hbytes;
    return true;
  }
  return false;
}

// skip_tail: the Horner tail for theta is already in w_buf (carried by the
// previous iteration's restriction tail)
template <typename T>
static hipError_t horner_t(modil_ctx *c, const void *theta_v, void *fine_dst_v, bool skip_fine,
                           bool skip_tail) {
  const Levels G = levels_of(c);
  const T *theta = (const T *)theta_v;
  T *w = (T *)c->w_buf;
  T *fine_dst = fine_dst_v ? (T *)fine_dst_v : w;
  if (G.L == 1) return hipSuccess;
  int l = G.L - 2;
  HornerPlan hp;
  if (skip_tail) {
    l = c->carry_stop - 1;  // w_{L-2} .. w_{carry_stop} came with the restriction tail
  } else if (horner_plan(c, G, sizeof(T), hp) && lds_ready(horner_tail_kernel<T>, hp.hbytes)) {
    horner_tail_kernel<T><<<G.batch * G.nf * hp.parts, 1024, hp.hbytes, c->stream>>>(
        G, hp.l_stop, hp.parts, theta, w);
    l = hp.l_stop - 1;
  }
  const int l_end = skip_fine ? 1 : 0;
  for (; l >= l_end; --l) {
    const T *src = (l == G.L - 2) ? theta + G.off[l + 1] : w + G.off[l + 1];
    // two steps at once where the levels admit it (w_l is then never written)
    if (l - 1 >= l_end && c->march_enabled &&
        launch_prolong2<T>(G, l - 1, theta + G.off[l - 1], theta + G.off[l], src,
                           (l - 1 == 0) ? fine_dst : w + G.off[l - 1], c->stream)) {
      --l;
      continue;
    }
    T *dst = (l == 0) ? fine_dst : w + G.off[l];
    if (c->march_enabled && launch_prolong_block<T>(G, l, theta + G.off[l], src, dst, c->stream))
      continue;
    if (c->march_enabled && launch_prolong_node<T>(G, l, theta + G.off[l], src, dst, c->stream))
      continue;
    const long total = (long)G.stride[l] * G.batch;
    prolong_kernel<T><<<nblk(total), kBlock, 0, c->stream>>>(G, l, theta, src, dst);
  }
  return hipGetLastError();
}

hipError_t launch_horner(modil_ctx *c, const void *theta, void *fine_dst, bool skip_fine,
                         bool skip_tail) {
  return c->prob.dtype == MODIL_F64 ? horner_t<double>(c, theta, fine_dst, skip_fine, skip_tail)
                                    : horner_t<float>(c, theta, fine_dst, skip_fine, skip_tail);
}

template <typename T>
static hipError_t restrict_t(modil_ctx *c, void *g_v, int from, const void *th_in, void *th_out,
                             void *m, void *v, const AdamHost *ad, const TermSum *sum,
                             bool *summed, bool carry, bool *carried, bool colsum) {
  if (summed) *summed = false;
  if (carried) *carried = false;
  const Levels G = levels_of(c);
  T *g = (T *)g_v;
  AdamArgs<T> A{};
  if (ad) {
    A.th_in = (const T *)th_in; A.th_out = (T *)th_out; A.m = (T *)m; A.v = (T *)v;
    A.b1 = T(ad->b1); A.b2 = T(ad->b2); A.step = T(ad->step); A.isb2 = T(ad->isb2); A.eps = T(ad->eps);
  }
  // levels lt+1 .. L-1 come from one launch of the LDS tail kernel
  // (less 1 KB of the LDS budget for the kernel's static arrays)
  int lt = c->tail_enabled
               ? tail_level(G, from, sizeof(T), c->lds_budget - 1024, kTailCapRestrict)
               : G.L - 1;
  int cap0 = lt + 1 < G.L ? (int)max_field(G, lt) : 0;
  // Fields past a leading group of one shape that are small enough to start
  // the tail at level `from` (the heat problem's 1-D q beside its 2-D u):
  // the marching kernel then restricts the leading group alone, levels
  // from .. lt-1, where mixed shapes would take the per-cell kernel.  Taken
  // only when the marching kernel applies at every one of those levels.
  int nf_big = G.nf;
  Levels Gb = G;
  if (c->march_enabled && lt > from && lt + 1 < G.L) {
    int k = 1;
    while (k < G.nf && G.n[from][k][0] == G.n[from][0][0] && G.n[from][k][1] == G.n[from][0][1] &&
           G.n[from][k][2] == G.n[from][0][2])
      ++k;
    bool ok = k < G.nf;
    long cap_small = 0;
    for (int f = k; ok && f < G.nf; ++f) {
      long work = 0;
      for (int j = from + 1; j < G.L; ++j) work += field_size(G, j, f);
      cap_small = std::max(cap_small, field_size(G, from, f));
      ok = work <= kTailCapRestrict;
    }
    Gb.nf = k;
    for (int l = from; ok && l < lt; ++l) ok = restrict_march_applies(Gb, l, g, sizeof(T), c->march_tile);
    if (ok) {
      nf_big = k;
      cap0 = (int)std::max<long>(cap0, cap_small);
    }
  }
  const size_t bytes = (size_t)2 * cap0 * sizeof(T);
  if (lt + 1 < G.L && !(ad ? lds_ready(restrict_tail_kernel<T, true>, bytes)
                          : lds_ready(restrict_tail_kernel<T, false>, bytes))) {
    lt = G.L - 1;
    nf_big = G.nf;
  }
  const int l_small = nf_big < G.nf ? from : lt;
  // the x-only field's column sums (and its level-0 Adam): in the tail when
  // that field starts there at level 0, else by their own launch first
  ColFold<T> Q;
  if (colsum) {
    int xf = -1;
    for (int f = 0; f < G.nf; ++f)
      if (field_is_x_only(c->prob, f)) xf = f;
    const int start = xf >= nf_big ? l_small : lt;
    if (xf >= 0 && from == 0 && start == 0 && lt + 1 < G.L && field_size(G, 0, xf) <= kTailThreads &&
        field_size(G, 0, xf) <= cap0) {
      Q.gq = (const T *)c->gq_buf;
      Q.rows = c->gq_rows;
      Q.f = xf;
    } else {
      const hipError_t e = launch_colsum(c, g_v, ad, th_in, th_out, m, v);
      if (e != hipSuccess) return e;
    }
  }
  for (int l = from; l + 1 < G.L && l < lt; ++l) {
    if (nf_big < G.nf) {
      // checked above: applies at every level of the range
      launch_restrict_march<T>(Gb, l, g, A, ad != nullptr, c->march_tile, c->stream);
      continue;
    }
    if (c->march_enabled &&
        launch_restrict_march<T>(G, l, g, A, ad != nullptr, c->march_tile, c->stream))
      continue;
    if (c->march_enabled && launch_restrict_march_node<T>(G, l, g, A, ad != nullptr, c->stream))
      continue;
    const long total = (long)G.stride[l + 1] * G.batch;
    if (ad)
      restrict_kernel<T, true><<<nblk(total), kBlock, 0, c->stream>>>(G, l, g, A);
    else
      restrict_kernel<T, false><<<nblk(total), kBlock, 0, c->stream>>>(G, l, g, A);
  }
  if (lt + 1 < G.L) {
    const TermSum S = sum ? *sum : TermSum{};
    // carry the next iteration's Horner tail when its LDS fits beside
    CarryTail<T> H;
    size_t lds = bytes;
    HornerPlan hp;
    if (carry && ad && horner_plan(c, G, sizeof(T), hp)) {
      // LDS: the restriction's regions or the Horner buffers, then the theta
      // of the part's slice of l_stop and of the levels above
      const size_t toff = (std::max(bytes, hp.hbytes) + 15) / 16 * 16 / sizeof(T);
      const size_t lds_c = (toff + (size_t)(hp.slice + hp.above)) * sizeof(T);
      if (lds_c + 1024 <= c->lds_budget && lds_ready(restrict_tail_kernel<T, true>, lds_c)) {
        H.w = (T *)c->w_buf;
        H.l_stop = hp.l_stop;
        H.toff = (int)toff;
        H.parts = hp.parts;
        lds = lds_c;
        c->carry_stop = hp.l_stop;
        if (carried) *carried = true;
      }
    }
    const int blocks = G.batch * G.nf * H.parts + (sum ? G.batch : 0);
    if (ad)
      restrict_tail_kernel<T, true><<<blocks, kTailThreads, lds, c->stream>>>(G, lt, l_small, nf_big, cap0,
                                                                             g, A, S, H, Q);
    else
      restrict_tail_kernel<T, false><<<blocks, kTailThreads, lds, c->stream>>>(G, lt, l_small, nf_big, cap0,
                                                                              g, A, S, H, Q);
    if (summed) *summed = sum != nullptr;
  }
  return hipGetLastError();
}

hipError_t launch_restrict_chain(modil_ctx *c, void *g, int from, const void *th_in, void *th_out,
                                 void *m, void *v, const AdamHost *adam, const TermSum *sum,
                                 bool *summed, bool carry, bool *carried, bool colsum) {
  return c->prob.dtype == MODIL_F64
             ? restrict_t<double>(c, g, from, th_in, th_out, m, v, adam, sum, summed, carry, carried, colsum)
             : restrict_t<float>(c, g, from, th_in, th_out, m, v, adam, sum, summed, carry, carried, colsum);
}

hipError_t launch_adam(modil_ctx *c, const void *th_in, void *th_out, void *m, void *v,
                       const void *g, long n, const AdamHost &h) {
  if (c->prob.dtype == MODIL_F64) {
    adam_kernel<double><<<nblk(n), kBlock, 0, c->stream>>>(
        (const double *)th_in, (double *)th_out, (double *)m, (double *)v, (const double *)g, n,
        h.b1, h.b2, h.step, h.isb2, h.eps);
  } else {
    adam_kernel<float><<<nblk(n), kBlock, 0, c->stream>>>(
        (const float *)th_in, (float *)th_out, (float *)m, (float *)v, (const float *)g, n,
        (float)h.b1, (float)h.b2, (float)h.step, (float)h.isb2, (float)h.eps);
  }
  return hipGetLastError();
}

template <typename T>
static FineArgs<T> fine_args(modil_ctx *c, const void *u, void *g, bool want_grad) {
  FineArgs<T> A{};
  const modil_problem &P = c->prob;
  OpParams &p = A.p;
  p.ndim = (P.op == MODIL_OP_POISSON) ? P.ndim : (P.op == MODIL_OP_NS3D ? 3 : 2);
  for (int a = 0; a < 3; ++a) { p.n[a] = 1; p.h[a] = 1.0; }
  const int extra = P.centering == MODIL_NODE ? 1 : 0;  // nodes: one more value per axis
  for (int k = 0; k < P.ndim; ++k) {
    const int a = 3 - P.ndim + k;
    p.n[a] = P.dims[k] + extra;
    p.h[a] = P.lengths[k] / P.dims[k];
  }
  p.V = 1.0;
  for (int a = 3 - p.ndim; a < 3; ++a) p.V *= p.h[a];
  p.w_pde = P.w_pde; p.w_reg = P.w_reg; p.w_bc = P.w_bc;
  p.re = P.re; p.diam = P.diam; p.lam = P.lambda_; p.chi_shift = P.chi_shift;
  p.tau_coef = P.tau_coef; p.u_ref = P.u_ref;
  p.inst_re = c->inst_re;
  FineFields &ff = A.ff;
  ff.nf = c->lay.n_fields;
  ff.inst_stride = c->lay.level_stride[0];
  A.xonly_field = -1;
  for (int f = 0; f < ff.nf; ++f) {
    ff.off[f] = c->lay.field_offset[0][f];
    const FieldGeom fg = field_geom(P, 0, f);
    for (int a = 0; a < 3; ++a) ff.stride[f][a] = (fg.n[a] == 1 && p.n[a] != 1) ? 0 : fg.stride[a];
    if (field_is_x_only(P, f)) A.xonly_field = f;
  }
  A.u = (const T *)u;
  A.g = (T *)g;
  A.gq = (T *)c->gq_buf;
  for (int e = 0; e < 4; ++e) A.forcing[e] = (const T *)c->forcing[e];
  A.chi = (const T *)c->chi;
  A.partials = c->partials;
  A.n_part_blocks = c->n_part_blocks;
  A.ncell = c->lay.fine_cells;
  A.want_grad = want_grad ? 1 : 0;
  return A;
}

void fine_2d(const modil_problem &P, int &ny, int &nx) {
  const int extra = P.centering == MODIL_NODE ? 1 : 0;
  ny = P.dims[0] + extra;
  nx = P.dims[1] + extra;
}

bool fine_is_2d(const modil_problem &P) {
  return P.op == MODIL_OP_BURGERS || P.op == MODIL_OP_HEAT_KX || P.op == MODIL_OP_CAVITY ||
         (P.op == MODIL_OP_POISSON && P.ndim == 2);
}

void fine_tile_shape(const modil_problem &P, int &tx, int &ty, int &tiles_x, int &tiles_y) {
  int ny, nx;
  fine_2d(P, ny, nx);
  tx = 32;
  ty = 8;
  tiles_x = (nx + tx - 1) / tx;
  tiles_y = (ny + ty - 1) / ty;
  if ((long)tiles_x * tiles_y * P.batch < 256) {
    tx = 16;
    ty = 4;
    tiles_x = (nx + tx - 1) / tx;
    tiles_y = (ny + ty - 1) / ty;
  }
}

int sens_fields(const modil_problem &P) {
  if (P.op == MODIL_OP_NS3D) return 4;  // u, v, w, p (chihat enters at the centre only)
  if (P.op == MODIL_OP_POISSON && P.ndim == 3) return 1;
  return 0;
}

bool two_pass_adjoint(const modil_problem &P) {
  if (sens_fields(P) == 0) return false;
  return !(P.op == MODIL_OP_NS3D && P.centering == MODIL_CELL && P.dtype == MODIL_F32);
}

long fine_partial_slots(const modil_problem &P) {
  long cells = 1;
  for (int k = 0; k < P.ndim; ++k) cells *= P.dims[k] + (P.centering == MODIL_NODE ? 1 : 0);
  long slots = (cells + kBlock - 1) / kBlock;
  if (fine_is_2d(P)) {
    int ny, nx;
    fine_2d(P, ny, nx);
    slots = std::max(slots, (long)((nx + 15) / 16) * ((ny + 3) / 4));  // the smaller tile
  }
  return slots;
}

template <typename T>
static AdamArgs<T> adam_args(const AdamHost *ad, const void *th_in, void *th_out, void *m, void *v) {
  AdamArgs<T> A{};
  if (ad) {
    A.th_in = (const T *)th_in; A.th_out = (T *)th_out; A.m = (T *)m; A.v = (T *)v;
    A.b1 = T(ad->b1); A.b2 = T(ad->b2); A.step = T(ad->step); A.isb2 = T(ad->isb2); A.eps = T(ad->eps);
  }
  return A;
}

// the tiled engine for one operator (tile shape from fine_tile_shape)
template <class Op, typename T>
static void launch_fine_tile(modil_ctx *c, const FineArgs<T> &A, const AdamArgs<T> &A0, bool adam) {
  int tx, ty, nbx, nby;
  fine_tile_shape(c->prob, tx, ty, nbx, nby);
  c->fine_slots = (long)nbx * nby;
  c->gq_rows = nby;  // the x-only field's contributions come summed per row of tiles
  const TileMeas M{c->tm_ptr, c->tm_rec};
  const dim3 grid(nbx * nby, c->prob.batch);
  // residuals are formed on the tile plus a one-cell ring (34 x 10, 18 x 6
  // cells): six and two waves take them in one pass
  if (tx == 32) {
    if (adam) fine_tile_kernel<Op, T, 32, 8, 384, true><<<grid, 384, 0, c->stream>>>(A, nbx, M, A0);
    else fine_tile_kernel<Op, T, 32, 8, 384, false><<<grid, 384, 0, c->stream>>>(A, nbx, M, A0);
  } else {
    if (adam) fine_tile_kernel<Op, T, 16, 4, 128, true><<<grid, 128, 0, c->stream>>>(A, nbx, M, A0);
    else fine_tile_kernel<Op, T, 16, 4, 128, false><<<grid, 128, 0, c->stream>>>(A, nbx, M, A0);
  }
}

template <typename T>
static hipError_t launch_fine_t(modil_ctx *c, const void *u, void *g, bool want_grad,
                                const AdamHost *adam, const void *th_in, void *th_out, void *m,
                                void *v, bool prolong) {
  FineArgs<T> A = fine_args<T>(c, u, g, want_grad);
  if (prolong && c->prob.n_levels > 1) {
    // u is theta; level 1 of the prolonged levels is theta's own when L = 2
    const T *wb = c->prob.n_levels == 2 ? (const T *)u : (const T *)c->w_buf;
    A.w1 = wb + c->lay.level_offset[1];
    A.w1_inst = c->lay.level_stride[1];
    A.node = c->prob.centering == MODIL_NODE;
    for (int f = 0; f < c->lay.n_fields; ++f) {
      A.w1_off[f] = (int)c->lay.field_offset[1][f];
      const FieldGeom g1 = field_geom(c->prob, 1, f);
      A.w1_n[f][0] = g1.n[1];
      A.w1_n[f][1] = g1.n[2];
    }
  }
  const AdamArgs<T> A0 = adam_args<T>(adam, th_in, th_out, m, v);
  const bool ad = adam != nullptr;
  const dim3 grid(nblk(A.ncell), c->prob.batch);
  const modil_problem &P = c->prob;
  c->fine_slots = nblk(A.ncell);
  c->gq_rows = P.dims[0];  // per-cell contributions (the tile launcher sets its own)
  if (fine_uses_tiles(c)) {
    switch (P.op) {
      case MODIL_OP_POISSON:
        if (P.centering == MODIL_NODE) launch_fine_tile<OpPoissonNode, T>(c, A, A0, ad);
        else launch_fine_tile<OpPoisson, T>(c, A, A0, ad);
        break;
      case MODIL_OP_BURGERS: launch_fine_tile<OpBurgers, T>(c, A, A0, ad); break;
      case MODIL_OP_HEAT_KX: launch_fine_tile<OpHeat, T>(c, A, A0, ad); break;
      case MODIL_OP_CAVITY:
        if (P.centering == MODIL_NODE) launch_fine_tile<OpCavityNode, T>(c, A, A0, ad);
        else launch_fine_tile<OpNS<2, 0>, T>(c, A, A0, ad);
        break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  if (ad) return hipErrorInvalidValue;  // the per-cell kernel has no Adam
  switch (P.op) {
    case MODIL_OP_POISSON:
      if (P.centering == MODIL_NODE)
        launch_fine_3d<OpPoissonNode, T>(c, A, grid);
      else
        launch_fine_3d<OpPoisson, T>(c, A, grid);
      break;
    case MODIL_OP_BURGERS:
      fine_kernel<OpBurgers, T><<<grid, kBlock, 0, c->stream>>>(A);
      break;
    case MODIL_OP_HEAT_KX:
      fine_kernel<OpHeat, T><<<grid, kBlock, 0, c->stream>>>(A);
      break;
    case MODIL_OP_NS3D:
      if (P.centering == MODIL_NODE) {
        if (P.flags & MODIL_FLAG_CHI_FIXED)
          launch_fine_3d<OpChannelNode<1>, T>(c, A, grid);
        else
          launch_fine_3d<OpChannelNode<2>, T>(c, A, grid);
      } else if (P.flags & MODIL_FLAG_CHI_FIXED) {
        launch_fine_3d<OpNS<3, 1>, T>(c, A, grid);
      } else {
        launch_fine_3d<OpNS<3, 2>, T>(c, A, grid);
      }
      break;
    case MODIL_OP_CAVITY:
      if (P.centering == MODIL_NODE)
        fine_kernel<OpCavityNode, T><<<grid, kBlock, 0, c->stream>>>(A);
      else
        fine_kernel<OpNS<2, 0>, T><<<grid, kBlock, 0, c->stream>>>(A);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

bool fine_uses_tiles(const modil_ctx *c) { return c->tile_enabled && fine_is_2d(c->prob); }

hipError_t launch_fine(modil_ctx *c, const void *u, void *g, bool want_grad, const AdamHost *adam,
                       const void *th_in, void *th_out, void *m, void *v, bool prolong) {
  return c->prob.dtype == MODIL_F64
             ? launch_fine_t<double>(c, u, g, want_grad, adam, th_in, th_out, m, v, prolong)
             : launch_fine_t<float>(c, u, g, want_grad, adam, th_in, th_out, m, v, prolong);
}

hipError_t launch_colsum(modil_ctx *c, void *g_fine, const AdamHost *adam, const void *th_in,
                         void *th_out, void *m, void *v) {
  int xf = -1;
  for (int f = 0; f < c->lay.n_fields; ++f)
    if (field_is_x_only(c->prob, f)) xf = f;
  if (xf < 0) return hipSuccess;
  const int nt = c->gq_rows, nx = c->prob.dims[1];
  const dim3 grid((nx + kColX - 1) / kColX, c->prob.batch), block(kColX, kColY);
  const long st = c->lay.level_stride[0], fo = c->lay.field_offset[0][xf];
  if (c->prob.dtype == MODIL_F64) {
    const AdamArgs<double> A0 = adam_args<double>(adam, th_in, th_out, m, v);
    if (adam)
      colsum_kernel<double, true><<<grid, block, 0, c->stream>>>(
          (const double *)c->gq_buf, (double *)g_fine, st, fo, nt, nx, A0);
    else
      colsum_kernel<double, false><<<grid, block, 0, c->stream>>>(
          (const double *)c->gq_buf, (double *)g_fine, st, fo, nt, nx, A0);
  } else {
    const AdamArgs<float> A0 = adam_args<float>(adam, th_in, th_out, m, v);
    if (adam)
      colsum_kernel<float, true><<<grid, block, 0, c->stream>>>(
          (const float *)c->gq_buf, (float *)g_fine, st, fo, nt, nx, A0);
    else
      colsum_kernel<float, false><<<grid, block, 0, c->stream>>>(
          (const float *)c->gq_buf, (float *)g_fine, st, fo, nt, nx, A0);
  }
  return hipGetLastError();
}

hipError_t launch_data(modil_ctx *c, const void *u, void *g, bool want_grad, double *terms,
                       bool &summed) {
  const long n_fine = c->fine_slots;
  summed = c->n_data_blocks == 1;
  if (!summed) terms = nullptr;
  FineFields ff{};
  ff.nf = c->lay.n_fields;
  ff.inst_stride = c->lay.level_stride[0];
  for (int f = 0; f < ff.nf; ++f) ff.off[f] = c->lay.field_offset[0][f];
  const dim3 grid((unsigned)c->n_data_blocks, c->prob.batch);
  if (c->prob.dtype == MODIL_F64)
    data_kernel<double><<<grid, kBlock, 0, c->stream>>>(
        (const double *)u, (double *)g, ff, c->m_inst_ptr, c->m_field, c->m_idx, c->m_term,
        c->m_val, c->m_w, c->partials, c->n_part_blocks, c->n_fine_blocks, want_grad ? 1 : 0,
        n_fine, terms, c->flag);
  else
    data_kernel<float><<<grid, kBlock, 0, c->stream>>>(
        (const float *)u, (float *)g, ff, c->m_inst_ptr, c->m_field, c->m_idx, c->m_term,
        c->m_val, c->m_w, c->partials, c->n_part_blocks, c->n_fine_blocks, want_grad ? 1 : 0,
        n_fine, terms, c->flag);
  return hipGetLastError();
}

hipError_t launch_reduce(modil_ctx *c, double *terms, long n_a, long off_b, long n_b) {
  reduce_kernel<<<c->prob.batch, kBlock, 0, c->stream>>>(c->partials, c->n_part_blocks, n_a, off_b,
                                                         n_b, terms, c->flag);
  return hipGetLastError();
}

hipError_t launch_metric(modil_ctx *c, const double *terms, double *r) {
  const modil_problem &P = c->prob;
  double V = 1.0;
  for (int k = 0; k < P.ndim; ++k) V *= P.lengths[k] / P.dims[k];
  // points carrying the PDE equations: every cell; the interior nodes of
  // node-based grids; the inner points n >= 1, 1 <= i <= N - 2 of space-time grids
  double rows = (double)c->lay.fine_cells;
  if (P.centering == MODIL_NODE) {
    rows = 1.0;
    for (int k = 0; k < P.ndim; ++k) rows *= P.dims[k] - 1;
  } else if (P.op == MODIL_OP_BURGERS || P.op == MODIL_OP_HEAT_KX) {
    rows = (double)(P.dims[0] - 1) * (double)(P.dims[1] - 2);
  }
  const double scale = V / (P.w_pde * (double)op_pde_equations(P) * rows);
  metric_kernel<<<(P.batch + 63) / 64, 64, 0, c->stream>>>(terms, r, P.batch, scale);
  return hipGetLastError();
}

}  // namespace modil
