// Marching restriction with Adam: g_{l+1} = T^T g_l on one level, followed by
// Adam on the level-(l+1) parameters, for fields that span every axis they
// have (Section 2.2: T is the tensor product of the 1-D cell-based
// interpolation, so T^T is applied one axis at a time).
//
// A wave owns a run of coarse cells along x (one lane per coarse cell, up to
// 64 per row; narrower rows pack several row groups into a wave), YR coarse
// rows and ZR coarse planes.  Each fine value is loaded once per wave:
//   x  a lane loads its two fine cells 2J, 2J+1 as one vector load and takes
//      the neighbours 2J-1, 2J+2 (and the extrapolated end cells) from the
//      adjacent lanes by DPP wave shifts;
//   y  the fine rows of a plane are scattered into the YR coarse rows with the
//      weights of T (each fine row feeds two coarse rows);
//   z  the wave marches through the fine planes two at a time; a fine plane
//      feeds the previous, current and next coarse plane accumulators, and the
//      previous one is complete once both planes of a step are in.
// The loads of both planes of a step are issued before any of them is used.
// Every address is a wave-uniform base (the wave's task is read into scalar
// registers) plus a 32-bit byte offset per lane.  Summation order is fixed,
// so results are deterministic.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "multigrid.h"

namespace modil {

template <typename T> struct Pair;
template <> struct Pair<float> { using type = float2; };
template <> struct Pair<double> { using type = double2; };

constexpr int kMarchWaves = 4;  // waves per block

struct MarchPlan {
  int W;          // lanes per coarse row (min(64, coarse nx))
  int wshift;     // log2(W)
  int groups;     // row groups per wave (64 / W)
  int nseg;       // 64-lane segments per coarse row (coarse nx / 64, or 1)
  int nyc, nzc;   // y and z chunks
  int n_tasks;    // waves with work
};

// One fine row of a plane: the lane's two cells and, with SEG, the cell just
// outside the lane's 64-wide segment (the first lane takes the one to its
// left, the last lane the one to its right; the others reload their own
// cell, in the same cache line).
template <typename T, bool SEG>
struct RowLoad {
  T a, b, e;
};

// Loads address a wave-uniform base plus a 32-bit byte offset per lane.
template <typename T>
__device__ inline T ld_off(const T *base, uint32_t byte_off) {
  return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte_off);
}
template <typename T>
__device__ inline void st_off(T *base, uint32_t byte_off, T v) {
  *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + byte_off) = v;
}

template <typename T, bool SEG>
__device__ inline RowLoad<T, SEG> load_row(const T *base, uint32_t off, uint32_t eoff) {
  using P2 = typename Pair<T>::type;
  RowLoad<T, SEG> v;
  const P2 ab = ld_off(reinterpret_cast<const P2 *>(base), off);
  v.a = ab.x;
  v.b = ab.y;
  v.e = SEG ? ld_off(base, eoff) : T(0);
  return v;
}

// The value of the lane below (wave_prev: lane i gets lane i - 1) or above
// (wave_next: lane i gets lane i + 1) by a DPP wave shift, an operand
// modifier of a VALU move with no LDS round trip.  The first (last) lane
// keeps its own value; callers never use it there.  Every lane of the wave
// must be active.
__device__ inline uint32_t dpp_prev(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x138, 0xf, 0xf, false);  // wave_shr:1
}
__device__ inline uint32_t dpp_next(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x130, 0xf, 0xf, false);  // wave_shl:1
}
__device__ inline float wave_prev(float v) { return __uint_as_float(dpp_prev(__float_as_uint(v))); }
__device__ inline float wave_next(float v) { return __uint_as_float(dpp_next(__float_as_uint(v))); }
__device__ inline double wave_prev(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned long long r = (unsigned long long)dpp_prev((uint32_t)u) |
                               ((unsigned long long)dpp_prev((uint32_t)(u >> 32)) << 32);
  return __longlong_as_double((long long)r);
}
__device__ inline double wave_next(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned long long r = (unsigned long long)dpp_next((uint32_t)u) |
                               ((unsigned long long)dpp_next((uint32_t)(u >> 32)) << 32);
  return __longlong_as_double((long long)r);
}

// Column value (T^T along x) of one row: every lane executes the shifts.  A
// row group of W < 64 lanes takes its neighbours from within the group: the
// lanes whose shifted value would come from the next group (its first and
// last lane) do not use it.
template <typename T, bool SEG>
__device__ inline T x_restrict(const RowLoad<T, SEG> &v, int W, int gl, int cx, int cnx) {
  T left = wave_prev(v.b);     // fine 2J-1
  T right = wave_next(v.a);    // fine 2J+2
  const T e0 = wave_prev(v.a);  // fine 0, for J = 1
  const T e1 = wave_next(v.b);  // fine 2n-1, for J = n-2
  if (SEG) {
    if (gl == 0) left = v.e;
    if (gl == W - 1) right = v.e;
  }
  T x = (cx == 0 ? T(1.25) : T(0.75)) * v.a + (cx == cnx - 1 ? T(1.25) : T(0.75)) * v.b;
  if (cx > 0) x += T(0.25) * left;
  if (cx < cnx - 1) x += T(0.25) * right;
  if (cx == 1) x -= T(0.25) * e0;
  if (cx == cnx - 2) x -= T(0.25) * e1;
  return x;
}

// Rows of a plane, in order: k = 0 is fine row 2 Y0 - 1 (it feeds coarse row
// Y0 with 1/4); k = 1 .. 2 YR are the rows 2 Y0 .. 2 (Y0 + YR) - 1 the wave
// owns; k = 2 YR + 1 is row 2 (Y0 + YR) (1/4 to coarse row Y0 + YR - 1).  With
// YR >= 2 the two extrapolated end rows (fine row 0 feeding coarse row 1, the
// last fine row feeding coarse row ny/2 - 2) lie inside the owned rows.  A row
// outside the grid is clamped onto an owned one (same cache lines) and skipped.
template <int YR>
__device__ inline int row_of(int k, int Y0, int ny) {
  if (k == 0) return Y0 > 0 ? 2 * Y0 - 1 : 0;
  if (k <= 2 * YR) return 2 * Y0 + k - 1;
  return 2 * (Y0 + YR) < ny ? 2 * (Y0 + YR) : ny - 1;
}

// T^T along y of one plane from its loaded rows into P[0..YR-1]
template <typename T, int YR, bool SEG>
__device__ inline void y_restrict(const RowLoad<T, SEG> (&rows)[2 * YR + 2], int W, int gl, int cx,
                                  int cnx, int Y0, int ny, T (&P)[YR]) {
  static_assert(YR >= 2, "the end rows must fall inside the owned rows");
  const int cny = ny >> 1;
#pragma unroll
  for (int j = 0; j < YR; ++j) P[j] = T(0);
#pragma unroll
  for (int k = 0; k < 2 * YR + 2; ++k) {
    const T x = x_restrict<T, SEG>(rows[k], W, gl, cx, cnx);
    if (k == 0) {
      if (Y0 > 0) P[0] += T(0.25) * x;
    } else if (k <= 2 * YR) {
      const int j = (k - 1) >> 1;  // coarse row (relative) of fine row 2 Y0 + k - 1
      if (k & 1) {                 // even fine row 2 (Y0 + j)
        const bool end = Y0 + j == 0;
        P[j] += (end ? T(1.25) : T(0.75)) * x;
        if (end) {
          if (j + 1 < YR) P[j + 1] -= T(0.25) * x;
        } else if (j >= 1) {
          P[j - 1] += T(0.25) * x;
        }
      } else {  // odd fine row 2 (Y0 + j) + 1
        const bool end = Y0 + j == cny - 1;
        P[j] += (end ? T(1.25) : T(0.75)) * x;
        if (end) {
          if (j >= 1) P[j - 1] -= T(0.25) * x;
        } else if (j + 1 < YR) {
          P[j + 1] += T(0.25) * x;
        }
      }
    } else {
      if (Y0 + YR < cny) P[YR - 1] += T(0.25) * x;
    }
  }
}

// The rows of one fine plane: pb is the field's base (wave-uniform), zoff the
// plane's byte offset, loff the lane's pair offset within a row, eoff - loff
// the lane's edge cell relative to its pair.
template <typename T, int YR, bool SEG>
__device__ inline void load_plane(const T *pb, uint32_t zoff, uint32_t rowb, int Y0, int ny,
                                  uint32_t loff, uint32_t edelta, RowLoad<T, SEG> (&rows)[2 * YR + 2]) {
#pragma unroll
  for (int k = 0; k < 2 * YR + 2; ++k) {
    const uint32_t off = zoff + (uint32_t)row_of<YR>(k, Y0, ny) * rowb + loff;
    rows[k] = load_row<T, SEG>(pb, off, off + edelta);
  }
}

// Coarse-level arrays of one field of one instance (wave-uniform bases).
template <typename T>
struct CoarseBase {
  T *g;
  const T *th_in;
  T *th_out, *m, *v;
};

template <typename T, int YR, bool ADAM>
__device__ inline void emit_rows(const CoarseBase<T> &C, const AdamArgs<T> &A, uint32_t e0, uint32_t rowb,
                                 const T (&val)[YR], const T (&th)[YR], const T (&m)[YR],
                                 const T (&v)[YR]) {
#pragma unroll
  for (int j = 0; j < YR; ++j) {
    const uint32_t e = e0 + (uint32_t)j * rowb;
    st_off(C.g, e, val[j]);
    if (ADAM) {
      const T mm = A.b1 * m[j] + (T(1) - A.b1) * val[j];
      const T vv = A.b2 * v[j] + (T(1) - A.b2) * val[j] * val[j];
      st_off(C.m, e, mm);
      st_off(C.v, e, vv);
      st_off(C.th_out, e, adam_theta(th[j], mm, vv, A.step, A.isb2, A.eps));
    }
  }
}

template <typename T, int YR, bool ADAM>
__device__ inline void load_adam(const CoarseBase<T> &C, uint32_t e0, uint32_t rowb, T (&th)[YR],
                                 T (&m)[YR], T (&v)[YR]) {
#pragma unroll
  for (int j = 0; j < YR; ++j) {
    if (ADAM) {
      const uint32_t e = e0 + (uint32_t)j * rowb;
      th[j] = ld_off(C.th_in, e);
      m[j] = ld_off(C.m, e);
      v[j] = ld_off(C.v, e);
    } else {
      th[j] = m[j] = v[j] = T(0);
    }
  }
}

template <typename T, int YR, int ZR, bool SPANZ, bool SEG, bool ADAM>
__global__ __launch_bounds__(64 * kMarchWaves) void restrict_march_kernel(Levels G, int l, T *g,
                                                                          AdamArgs<T> A, MarchPlan P) {
  // blocks with consecutive logical indices land on the same XCD (blocks are
  // dealt round-robin over the 8 XCDs), so neighbouring tiles share an L2
  const int B = gridDim.x, b = blockIdx.x, xcd = b & 7;
  const int q = B >> 3, r = B & 7;
  const int lb = xcd * q + (xcd < r ? xcd : r) + (b >> 3);
  // the wave's task, held in scalar registers: every base address below is
  // wave-uniform and each lane adds a 32-bit byte offset
  const int task = __builtin_amdgcn_readfirstlane(lb * kMarchWaves + (int)(threadIdx.x >> 6));
  if (task >= P.n_tasks) return;  // whole waves
  const int lane = threadIdx.x & 63;
  int t = task;
  const int yc = t % P.nyc;
  t /= P.nyc;
  const int zc = t % P.nzc;
  t /= P.nzc;
  const int seg = t % P.nseg;
  t /= P.nseg;
  const int f = t % G.nf;
  const int inst = t / G.nf;

  const int W = P.W;
  const int grp = lane >> P.wshift, gl = lane & (W - 1);
  const int nz = G.n[l][f][0], ny = G.n[l][f][1], nx = G.n[l][f][2];
  const int cnx = nx >> 1, cny = ny >> 1;
  const int cx = seg * 64 + gl;
  const int Y0 = (yc * P.groups + grp) * YR;
  // the edge lanes' cell beyond the segment, relative to the lane's pair
  const int ed = (SEG && gl == 0 && cx > 0) ? -1 : (SEG && gl == W - 1 && cx < cnx - 1) ? 2 : 0;
  const uint32_t edelta = (uint32_t)(ed * (int)sizeof(T));

  const T *fb = g + G.off[l] + (long)inst * G.stride[l] + G.foff[l][f];
  const long cbase = G.off[l + 1] + (long)inst * G.stride[l + 1] + G.foff[l + 1][f];
  const CoarseBase<T> C{g + cbase, A.th_in + cbase, A.th_out + cbase, A.m + cbase, A.v + cbase};
  const uint32_t rowb = (uint32_t)nx * sizeof(T), crowb = (uint32_t)cnx * sizeof(T);
  const uint32_t plane_fb = (uint32_t)ny * rowb, plane_cb = (uint32_t)cny * crowb;
  const uint32_t loff = 2u * (uint32_t)cx * sizeof(T);
  const uint32_t row0 = (uint32_t)Y0 * crowb + (uint32_t)cx * sizeof(T);

  T th[YR], m[YR], v[YR];
  if (!SPANZ) {
    RowLoad<T, SEG> rows[2 * YR + 2];
    load_adam<T, YR, ADAM>(C, row0, crowb, th, m, v);
    load_plane<T, YR, SEG>(fb, 0u, rowb, Y0, ny, loff, edelta, rows);
    T Pl[YR];
    y_restrict<T, YR, SEG>(rows, W, gl, cx, cnx, Y0, ny, Pl);
    emit_rows<T, YR, ADAM>(C, A, row0, crowb, Pl, th, m, v);
    return;
  }

  const int cnz = nz >> 1;
  const int Z0 = zc * ZR;
  if (ZR == 1) {
    // one coarse plane per wave: every fine plane it gathers (a window of four
    // and the end planes, restrict_taps6; zero weights are skipped, uniformly
    // over the wave) is loaded before any is used, so the wave waits on memory
    // once instead of once per step of the march
    int iz[6];
    T wz[6];
    restrict_taps6(Z0, cnz, iz, wz);
    const uint32_t e0 = (uint32_t)Z0 * plane_cb + row0;
    load_adam<T, YR, ADAM>(C, e0, crowb, th, m, v);
    RowLoad<T, SEG> rows[6][2 * YR + 2];
#pragma unroll
    for (int t = 0; t < 6; ++t)
      if (wz[t] != T(0)) load_plane<T, YR, SEG>(fb, (uint32_t)iz[t] * plane_fb, rowb, Y0, ny, loff, edelta, rows[t]);
    T acc[YR];
#pragma unroll
    for (int j = 0; j < YR; ++j) acc[j] = T(0);
#pragma unroll
    for (int t = 0; t < 6; ++t)
      if (wz[t] != T(0)) {
        T P[YR];
        y_restrict<T, YR, SEG>(rows[t], W, gl, cx, cnx, Y0, ny, P);
#pragma unroll
        for (int j = 0; j < YR; ++j) acc[j] += wz[t] * P[j];
      }
    emit_rows<T, YR, ADAM>(C, A, e0, crowb, acc, th, m, v);
    return;
  }
  T Ap[YR], Ac[YR], An[YR];
#pragma unroll
  for (int j = 0; j < YR; ++j) Ap[j] = Ac[j] = An[j] = T(0);
  const int Jbeg = Z0 - 1 > 0 ? Z0 - 1 : 0;
  const int Jend = Z0 + ZR < cnz - 1 ? Z0 + ZR : cnz - 1;
  for (int J = Jbeg; J <= Jend; ++J) {
    // step J takes fine planes 2J and 2J+1; they feed coarse planes J-1, J, J+1
    const int za = 2 * J, zb = 2 * J + 1;
    const bool emit = J - 1 >= Z0 && J - 1 < Z0 + ZR;
    const bool needA = !(J == Z0 - 1 && za != 0);       // plane 2J feeds only J-1, J-2 there
    const bool needB = !(J == Z0 + ZR && zb != nz - 1);  // plane 2J+1 feeds only J, J+1 there
    const uint32_t ec = (uint32_t)(J - 1) * plane_cb + row0;
    if (emit) load_adam<T, YR, ADAM>(C, ec, crowb, th, m, v);
    RowLoad<T, SEG> ra[2 * YR + 2], rb[2 * YR + 2];
    if (needA) load_plane<T, YR, SEG>(fb, (uint32_t)za * plane_fb, rowb, Y0, ny, loff, edelta, ra);
    if (needB) load_plane<T, YR, SEG>(fb, (uint32_t)zb * plane_fb, rowb, Y0, ny, loff, edelta, rb);
    if (needA) {
      T Pa[YR];
      y_restrict<T, YR, SEG>(ra, W, gl, cx, cnx, Y0, ny, Pa);
      const T wa = za == 0 ? T(1.25) : T(0.75);
#pragma unroll
      for (int j = 0; j < YR; ++j) {
        Ac[j] += wa * Pa[j];
        if (za == 0)
          An[j] -= T(0.25) * Pa[j];
        else
          Ap[j] += T(0.25) * Pa[j];
      }
    }
    if (needB) {
      T Pb[YR];
      y_restrict<T, YR, SEG>(rb, W, gl, cx, cnx, Y0, ny, Pb);
      const bool last = zb == nz - 1;
      const T wb = last ? T(1.25) : T(0.75);
#pragma unroll
      for (int j = 0; j < YR; ++j) {
        Ac[j] += wb * Pb[j];
        if (last)
          Ap[j] -= T(0.25) * Pb[j];
        else
          An[j] += T(0.25) * Pb[j];
      }
    }
    if (emit) emit_rows<T, YR, ADAM>(C, A, ec, crowb, Ap, th, m, v);
#pragma unroll
    for (int j = 0; j < YR; ++j) {
      Ap[j] = Ac[j];
      Ac[j] = An[j];
      An[j] = T(0);
    }
  }
  // the last coarse plane is complete after the last step
  if (Jend == cnz - 1 && cnz - 1 >= Z0 && cnz - 1 < Z0 + ZR) {
    const uint32_t e0 = (uint32_t)(cnz - 1) * plane_cb + row0;
    load_adam<T, YR, ADAM>(C, e0, crowb, th, m, v);
    emit_rows<T, YR, ADAM>(C, A, e0, crowb, Ap, th, m, v);
  }
}

// ------------------------------------------------------------------ host side
// Tile choice: rows per wave YR and planes per wave ZR, 0 = automatic.
static void choose_tile(int cnx, int cny, int cnz, int groups, bool spanz, int req, int &YR, int &ZR) {
  YR = req ? (req >> 6) : 2;
  ZR = req ? (req & 63) : 4;
  if (!req && spanz) {
    // measured on MI355X, 5 FP32 fields with Adam (us per launch):
    //   128^3 coarse cells: (4, 8) 152, (4, 4) 158, (2, 8) 161, (2, 4) 167
    //   64^3: (2, 4) 16.0, (2, 2) 16.4, (4, 2) 16.6, (4, 4) 17.5
    //   32^3 and smaller: (2, 1) fastest (more waves in flight)
    const long cells = (long)cnx * cny * cnz;
    if (cells >= 128L * 128 * 128) {
      YR = 4;
      ZR = 8;
    } else if (cells > 32L * 32 * 32) {
      YR = 2;
      ZR = 4;
    } else {
      YR = 2;
      ZR = 1;
    }
    // a tile that does not divide the level falls back to one that does
    if (cny % (groups * YR) || cnz % ZR) {
      YR = 2;
      ZR = 1;
    }
  }
  if (!spanz) ZR = 1;
}

// The marching kernel applies to level l -> l+1 when every field has the
// same shape, spans x and y (and z, or no z at all), the coarse rows are
// whole 64-lane segments or a power of two of at least 16 cells, the tiles
// divide the coarse grid, and g admits paired loads.
bool restrict_march_ok(const Levels &G, int l, const void *g, size_t elem, int req, int &YR, int &ZR,
                       bool &spanz, MarchPlan &P) {
  if (l + 1 >= G.L) return false;
  if (reinterpret_cast<uintptr_t>(g) % (2 * elem)) return false;
  for (int f = 1; f < G.nf; ++f)
    for (int a = 0; a < 3; ++a)
      if (G.n[l][f][a] != G.n[l][0][a] || G.n[l + 1][f][a] != G.n[l + 1][0][a]) return false;
  const int nz = G.n[l][0][0], ny = G.n[l][0][1], nx = G.n[l][0][2];
  const int cnz = G.n[l + 1][0][0], cny = G.n[l + 1][0][1], cnx = G.n[l + 1][0][2];
  if (nx != 2 * cnx || ny != 2 * cny) return false;
  spanz = nz > 1;
  if (spanz ? nz != 2 * cnz : cnz != 1) return false;
  if (cnx % 64 == 0) {
    P.W = 64;
    P.nseg = cnx / 64;
  } else if (cnx >= 16 && cnx < 64 && (cnx & (cnx - 1)) == 0) {
    P.W = cnx;
    P.nseg = 1;
  } else {
    return false;
  }
  P.wshift = 0;
  while ((1 << P.wshift) < P.W) ++P.wshift;
  P.groups = 64 / P.W;
  choose_tile(cnx, cny, spanz ? cnz : 1, P.groups, spanz, req, YR, ZR);
  if (cny % (P.groups * YR)) return false;
  if (spanz && cnz % ZR) return false;
  // byte offsets within one field of a level are 32-bit
  if ((long)nz * ny * nx * (long)elem >= (1L << 31)) return false;
  P.nyc = cny / (P.groups * YR);
  P.nzc = spanz ? cnz / ZR : 1;
  const long tasks = (long)G.batch * G.nf * P.nseg * P.nyc * P.nzc;
  if (tasks > (1L << 30)) return false;
  P.n_tasks = (int)tasks;
  return true;
}

bool restrict_march_applies(const Levels &G, int l, const void *g, size_t elem, int tile) {
  int YR, ZR;
  bool spanz;
  MarchPlan P{};
  return restrict_march_ok(G, l, g, elem, tile, YR, ZR, spanz, P);
}

template <typename T, int YR, int ZR, bool ADAM>
static void launch_march_yz(const Levels &G, int l, T *g, const AdamArgs<T> &A, const MarchPlan &P,
                            bool spanz, hipStream_t s) {
  const unsigned blocks = (unsigned)((P.n_tasks + kMarchWaves - 1) / kMarchWaves);
  const dim3 grid(blocks), block(64 * kMarchWaves);
  const bool seg = P.nseg > 1;
  if (spanz) {
    if (seg)
      restrict_march_kernel<T, YR, ZR, true, true, ADAM><<<grid, block, 0, s>>>(G, l, g, A, P);
    else
      restrict_march_kernel<T, YR, ZR, true, false, ADAM><<<grid, block, 0, s>>>(G, l, g, A, P);
  } else {
    if (seg)
      restrict_march_kernel<T, YR, 1, false, true, ADAM><<<grid, block, 0, s>>>(G, l, g, A, P);
    else
      restrict_march_kernel<T, YR, 1, false, false, ADAM><<<grid, block, 0, s>>>(G, l, g, A, P);
  }
}

template <typename T, bool ADAM>
static bool launch_march_t(const Levels &G, int l, T *g, const AdamArgs<T> &A, const MarchPlan &P,
                           int YR, int ZR, bool spanz, hipStream_t s) {
  switch (YR * 64 + (spanz ? ZR : 1)) {
    case 2 * 64 + 1: launch_march_yz<T, 2, 1, ADAM>(G, l, g, A, P, spanz, s); return true;
    case 2 * 64 + 2: launch_march_yz<T, 2, 2, ADAM>(G, l, g, A, P, spanz, s); return true;
    case 2 * 64 + 4: launch_march_yz<T, 2, 4, ADAM>(G, l, g, A, P, spanz, s); return true;
    case 2 * 64 + 8: launch_march_yz<T, 2, 8, ADAM>(G, l, g, A, P, spanz, s); return true;
    case 4 * 64 + 1: launch_march_yz<T, 4, 1, ADAM>(G, l, g, A, P, spanz, s); return true;
    case 4 * 64 + 2: launch_march_yz<T, 4, 2, ADAM>(G, l, g, A, P, spanz, s); return true;
    case 4 * 64 + 4: launch_march_yz<T, 4, 4, ADAM>(G, l, g, A, P, spanz, s); return true;
    case 4 * 64 + 8: launch_march_yz<T, 4, 8, ADAM>(G, l, g, A, P, spanz, s); return true;
    case 4 * 64 + 16: launch_march_yz<T, 4, 16, ADAM>(G, l, g, A, P, spanz, s); return true;
    case 8 * 64 + 4: launch_march_yz<T, 8, 4, ADAM>(G, l, g, A, P, spanz, s); return true;
    case 8 * 64 + 8: launch_march_yz<T, 8, 8, ADAM>(G, l, g, A, P, spanz, s); return true;
    default: return false;
  }
}

// Launch the marching restriction (and Adam) of level l -> l+1 if it
// applies; returns false (nothing launched) otherwise.
template <typename T>
bool launch_restrict_march(const Levels &G, int l, T *g, const AdamArgs<T> &A, bool adam, int req,
                           hipStream_t s) {
  int YR, ZR;
  bool spanz;
  MarchPlan P{};
  if (!restrict_march_ok(G, l, g, sizeof(T), req, YR, ZR, spanz, P)) return false;
  return adam ? launch_march_t<T, true>(G, l, g, A, P, YR, ZR, spanz, s)
              : launch_march_t<T, false>(G, l, g, A, P, YR, ZR, spanz, s);
}

// ------------------------------------------------- node-based values
// Node-based T^T (Section 2.2): coarse node J gathers the fine nodes 2J - 1,
// 2J, 2J + 1 with weights 1/2, 1, 1/2 (clipped at the ends) along every
// spanned axis.  Node counts are 2^k + 1, which rows of 64-lane segments do
// not tile, so a wave's 64 lanes take 64 consecutive nodes of the flattened
// coarse plane (y, x) and the wave marches along z through ZR coarse planes:
//   x  a lane loads fine nodes 2J and 2J + 1 of a fine row and takes 2J - 1
//      from the previous lane (the same row when J > 0); the wave's first
//      lane loads it itself;
//   y  a lane gathers the three fine rows 2Y - 1, 2Y, 2Y + 1 of its coarse row;
//   z  each fine plane is formed once per wave: an even plane 2J feeds coarse
//      plane J, an odd plane 2J + 1 feeds J and J + 1 with 1/2 each.
// Lanes past the plane's last node load nothing and store nothing but still
// run the shifts.  Fine rows have an odd count, so loads are per value.
struct NodeMarchPlan {
  int lanes_per_plane;  // coarse nodes of one coarse plane (ncy * ncx)
  int tasks_plane;      // waves per coarse plane chunk
  int zr, nzc;          // coarse planes per wave, chunks along z
  int spanz;
  int n_tasks;
};

template <typename T, int ZR, bool ADAM>
__global__ __launch_bounds__(64 * kMarchWaves) void restrict_march_node_kernel(Levels G, int l, T *g,
                                                                               AdamArgs<T> A,
                                                                               NodeMarchPlan P) {
  const int B = gridDim.x, b = blockIdx.x, xcd = b & 7;
  const int q8 = B >> 3, r8 = B & 7;
  const int lb = xcd * q8 + (xcd < r8 ? xcd : r8) + (b >> 3);
  const int task = __builtin_amdgcn_readfirstlane(lb * kMarchWaves + (int)(threadIdx.x >> 6));
  if (task >= P.n_tasks) return;  // whole waves
  const int lane = threadIdx.x & 63;
  int t = task;
  const int tp = t % P.tasks_plane;
  t /= P.tasks_plane;
  const int zc = t % P.nzc;
  t /= P.nzc;
  const int f = t % G.nf, inst = t / G.nf;
  const int nfy = G.n[l][f][1], nfx = G.n[l][f][2], nfz = G.n[l][f][0];
  const int ncz = G.n[l + 1][f][0], ncx = G.n[l + 1][f][2];
  // this lane's coarse node of the plane: row Y, column J
  const int qn = tp * 64 + lane;
  const bool on = qn < P.lanes_per_plane;
  const int qc = on ? qn : P.lanes_per_plane - 1;  // idle lanes mirror the last node
  const int Y = small_div(qc, ncx, 1.0f / (float)ncx), J = qc - Y * ncx;
  const T *fb = g + G.off[l] + (long)inst * G.stride[l] + G.foff[l][f];
  const long cbase = G.off[l + 1] + (long)inst * G.stride[l + 1] + G.foff[l + 1][f];
  const CoarseBase<T> C{g + cbase, A.th_in + cbase, A.th_out + cbase, A.m + cbase, A.v + cbase};
  const uint32_t rowb = (uint32_t)nfx * sizeof(T), plane_fb = (uint32_t)nfy * rowb;
  const uint32_t plane_cb = (uint32_t)P.lanes_per_plane * sizeof(T);
  const uint32_t cofs = (uint32_t)qc * sizeof(T);
  const bool has_b = 2 * J + 1 < nfx;                    // fine node 2J + 1 exists
  const bool self_left = lane == 0 && J > 0;              // 2J - 1 not on the previous lane
  // the three fine rows of coarse row Y (clipped rows get weight 0)
  int rows[3];
  T wy[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int r = 2 * Y - 1 + k;
    rows[k] = r < 0 ? 0 : (r >= nfy ? nfy - 1 : r);
    wy[k] = (r < 0 || r >= nfy) ? T(0) : (k == 1 ? T(1) : T(0.5));
  }
  // T^T along y and x of fine plane z for this lane
  auto plane_value = [&](int z) {
    const uint32_t zo = (uint32_t)z * plane_fb;
    T a[3], bb[3], e[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const uint32_t o = zo + (uint32_t)rows[k] * rowb + (uint32_t)(2 * J) * sizeof(T);
      a[k] = ld_off(fb, o);
      bb[k] = has_b ? ld_off(fb, o + sizeof(T)) : T(0);
      e[k] = self_left ? ld_off(fb, o - sizeof(T)) : T(0);
    }
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      T left = wave_prev(bb[k]);
      if (self_left) left = e[k];
      if (J == 0) left = T(0);
      acc += wy[k] * (a[k] + T(0.5) * left + T(0.5) * bb[k]);
    }
    return acc;
  };
  auto finish = [&](int Jz, T val) {
    if (!on) return;
    const uint32_t e = (uint32_t)Jz * plane_cb + cofs;
    T th = T(0), m = T(0), v = T(0);
    if (ADAM) {
      th = ld_off(C.th_in, e);
      m = ld_off(C.m, e);
      v = ld_off(C.v, e);
    }
    st_off(C.g, e, val);
    if (ADAM) {
      const T mm = A.b1 * m + (T(1) - A.b1) * val;
      const T vv = A.b2 * v + (T(1) - A.b2) * val * val;
      st_off(C.m, e, mm);
      st_off(C.v, e, vv);
      st_off(C.th_out, e, adam_theta(th, mm, vv, A.step, A.isb2, A.eps));
    }
  };
  if (!P.spanz) {
    finish(0, plane_value(0));
    return;
  }
  const int Z0 = zc * ZR;
  const int Z1 = Z0 + ZR < ncz ? Z0 + ZR : ncz;
  T odd = Z0 > 0 ? plane_value(2 * Z0 - 1) : T(0);  // fine plane 2 Z0 - 1
  for (int Jz = Z0; Jz < Z1; ++Jz) {
    const T even = plane_value(2 * Jz);
    const T nxt = 2 * Jz + 1 < nfz ? plane_value(2 * Jz + 1) : T(0);
    finish(Jz, T(0.5) * odd + even + T(0.5) * nxt);
    odd = nxt;
  }
}

// Node-based levels of one shape spanning every axis they have (2-D: y and
// x; 3-D: all three), node counts 2 n + 1 -> n + 1.
static bool restrict_march_node_ok(const Levels &G, int l, size_t elem, NodeMarchPlan &P) {
  if (!G.node || l + 1 >= G.L) return false;
  for (int f = 1; f < G.nf; ++f)
    for (int a = 0; a < 3; ++a)
      if (G.n[l][f][a] != G.n[l][0][a] || G.n[l + 1][f][a] != G.n[l + 1][0][a]) return false;
  const int nz = G.n[l][0][0], ny = G.n[l][0][1], nx = G.n[l][0][2];
  const int cnz = G.n[l + 1][0][0], cny = G.n[l + 1][0][1], cnx = G.n[l + 1][0][2];
  if (nx != 2 * cnx - 1 || ny != 2 * cny - 1 || cnx < 2 || cny < 2) return false;
  const bool spanz = nz > 1;
  if (spanz ? nz != 2 * cnz - 1 : cnz != 1) return false;
  if ((long)nz * ny * nx * (long)elem >= (1L << 31)) return false;  // 32-bit byte offsets
  const long plane = (long)cny * cnx;
  if (plane >= (1L << 22)) return false;  // the float-reciprocal split of a plane index
  P.lanes_per_plane = (int)plane;
  P.tasks_plane = (int)((plane + 63) / 64);
  P.spanz = spanz ? 1 : 0;
  // two coarse planes per wave (five fine planes formed for two outputs)
  // while that still gives 2048 waves, else one (three for one)
  P.zr = spanz ? 2 : 1;
  if (spanz && (long)G.batch * G.nf * ((cnz + 1) / 2) * P.tasks_plane < 2048) P.zr = 1;
  P.nzc = spanz ? (cnz + P.zr - 1) / P.zr : 1;
  const long tasks = (long)G.batch * G.nf * P.nzc * P.tasks_plane;
  if (tasks > (1L << 30)) return false;
  P.n_tasks = (int)tasks;
  return true;
}

template <typename T>
bool launch_restrict_march_node(const Levels &G, int l, T *g, const AdamArgs<T> &A, bool adam,
                                hipStream_t s) {
  NodeMarchPlan P{};
  if (!restrict_march_node_ok(G, l, sizeof(T), P)) return false;
  const unsigned blocks = (unsigned)((P.n_tasks + kMarchWaves - 1) / kMarchWaves);
  auto go = [&](auto kernel) { kernel<<<blocks, 64 * kMarchWaves, 0, s>>>(G, l, g, A, P); };
  if (P.zr == 2)
    adam ? go(restrict_march_node_kernel<T, 2, true>) : go(restrict_march_node_kernel<T, 2, false>);
  else
    adam ? go(restrict_march_node_kernel<T, 1, true>) : go(restrict_march_node_kernel<T, 1, false>);
  return true;
}

template bool launch_restrict_march_node<float>(const Levels &, int, float *, const AdamArgs<float> &,
                                                bool, hipStream_t);
template bool launch_restrict_march_node<double>(const Levels &, int, double *,
                                                 const AdamArgs<double> &, bool, hipStream_t);

template bool launch_restrict_march<float>(const Levels &, int, float *, const AdamArgs<float> &,
                                           bool, int, hipStream_t);
template bool launch_restrict_march<double>(const Levels &, int, double *,
                                            const AdamArgs<double> &, bool, int, hipStream_t);

}  // namespace modil
