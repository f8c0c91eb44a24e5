// Kernels of one mODIL iteration on gfx950.
//
//   prolong_level   w_l = theta_l + T w_{l+1}          (Horner step, Section 2.2)
//   restrict_level  g_{l+1} = T^T g_l                  (exact transpose of T)
//   fine_kernel     residuals, FP64 loss partials and the gathered adjoint
//                   g(c) = sum_o s_o(c - o) of every equation whose stencil
//                   touches c (Section 2.1 loss, adjoint by hand)
//   data_kernel     measurement misfits and their adjoint
//   colsum_kernel   sums the per-cell contributions of a field that spans x only
//   reduce_kernel   fixed-order reduction of the FP64 partials per instance
//   adam_kernel     elementwise Adam over a pack
//
// Every reduction is deterministic: wave shuffles in a fixed pattern, LDS
// across the waves of a block, and one block per instance for the final sum.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"
#include "ops.h"

namespace modil {

// ---------------------------------------------------------------- geometry
struct LevelGeom {
  int nf;
  long inst_stride;     // elements of one instance on this level
  long foff[kMaxF];     // field offsets inside one instance
  int n[kMaxF][3];      // cells per axis of every field (1 where not spanned)
};

static LevelGeom level_geom(const modil_ctx *c, int level) {
  LevelGeom g{};
  g.nf = c->lay.n_fields;
  g.inst_stride = c->lay.level_stride[level];
  for (int f = 0; f < g.nf; ++f) {
    g.foff[f] = c->lay.field_offset[level][f];
    for (int a = 0; a < 3; ++a) g.n[f][a] = c->lay.field_dims[level][f][a];
  }
  return g;
}

__device__ inline void locate(const LevelGeom &g, long e, int &inst, int &f, int (&i)[3]) {
  inst = (int)(e / g.inst_stride);
  long rem = e - (long)inst * g.inst_stride;
  f = 0;
  for (int k = 1; k < g.nf; ++k)
    if (rem >= g.foff[k]) f = k;
  long cell = rem - g.foff[f];
  i[2] = (int)(cell % g.n[f][2]);
  cell /= g.n[f][2];
  i[1] = (int)(cell % g.n[f][1]);
  i[0] = (int)(cell / g.n[f][1]);
}

// 1-D taps of the cell-based T: fine cell i of 2n fine cells from n coarse.
__device__ inline int prolong_taps(int i, int n, int (&idx)[2], double (&w)[2]) {
  const int J = i >> 1;
  const int nb = (i & 1) ? J + 1 : J - 1;
  if (nb < 0) {
    idx[0] = J; w[0] = 1.25; idx[1] = J + 1; w[1] = -0.25;
  } else if (nb >= n) {
    idx[0] = J; w[0] = 1.25; idx[1] = J - 1; w[1] = -0.25;
  } else {
    idx[0] = J; w[0] = 0.75; idx[1] = nb; w[1] = 0.25;
  }
  return 2;
}

// 1-D taps of T^T: coarse cell J of n coarse cells gathers from 2n fine.
__device__ inline int restrict_taps(int J, int n, int (&idx)[6], double (&w)[6]) {
  int k = 0;
  if (J >= 1) { idx[k] = 2 * J - 1; w[k++] = 0.25; }
  idx[k] = 2 * J; w[k++] = (J == 0) ? 1.25 : 0.75;
  idx[k] = 2 * J + 1; w[k++] = (J == n - 1) ? 1.25 : 0.75;
  if (J <= n - 2) { idx[k] = 2 * J + 2; w[k++] = 0.25; }
  if (J == 1) { idx[k] = 0; w[k++] = -0.25; }
  if (J == n - 2) { idx[k] = 2 * n - 1; w[k++] = -0.25; }
  return k;
}

// ------------------------------------------------------------- prolongation
template <typename T>
__global__ __launch_bounds__(kBlock) void prolong_level_kernel(
    LevelGeom fine, LevelGeom coarse, const T *__restrict__ theta_l, const T *__restrict__ csrc,
    T *__restrict__ dst, long total) {
  const long e = (long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= total) return;
  int inst, f, i[3];
  locate(fine, e, inst, f, i);
  int ti[3][2];
  double tw[3][2];
  int nt[3];
  for (int a = 0; a < 3; ++a) {
    if (fine.n[f][a] == coarse.n[f][a]) {  // axis not spanned by this field
      ti[a][0] = i[a]; tw[a][0] = 1.0; nt[a] = 1;
    } else {
      nt[a] = prolong_taps(i[a], coarse.n[f][a], ti[a], tw[a]);
    }
  }
  const T *cb = csrc + (long)inst * coarse.inst_stride + coarse.foff[f];
  const long sy = coarse.n[f][2], sz = (long)coarse.n[f][1] * coarse.n[f][2];
  T acc = T(0);
  for (int a = 0; a < nt[0]; ++a)
    for (int b = 0; b < nt[1]; ++b)
      for (int d = 0; d < nt[2]; ++d)
        acc += T(tw[0][a] * tw[1][b] * tw[2][d]) * cb[ti[0][a] * sz + ti[1][b] * sy + ti[2][d]];
  dst[e] = theta_l[e] + acc;
}

// --------------------------------------------------------------- restriction
template <typename T>
__global__ __launch_bounds__(kBlock) void restrict_level_kernel(
    LevelGeom fine, LevelGeom coarse, const T *__restrict__ gsrc, T *__restrict__ dst, long total) {
  const long e = (long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= total) return;
  int inst, f, I[3];
  locate(coarse, e, inst, f, I);
  int ti[3][6];
  double tw[3][6];
  int nt[3];
  for (int a = 0; a < 3; ++a) {
    if (fine.n[f][a] == coarse.n[f][a]) {
      ti[a][0] = I[a]; tw[a][0] = 1.0; nt[a] = 1;
    } else {
      nt[a] = restrict_taps(I[a], coarse.n[f][a], ti[a], tw[a]);
    }
  }
  const T *fb = gsrc + (long)inst * fine.inst_stride + fine.foff[f];
  const long sy = fine.n[f][2], sz = (long)fine.n[f][1] * fine.n[f][2];
  T acc = T(0);
  for (int a = 0; a < nt[0]; ++a)
    for (int b = 0; b < nt[1]; ++b) {
      T row = T(0);
      for (int d = 0; d < nt[2]; ++d) row += T(tw[2][d]) * fb[ti[0][a] * sz + ti[1][b] * sy + ti[2][d]];
      acc += T(tw[0][a] * tw[1][b]) * row;
    }
  dst[e] = acc;
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
  const T gg = g[e];
  const T mm = b1 * m[e] + (T(1) - b1) * gg;
  const T vv = b2 * v[e] + (T(1) - b2) * gg * gg;
  m[e] = mm;
  v[e] = vv;
  th_out[e] = th_in[e] - step * mm / (sqrt(vv) * inv_sqrt_bc2 + eps);
}

// ------------------------------------------------------- block-sum of terms
__device__ inline void block_terms(double (&t)[kTerms], double *out) {
  __shared__ double sh[kBlock / 64][kTerms];
  for (int k = 0; k < kTerms; ++k) {
    double x = t[k];
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_down(x, off, 64);
    t[k] = x;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
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
};

template <class Op, typename T>
__device__ inline void load_star(const OpParams &p, const FineFields &ff, const T *ub,
                                 const int (&i)[3], T (&U)[Op::NF][7]) {
  for (int f = 0; f < Op::NF; ++f) {
    const T *base = ub + ff.off[f];
    const long lin = i[0] * ff.stride[f][0] + i[1] * ff.stride[f][1] + i[2] * ff.stride[f][2];
    const T c = base[lin];
    for (int s = 0; s < 7; ++s) U[f][s] = c;
    if (!Op::needs_nb(f)) continue;
    for (int a = 3 - p.ndim; a < 3; ++a) {
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

template <class Op, typename T>
__device__ inline void fold_ghosts(const OpParams &p, const FineFields &ff, const int (&i)[3],
                                   T (&s)[Op::NF][7]) {
  for (int f = 0; f < Op::NF; ++f) {
    if (!Op::needs_nb(f)) continue;
    for (int a = 3 - p.ndim; a < 3; ++a) {
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
template <class Op, typename T>
__device__ inline void cell_residual(const FineArgs<T> &A, int inst, const int (&j)[3],
                                     T (&U)[Op::NF][7], T &chi, T (&r)[Op::NE], T (&wv)[Op::NE],
                                     int (&term)[Op::NE]) {
  const long lin = ((long)j[0] * A.p.n[1] + j[1]) * A.p.n[2] + j[2];
  load_star<Op>(A.p, A.ff, A.u + (long)inst * A.ff.inst_stride, j, U);
  chi = A.chi ? A.chi[(long)inst * A.ncell + lin] : T(0);
  Op::eval(A.p, j, inst, U, chi, r, wv, term);
  for (int e = 0; e < Op::NE && e < 4; ++e)
    if (A.forcing[e] && wv[e] != T(0)) r[e] -= A.forcing[e][(long)inst * A.ncell + lin];
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

// column sums of the x-only field's per-cell contributions (rows = t)
template <typename T>
__global__ __launch_bounds__(kBlock) void colsum_kernel(const T *__restrict__ gq, T *__restrict__ g,
                                                        long inst_stride, long foff, int nt, int nx,
                                                        int batch) {
  const long e = (long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= (long)batch * nx) return;
  const int inst = (int)(e / nx), ix = (int)(e % nx);
  const T *src = gq + (long)inst * nt * nx + ix;
  T acc = T(0);
  for (int it = 0; it < nt; ++it) acc += src[(long)it * nx];
  g[(long)inst * inst_stride + foff + ix] = acc;
}

// measurement misfits; entries sorted by (instance, field, index, term)
template <typename T>
__global__ __launch_bounds__(kBlock) void data_kernel(
    const T *__restrict__ u, T *__restrict__ g, FineFields ff, const int32_t *__restrict__ ptr,
    const int32_t *__restrict__ fld, const int32_t *__restrict__ idx, const int32_t *__restrict__ trm,
    const double *__restrict__ val, const double *__restrict__ wt, double *partials,
    long n_part_blocks, long first_block, int want_grad) {
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
  block_terms(part, partials + ((long)inst * n_part_blocks + first_block + blockIdx.x) * kTerms);
}

// fixed-order sum of all partial blocks of one instance
__global__ __launch_bounds__(kBlock) void reduce_kernel(const double *__restrict__ partials,
                                                        long n_part_blocks, double *terms,
                                                        int32_t *flag) {
  const int inst = blockIdx.x;
  double t[kTerms] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const double *src = partials + (long)inst * n_part_blocks * kTerms;
  for (long b = threadIdx.x; b < n_part_blocks; b += kBlock)
    for (int k = 0; k < kTerms; ++k) t[k] += src[b * kTerms + k];
  __shared__ double out[kTerms];
  block_terms(t, out);
  __syncthreads();
  if (threadIdx.x < kTerms) {
    const double x = out[threadIdx.x];
    terms[(long)inst * kTerms + threadIdx.x] = x;
    if (!isfinite(x)) flag[0] = 1;
  }
}

__global__ void metric_kernel(const double *terms, double *r, int batch, double scale) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < batch) r[b] = sqrt(fmax(terms[(long)b * kTerms + MODIL_TERM_PDE], 0.0) * scale);
}

// -------------------------------------------------------------- launchers
static inline unsigned nblk(long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

hipError_t launch_prolong_level(modil_ctx *c, const void *theta, const void *coarse_src,
                                long coarse_off, void *dst, long dst_off, int level) {
  const LevelGeom fg = level_geom(c, level), cg = level_geom(c, level + 1);
  const long total = fg.inst_stride * c->prob.batch;
  const long toff = c->lay.level_offset[level];
  if (c->prob.dtype == MODIL_F64) {
    prolong_level_kernel<double><<<nblk(total), kBlock, 0, c->stream>>>(
        fg, cg, (const double *)theta + toff, (const double *)coarse_src + coarse_off,
        (double *)dst + dst_off, total);
  } else {
    prolong_level_kernel<float><<<nblk(total), kBlock, 0, c->stream>>>(
        fg, cg, (const float *)theta + toff, (const float *)coarse_src + coarse_off,
        (float *)dst + dst_off, total);
  }
  return hipGetLastError();
}

hipError_t launch_restrict_level(modil_ctx *c, const void *fine_src, long fine_off, void *dst,
                                 long dst_off, int level) {
  const LevelGeom fg = level_geom(c, level), cg = level_geom(c, level + 1);
  const long total = cg.inst_stride * c->prob.batch;
  if (c->prob.dtype == MODIL_F64) {
    restrict_level_kernel<double><<<nblk(total), kBlock, 0, c->stream>>>(
        fg, cg, (const double *)fine_src + fine_off, (double *)dst + dst_off, total);
  } else {
    restrict_level_kernel<float><<<nblk(total), kBlock, 0, c->stream>>>(
        fg, cg, (const float *)fine_src + fine_off, (float *)dst + dst_off, total);
  }
  return hipGetLastError();
}

hipError_t launch_adam(modil_ctx *c, const void *th_in, void *th_out, void *m, void *v,
                       const void *g, long n, double lr, double b1, double b2, double eps,
                       double bc1, double bc2) {
  const double step = lr / bc1, isb = 1.0 / std::sqrt(bc2);
  if (c->prob.dtype == MODIL_F64) {
    adam_kernel<double><<<nblk(n), kBlock, 0, c->stream>>>(
        (const double *)th_in, (double *)th_out, (double *)m, (double *)v, (const double *)g, n,
        b1, b2, step, isb, eps);
  } else {
    adam_kernel<float><<<nblk(n), kBlock, 0, c->stream>>>(
        (const float *)th_in, (float *)th_out, (float *)m, (float *)v, (const float *)g, n,
        (float)b1, (float)b2, (float)step, (float)isb, (float)eps);
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
  for (int k = 0; k < P.ndim; ++k) {
    const int a = 3 - P.ndim + k;
    p.n[a] = P.dims[k];
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

template <typename T>
static hipError_t launch_fine_t(modil_ctx *c, const void *u, void *g, bool want_grad) {
  const FineArgs<T> A = fine_args<T>(c, u, g, want_grad);
  const dim3 grid(nblk(A.ncell), c->prob.batch);
  const modil_problem &P = c->prob;
  switch (P.op) {
    case MODIL_OP_POISSON:
      fine_kernel<OpPoisson, T><<<grid, kBlock, 0, c->stream>>>(A);
      break;
    case MODIL_OP_BURGERS:
      fine_kernel<OpBurgers, T><<<grid, kBlock, 0, c->stream>>>(A);
      break;
    case MODIL_OP_HEAT_KX:
      fine_kernel<OpHeat, T><<<grid, kBlock, 0, c->stream>>>(A);
      break;
    case MODIL_OP_NS3D:
      if (P.flags & MODIL_FLAG_CHI_FIXED)
        fine_kernel<OpNS<3, 1>, T><<<grid, kBlock, 0, c->stream>>>(A);
      else
        fine_kernel<OpNS<3, 2>, T><<<grid, kBlock, 0, c->stream>>>(A);
      break;
    case MODIL_OP_CAVITY:
      fine_kernel<OpNS<2, 0>, T><<<grid, kBlock, 0, c->stream>>>(A);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fine(modil_ctx *c, const void *u, void *g, bool want_grad) {
  return c->prob.dtype == MODIL_F64 ? launch_fine_t<double>(c, u, g, want_grad)
                                    : launch_fine_t<float>(c, u, g, want_grad);
}

hipError_t launch_colsum(modil_ctx *c, void *g_fine) {
  int xf = -1;
  for (int f = 0; f < c->lay.n_fields; ++f)
    if (field_is_x_only(c->prob, f)) xf = f;
  if (xf < 0) return hipSuccess;
  const int nt = c->prob.dims[0], nx = c->prob.dims[1];
  const long n = (long)c->prob.batch * nx;
  if (c->prob.dtype == MODIL_F64)
    colsum_kernel<double><<<nblk(n), kBlock, 0, c->stream>>>(
        (const double *)c->gq_buf, (double *)g_fine, c->lay.level_stride[0],
        c->lay.field_offset[0][xf], nt, nx, c->prob.batch);
  else
    colsum_kernel<float><<<nblk(n), kBlock, 0, c->stream>>>(
        (const float *)c->gq_buf, (float *)g_fine, c->lay.level_stride[0],
        c->lay.field_offset[0][xf], nt, nx, c->prob.batch);
  return hipGetLastError();
}

hipError_t launch_data(modil_ctx *c, const void *u, void *g, bool want_grad) {
  FineFields ff{};
  ff.nf = c->lay.n_fields;
  ff.inst_stride = c->lay.level_stride[0];
  for (int f = 0; f < ff.nf; ++f) ff.off[f] = c->lay.field_offset[0][f];
  const dim3 grid((unsigned)c->n_data_blocks, c->prob.batch);
  if (c->prob.dtype == MODIL_F64)
    data_kernel<double><<<grid, kBlock, 0, c->stream>>>(
        (const double *)u, (double *)g, ff, c->m_inst_ptr, c->m_field, c->m_idx, c->m_term,
        c->m_val, c->m_w, c->partials, c->n_part_blocks, c->n_fine_blocks, want_grad ? 1 : 0);
  else
    data_kernel<float><<<grid, kBlock, 0, c->stream>>>(
        (const float *)u, (float *)g, ff, c->m_inst_ptr, c->m_field, c->m_idx, c->m_term,
        c->m_val, c->m_w, c->partials, c->n_part_blocks, c->n_fine_blocks, want_grad ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_reduce(modil_ctx *c, double *terms) {
  reduce_kernel<<<c->prob.batch, kBlock, 0, c->stream>>>(c->partials, c->n_part_blocks, terms,
                                                         c->flag);
  return hipGetLastError();
}

hipError_t launch_metric(modil_ctx *c, const double *terms, double *r) {
  const modil_problem &P = c->prob;
  double V = 1.0;
  for (int k = 0; k < P.ndim; ++k) V *= P.lengths[k] / P.dims[k];
  const double scale =
      V / (P.w_pde * (double)op_pde_equations(P) * (double)c->lay.fine_cells);
  metric_kernel<<<(P.batch + 63) / 64, 64, 0, c->stream>>>(terms, r, P.batch, scale);
  return hipGetLastError();
}

}  // namespace modil
