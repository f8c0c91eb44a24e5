// Internal declarations shared by the host side of libmodil and its kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "modil.h"

namespace modil {

constexpr int kBlock = 256;       // threads per block of the flat kernels
constexpr int kMaxF = MODIL_MAX_FIELDS;
constexpr int kMaxL = MODIL_MAX_LEVELS;
constexpr int kTerms = MODIL_N_TERMS;

// Geometry of one field on one level: cells per axis (z, y, x; 1 for axes the
// field or the grid does not span) and C-order strides.
struct FieldGeom {
  int n[3];
  long stride[3];
  long size;
};

// Constants of the residual operator, passed by value to the kernels.
struct OpParams {
  int ndim;          // active axes are the last ndim of (z, y, x)
  int n[3];          // fine cells per axis (1 on inactive axes)
  double h[3];       // cell size per axis
  double V;          // cell measure (product of active h)
  double w_pde, w_reg, w_bc;
  double re, diam, lam, chi_shift, tau_coef, u_ref;
  const double *inst_re;  // per-instance Reynolds number (device) or null
};

// Per-field description of the finest grid for the stencil engine.
struct FineFields {
  int nf;
  long off[kMaxF];      // element offset of field f inside one instance
  long stride[kMaxF][3];  // strides of field f (0 on axes it does not span)
  long inst_stride;     // elements of all fields of one instance
};

// Geometry of every level of a parameter pack, 32-bit (validated to fit).
struct Levels {
  int L, nf, batch;
  int node;                // node-based values (Section 2.2); else cell-based
  int off[kMaxL];          // pack offset of level l
  int stride[kMaxL];       // elements of one instance on level l
  int foff[kMaxL][kMaxF];  // field offsets inside one instance
  int n[kMaxL][kMaxF][3];  // cells per axis (z, y, x) of every field
};

// The Adam parameter update theta - step * m / (sqrt(v) * isb2 + eps), with
// step = lr / (1 - b1^t) and isb2 = 1 / sqrt(1 - b2^t) folded on the host.  In
// FP32 the square root and the reciprocal are the hardware approximations
// (about 1 ulp each) instead of correctly rounded sequences; FP64 is exact.
// Every kernel that applies Adam uses this one function, so all of them give
// the same bits.
template <typename T>
__device__ inline T adam_theta(T th, T m, T v, T step, T isb2, T eps) {
  return th - step * m / (sqrt(v) * isb2 + eps);
}
template <>
__device__ inline float adam_theta<float>(float th, float m, float v, float step, float isb2,
                                          float eps) {
  return th - step * m * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(v) * isb2 + eps);
}

// Barrier for data exchanged through LDS only: it waits for the wave's own
// LDS accesses, not for its global stores as __syncthreads does, so blocks
// that write results level after level do not wait for each level's stores.
// The memory clobber keeps the compiler from moving memory accesses across it.
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Makes a loaded value count as used at this point: its load is issued
// before here and waited for here.  Keeps the compiler from sinking a load
// past a barrier to its first real use, where the wait for it (one counter
// tracks loads and stores in issue order) would also cover later loads and
// stores.
template <typename T>
__device__ inline void settle(const T &v) {
  asm volatile("" ::"v"(v));
}

// e / m for 0 <= e < 2^22 and m >= 1 with rcp = 1 / m (rounded): e is exact
// in float and the product is within 2^-23 relative of e / m, i.e. less than
// 1/2 from it, so the truncated quotient is off by at most one, which one
// correction step fixes (the LDS tail kernels index arrays of far fewer than
// 2^22 elements this way, several times cheaper than an integer division)
__device__ inline int small_div(int e, int m, float rcp) {
  int q = (int)((float)e * rcp);
  const int r = e - q * m;
  q += (r >= m ? 1 : 0) - (r < 0 ? 1 : 0);
  return q;
}

// 3-D index (z, y, x) of element e < 2^22 of an array with dims (., n1, n2)
__device__ inline void small_index(int e, int n1, int n2, float r1, float r2, int (&i)[3]) {
  const int q = small_div(e, n2, r2);
  i[2] = e - q * n2;
  i[0] = small_div(q, n1, r1);
  i[1] = q - i[0] * n1;
}

// x of the lane that DPP control CTRL names, on the rows and banks (groups of
// four lanes) that ROW and BANK enable; 0 elsewhere.  A double moves as its two
// 32-bit halves under the same control.
template <int CTRL, int ROW, int BANK>
__device__ inline double dpp_take(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW, BANK, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW, BANK, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum of x over the 64 lanes of a wave, in a fixed order, left in lane 63
// (other lanes hold partial sums).  Within each row of 16 lanes: every lane
// adds the three before it (row shifts 1, 2, 3 of x), then the partial four
// (shift 4, upper three banks) and eight (shift 8, upper two banks) before
// it, so lane 15 of the row holds the row's sum; then lane 15 of rows 0 and 2
// is added across to rows 1 and 3, and lane 31 to rows 2 and 3.  Each step is
// one DPP move per 32-bit half and one add, with no LDS round trip.
__device__ inline double wave_sum(double x) {
  double s = x + dpp_take<0x111, 0xf, 0xf>(x);  // row_shr:1
  s += dpp_take<0x112, 0xf, 0xf>(x);           // row_shr:2
  s += dpp_take<0x113, 0xf, 0xf>(x);           // row_shr:3
  s += dpp_take<0x114, 0xf, 0xe>(s);           // row_shr:4, banks 1-3
  s += dpp_take<0x118, 0xf, 0xc>(s);           // row_shr:8, banks 2-3
  s += dpp_take<0x142, 0xa, 0xf>(s);           // row_bcast:15 into rows 1 and 3
  s += dpp_take<0x143, 0xc, 0xf>(s);           // row_bcast:31 into rows 2 and 3
  return s;
}

// Fixed-order final sum of one instance's FP64 loss partials: slots [0, n_a)
// and [off_b, off_b + n_b) of src.  The first kBlock threads of the calling
// block add kBlock-strided slots, then each wave's lanes (wave_sum), then the
// waves in order, so every caller sums in the same order.  Writes the kTerms
// sums to terms and raises flag on a non-finite one.  Every thread of the
// block calls it (it holds a barrier); the block has at least kBlock threads.
__device__ inline void final_terms(const double *src, long n_a, long off_b, long n_b,
                                   double *terms, int32_t *flag) {
  __shared__ double sh[kBlock / 64][kTerms];
  const int tid = threadIdx.x;
  double t[kTerms];
  for (int k = 0; k < kTerms; ++k) t[k] = 0.0;
  if (tid < kBlock)
    for (long b = tid; b < n_a + n_b; b += kBlock) {
      const long slot = b < n_a ? b : off_b + (b - n_a);
      for (int k = 0; k < kTerms; ++k) t[k] += src[slot * kTerms + k];
    }
  for (int k = 0; k < kTerms; ++k) t[k] = wave_sum(t[k]);
  if (tid < kBlock && (tid & 63) == 63)
    for (int k = 0; k < kTerms; ++k) sh[tid >> 6][k] = t[k];
  __syncthreads();
  if (tid < kTerms) {
    double s = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) s += sh[w][tid];
    terms[tid] = s;
    if (!isfinite(s)) flag[0] = 1;
  }
}

// Adam on pack elements: theta_out[e] = adam_theta(theta_in[e], m, v, ...)
template <typename T>
struct AdamArgs {
  const T *th_in;
  T *th_out, *m, *v;
  T b1, b2, step, isb2, eps;
};

// A measurement as the fused channel-flow kernel reads it: field, flat cell
// index (to find repeated cells), loss term, position in its tile (halo
// included), value and weight.
struct FusedMeas {
  int32_t field, cell, term;
  int16_t lx, ly;
  double val, w;
};
static_assert(sizeof(FusedMeas) == 32, "32-byte records");

struct Meas {
  int32_t inst, field, term, idx;
  double val, w;
};

struct EventPair {
  hipEvent_t a, b;
};

struct ProfileClass {
  std::vector<EventPair> pending;
  std::vector<EventPair> pool;
  double ms = 0.0;
  int64_t count = 0;
};

// launch classes timed by modil_profile: 0 fine level, 1 Horner, 2 restriction,
// 3 Adam, 4 reductions / data terms, 5 L-BFGS dot products, 6 L-BFGS vector updates
constexpr int kProfileClasses = 7;

}  // namespace modil

struct modil_ctx {
  modil_problem prob;
  modil_pack_layout lay;
  hipStream_t stream = nullptr;
  int device = 0;
  char *ws = nullptr;
  size_t ws_bytes = 0;

  // workspace carve-up
  void *w_buf = nullptr;     // Horner intermediates, levels 0..L-2 (level 0 = fine u)
  void *g_buf = nullptr;     // gradient pack used by modil_step
  void *gq_buf = nullptr;    // per-cell contributions of 1-D fields (heat q)
  int gq_rows = 0;           // rows in gq_buf: grid rows, or rows of tiles (their sums)
  void *sens_buf = nullptr;  // 3-D adjoint: face-slot sensitivities [6][nnb][batch][cells]
  void *cpart = nullptr;     // fused channel flow: level-1 gradient partials of every tile
  void *fine_tmp = nullptr;  // one fine-field array (scratch)
  double *partials = nullptr;  // [batch][n_part_blocks][kTerms]
  double *terms_tmp = nullptr; // [batch][kTerms]
  int32_t *flag = nullptr;     // non-finite flag
  int32_t *m_idx = nullptr, *m_field = nullptr, *m_term = nullptr, *m_inst_ptr = nullptr;
  double *m_val = nullptr, *m_w = nullptr;
  double *inst_re = nullptr;

  // measurements bucketed per (tile, plane) for the fused channel-flow kernel
  int32_t *fm_ptr = nullptr;
  modil::FusedMeas *fm_rec = nullptr;
  // measurements bucketed per (instance, tile) for the 2-D tiled engine
  int32_t *tm_ptr = nullptr;
  modil::FusedMeas *tm_rec = nullptr;
  bool fused_enabled = true;  // MODIL_OPT_FUSED
  bool fused_ok = false;      // measurements admit the fused kernel
  bool march_enabled = true;  // MODIL_OPT_MARCH
  int march_tile = 0;         // MODIL_OPT_MARCH_TILE
  bool tail_enabled = true;   // MODIL_OPT_TAIL
  int carry_stop = 0;  // lowest level of the Horner tail the last restriction tail carried
  bool tile_enabled = true;   // MODIL_OPT_TILE
  bool two_pass_enabled = true;  // MODIL_OPT_TWO_PASS
  size_t lds_budget = 64 * 1024;  // LDS bytes one block of the tail kernels may use

  long n_fine_blocks = 0;   // partial blocks of the fine kernel per instance
  long fine_slots = 0;      // partial slots the last generic fine-kernel launch wrote
  long n_data_blocks = 0;   // partial blocks of the data kernel per instance
  long n_part_blocks = 0;   // n_fine_blocks + n_data_blocks

  std::vector<modil::Meas> meas;
  int n_meas_dev = 0;
  int max_list_len = 0;
  std::vector<double> inst_re_host;
  const void *forcing[4] = {nullptr, nullptr, nullptr, nullptr};
  const void *chi = nullptr;

  bool profiling = false;
  modil::ProfileClass prof[modil::kProfileClasses];
  std::string err;
};

namespace modil {

// RAII timing of one launch class with HIP events on the context's stream
// (only while profiling is enabled).
struct Timed {
  modil_ctx *c;
  EventPair ev{};
  bool on;
  int cls_;
  Timed(modil_ctx *ctx, int cls) : c(ctx), on(ctx->profiling), cls_(cls) {
    if (!on) return;
    ProfileClass &pc = c->prof[cls_];
    if (!pc.pool.empty()) {
      ev = pc.pool.back();
      pc.pool.pop_back();
    } else {
      (void)hipEventCreate(&ev.a);
      (void)hipEventCreate(&ev.b);
    }
    (void)hipEventRecord(ev.a, c->stream);
  }
  ~Timed() {
    if (!on) return;
    (void)hipEventRecord(ev.b, c->stream);
    c->prof[cls_].pending.push_back(ev);
  }
};

// layout helpers (api.cpp)
int op_fields(const modil_problem &p);
int op_equations(const modil_problem &p);
int op_pde_equations(const modil_problem &p);
bool field_is_x_only(const modil_problem &p, int f);
FieldGeom field_geom(const modil_problem &p, int level, int f);

Levels levels_of(const modil_ctx *c);

// record the message returned by modil_last_error(NULL); returns status
int set_global_error(int status, const std::string &msg);
// record an error on a context (and globally); returns status
int set_ctx_error(modil_ctx *c, int status, const std::string &msg);
// loss terms [batch][5] and, if grad is not null, the gradient pack at theta
int eval_loss_grad(modil_ctx *c, const void *theta, void *grad, double *terms);

// Adam hyper-parameters as passed to the kernels (bias corrections folded in)
struct AdamHost {
  double b1, b2, step, isb2, eps;
};

// kernel launchers (kernels.hip, ns3d_fused.hip); all enqueue on ctx->stream
// and return hipSuccess or the launch error.
// Horner chain: w_l for every coarse level into w_buf and the finest field
// into fine_dst (w_buf level 0 if null); stops at level 1 when skip_fine.
// skip_tail: the small levels' w are in w_buf already (carried)
hipError_t launch_horner(modil_ctx *c, const void *theta, void *fine_dst, bool skip_fine,
                         bool skip_tail = false);
// g_{l+1} = T^T g_l for l >= from_level (pack layout in g); with adam also
// Adam on every level it produces.
// A final sum of loss partials that a later kernel can carry out:
// final_terms(partials + instance * n_part_blocks * kTerms, n_a, off_b, n_b, ...)
// for every instance.
struct TermSum {
  const double *partials = nullptr;
  long n_part_blocks = 0, n_a = 0, off_b = 0, n_b = 0;
  double *terms = nullptr;
  int32_t *flag = nullptr;
};
// Restriction of the gradient from level from_level down, with Adam on every
// level produced when adam is given.  With sum given, the chain's last kernel
// also does that sum when it can (summed tells whether it did).  With colsum,
// the x-only field's column sums of the tile kernel's contributions (and its
// level-0 Adam) come first: in the restriction tail where it can, else by
// launch_colsum.
hipError_t launch_restrict_chain(modil_ctx *c, void *g, int from_level, const void *th_in,
                                 void *th_out, void *m, void *v, const AdamHost *adam,
                                 const TermSum *sum = nullptr, bool *summed = nullptr,
                                 bool carry = false, bool *carried = nullptr, bool colsum = false);
// Marching restriction of level l -> l+1 with optional Adam (restrict_march.hip);
// returns false, launching nothing, when the level's shape does not admit it.
// tile: 64 * rows + planes per wave, 0 = automatic.
template <typename T>
bool launch_restrict_march(const Levels &G, int l, T *g, const AdamArgs<T> &A, bool adam, int tile,
                           hipStream_t s);
// whether launch_restrict_march would launch for this level (host only)
bool restrict_march_applies(const Levels &G, int l, const void *g, size_t elem, int tile);
// the same for node-based fields of one shape spanning every axis they have
// (lanes over the flattened coarse plane); false when the level does not qualify
template <typename T>
bool launch_restrict_march_node(const Levels &G, int l, T *g, const AdamArgs<T> &A, bool adam,
                                hipStream_t s);
// Horner step of level l by coarse-cell blocks (prolong_block.hip): theta and
// dst are level-l bases, csrc the level-(l+1) base; false (nothing launched)
// when the level's shape does not admit it.
template <typename T>
bool launch_prolong_block(const Levels &G, int l, const T *theta, const T *csrc, T *dst,
                          hipStream_t s);
// the same for node-based fields of one shape spanning three axes; false when
// the level does not qualify
template <typename T>
bool launch_prolong_node(const Levels &G, int l, const T *theta, const T *csrc, T *dst,
                         hipStream_t s);
// Two Horner steps (levels l + 2 -> l) in one launch where the levels admit it.
template <typename T>
bool launch_prolong2(const Levels &G, int l, const T *th_l, const T *th_m, const T *csrc, T *dst,
                     hipStream_t s);
hipError_t launch_adam(modil_ctx *c, const void *theta_in, void *theta_out, void *m, void *v,
                       const void *g, long n, const AdamHost &h);
// generic finest-level kernel (tiled on 2-D problems); with adam given (tiled
// engine only) also Adam on level 0 of the fields spanning the grid; with
// prolong (tiled engine only) u is theta and the kernel forms the finest
// level itself, theta_0 + T w_1, from level 1 of the prolonged levels
hipError_t launch_fine(modil_ctx *c, const void *u, void *g, bool want_grad,
                       const AdamHost *adam = nullptr, const void *th_in = nullptr,
                       void *th_out = nullptr, void *m = nullptr, void *v = nullptr,
                       bool prolong = false);
// the 2-D engine by tiles: the problems it takes, their fine grid, tile shape
bool fine_is_2d(const modil_problem &P);
void fine_2d(const modil_problem &P, int &ny, int &nx);
void fine_tile_shape(const modil_problem &P, int &tx, int &ty, int &tiles_x, int &tiles_y);
bool fine_uses_tiles(const modil_ctx *c);
// most partial slots per instance the generic fine kernels use
long fine_partial_slots(const modil_problem &P);
// fields whose neighbours enter the stencil (a prefix of the fields), for the
// two-pass 3-D adjoint; 0 when the problem is not 3-D
int sens_fields(const modil_problem &P);
// whether the workspace holds the two-pass adjoint's face-sensitivity scratch:
// 3-D problems that can run the generic engine with a gradient, except FP32
// cell-based channel flow, which runs the fused kernel (or, when that does
// not apply, the single-pass per-cell kernel)
bool two_pass_adjoint(const modil_problem &P);
// column sums of the x-only field's contributions; with adam given also Adam
// on that field's level 0
hipError_t launch_colsum(modil_ctx *c, void *g_fine, const AdamHost *adam = nullptr,
                         const void *th_in = nullptr, void *th_out = nullptr, void *m = nullptr,
                         void *v = nullptr);
// measurement misfits; with one data block per instance that block also sums
// the fine and data partials into terms (returns whether it did)
hipError_t launch_data(modil_ctx *c, const void *u, void *g, bool want_grad, double *terms,
                       bool &summed);
// fixed-order sum of the partials [0, n_a) and [off_b, off_b + n_b) per instance
hipError_t launch_reduce(modil_ctx *c, double *terms, long n_a, long off_b, long n_b);
hipError_t launch_ns3d_fused(modil_ctx *c, const void *theta, void *g, const AdamHost *adam,
                             void *th_out, void *m, void *v);
void ns3d_tiles(const modil_problem &P, int &tz, int &nzt, int &ntx, int &nty, int &ox, int &oy);
// bytes of the fused kernel's level-1 gradient partials (0 where it has none)
size_t fused_partial_bytes(const modil_problem &P);
// level 1 of the gradient from those partials (and, with adam, Adam on level 1)
hipError_t launch_fused_assemble(modil_ctx *c, void *g, const AdamHost *adam, const void *th_in,
                                 void *th_out, void *m, void *v);
// the fused kernel addresses a plane's fields by 32-bit byte offsets
bool ns3d_offsets_fit(const modil_problem &P);
hipError_t launch_metric(modil_ctx *c, const double *terms, double *r);

}  // namespace modil
