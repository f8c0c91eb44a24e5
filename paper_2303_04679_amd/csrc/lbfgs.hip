// Limited-memory BFGS on the loss of a context (the optimiser of most results
// of the paper, Sections 2.1, 3.1, 3.3, 3.5).
//
// Device side: streaming kernels over pack-sized vectors --
//   multidot  up to 2 "right" vectors against up to 8 "left" vectors per grid
//             row (FP64 products, fixed-order block partials), reduced by
//   dot_reduce  one block per output, partials summed in block order
//   combine   d = c_g g + sum_k c_k v_k over the stored pairs
//   axpy      x_trial = x + alpha d
//   pair      s = alpha d, y = g_new - g into a ring slot
// Host side: the compact representation of the L-BFGS matrix (Byrd, Nocedal &
// Schnabel 1994) from the FP64 scalars S^T Y, Y^T Y, S^T g, Y^T g, and the
// strong-Wolfe line search (Nocedal & Wright, Algorithms 3.5 and 3.6).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

namespace modil {

constexpr int kLbBlock = 256;
constexpr int kLbChunk = 8;                              // left vectors per grid row
constexpr int kLbMaxLeft = 2 * (MODIL_LBFGS_MAX_HISTORY + 1) + 1;  // S, Y (+ new pair) and g
constexpr int kLbMaxChunks = (kLbMaxLeft + kLbChunk - 1) / kLbChunk;
constexpr int kLbBlocks = 1024;                          // blocks per grid row

template <typename T>
struct MultiDotArgs {
  const T *left[kLbMaxChunks * kLbChunk];
  const T *right[2];
  int n_left, n_right;
  long n;
  double *partials;  // [chunk][block][right][kLbChunk]
};

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; static constexpr int n = 4; };
template <> struct Vec4<double> { using type = double2; static constexpr int n = 2; };

template <typename V>
__device__ inline double lane_of(const V &v, int i);
template <>
__device__ inline double lane_of<float4>(const float4 &v, int i) {
  return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}
template <>
__device__ inline double lane_of<double2>(const double2 &v, int i) {
  return i == 0 ? v.x : v.y;
}

// Every block covers a fixed contiguous range of elements, read as 16-byte
// vectors (all vectors are 256-byte aligned); products are accumulated in FP64
// per thread, then summed over the block in a fixed tree.  The elements past
// the last whole vector are added by block 0.
template <typename T>
__global__ __launch_bounds__(kLbBlock) void multidot_kernel(MultiDotArgs<T> A) {
  using V = typename Vec4<T>::type;
  constexpr int NV = Vec4<T>::n;
  const int chunk = blockIdx.y;
  const int l0 = chunk * kLbChunk;
  const int nl = min(kLbChunk, A.n_left - l0);
  const long groups = A.n / NV;
  const long per = (groups + gridDim.x - 1) / gridDim.x;
  const long q0 = (long)blockIdx.x * per, q1 = min(groups, q0 + per);
  double acc[2][kLbChunk];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int k = 0; k < kLbChunk; ++k) acc[r][k] = 0.0;
  for (long q = q0 + threadIdx.x; q < q1; q += kLbBlock) {
    const V r0 = reinterpret_cast<const V *>(A.right[0])[q];
    V r1 = r0;
    if (A.n_right > 1) r1 = reinterpret_cast<const V *>(A.right[1])[q];
#pragma unroll
    for (int k = 0; k < kLbChunk; ++k) {
      if (k < nl) {
        const V lv = reinterpret_cast<const V *>(A.left[l0 + k])[q];
#pragma unroll
        for (int i = 0; i < NV; ++i) {
          acc[0][k] += lane_of(lv, i) * lane_of(r0, i);
          acc[1][k] += lane_of(lv, i) * lane_of(r1, i);
        }
      }
    }
  }
  if (blockIdx.x == 0) {
    for (long e = groups * NV + threadIdx.x; e < A.n; e += kLbBlock) {
      const double r0 = (double)A.right[0][e];
      const double r1 = A.n_right > 1 ? (double)A.right[1][e] : r0;
#pragma unroll
      for (int k = 0; k < kLbChunk; ++k) {
        if (k < nl) {
          const double lv = (double)A.left[l0 + k][e];
          acc[0][k] += lv * r0;
          acc[1][k] += lv * r1;
        }
      }
    }
  }
  __shared__ double sh[kLbBlock / 64][2][kLbChunk];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int k = 0; k < kLbChunk; ++k) {
      const double v = wave_sum(acc[r][k]);  // fixed order, in lane 63
      if (lane == 63) sh[wave][r][k] = v;
    }
  __syncthreads();
  if (threadIdx.x < 2 * kLbChunk) {
    const int r = threadIdx.x / kLbChunk, k = threadIdx.x % kLbChunk;
    double v = 0.0;
    for (int w = 0; w < kLbBlock / 64; ++w) v += sh[w][r][k];
    A.partials[(((long)chunk * gridDim.x + blockIdx.x) * 2 + r) * kLbChunk + k] = v;
  }
}

// out[r][l] = sum over blocks of the partials of left vector l, right vector r
__global__ __launch_bounds__(256) void dot_reduce_kernel(const double *__restrict__ partials,
                                                         int blocks, int n_left, double *out) {
  const int l = blockIdx.x, r = blockIdx.y;
  const int chunk = l / kLbChunk, k = l % kLbChunk;
  double v = 0.0;
  for (int b = threadIdx.x; b < blocks; b += 256)
    v += partials[(((long)chunk * blocks + b) * 2 + r) * kLbChunk + k];
  __shared__ double sh[4];
  v = wave_sum(v);  // fixed order, in lane 63
  if ((threadIdx.x & 63) == 63) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) out[r * kLbMaxLeft + l] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

template <typename T>
struct CombineArgs {
  const T *v[2 * MODIL_LBFGS_MAX_HISTORY];
  int nv;
  const T *g;
  T *d;
  const double *coef;  // [0] for g, [1 + k] for v[k]
  long n;
};

// d = c_g g + sum_k c_k v_k, 16-byte vectors per thread (FP64 sums), the
// elements past the last whole vector one per thread
template <typename T>
__global__ __launch_bounds__(kLbBlock) void combine_kernel(CombineArgs<T> A) {
  using V = typename Vec4<T>::type;
  constexpr int NV = Vec4<T>::n;
  const long groups = A.n / NV;
  const long q = (long)blockIdx.x * kLbBlock + threadIdx.x;
  if (q < groups) {
    const V gv = reinterpret_cast<const V *>(A.g)[q];
    double acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = A.coef[0] * lane_of(gv, i);
    for (int k = 0; k < A.nv; ++k) {
      const V x = reinterpret_cast<const V *>(A.v[k])[q];
      const double c = A.coef[1 + k];
#pragma unroll
      for (int i = 0; i < NV; ++i) acc[i] += c * lane_of(x, i);
    }
    V out;
    T *o = reinterpret_cast<T *>(&out);
#pragma unroll
    for (int i = 0; i < NV; ++i) o[i] = (T)acc[i];
    reinterpret_cast<V *>(A.d)[q] = out;
  } else {
    const long e = groups * NV + (q - groups);
    if (q - groups < NV && e < A.n) {
      double acc = A.coef[0] * (double)A.g[e];
      for (int k = 0; k < A.nv; ++k) acc += A.coef[1 + k] * (double)A.v[k][e];
      A.d[e] = (T)acc;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kLbBlock) void axpy_kernel(const T *__restrict__ x,
                                                        const T *__restrict__ d, double alpha,
                                                        T *__restrict__ out, long n) {
  const long e = (long)blockIdx.x * kLbBlock + threadIdx.x;
  if (e >= n) return;
  out[e] = (T)((double)x[e] + alpha * (double)d[e]);
}

template <typename T>
__global__ __launch_bounds__(kLbBlock) void pair_kernel(const T *__restrict__ d, double alpha,
                                                        const T *__restrict__ g_new,
                                                        const T *__restrict__ g, T *__restrict__ s,
                                                        T *__restrict__ y, long n) {
  const long e = (long)blockIdx.x * kLbBlock + threadIdx.x;
  if (e >= n) return;
  s[e] = (T)(alpha * (double)d[e]);
  y[e] = g_new[e] - g[e];
}

}  // namespace modil

using namespace modil;

struct modil_lbfgs {
  modil_ctx *c = nullptr;
  modil_lbfgs_params prm{};
  long n = 0, n_pad = 0;
  size_t elem = 4;
  char *S = nullptr, *Y = nullptr;        // ring slots, slot i at base + i * n_pad * elem
  char *g = nullptr, *gt = nullptr, *d = nullptr, *xt = nullptr;
  double *partials = nullptr, *dots = nullptr, *coef = nullptr, *terms = nullptr;
  double *h_dots = nullptr, *h_coef = nullptr, *h_terms = nullptr;  // pinned host
  // host state, pairs in logical order (oldest first)
  std::vector<int> slot;            // ring slot of each stored pair
  std::vector<double> R, YY;        // R[i][j] = s_i^T y_j (i <= j), YY[i][j] = y_i^T y_j, m x m
  std::vector<double> a, b;         // S^T g, Y^T g
  double f = 0.0, gg = 0.0;
  bool have = false;
  int iteration = 0;
};

namespace {

int lb_fail(modil_lbfgs *lb, int status, const std::string &msg) {
  return lb && lb->c ? set_ctx_error(lb->c, status, msg) : set_global_error(status, msg);
}

#define LB_HIP(lb, expr, where)                                                          \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return lb_fail(lb, MODIL_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

struct LbCarve {
  size_t S, Y, g, gt, d, xt, partials, dots, coef, terms, end;
};

LbCarve lb_carve(long n_pad, size_t elem, int m, int batch) {
  LbCarve k{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = a256(off + bytes);
    return at;
  };
  const size_t vec = (size_t)n_pad * elem;
  k.S = take(vec * (m + 1));  // one spare slot: a new pair never overwrites a stored one
  k.Y = take(vec * (m + 1));
  k.g = take(vec);
  k.gt = take(vec);
  k.d = take(vec);
  k.xt = take(vec);
  k.partials = take((size_t)kLbMaxChunks * kLbBlocks * 2 * kLbChunk * 8);
  k.dots = take((size_t)2 * kLbMaxLeft * 8);
  k.coef = take((size_t)(2 * MODIL_LBFGS_MAX_HISTORY + 1) * 8);
  k.terms = take((size_t)batch * MODIL_N_TERMS * 8);
  k.end = off;
  return k;
}

void *vec_at(modil_lbfgs *lb, char *base, int slot_i) {
  return base + (size_t)slot_i * lb->n_pad * lb->elem;
}

unsigned nblk_lb(long n) { return (unsigned)((n + kLbBlock - 1) / kLbBlock); }

// dots[r][l] = left[l] . right[r] for the listed vectors (device results)
template <typename T>
hipError_t multidot(modil_lbfgs *lb, const std::vector<const void *> &left,
                    const std::vector<const void *> &right) {
  MultiDotArgs<T> A{};
  A.n_left = (int)left.size();
  A.n_right = (int)right.size();
  for (int i = 0; i < A.n_left; ++i) A.left[i] = (const T *)left[i];
  for (int r = 0; r < A.n_right; ++r) A.right[r] = (const T *)right[r];
  A.n = lb->n;
  A.partials = lb->partials;
  const int chunks = (A.n_left + kLbChunk - 1) / kLbChunk;
  const long groups = lb->n / Vec4<T>::n;
  const int blocks = (int)std::min<long>(kLbBlocks, std::max<long>(1, (groups + kLbBlock - 1) / kLbBlock));
  hipStream_t s = lb->c->stream;
  Timed tm(lb->c, 5);
  multidot_kernel<T><<<dim3(blocks, chunks), kLbBlock, 0, s>>>(A);
  dot_reduce_kernel<<<dim3(A.n_left, A.n_right), 256, 0, s>>>(lb->partials, blocks, A.n_left,
                                                               lb->dots);
  return hipGetLastError();
}

hipError_t multidot_any(modil_lbfgs *lb, const std::vector<const void *> &l,
                        const std::vector<const void *> &r) {
  return lb->elem == 8 ? multidot<double>(lb, l, r) : multidot<float>(lb, l, r);
}

hipError_t fetch(modil_lbfgs *lb, int n_left, int n_right) {
  hipStream_t s = lb->c->stream;
  for (int r = 0; r < n_right; ++r) {
    hipError_t e = hipMemcpyAsync(lb->h_dots + r * kLbMaxLeft, lb->dots + r * kLbMaxLeft,
                                  (size_t)n_left * 8, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
  }
  return hipStreamSynchronize(s);
}

// objective and d-derivative at theta: loss terms and gradient into grad,
// dot(grad, d) when d is given
int objective(modil_lbfgs *lb, const void *theta, void *grad, const void *d, double &f,
              double &dphi) {
  modil_ctx *c = lb->c;
  const int st = eval_loss_grad(c, theta, grad, lb->terms);
  if (st != MODIL_OK) return st;
  const int nt = c->prob.batch * MODIL_N_TERMS;
  LB_HIP(lb, hipMemcpyAsync(lb->h_terms, lb->terms, (size_t)nt * 8, hipMemcpyDeviceToHost, c->stream),
         "terms");
  if (d) {
    LB_HIP(lb, multidot_any(lb, {grad}, {d}), "dot");
    LB_HIP(lb, hipMemcpyAsync(lb->h_dots, lb->dots, 8, hipMemcpyDeviceToHost, c->stream), "dot");
  }
  LB_HIP(lb, hipStreamSynchronize(c->stream), "objective");
  f = 0.0;
  for (int i = 0; i < nt; ++i) f += lb->h_terms[i];
  dphi = d ? lb->h_dots[0] : 0.0;
  return MODIL_OK;
}

template <typename T>
hipError_t launch_axpy(modil_lbfgs *lb, const void *x, double alpha, void *out) {
  Timed tm(lb->c, 6);
  axpy_kernel<T><<<nblk_lb(lb->n), kLbBlock, 0, lb->c->stream>>>((const T *)x, (const T *)lb->d,
                                                                  alpha, (T *)out, lb->n);
  return hipGetLastError();
}

hipError_t axpy(modil_lbfgs *lb, const void *x, double alpha, void *out) {
  return lb->elem == 8 ? launch_axpy<double>(lb, x, alpha, out) : launch_axpy<float>(lb, x, alpha, out);
}

template <typename T>
hipError_t launch_combine(modil_lbfgs *lb, int k) {
  CombineArgs<T> A{};
  A.nv = 2 * k;
  for (int i = 0; i < k; ++i) {
    A.v[i] = (const T *)vec_at(lb, lb->S, lb->slot[i]);
    A.v[k + i] = (const T *)vec_at(lb, lb->Y, lb->slot[i]);
  }
  A.g = (const T *)lb->g;
  A.d = (T *)lb->d;
  A.coef = lb->coef;
  A.n = lb->n;
  Timed tm(lb->c, 6);
  const long groups = lb->n / Vec4<T>::n;
  combine_kernel<T><<<nblk_lb(groups + Vec4<T>::n), kLbBlock, 0, lb->c->stream>>>(A);
  return hipGetLastError();
}

// d = -H g through the compact representation; returns g^T d
int direction(modil_lbfgs *lb, double &dphi0) {
  const int k = (int)lb->slot.size();
  const int m = lb->prm.history;
  std::vector<double> coef(1 + 2 * k, 0.0);
  if (k == 0) {
    coef[0] = -1.0;
    dphi0 = -lb->gg;
  } else {
    auto Rr = [&](int i, int j) { return lb->R[(size_t)i * m + j]; };
    auto YYr = [&](int i, int j) { return lb->YY[(size_t)i * m + j]; };
    const double gamma = Rr(k - 1, k - 1) / YYr(k - 1, k - 1);
    std::vector<double> q(k), t(k), w(k);
    for (int i = k - 1; i >= 0; --i) {  // R q = a (R upper triangular)
      double s = lb->a[i];
      for (int j = i + 1; j < k; ++j) s -= Rr(i, j) * q[j];
      q[i] = s / Rr(i, i);
    }
    for (int i = 0; i < k; ++i) {
      double s = Rr(i, i) * q[i] - gamma * lb->b[i];
      for (int j = 0; j < k; ++j) s += gamma * YYr(i, j) * q[j];
      t[i] = s;
    }
    for (int i = 0; i < k; ++i) {  // R^T w = t (R^T lower triangular)
      double s = t[i];
      for (int j = 0; j < i; ++j) s -= Rr(j, i) * w[j];
      w[i] = s / Rr(i, i);
    }
    coef[0] = -gamma;
    dphi0 = -gamma * lb->gg;
    for (int i = 0; i < k; ++i) {
      coef[1 + i] = -w[i];
      coef[1 + k + i] = gamma * q[i];
      dphi0 += -w[i] * lb->a[i] + gamma * q[i] * lb->b[i];
    }
  }
  std::memcpy(lb->h_coef, coef.data(), coef.size() * 8);
  hipStream_t s = lb->c->stream;
  LB_HIP(lb, hipMemcpyAsync(lb->coef, lb->h_coef, coef.size() * 8, hipMemcpyHostToDevice, s), "coef");
  LB_HIP(lb, lb->elem == 8 ? launch_combine<double>(lb, k) : launch_combine<float>(lb, k), "combine");
  // the coefficients are read by the kernel before the host buffer is reused:
  // the line search synchronises the stream before the next direction
  return MODIL_OK;
}

// after a pair was written to `new_slot` (or none, new_slot < 0): the dot
// products of the new gradient (and the new y) with every stored vector
int refresh(modil_lbfgs *lb, int new_slot) {
  const int k = (int)lb->slot.size();
  std::vector<const void *> left;
  for (int i = 0; i < k; ++i) left.push_back(vec_at(lb, lb->S, lb->slot[i]));
  if (new_slot >= 0) left.push_back(vec_at(lb, lb->S, new_slot));
  for (int i = 0; i < k; ++i) left.push_back(vec_at(lb, lb->Y, lb->slot[i]));
  if (new_slot >= 0) left.push_back(vec_at(lb, lb->Y, new_slot));
  left.push_back(lb->g);
  std::vector<const void *> right = {lb->g};
  if (new_slot >= 0) right.push_back(vec_at(lb, lb->Y, new_slot));
  LB_HIP(lb, multidot_any(lb, left, right), "dots");
  LB_HIP(lb, fetch(lb, (int)left.size(), (int)right.size()), "dots");
  const int kk = k + (new_slot >= 0 ? 1 : 0);
  const double *dg = lb->h_dots;                 // right = g
  const double *dy = lb->h_dots + kLbMaxLeft;    // right = y_new
  const int m = lb->prm.history;
  bool keep = false;
  if (new_slot >= 0) {
    const double sy = dy[k], yy = dy[kk + k];
    keep = sy > std::numeric_limits<double>::epsilon() * yy;
  }
  if (keep) {
    // drop the oldest pair when full, then append the new one
    std::vector<double> sg(dg, dg + kk), yg(dg + kk, dg + 2 * kk), sy(dy, dy + kk), yy(dy + kk, dy + 2 * kk);
    int first = 0;
    if (kk > m) {
      first = 1;
      std::vector<double> R2((size_t)m * m, 0.0), Y2((size_t)m * m, 0.0);
      for (int i = 1; i < k; ++i)
        for (int j = 1; j < k; ++j) {
          R2[(size_t)(i - 1) * m + (j - 1)] = lb->R[(size_t)i * m + j];
          Y2[(size_t)(i - 1) * m + (j - 1)] = lb->YY[(size_t)i * m + j];
        }
      lb->R.swap(R2);
      lb->YY.swap(Y2);
      lb->slot.erase(lb->slot.begin());
    }
    const int kn = kk - first;  // pairs after the update
    for (int i = 0; i < kn; ++i) {
      lb->R[(size_t)i * m + (kn - 1)] = sy[first + i];
      lb->YY[(size_t)i * m + (kn - 1)] = yy[first + i];
      lb->YY[(size_t)(kn - 1) * m + i] = yy[first + i];
    }
    lb->slot.push_back(new_slot);
    lb->a.assign(sg.begin() + first, sg.end());
    lb->b.assign(yg.begin() + first, yg.end());
    lb->gg = dg[2 * kk];
  } else {
    // the new pair (if any) is not stored: keep the old pairs' products with g
    lb->a.assign(dg, dg + k);
    lb->b.assign(dg + kk, dg + kk + k);
    lb->gg = dg[2 * kk];
  }
  return MODIL_OK;
}

void clear_pairs(modil_lbfgs *lb) {
  lb->slot.clear();
  lb->a.clear();
  lb->b.clear();
  std::fill(lb->R.begin(), lb->R.end(), 0.0);
  std::fill(lb->YY.begin(), lb->YY.end(), 0.0);
}

// a ring slot that holds no stored pair (there are history + 1 slots)
int free_slot(const modil_lbfgs *lb) {
  for (int s = 0; s <= lb->prm.history; ++s)
    if (std::find(lb->slot.begin(), lb->slot.end(), s) == lb->slot.end()) return s;
  return -1;  // unreachable: at most `history` slots are in use
}

// cubic minimiser through (a, fa, da), (b, fb, db); NaN if there is none
double cubic_step(double a, double fa, double da, double b, double fb, double db) {
  const double v[6] = {a, fa, da, b, fb, db};
  for (double x : v)
    if (!std::isfinite(x)) return NAN;
  if (a == b) return NAN;
  const double d1 = da + db - 3.0 * (fa - fb) / (a - b);
  const double disc = d1 * d1 - da * db;
  if (disc < 0.0) return NAN;
  const double d2 = std::copysign(std::sqrt(disc), b - a);
  const double den = db - da + 2.0 * d2;
  if (den == 0.0) return NAN;
  return b - (b - a) * (db + d2 - d1) / den;
}

double trial_step(double lo, double flo, double dlo, double hi, double fhi, double dhi) {
  const double a = std::min(lo, hi), b = std::max(lo, hi), w = b - a;
  double t = cubic_step(lo, flo, dlo, hi, fhi, dhi);
  if (!(t >= a + 0.1 * w && t <= b - 0.1 * w)) t = 0.5 * (lo + hi);
  return t;
}

struct LsOut {
  double alpha = 0.0, f = 0.0;
  int status = 2, evals = 0;
  bool grad_current = false;  // gt holds the gradient at alpha
};

// strong-Wolfe line search along d from theta (Nocedal & Wright 3.5 / 3.6)
int line_search(modil_lbfgs *lb, const void *theta, double dphi0, double alpha1, LsOut &out) {
  const double f0 = lb->f, c1 = lb->prm.c1, c2 = lb->prm.c2;
  const int max_evals = lb->prm.max_evals;
  int evals = 0;
  double last_alpha = -1.0;
  auto phi = [&](double a, double &fa, double &da) -> int {
    ++evals;
    hipError_t e = axpy(lb, theta, a, lb->xt);
    if (e != hipSuccess) return lb_fail(lb, MODIL_ERR_HIP, std::string("axpy: ") + hipGetErrorString(e));
    const int st = objective(lb, lb->xt, lb->gt, lb->d, fa, da);
    last_alpha = a;
    return st;
  };
  auto decrease = [&](double a, double fa) { return std::isfinite(fa) && fa <= f0 + c1 * a * dphi0; };
  auto finish = [&](double a, double fa, int status) {
    out.alpha = a;
    out.f = fa;
    out.status = status;
    out.evals = evals;
    out.grad_current = last_alpha == a;
    return MODIL_OK;
  };
  auto zoom = [&](double lo, double flo, double dlo, double hi, double fhi, double dhi) -> int {
    while (evals < max_evals) {
      const double a = trial_step(lo, flo, dlo, hi, fhi, dhi);
      double fa, da;
      const int st = phi(a, fa, da);
      if (st != MODIL_OK) return st;
      if (!decrease(a, fa) || fa >= flo) {
        hi = a; fhi = fa; dhi = da;
      } else {
        if (std::fabs(da) <= -c2 * dphi0) return finish(a, fa, 0);
        if (da * (hi - lo) >= 0.0) { hi = lo; fhi = flo; dhi = dlo; }
        lo = a; flo = fa; dlo = da;
      }
    }
    if (lo > 0.0) return finish(lo, flo, 1);
    return finish(0.0, f0, 2);
  };
  double a_prev = 0.0, f_prev = f0, d_prev = dphi0, a = alpha1;
  bool first = true;
  while (evals < max_evals) {
    double fa, da;
    const int st = phi(a, fa, da);
    if (st != MODIL_OK) return st;
    if (!decrease(a, fa) || (!first && fa >= f_prev)) return zoom(a_prev, f_prev, d_prev, a, fa, da);
    if (std::fabs(da) <= -c2 * dphi0) return finish(a, fa, 0);
    if (da >= 0.0) return zoom(a, fa, da, a_prev, f_prev, d_prev);
    a_prev = a; f_prev = fa; d_prev = da;
    a = 2.0 * a;
    first = false;
  }
  if (a_prev > 0.0) return finish(a_prev, f_prev, 1);
  return finish(0.0, f0, 2);
}

int validate_params(const modil_lbfgs_params *p, std::string &msg) {
  if (!p) { msg = "params is NULL"; return MODIL_ERR_INVALID_ARG; }
  if (p->history < 1 || p->history > MODIL_LBFGS_MAX_HISTORY) {
    msg = "history must be in 1..64";
    return MODIL_ERR_INVALID_ARG;
  }
  if (p->max_evals < 2) { msg = "max_evals must be >= 2"; return MODIL_ERR_INVALID_ARG; }
  if (!(p->c1 > 0.0 && p->c1 < p->c2 && p->c2 < 1.0)) {
    msg = "Wolfe constants must satisfy 0 < c1 < c2 < 1";
    return MODIL_ERR_INVALID_ARG;
  }
  return MODIL_OK;
}

}  // namespace

extern "C" {

int modil_lbfgs_workspace(const modil_ctx *c, int32_t history, size_t *bytes) {
  if (!c || !bytes) return set_global_error(MODIL_ERR_INVALID_ARG, "ctx or bytes is NULL");
  if (history < 1 || history > MODIL_LBFGS_MAX_HISTORY)
    return set_global_error(MODIL_ERR_INVALID_ARG, "history must be in 1..64");
  const size_t elem = c->prob.dtype == MODIL_F64 ? 8 : 4;
  const long n = c->lay.total;
  const long n_pad = (n + 63) / 64 * 64;
  *bytes = lb_carve(n_pad, elem, history, c->prob.batch).end;
  return MODIL_OK;
}

int modil_lbfgs_create(modil_ctx *c, const modil_lbfgs_params *prm, void *ws, size_t ws_bytes,
                       modil_lbfgs **out) {
  if (!c || !out) return set_global_error(MODIL_ERR_INVALID_ARG, "ctx or out is NULL");
  *out = nullptr;
  std::string msg;
  int st = validate_params(prm, msg);
  if (st != MODIL_OK) return set_ctx_error(c, st, msg);
  size_t need = 0;
  st = modil_lbfgs_workspace(c, prm->history, &need);
  if (st != MODIL_OK) return st;
  if (!ws || ws_bytes < need || reinterpret_cast<uintptr_t>(ws) % 256)
    return set_ctx_error(c, MODIL_ERR_INVALID_ARG,
                         "workspace must be 256-byte aligned and hold " + std::to_string(need) + " bytes");
  modil_lbfgs *lb = new (std::nothrow) modil_lbfgs();
  if (!lb) return set_ctx_error(c, MODIL_ERR_STATE, "out of host memory");
  lb->c = c;
  lb->prm = *prm;
  lb->elem = c->prob.dtype == MODIL_F64 ? 8 : 4;
  lb->n = c->lay.total;
  lb->n_pad = (lb->n + 63) / 64 * 64;
  const LbCarve k = lb_carve(lb->n_pad, lb->elem, prm->history, c->prob.batch);
  char *base = static_cast<char *>(ws);
  lb->S = base + k.S;
  lb->Y = base + k.Y;
  lb->g = base + k.g;
  lb->gt = base + k.gt;
  lb->d = base + k.d;
  lb->xt = base + k.xt;
  lb->partials = reinterpret_cast<double *>(base + k.partials);
  lb->dots = reinterpret_cast<double *>(base + k.dots);
  lb->coef = reinterpret_cast<double *>(base + k.coef);
  lb->terms = reinterpret_cast<double *>(base + k.terms);
  const size_t host_bytes = (2 * kLbMaxLeft + (2 * MODIL_LBFGS_MAX_HISTORY + 1) +
                             (size_t)c->prob.batch * MODIL_N_TERMS) * 8;
  void *h = nullptr;
  if (hipHostMalloc(&h, host_bytes, hipHostMallocDefault) != hipSuccess) {
    delete lb;
    return set_ctx_error(c, MODIL_ERR_HIP, "pinned host buffer");
  }
  lb->h_dots = static_cast<double *>(h);
  lb->h_coef = lb->h_dots + 2 * kLbMaxLeft;
  lb->h_terms = lb->h_coef + (2 * MODIL_LBFGS_MAX_HISTORY + 1);
  const int m = prm->history;
  lb->R.assign((size_t)m * m, 0.0);
  lb->YY.assign((size_t)m * m, 0.0);
  *out = lb;
  return MODIL_OK;
}

int modil_lbfgs_destroy(modil_lbfgs *lb) {
  if (!lb) return MODIL_OK;
  // every call ends synchronised, so no copy into the pinned buffer is pending
  if (lb->h_dots) (void)hipHostFree(lb->h_dots);
  delete lb;
  return MODIL_OK;
}

int modil_lbfgs_reset(modil_lbfgs *lb) {
  if (!lb) return set_global_error(MODIL_ERR_INVALID_ARG, "lbfgs is NULL");
  clear_pairs(lb);
  lb->have = false;
  lb->iteration = 0;
  return MODIL_OK;
}

int modil_lbfgs_step(modil_lbfgs *lb, void *theta, modil_lbfgs_info *info) {
  if (!lb || !theta) return set_global_error(MODIL_ERR_INVALID_ARG, "lbfgs or theta is NULL");
  if (reinterpret_cast<uintptr_t>(theta) % lb->elem)
    return lb_fail(lb, MODIL_ERR_INVALID_ARG, "theta is not aligned to its element size");
  int evals = 0;
  if (!lb->have) {
    double f, unused;
    const int st = objective(lb, theta, lb->g, nullptr, f, unused);
    if (st != MODIL_OK) return st;
    ++evals;
    lb->f = f;
    const int st2 = refresh(lb, -1);
    if (st2 != MODIL_OK) return st2;
    lb->have = true;
  }
  double dphi0 = 0.0;
  int st = direction(lb, dphi0);
  if (st != MODIL_OK) return st;
  if (!(dphi0 < 0.0) && !lb->slot.empty()) {  // not a descent direction: forget the pairs
    clear_pairs(lb);
    st = direction(lb, dphi0);
    if (st != MODIL_OK) return st;
  }
  LsOut ls;
  if (dphi0 < 0.0) {
    const double alpha1 = lb->slot.empty() ? std::min(1.0, 1.0 / std::sqrt(lb->gg)) : 1.0;
    st = line_search(lb, theta, dphi0, alpha1, ls);
    if (st != MODIL_OK) return st;
  }
  evals += ls.evals;
  if (ls.status == 2) {
    clear_pairs(lb);
    st = refresh(lb, -1);
    if (st != MODIL_OK) return st;
  } else {
    if (!ls.grad_current) {  // the accepted point was evaluated earlier: evaluate it again
      LB_HIP(lb, axpy(lb, theta, ls.alpha, lb->xt), "axpy");
      double f, unused;
      st = objective(lb, lb->xt, lb->gt, nullptr, f, unused);
      if (st != MODIL_OK) return st;
      ++evals;
    }
    const int sl = free_slot(lb);
    {
      hipStream_t s = lb->c->stream;
      Timed tm(lb->c, 6);
      if (lb->elem == 8)
        pair_kernel<double><<<nblk_lb(lb->n), kLbBlock, 0, s>>>(
            (const double *)lb->d, ls.alpha, (const double *)lb->gt, (const double *)lb->g,
            (double *)vec_at(lb, lb->S, sl), (double *)vec_at(lb, lb->Y, sl), lb->n);
      else
        pair_kernel<float><<<nblk_lb(lb->n), kLbBlock, 0, s>>>(
            (const float *)lb->d, ls.alpha, (const float *)lb->gt, (const float *)lb->g,
            (float *)vec_at(lb, lb->S, sl), (float *)vec_at(lb, lb->Y, sl), lb->n);
      LB_HIP(lb, hipGetLastError(), "pair");
      LB_HIP(lb, hipMemcpyAsync(theta, lb->xt, (size_t)lb->n * lb->elem, hipMemcpyDeviceToDevice, s),
             "accept");
    }
    std::swap(lb->g, lb->gt);
    lb->f = ls.f;
    st = refresh(lb, sl);  // stores the pair (dropping the oldest when full) or discards it
    if (st != MODIL_OK) return st;
    ++lb->iteration;
  }
  if (info) {
    info->loss = lb->f;
    info->grad_norm = std::sqrt(lb->gg);
    info->step = ls.status == 2 ? 0.0 : ls.alpha;
    info->evals = evals;
    info->status = ls.status;
    info->pairs = (int)lb->slot.size();
    info->iteration = lb->iteration;
  }
  return MODIL_OK;
}

}  // extern "C"
