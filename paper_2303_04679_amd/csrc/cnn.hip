// Warm-start network: rasterisation of measurements, direct convolutions
// (bf16 weights widened to float, float accumulation), ReLU, mean squared
// error, backward data / weight passes and Adam with bf16 re-rounding.
//
// All reductions are deterministic: every output element (or weight
// gradient) is owned by one thread or one block that sums its terms in a
// fixed order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "internal.h"

struct modil_cnn {
  modil_cnn_desc d;
  modil_cnn_layout_t lay;
  hipStream_t stream;
  char *ws;
  float *dact;      // [batch][act_size] gradients of the trunk activations
  float *dout;      // [batch][out_size] gradient of the loss w.r.t. the head maps
  double *lpart;    // loss partial sums
  long n_lpart;
};

namespace modil {
namespace {

constexpr int kB = 256;

struct Layer {
  int ci, co, k, s, p, hin, hout, relu;
  long w_off, b_off;
};

// the six layers for one descriptor: 0..2 trunk, 3..5 heads
void layers(const modil_cnn_desc &d, Layer (&L)[6]) {
  const int s1 = d.size / 4, s2 = d.size / 8, s3 = d.size / 16;
  L[0] = {4, d.width1, 4, 4, 0, d.size, s1, 1, 0, 0};
  L[1] = {d.width1, d.width2, 3, 2, 1, s1, s2, 1, 0, 0};
  L[2] = {d.width2, d.width3, 3, 2, 1, s2, s3, 1, 0, 0};
  L[3] = {d.width1, d.out_ch, 3, 1, 1, s1, s1, 0, 0, 0};
  L[4] = {d.width2, d.out_ch, 3, 1, 1, s2, s2, 0, 0, 0};
  L[5] = {d.width3, d.out_ch, 3, 1, 1, s3, s3, 0, 0, 0};
  long off = 0;
  for (auto &l : L) {
    l.w_off = off;
    off += (long)l.co * l.ci * l.k * l.k;
    l.b_off = off;
    off += l.co;
  }
}

__device__ inline float bf16_to_f32(uint16_t h) {
  return __uint_as_float((uint32_t)h << 16);
}

// round to nearest, ties to even
__device__ inline uint16_t f32_to_bf16(float x) {
  const uint32_t u = __float_as_uint(x);
  const uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(r >> 16);
}

// ---------------------------------------------------------------- kernels
__global__ __launch_bounds__(kB) void raster_bg_kernel(float *img, int B, int S, const float *re,
                                                       float c, float sc) {
  const long n = (long)B * 4 * S * S;
  const long e = (long)blockIdx.x * kB + threadIdx.x;
  if (e >= n) return;
  const long plane = (long)S * S;
  const int ch = (int)((e / plane) % 4);
  const int b = (int)(e / (4 * plane));
  img[e] = ch == 3 ? (re[b] - c) / sc : 0.f;
}

__global__ __launch_bounds__(kB) void raster_obs_kernel(float *img, int B, int S, int n_obs,
                                                        const int32_t *idx, const float *u,
                                                        const float *v) {
  const int e = blockIdx.x * kB + threadIdx.x;
  if (e >= B * n_obs) return;
  const int b = e / n_obs;
  const long plane = (long)S * S;
  const int k = idx[e];
  float *base = img + (long)b * 4 * plane;
  base[k] = u[e];
  base[plane + k] = v[e];
  base[2 * plane + k] = 1.f;
}

// out[b][co][y][x] = bias + sum W * in (zero padding), optional ReLU
__global__ __launch_bounds__(kB) void conv_fwd_kernel(const float *__restrict__ in,
                                                      const uint16_t *__restrict__ P, Layer L,
                                                      float *__restrict__ out, int B, long in_bs,
                                                      long out_bs) {
  const long n = (long)B * L.co * L.hout * L.hout;
  const long e = (long)blockIdx.x * kB + threadIdx.x;
  if (e >= n) return;
  const int x = (int)(e % L.hout), y = (int)((e / L.hout) % L.hout);
  const int co = (int)((e / ((long)L.hout * L.hout)) % L.co);
  const int b = (int)(e / ((long)L.hout * L.hout * L.co));
  const float *ib = in + b * in_bs;
  const uint16_t *w = P + L.w_off + (long)co * L.ci * L.k * L.k;
  float acc = bf16_to_f32(P[L.b_off + co]);
  for (int ci = 0; ci < L.ci; ++ci) {
    const float *ic = ib + (long)ci * L.hin * L.hin;
    for (int ky = 0; ky < L.k; ++ky) {
      const int iy = y * L.s - L.p + ky;
      if (iy < 0 || iy >= L.hin) continue;
      for (int kx = 0; kx < L.k; ++kx) {
        const int ix = x * L.s - L.p + kx;
        if (ix < 0 || ix >= L.hin) continue;
        acc += bf16_to_f32(w[(ci * L.k + ky) * L.k + kx]) * ic[iy * L.hin + ix];
      }
    }
  }
  if (L.relu) acc = acc > 0.f ? acc : 0.f;
  out[b * out_bs + ((long)co * L.hout + y) * L.hout + x] = acc;
}

// gradient at the layer's pre-activation: dout, masked by the ReLU of the output
__device__ inline float dpre(const float *dout, const float *out, long i, int relu) {
  return relu ? (out[i] > 0.f ? dout[i] : 0.f) : dout[i];
}

// din[b][ci][y][x] (+)= sum_{co,ky,kx} W[co][ci][ky][kx] dpre[b][co][oy][ox]
__global__ __launch_bounds__(kB) void conv_bwd_data_kernel(const float *__restrict__ dout,
                                                           const float *__restrict__ out,
                                                           const uint16_t *__restrict__ P, Layer L,
                                                           float *__restrict__ din, int B,
                                                           long in_bs, long out_bs, int accumulate) {
  const long n = (long)B * L.ci * L.hin * L.hin;
  const long e = (long)blockIdx.x * kB + threadIdx.x;
  if (e >= n) return;
  const int x = (int)(e % L.hin), y = (int)((e / L.hin) % L.hin);
  const int ci = (int)((e / ((long)L.hin * L.hin)) % L.ci);
  const int b = (int)(e / ((long)L.hin * L.hin * L.ci));
  float acc = 0.f;
  for (int co = 0; co < L.co; ++co) {
    const uint16_t *w = P + L.w_off + ((long)co * L.ci + ci) * L.k * L.k;
    const long ob = b * out_bs + (long)co * L.hout * L.hout;
    for (int ky = 0; ky < L.k; ++ky) {
      const int t = y + L.p - ky;
      if (t < 0 || t % L.s) continue;
      const int oy = t / L.s;
      if (oy >= L.hout) continue;
      for (int kx = 0; kx < L.k; ++kx) {
        const int u = x + L.p - kx;
        if (u < 0 || u % L.s) continue;
        const int ox = u / L.s;
        if (ox >= L.hout) continue;
        acc += bf16_to_f32(w[ky * L.k + kx]) * dpre(dout, out, ob + (long)oy * L.hout + ox, L.relu);
      }
    }
  }
  float *d = din + b * in_bs + ((long)ci * L.hin + y) * L.hin + x;
  *d = accumulate ? *d + acc : acc;
}

// one block per weight (and one per bias): sum over (b, oy, ox) in a fixed order
__global__ __launch_bounds__(kB) void conv_bwd_weight_kernel(const float *__restrict__ dout,
                                                             const float *__restrict__ out,
                                                             const float *__restrict__ in, Layer L,
                                                             float *__restrict__ grad, int B,
                                                             long in_bs, long out_bs) {
  const long nw = (long)L.co * L.ci * L.k * L.k;
  const long widx = blockIdx.x;  // < nw: weight, else bias of co = widx - nw
  const long m = (long)B * L.hout * L.hout;
  float acc = 0.f;
  if (widx < nw) {
    const int kx = (int)(widx % L.k), ky = (int)((widx / L.k) % L.k);
    const int ci = (int)((widx / ((long)L.k * L.k)) % L.ci);
    const int co = (int)(widx / ((long)L.k * L.k * L.ci));
    for (long t = threadIdx.x; t < m; t += kB) {
      const int ox = (int)(t % L.hout), oy = (int)((t / L.hout) % L.hout);
      const int b = (int)(t / ((long)L.hout * L.hout));
      const int iy = oy * L.s - L.p + ky, ix = ox * L.s - L.p + kx;
      if (iy < 0 || iy >= L.hin || ix < 0 || ix >= L.hin) continue;
      const long oi = b * out_bs + ((long)co * L.hout + oy) * L.hout + ox;
      acc += dpre(dout, out, oi, L.relu) * in[b * in_bs + ((long)ci * L.hin + iy) * L.hin + ix];
    }
  } else {
    const int co = (int)(widx - nw);
    for (long t = threadIdx.x; t < m; t += kB) {
      const int ox = (int)(t % L.hout), oy = (int)((t / L.hout) % L.hout);
      const int b = (int)(t / ((long)L.hout * L.hout));
      acc += dpre(dout, out, b * out_bs + ((long)co * L.hout + oy) * L.hout + ox, L.relu);
    }
  }
  __shared__ float sh[kB];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) grad[widx < nw ? L.w_off + widx : L.b_off + (widx - nw)] = sh[0];
}

// d = 2 (y - t) / n; per-block FP64 partial sums of (y - t)^2 / n
__global__ __launch_bounds__(kB) void mse_kernel(const float *y, const float *t, float *d, long n,
                                                 double *part) {
  const long e = (long)blockIdx.x * kB + threadIdx.x;
  double s = 0.0;
  if (e < n) {
    const float r = y[e] - t[e];
    d[e] = 2.f * r / (float)n;
    s = (double)r * (double)r / (double)n;
  }
  __shared__ double sh[kB];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kB) void sum_kernel(const double *part, long n, double *out) {
  double s = 0.0;
  for (long i = threadIdx.x; i < n; i += kB) s += part[i];
  __shared__ double sh[kB];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

__global__ __launch_bounds__(kB) void cnn_adam_kernel(float *w, uint16_t *wb, float *m, float *v,
                                                      const float *g, long n, float b1, float b2,
                                                      float step, float isb2, float eps) {
  const long e = (long)blockIdx.x * kB + threadIdx.x;
  if (e >= n) return;
  const float gg = g[e];
  const float mm = b1 * m[e] + (1.f - b1) * gg;
  const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
  m[e] = mm;
  v[e] = vv;
  const float x = w[e] - step * mm / (sqrtf(vv) * isb2 + eps);
  w[e] = x;
  wb[e] = f32_to_bf16(x);
}

__global__ __launch_bounds__(kB) void to_bf16_kernel(const float *w, uint16_t *wb, long n) {
  const long e = (long)blockIdx.x * kB + threadIdx.x;
  if (e < n) wb[e] = f32_to_bf16(w[e]);
}

inline unsigned nb(long n) { return (unsigned)((n + kB - 1) / kB); }

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int validate(const modil_cnn_desc *d, std::string &msg) {
  if (!d) { msg = "descriptor is NULL"; return MODIL_ERR_INVALID_ARG; }
  if (d->batch < 1 || d->size < 16 || d->size % 16 || d->n_obs < 0 || d->n_obs > d->size * d->size ||
      d->width1 < 1 || d->width2 < 1 || d->width3 < 1 || d->out_ch < 1 || !(d->re_scale != 0.0)) {
    msg = "bad network descriptor";
    return MODIL_ERR_INVALID_ARG;
  }
  return MODIL_OK;
}

void fill(const modil_cnn_desc &d, modil_cnn_layout_t &lay, long &n_lpart) {
  Layer L[6];
  layers(d, L);
  std::memset(&lay, 0, sizeof(lay));
  for (int i = 0; i < 6; ++i) {
    lay.w_offset[i] = L[i].w_off;
    lay.b_offset[i] = L[i].b_off;
  }
  lay.n_params = L[5].b_off + L[5].co;
  lay.img_size = 4L * d.size * d.size;
  const long s1 = d.size / 4, s2 = d.size / 8, s3 = d.size / 16;
  lay.act_size = d.width1 * s1 * s1 + d.width2 * s2 * s2 + d.width3 * s3 * s3;
  lay.out_size = (long)d.out_ch * (s1 * s1 + s2 * s2 + s3 * s3);
  n_lpart = ((long)d.batch * lay.out_size + kB - 1) / kB;
  size_t off = 0;
  off = align256(off + (size_t)d.batch * lay.act_size * 4);
  off = align256(off + (size_t)d.batch * lay.out_size * 4);
  off = align256(off + (size_t)n_lpart * 8);
  lay.workspace_bytes = off;
}

#define CNN_HIP(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return set_global_error(MODIL_ERR_HIP, std::string("cnn: ") + hipGetErrorString(e_)); \
  } while (0)

}  // namespace
}  // namespace modil

using namespace modil;

extern "C" {

int modil_cnn_layout(const modil_cnn_desc *d, modil_cnn_layout_t *out) {
  std::string msg;
  const int st = validate(d, msg);
  if (st) return set_global_error(st, msg);
  if (!out) return set_global_error(MODIL_ERR_INVALID_ARG, "layout output is NULL");
  long np;
  fill(*d, *out, np);
  return MODIL_OK;
}

int modil_cnn_create(const modil_cnn_desc *d, void *ws, size_t ws_bytes, void *stream,
                     modil_cnn **out) {
  std::string msg;
  const int st = validate(d, msg);
  if (st) return set_global_error(st, msg);
  if (!out) return set_global_error(MODIL_ERR_INVALID_ARG, "output handle is NULL");
  modil_cnn_layout_t lay;
  long np;
  fill(*d, lay, np);
  if (!ws || ws_bytes < lay.workspace_bytes || reinterpret_cast<uintptr_t>(ws) % 256)
    return set_global_error(MODIL_ERR_INVALID_ARG, "workspace NULL, too small or not 256-byte aligned");
  modil_cnn *n = new (std::nothrow) modil_cnn();
  if (!n) return set_global_error(MODIL_ERR_STATE, "out of host memory");
  n->d = *d;
  n->lay = lay;
  n->stream = (hipStream_t)stream;
  n->ws = (char *)ws;
  n->n_lpart = np;
  size_t off = 0;
  n->dact = (float *)(n->ws + off);
  off = align256(off + (size_t)d->batch * lay.act_size * 4);
  n->dout = (float *)(n->ws + off);
  off = align256(off + (size_t)d->batch * lay.out_size * 4);
  n->lpart = (double *)(n->ws + off);
  *out = n;
  return MODIL_OK;
}

int modil_cnn_destroy(modil_cnn *n) {
  delete n;
  return MODIL_OK;
}

static int check_batch(const modil_cnn *n, int32_t batch) {
  if (!n) return set_global_error(MODIL_ERR_INVALID_ARG, "net is NULL");
  if (batch < 1 || batch > n->d.batch) return set_global_error(MODIL_ERR_SHAPE, "batch out of range");
  return MODIL_OK;
}

int modil_cnn_rasterize(modil_cnn *n, int32_t batch, const int32_t *idx, const float *u,
                        const float *v, const float *re, float *img) {
  int st = check_batch(n, batch);
  if (st) return st;
  if (!re || !img || (n->d.n_obs && (!idx || !u || !v)))
    return set_global_error(MODIL_ERR_INVALID_ARG, "NULL pointer");
  const int S = n->d.size;
  raster_bg_kernel<<<nb((long)batch * 4 * S * S), kB, 0, n->stream>>>(
      img, batch, S, re, (float)n->d.re_center, (float)n->d.re_scale);
  if (n->d.n_obs)
    raster_obs_kernel<<<nb((long)batch * n->d.n_obs), kB, 0, n->stream>>>(img, batch, S, n->d.n_obs,
                                                                          idx, u, v);
  CNN_HIP(hipGetLastError());
  return MODIL_OK;
}

// trunk activation and head-map bases inside the per-image act / out arrays
static void bases(const modil_cnn *n, long (&act_off)[3], long (&out_off)[3]) {
  const long s1 = n->d.size / 4, s2 = n->d.size / 8;
  act_off[0] = 0;
  act_off[1] = n->d.width1 * s1 * s1;
  act_off[2] = act_off[1] + n->d.width2 * s2 * s2;
  out_off[0] = 0;
  out_off[1] = n->d.out_ch * s1 * s1;
  out_off[2] = out_off[1] + n->d.out_ch * s2 * s2;
}

int modil_cnn_forward(modil_cnn *n, int32_t batch, const uint16_t *P, const float *img, float *acts,
                      float *out) {
  int st = check_batch(n, batch);
  if (st) return st;
  if (!P || !img || !acts || !out) return set_global_error(MODIL_ERR_INVALID_ARG, "NULL pointer");
  Layer L[6];
  layers(n->d, L);
  long ao[3], oo[3];
  bases(n, ao, oo);
  const long A = n->lay.act_size, O = n->lay.out_size, I = n->lay.img_size;
  const float *src[3] = {img, acts + ao[0], acts + ao[1]};
  const long src_bs[3] = {I, A, A};
  for (int i = 0; i < 3; ++i) {
    const long cnt = (long)batch * L[i].co * L[i].hout * L[i].hout;
    conv_fwd_kernel<<<nb(cnt), kB, 0, n->stream>>>(src[i], P, L[i], acts + ao[i], batch, src_bs[i], A);
  }
  for (int h = 0; h < 3; ++h) {
    const long cnt = (long)batch * L[3 + h].co * L[3 + h].hout * L[3 + h].hout;
    conv_fwd_kernel<<<nb(cnt), kB, 0, n->stream>>>(acts + ao[h], P, L[3 + h], out + oo[h], batch, A, O);
  }
  CNN_HIP(hipGetLastError());
  return MODIL_OK;
}

int modil_cnn_loss_backward(modil_cnn *n, int32_t batch, const uint16_t *P, const float *img,
                            const float *acts, const float *out, const float *target, double *loss,
                            float *grad) {
  int st = check_batch(n, batch);
  if (st) return st;
  if (!P || !img || !acts || !out || !target || !loss || !grad)
    return set_global_error(MODIL_ERR_INVALID_ARG, "NULL pointer");
  Layer L[6];
  layers(n->d, L);
  long ao[3], oo[3];
  bases(n, ao, oo);
  const long A = n->lay.act_size, O = n->lay.out_size, I = n->lay.img_size;
  const long nout = (long)batch * O;
  const long np = (nout + kB - 1) / kB;
  mse_kernel<<<nb(nout), kB, 0, n->stream>>>(out, target, n->dout, nout, n->lpart);
  sum_kernel<<<1, kB, 0, n->stream>>>(n->lpart, np, loss);
  // heads: weight gradients and the data gradient into the trunk activations
  for (int h = 0; h < 3; ++h) {
    const Layer &l = L[3 + h];
    conv_bwd_weight_kernel<<<(unsigned)((long)l.co * l.ci * l.k * l.k + l.co), kB, 0, n->stream>>>(
        n->dout + oo[h], out + oo[h], acts + ao[h], l, grad, batch, A, O);
    conv_bwd_data_kernel<<<nb((long)batch * l.ci * l.hin * l.hin), kB, 0, n->stream>>>(
        n->dout + oo[h], out + oo[h], P, l, n->dact + ao[h], batch, A, O, 0);
  }
  // trunk, deepest first: layer i consumes activation i-1 (or the image)
  for (int i = 2; i >= 0; --i) {
    const Layer &l = L[i];
    const float *in = i == 0 ? img : acts + ao[i - 1];
    const long in_bs = i == 0 ? I : A;
    conv_bwd_weight_kernel<<<(unsigned)((long)l.co * l.ci * l.k * l.k + l.co), kB, 0, n->stream>>>(
        n->dact + ao[i], acts + ao[i], in, l, grad, batch, in_bs, A);
    if (i > 0)
      conv_bwd_data_kernel<<<nb((long)batch * l.ci * l.hin * l.hin), kB, 0, n->stream>>>(
          n->dact + ao[i], acts + ao[i], P, l, n->dact + ao[i - 1], batch, A, A, 1);
  }
  CNN_HIP(hipGetLastError());
  return MODIL_OK;
}

int modil_cnn_adam(modil_cnn *n, float *w, uint16_t *wb, float *m, float *v, const float *g,
                   const modil_adam_hp *hp, int64_t step) {
  if (!n) return set_global_error(MODIL_ERR_INVALID_ARG, "net is NULL");
  if (!w || !wb || !m || !v || !g || !hp || step < 1)
    return set_global_error(MODIL_ERR_INVALID_ARG, "bad Adam arguments");
  const double bc1 = 1.0 - std::pow(hp->beta1, (double)step);
  const double bc2 = 1.0 - std::pow(hp->beta2, (double)step);
  const long np = n->lay.n_params;
  cnn_adam_kernel<<<nb(np), kB, 0, n->stream>>>(w, wb, m, v, g, np, (float)hp->beta1,
                                                (float)hp->beta2, (float)(hp->lr / bc1),
                                                (float)(1.0 / std::sqrt(bc2)), (float)hp->eps);
  CNN_HIP(hipGetLastError());
  return MODIL_OK;
}

int modil_cnn_to_bf16(modil_cnn *n, const float *w, uint16_t *wb) {
  if (!n || !w || !wb) return set_global_error(MODIL_ERR_INVALID_ARG, "NULL pointer");
  to_bf16_kernel<<<nb(n->lay.n_params), kB, 0, n->stream>>>(w, wb, n->lay.n_params);
  CNN_HIP(hipGetLastError());
  return MODIL_OK;
}

}  // extern "C"
