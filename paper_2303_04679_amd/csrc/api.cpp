// C ABI of libmodil: validation, pack layout, workspace carve-up and the
// launch sequence of one mODIL iteration.  No exception crosses the ABI and
// no device memory is allocated here: the caller provides the workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

using namespace modil;

// Scratch of the allocation-free entry point (modil_prolong_noalloc): a fixed
// device array that every GPU the library runs on holds until the process
// ends.  Host code never passes the array's name to a kernel (on the host it
// stands for a host-side shadow, not a device address): it takes the device
// address of the current device's copy once, with hipGetSymbolAddress, and
// uses that address.
static __device__ __align__(256) unsigned char scratch[MODIL_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_last_error = "no error";

int fail_global(int status, const std::string &msg) {
  g_last_error = msg;
  return status;
}

int fail(modil_ctx *c, int status, const std::string &msg) {
  if (c) c->err = msg;
  g_last_error = msg;
  return status;
}

int hip_fail(modil_ctx *c, hipError_t e, const char *where) {
  return fail(c, MODIL_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_OR_RETURN(ctx, expr, where)              \
  do {                                              \
    hipError_t e_ = (expr);                         \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, where); \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

size_t dtype_size(const modil_problem &p) { return p.dtype == MODIL_F64 ? 8 : 4; }

int expected_ndim(int op) {
  switch (op) {
    case MODIL_OP_BURGERS:
    case MODIL_OP_HEAT_KX:
    case MODIL_OP_CAVITY:
      return 2;
    case MODIL_OP_NS3D:
      return 3;
    default:
      return 0;
  }
}

void fill_layout(const modil_problem &p, modil_pack_layout &L);

int validate(const modil_problem *p, std::string &msg) {
  if (!p) { msg = "problem is NULL"; return MODIL_ERR_INVALID_ARG; }
  if (p->op < MODIL_OP_POISSON || p->op > MODIL_OP_CAVITY) {
    msg = "unknown operator " + std::to_string(p->op);
    return MODIL_ERR_INVALID_ARG;
  }
  if (p->dtype != MODIL_F32 && p->dtype != MODIL_F64) {
    msg = "dtype must be MODIL_F32 or MODIL_F64";
    return MODIL_ERR_DTYPE;
  }
  if (p->centering != MODIL_CELL &&
      !(p->centering == MODIL_NODE && (p->op == MODIL_OP_POISSON || p->op == MODIL_OP_CAVITY ||
                                       p->op == MODIL_OP_NS3D))) {
    msg = "node-based values are implemented for MODIL_OP_POISSON, MODIL_OP_CAVITY and "
          "MODIL_OP_NS3D only";
    return MODIL_ERR_DTYPE;
  }
  const int want = expected_ndim(p->op);
  if (p->op == MODIL_OP_POISSON ? (p->ndim < 1 || p->ndim > 3) : p->ndim != want) {
    msg = "ndim " + std::to_string(p->ndim) + " does not match the operator";
    return MODIL_ERR_SHAPE;
  }
  if (p->n_levels < 1 || p->n_levels > MODIL_MAX_LEVELS) {
    msg = "n_levels must be in 1..8";
    return MODIL_ERR_SHAPE;
  }
  for (int a = 0; a < p->ndim; ++a) {
    const int n = p->dims[a];
    const int q = 1 << (p->n_levels - 1);
    if (n < 4 || n % q != 0 || n / q < 2) {
      msg = "dims[" + std::to_string(a) + "] = " + std::to_string(n) +
            " must be >= 4 and a multiple of 2^(n_levels-1) with >= 2 coarsest cells";
      return MODIL_ERR_SHAPE;
    }
    if (!(p->lengths[a] > 0.0) || !std::isfinite(p->lengths[a])) {
      msg = "lengths must be positive";
      return MODIL_ERR_INVALID_ARG;
    }
  }
  long cells = 1;
  for (int a = 0; a < p->ndim; ++a) cells *= p->dims[a];
  if (cells > (1L << 31) - 1) {
    msg = "grid too large for 32-bit measurement indices";
    return MODIL_ERR_SHAPE;
  }
  {
    modil_pack_layout L;
    fill_layout(*p, L);
    if (L.total > (1L << 31) - 1 || (long)p->batch * L.fine_cells > (1L << 31) - 1) {
      msg = "parameter pack too large for 32-bit indexing";
      return MODIL_ERR_SHAPE;
    }
  }
  if (p->batch < 1 || p->batch > 65535) {
    msg = "batch must be in 1..65535";
    return MODIL_ERR_INVALID_ARG;
  }
  if (p->max_meas < 0) {
    msg = "max_meas must be >= 0";
    return MODIL_ERR_INVALID_ARG;
  }
  if ((p->op == MODIL_OP_NS3D || p->op == MODIL_OP_CAVITY) && !(p->re > 0.0)) {
    msg = "re must be positive";
    return MODIL_ERR_INVALID_ARG;
  }
  if ((p->flags & MODIL_FLAG_CHI_FIXED) && p->op != MODIL_OP_NS3D) {
    msg = "MODIL_FLAG_CHI_FIXED applies to MODIL_OP_NS3D only";
    return MODIL_ERR_INVALID_ARG;
  }
  if (p->flags & ~(MODIL_FLAG_CHI_FIXED | MODIL_FLAG_FUSED_RESTRICT)) {
    msg = "unknown flags";
    return MODIL_ERR_INVALID_ARG;
  }
  return MODIL_OK;
}

struct Carve {
  size_t w, g, gq, partials, terms, flag, m_idx, m_field, m_term, m_ptr, m_val, m_w, inst_re;
  size_t fm_ptr, fm_rec, tm_ptr, tm_rec, sens, cpart, end;
  long n_fine_blocks, n_data_blocks, n_keys;
};

// per-instance partial-sum slots of the fused channel-flow kernel and its
// measurement buckets (0 for other operators)
void fused_geometry(const modil_problem &p, long &blocks, long &keys) {
  blocks = keys = 0;
  if (p.op != MODIL_OP_NS3D) return;
  int tz, nzt, ntx, nty, ox, oy;
  ns3d_tiles(p, tz, nzt, ntx, nty, ox, oy);
  blocks = (long)nzt * ntx * nty;
  keys = (long)p.batch * blocks * tz;
}

// (instance, tile) buckets of the 2-D tiled engine (0 for other problems)
long tile_keys(const modil_problem &p) {
  if (!fine_is_2d(p)) return 0;
  int tx, ty, nbx, nby;
  fine_tile_shape(p, tx, ty, nbx, nby);
  return (long)p.batch * nbx * nby;
}

Carve carve(const modil_problem &p, const modil_pack_layout &L) {
  Carve c{};
  const size_t ts = dtype_size(p);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align256(off + bytes);
    return at;
  };
  long fused_blocks, fused_keys;
  fused_geometry(p, fused_blocks, fused_keys);
  c.n_fine_blocks = std::max<long>(fine_partial_slots(p), fused_blocks);
  c.n_keys = fused_keys;
  c.n_data_blocks = std::max<long>(1, (p.max_meas + kBlock - 1) / kBlock);
  const long nl = p.n_levels;
  c.w = take(nl >= 2 ? (size_t)L.level_offset[nl - 1] * ts : 0);
  c.g = take((size_t)L.total * ts);
  bool xonly = false;
  for (int f = 0; f < L.n_fields; ++f) xonly |= field_is_x_only(p, f);
  c.gq = take(xonly ? (size_t)p.batch * L.fine_cells * ts : 0);
  c.sens = take(two_pass_adjoint(p) ? (size_t)6 * sens_fields(p) * p.batch * L.fine_cells * ts : 0);
  c.partials = take((size_t)p.batch * (c.n_fine_blocks + c.n_data_blocks) * kTerms * 8);
  c.terms = take((size_t)p.batch * kTerms * 8);
  c.flag = take(4);
  const size_t mm = (size_t)std::max(p.max_meas, 1);
  c.m_idx = take(mm * 4);
  c.m_field = take(mm * 4);
  c.m_term = take(mm * 4);
  c.m_ptr = take(((size_t)p.batch + 1) * 4);
  c.m_val = take(mm * 8);
  c.m_w = take(mm * 8);
  c.inst_re = take((size_t)p.batch * 8);
  const size_t fm = fused_keys ? mm : 0;
  c.fm_ptr = take(fused_keys ? ((size_t)fused_keys + 1) * 4 : 0);
  c.fm_rec = take(fm * sizeof(FusedMeas));
  const long tkeys = tile_keys(p);
  c.tm_ptr = take(tkeys ? ((size_t)tkeys + 1) * 4 : 0);
  c.tm_rec = take(tkeys ? mm * sizeof(FusedMeas) : 0);
  c.cpart = take(fused_partial_bytes(p));
  c.end = off;
  return c;
}

void fill_layout(const modil_problem &p, modil_pack_layout &L) {
  std::memset(&L, 0, sizeof(L));
  L.n_fields = op_fields(p);
  L.n_levels = p.n_levels;
  long off = 0;
  for (int l = 0; l < p.n_levels; ++l) {
    long stride = 0;
    for (int f = 0; f < L.n_fields; ++f) {
      const FieldGeom g = field_geom(p, l, f);
      L.field_offset[l][f] = stride;
      for (int a = 0; a < 3; ++a) L.field_dims[l][f][a] = g.n[a];
      stride += g.size;
    }
    L.level_stride[l] = stride;
    L.level_offset[l] = off;
    off += stride * p.batch;
  }
  L.total = off;
  L.fine_cells = 1;
  for (int a = 0; a < p.ndim; ++a) L.fine_cells *= p.dims[a] + (p.centering == MODIL_NODE ? 1 : 0);
  L.fine_total = L.level_stride[0] * p.batch;
  L.workspace_bytes = carve(p, L).end;
}

int upload_measurements(modil_ctx *c) {
  std::vector<Meas> m = c->meas;
  std::stable_sort(m.begin(), m.end(), [](const Meas &a, const Meas &b) {
    if (a.inst != b.inst) return a.inst < b.inst;
    if (a.field != b.field) return a.field < b.field;
    if (a.idx != b.idx) return a.idx < b.idx;
    return a.term < b.term;
  });
  const size_t n = m.size();
  std::vector<int32_t> idx(n), fld(n), trm(n), ptr(c->prob.batch + 1, 0);
  std::vector<double> val(n), w(n);
  for (size_t k = 0; k < n; ++k) {
    idx[k] = m[k].idx;
    fld[k] = m[k].field;
    trm[k] = m[k].term;
    val[k] = m[k].val;
    w[k] = m[k].w;
    ptr[m[k].inst + 1]++;
  }
  for (int b = 0; b < c->prob.batch; ++b) ptr[b + 1] += ptr[b];
  hipStream_t s = c->stream;
  if (n) {
    HIP_OR_RETURN(c, hipMemcpyAsync(c->m_idx, idx.data(), n * 4, hipMemcpyHostToDevice, s), "upload");
    HIP_OR_RETURN(c, hipMemcpyAsync(c->m_field, fld.data(), n * 4, hipMemcpyHostToDevice, s), "upload");
    HIP_OR_RETURN(c, hipMemcpyAsync(c->m_term, trm.data(), n * 4, hipMemcpyHostToDevice, s), "upload");
    HIP_OR_RETURN(c, hipMemcpyAsync(c->m_val, val.data(), n * 8, hipMemcpyHostToDevice, s), "upload");
    HIP_OR_RETURN(c, hipMemcpyAsync(c->m_w, w.data(), n * 8, hipMemcpyHostToDevice, s), "upload");
  }
  HIP_OR_RETURN(c, hipMemcpyAsync(c->m_inst_ptr, ptr.data(), ptr.size() * 4, hipMemcpyHostToDevice, s),
                "upload");
  // buckets of the fused channel-flow kernel: key = (tile, plane within the z-chunk)
  c->fused_ok = false;
  std::vector<int32_t> fptr;
  std::vector<FusedMeas> frec;
  if (c->prob.op == MODIL_OP_NS3D) {
    int tz, nzt, ntx, nty, ox, oy;
    ns3d_tiles(c->prob, tz, nzt, ntx, nty, ox, oy);
    // the fused kernel's grid: cells, or the interior nodes (measurements on
    // boundary nodes are rejected when they are set)
    const int e = c->prob.centering == MODIL_NODE ? 1 : 0;
    const int ny = c->prob.dims[1] + e, nx = c->prob.dims[2] + e;
    std::vector<std::pair<long, size_t>> order(n);
    bool ok = true;
    for (size_t k = 0; k < n; ++k) {
      const int cell = m[k].idx, x = cell % nx - e, y = (cell / nx) % ny - e, z = cell / (nx * ny) - e;
      const long tile = (((long)m[k].inst * nzt + z / tz) * nty + y / oy) * ntx + x / ox;
      order[k] = {tile * tz + z % tz, k};
      ok = ok && m[k].field < 4;
    }
    std::stable_sort(order.begin(), order.end(),
                     [](const std::pair<long, size_t> &a, const std::pair<long, size_t> &b) {
                       return a.first < b.first;
                     });
    const long keys = (long)c->prob.batch * nzt * ntx * nty * tz;
    fptr.assign(keys + 1, 0);
    const int ce = e;
    for (size_t k = 0; k < n; ++k) {
      const Meas &e = m[order[k].second];
      FusedMeas r{};
      r.field = e.field;
      r.cell = e.idx;
      r.term = e.term;
      // position in the tile, whose first column and row are a 2-cell halo
      r.lx = (int16_t)((e.idx % nx - ce) % ox + 2);
      r.ly = (int16_t)((e.idx / nx % ny - ce) % oy + 2);
      r.val = e.val;
      r.w = e.w;
      frec.push_back(r);
      fptr[order[k].first + 1]++;
    }
    for (long k = 0; k < keys; ++k) fptr[k + 1] += fptr[k];
    HIP_OR_RETURN(c, hipMemcpyAsync(c->fm_ptr, fptr.data(), fptr.size() * 4, hipMemcpyHostToDevice, s), "upload");
    if (n)
      HIP_OR_RETURN(c, hipMemcpyAsync(c->fm_rec, frec.data(), n * sizeof(FusedMeas),
                                      hipMemcpyHostToDevice, s),
                    "upload");
    for (double re : c->inst_re_host) ok = ok && re == c->prob.re;
    c->fused_ok = ok;
  }
  // buckets of the 2-D tiled engine: key = (instance, tile); within a key the
  // order of the list (field, cell, term) is kept
  if (fine_is_2d(c->prob)) {
    int tx, ty, nbx, nby, ny, nx;
    fine_tile_shape(c->prob, tx, ty, nbx, nby);
    fine_2d(c->prob, ny, nx);
    const long keys = (long)c->prob.batch * nbx * nby;
    std::vector<std::pair<long, size_t>> order(n);
    for (size_t k = 0; k < n; ++k) {
      const int x = m[k].idx % nx, y = m[k].idx / nx;
      order[k] = {((long)m[k].inst * nby + y / ty) * nbx + x / tx, k};
    }
    std::stable_sort(order.begin(), order.end(),
                     [](const std::pair<long, size_t> &a, const std::pair<long, size_t> &b) {
                       return a.first < b.first;
                     });
    std::vector<int32_t> tptr(keys + 1, 0);
    std::vector<FusedMeas> trec;
    trec.reserve(n);
    for (size_t k = 0; k < n; ++k) {
      const Meas &e = m[order[k].second];
      FusedMeas r{};
      r.field = e.field;
      r.cell = e.idx;
      r.term = e.term;
      r.lx = (int16_t)(e.idx % nx % tx);
      r.ly = (int16_t)(e.idx / nx % ty);
      r.val = e.val;
      r.w = e.w;
      trec.push_back(r);
      tptr[order[k].first + 1]++;
    }
    for (long k = 0; k < keys; ++k) tptr[k + 1] += tptr[k];
    HIP_OR_RETURN(c, hipMemcpyAsync(c->tm_ptr, tptr.data(), tptr.size() * 4, hipMemcpyHostToDevice, s),
                  "upload");
    if (n)
      HIP_OR_RETURN(c, hipMemcpyAsync(c->tm_rec, trec.data(), n * sizeof(FusedMeas),
                                      hipMemcpyHostToDevice, s),
                    "upload");
  }
  HIP_OR_RETURN(c, hipStreamSynchronize(s), "upload");
  c->n_meas_dev = (int)n;
  return MODIL_OK;
}

// a node index on the boundary of its field's grid (index 0 or n - 1 along an
// axis the field spans)
bool on_boundary_node(const FieldGeom &g, long idx) {
  for (int a = 2; a >= 0; --a) {
    const long i = idx % g.n[a];
    idx /= g.n[a];
    if (g.n[a] > 1 && (i == 0 || i == g.n[a] - 1)) return true;
  }
  return false;
}

bool use_fused(const modil_ctx *c) {
  return c->fused_enabled && c->fused_ok && c->prob.op == MODIL_OP_NS3D &&
         c->prob.dtype == MODIL_F32 && ns3d_offsets_fit(c->prob);
}

// Loss terms at theta; with grad the gradient of every level; with adam
// also one Adam step theta -> th_out on every level.
// carry_in: w_buf already holds the Horner tail for theta (carried by the
// previous iteration); carry_out: have the restriction tail also form the
// Horner tail for th_out (carried reports whether it did).
// whether launch_horner launches anything: the levels from L - 2 (or below
// the carried tail) down to level 1 (skip_fine) or 0
static bool horner_needed(const modil_ctx *c, bool skip_fine, bool skip_tail) {
  const int L = c->prob.n_levels, l_end = skip_fine ? 1 : 0;
  if (L == 1) return false;
  return (skip_tail ? c->carry_stop - 1 : L - 2) >= l_end;
}

int evaluate(modil_ctx *c, const void *theta, void *grad, double *terms, const AdamHost *adam = nullptr,
             void *th_out = nullptr, void *m = nullptr, void *v = nullptr, bool carry_in = false,
             bool carry_out = false, bool *carried = nullptr) {
  const bool want = grad != nullptr;
  if (carried) *carried = false;
  if (use_fused(c) && want) {
    if (horner_needed(c, true, carry_in)) {
      Timed t(c, 1);
      HIP_OR_RETURN(c, launch_horner(c, theta, nullptr, true, carry_in), "prolong");
    }
    {
      Timed t(c, 0);
      HIP_OR_RETURN(c, launch_ns3d_fused(c, theta, grad, adam, th_out, m, v), "fused kernel");
    }
    long blocks, keys;
    fused_geometry(c->prob, blocks, keys);
    TermSum sum;
    sum.partials = c->partials;
    sum.n_part_blocks = c->n_part_blocks;
    sum.n_a = blocks;
    sum.terms = terms;
    sum.flag = c->flag;
    bool summed = false;
    // with MODIL_FLAG_FUSED_RESTRICT the fused kernel summed the finest
    // gradient in z and the assembly kernel forms level 1
    const int from = fused_partial_bytes(c->prob) ? 1 : 0;
    {
      Timed t(c, 2);
      if (from == 1)
        HIP_OR_RETURN(c, launch_fused_assemble(c, grad, adam, theta, th_out, m, v), "assemble");
      HIP_OR_RETURN(c, launch_restrict_chain(c, grad, from, theta, th_out, m, v, adam, &sum, &summed,
                                             carry_out, carried),
                    "restrict");
    }
    if (!summed) {
      Timed t(c, 4);
      HIP_OR_RETURN(c, launch_reduce(c, terms, blocks, 0, 0), "reduce");
    }
    return MODIL_OK;
  }
  const void *u = theta;
  bool summed = false;  // the data kernel summed the partials
  const bool tiled = fine_uses_tiles(c);
  if (horner_needed(c, tiled, tiled && carry_in)) {
    // the tile kernel forms the finest level itself: Horner down to level 1
    Timed t(c, 1);
    HIP_OR_RETURN(c, launch_horner(c, theta, nullptr, tiled, tiled && carry_in), "prolong");
    if (!tiled) u = c->w_buf;
  }
  if (tiled) {
    // 2-D tiled engine: the tile kernel also forms the finest level (theta_0
    // + T w_1 while staging its tile), the data terms and, with Adam, updates
    // level 0; the restriction kernels update the coarse levels and the
    // restriction tail sums the loss partials
    {
      Timed t(c, 0);
      HIP_OR_RETURN(c, launch_fine(c, theta, grad, want, adam, theta, th_out, m, v, true), "fine kernel");
    }
    TermSum sum;
    sum.partials = c->partials;
    sum.n_part_blocks = c->n_part_blocks;
    sum.n_a = c->fine_slots;
    sum.terms = terms;
    sum.flag = c->flag;
    if (want) {
      bool xonly = false;
      for (int f = 0; f < c->lay.n_fields; ++f) xonly |= field_is_x_only(c->prob, f);
      Timed t(c, 2);
      HIP_OR_RETURN(c, launch_restrict_chain(c, grad, 0, theta, th_out, m, v, adam, &sum, &summed,
                                             carry_out, carried, xonly),
                    "restrict");
    }
    if (!summed) {
      Timed t(c, 4);
      HIP_OR_RETURN(c, launch_reduce(c, terms, c->fine_slots, 0, 0), "reduce");
    }
    return MODIL_OK;
  }
  {
    Timed t(c, 0);
    HIP_OR_RETURN(c, launch_fine(c, u, grad, want), "fine kernel");
  }
  {
    Timed t(c, 4);
    if (want) HIP_OR_RETURN(c, launch_colsum(c, grad), "column sum");
    HIP_OR_RETURN(c, launch_data(c, u, grad, want, terms, summed), "data kernel");
  }
  if (want) {
    Timed t(c, 2);
    HIP_OR_RETURN(c, launch_restrict_chain(c, grad, 0, nullptr, nullptr, nullptr, nullptr, nullptr),
                  "restrict");
  }
  if (!summed) {
    Timed t(c, 4);
    HIP_OR_RETURN(c, launch_reduce(c, terms, c->fine_slots, c->n_fine_blocks, c->n_data_blocks),
                  "reduce");
  }
  if (adam) {
    Timed t(c, 3);
    HIP_OR_RETURN(c, launch_adam(c, theta, th_out, m, v, grad, c->lay.total, *adam), "adam");
  }
  return MODIL_OK;
}

bool check_ctx(modil_ctx *c) { return c != nullptr; }

// device address of the current device's copy of `scratch`, taken once per
// device with that device current
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchDevices] = {};

hipError_t scratch_address(int device, void **out) {
  if (device < 0 || device >= kScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

}  // namespace

// ------------------------------------------------------------- op metadata
namespace modil {

int set_global_error(int status, const std::string &msg) { return fail_global(status, msg); }

int set_ctx_error(modil_ctx *c, int status, const std::string &msg) { return fail(c, status, msg); }

int eval_loss_grad(modil_ctx *c, const void *theta, void *grad, double *terms) {
  return evaluate(c, theta, grad, terms);
}

int op_fields(const modil_problem &p) {
  switch (p.op) {
    case MODIL_OP_POISSON:
    case MODIL_OP_BURGERS:
      return 1;
    case MODIL_OP_HEAT_KX:
      return 2;
    case MODIL_OP_NS3D:
      return (p.flags & MODIL_FLAG_CHI_FIXED) ? 4 : 5;
    case MODIL_OP_CAVITY:
      return 3;
  }
  return 0;
}

int op_pde_equations(const modil_problem &p) {
  switch (p.op) {
    case MODIL_OP_NS3D:
      return 4;
    case MODIL_OP_CAVITY:
      return 3;
    default:
      return 1;
  }
}

bool field_is_x_only(const modil_problem &p, int f) { return p.op == MODIL_OP_HEAT_KX && f == 1; }

FieldGeom field_geom(const modil_problem &p, int level, int f) {
  FieldGeom g{};
  for (int a = 0; a < 3; ++a) g.n[a] = 1;
  const int extra = p.centering == MODIL_NODE ? 1 : 0;  // nodes: cells + 1 per axis
  for (int k = 0; k < p.ndim; ++k) g.n[3 - p.ndim + k] = (p.dims[k] >> level) + extra;
  if (field_is_x_only(p, f)) g.n[0] = g.n[1] = 1;
  g.stride[2] = 1;
  g.stride[1] = g.n[2];
  g.stride[0] = (long)g.n[1] * g.n[2];
  g.size = (long)g.n[0] * g.n[1] * g.n[2];
  return g;
}

}  // namespace modil

// --------------------------------------------------------------------- ABI
extern "C" {

int modil_abi_version(void) { return MODIL_ABI_VERSION; }

const char *modil_status_str(int s) {
  switch (s) {
    case MODIL_OK: return "ok";
    case MODIL_ERR_INVALID_ARG: return "invalid argument";
    case MODIL_ERR_SHAPE: return "shape error";
    case MODIL_ERR_DTYPE: return "dtype error";
    case MODIL_ERR_HIP: return "HIP runtime error";
    case MODIL_ERR_NONFINITE: return "non-finite loss";
    case MODIL_ERR_STATE: return "invalid state";
  }
  return "unknown status";
}

const char *modil_last_error(const modil_ctx *c) {
  return c ? c->err.c_str() : g_last_error.c_str();
}

int modil_layout(const modil_problem *p, modil_pack_layout *out) {
  std::string msg;
  const int st = validate(p, msg);
  if (st) return fail_global(st, msg);
  if (!out) return fail_global(MODIL_ERR_INVALID_ARG, "layout output is NULL");
  fill_layout(*p, *out);
  return MODIL_OK;
}

int modil_create(const modil_problem *p, void *ws, size_t ws_bytes, void *stream, modil_ctx **out) {
  std::string msg;
  int st = validate(p, msg);
  if (st) return fail_global(st, msg);
  if (!out) return fail_global(MODIL_ERR_INVALID_ARG, "output handle is NULL");
  *out = nullptr;
  modil_pack_layout L;
  fill_layout(*p, L);
  if (!ws || ws_bytes < L.workspace_bytes)
    return fail_global(MODIL_ERR_INVALID_ARG, "workspace is NULL or smaller than layout.workspace_bytes (" +
                                                  std::to_string(L.workspace_bytes) + ")");
  if (reinterpret_cast<uintptr_t>(ws) % 256)
    return fail_global(MODIL_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  modil_ctx *c = new (std::nothrow) modil_ctx();
  if (!c) return fail_global(MODIL_ERR_STATE, "out of host memory");
  c->prob = *p;
  c->lay = L;
  c->stream = (hipStream_t)stream;
  c->ws = (char *)ws;
  c->ws_bytes = ws_bytes;
  (void)hipGetDevice(&c->device);
  {
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) ==
            hipSuccess &&
        lds > 0)
      c->lds_budget = std::min<size_t>((size_t)lds, 160 * 1024);
  }
  const Carve cv = carve(*p, L);
  c->w_buf = c->ws + cv.w;
  c->g_buf = c->ws + cv.g;
  c->gq_buf = c->ws + cv.gq;
  c->sens_buf = two_pass_adjoint(*p) ? c->ws + cv.sens : nullptr;
  c->cpart = fused_partial_bytes(*p) ? c->ws + cv.cpart : nullptr;
  c->partials = (double *)(c->ws + cv.partials);
  c->terms_tmp = (double *)(c->ws + cv.terms);
  c->flag = (int32_t *)(c->ws + cv.flag);
  c->m_idx = (int32_t *)(c->ws + cv.m_idx);
  c->m_field = (int32_t *)(c->ws + cv.m_field);
  c->m_term = (int32_t *)(c->ws + cv.m_term);
  c->m_inst_ptr = (int32_t *)(c->ws + cv.m_ptr);
  c->m_val = (double *)(c->ws + cv.m_val);
  c->m_w = (double *)(c->ws + cv.m_w);
  c->inst_re = (double *)(c->ws + cv.inst_re);
  c->fm_ptr = (int32_t *)(c->ws + cv.fm_ptr);
  c->fm_rec = (FusedMeas *)(c->ws + cv.fm_rec);
  c->tm_ptr = (int32_t *)(c->ws + cv.tm_ptr);
  c->tm_rec = (FusedMeas *)(c->ws + cv.tm_rec);
  c->n_fine_blocks = cv.n_fine_blocks;
  c->n_data_blocks = cv.n_data_blocks;
  c->n_part_blocks = cv.n_fine_blocks + cv.n_data_blocks;
  c->inst_re_host.assign(p->batch, p->re);
  // zero flag, empty measurement lists, default Reynolds numbers
  const int32_t zero = 0;
  hipError_t e = hipMemcpyAsync(c->flag, &zero, 4, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->inst_re, c->inst_re_host.data(), p->batch * 8, hipMemcpyHostToDevice,
                       c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    const std::string m = std::string("create: ") + hipGetErrorString(e);
    delete c;
    return fail_global(MODIL_ERR_HIP, m);
  }
  st = upload_measurements(c);
  if (st) {
    const std::string m = c->err;
    delete c;
    return fail_global(st, m);
  }
  *out = c;
  return MODIL_OK;
}

int modil_destroy(modil_ctx *c) {
  if (!c) return MODIL_OK;
  for (auto &pc : c->prof) {
    for (auto &ev : pc.pending) { (void)hipEventDestroy(ev.a); (void)hipEventDestroy(ev.b); }
    for (auto &ev : pc.pool) { (void)hipEventDestroy(ev.a); (void)hipEventDestroy(ev.b); }
  }
  delete c;
  return MODIL_OK;
}

int modil_set_stream(modil_ctx *c, void *stream) {
  if (!c) return fail_global(MODIL_ERR_INVALID_ARG, "ctx is NULL");
  c->stream = (hipStream_t)stream;
  return MODIL_OK;
}

int modil_set_measurements(modil_ctx *c, int32_t inst, int32_t field, int32_t term, int32_t n,
                           const int32_t *idx, const double *val, double weight) {
  if (!c) return fail_global(MODIL_ERR_INVALID_ARG, "ctx is NULL");
  if (inst < 0 || inst >= c->prob.batch) return fail(c, MODIL_ERR_INVALID_ARG, "instance out of range");
  if (field < 0 || field >= c->lay.n_fields) return fail(c, MODIL_ERR_INVALID_ARG, "field out of range");
  if (term != MODIL_TERM_DATA && term != MODIL_TERM_IC)
    return fail(c, MODIL_ERR_INVALID_ARG, "term must be MODIL_TERM_DATA or MODIL_TERM_IC");
  if (n < 0 || (n > 0 && (!idx || !val))) return fail(c, MODIL_ERR_INVALID_ARG, "bad list");
  if (!std::isfinite(weight) || weight < 0.0) return fail(c, MODIL_ERR_INVALID_ARG, "bad weight");
  if ((long)c->meas.size() + n > c->prob.max_meas)
    return fail(c, MODIL_ERR_INVALID_ARG, "measurement capacity max_meas exceeded");
  const FieldGeom g = field_geom(c->prob, 0, field);
  std::vector<int32_t> sorted(idx, idx + n);
  std::sort(sorted.begin(), sorted.end());
  for (int k = 0; k < n; ++k) {
    if (sorted[k] < 0 || sorted[k] >= g.size) return fail(c, MODIL_ERR_SHAPE, "cell index out of range");
    if (k && sorted[k] == sorted[k - 1]) return fail(c, MODIL_ERR_INVALID_ARG, "duplicate cell index in list");
    if (c->prob.centering == MODIL_NODE && on_boundary_node(g, sorted[k]))
      return fail(c, MODIL_ERR_SHAPE, "measurement on a boundary node (its value is imposed)");
  }
  for (int k = 0; k < n; ++k) c->meas.push_back(Meas{inst, field, term, idx[k], val[k], weight});
  return upload_measurements(c);
}

int modil_clear_measurements(modil_ctx *c) {
  if (!c) return fail_global(MODIL_ERR_INVALID_ARG, "ctx is NULL");
  c->meas.clear();
  return upload_measurements(c);
}

int modil_set_field(modil_ctx *c, int32_t which, const void *ptr) {
  if (!c) return fail_global(MODIL_ERR_INVALID_ARG, "ctx is NULL");
  if (which >= MODIL_FIELD_FORCING0 && which <= MODIL_FIELD_FORCING3) {
    c->forcing[which] = ptr;
    return MODIL_OK;
  }
  if (which == MODIL_FIELD_CHI) {
    if (!(c->prob.flags & MODIL_FLAG_CHI_FIXED))
      return fail(c, MODIL_ERR_INVALID_ARG, "chi array needs MODIL_FLAG_CHI_FIXED");
    c->chi = ptr;
    return MODIL_OK;
  }
  return fail(c, MODIL_ERR_INVALID_ARG, "unknown field slot");
}

int modil_set_instance_scalar(modil_ctx *c, int32_t inst, int32_t which, double value) {
  if (!c) return fail_global(MODIL_ERR_INVALID_ARG, "ctx is NULL");
  if (inst < 0 || inst >= c->prob.batch) return fail(c, MODIL_ERR_INVALID_ARG, "instance out of range");
  if (which != MODIL_SCALAR_RE || !(value > 0.0)) return fail(c, MODIL_ERR_INVALID_ARG, "bad scalar");
  c->inst_re_host[inst] = value;
  if (c->prob.op == MODIL_OP_NS3D) {
    int st = upload_measurements(c);  // re-evaluates whether the fused kernel applies
    if (st) return st;
  }
  HIP_OR_RETURN(c, hipMemcpyAsync(c->inst_re, c->inst_re_host.data(), c->prob.batch * 8,
                                  hipMemcpyHostToDevice, c->stream),
                "set scalar");
  HIP_OR_RETURN(c, hipStreamSynchronize(c->stream), "set scalar");
  return MODIL_OK;
}

static int ready(modil_ctx *c) {
  if (!c) return fail_global(MODIL_ERR_INVALID_ARG, "ctx is NULL");
  if ((c->prob.flags & MODIL_FLAG_CHI_FIXED) && !c->chi)
    return fail(c, MODIL_ERR_STATE, "fixed-chi problem needs modil_set_field(MODIL_FIELD_CHI)");
  return MODIL_OK;
}

int modil_prolong(modil_ctx *c, const void *theta, void *fine_out) {
  int st = ready(c);
  if (st) return st;
  if (!theta || !fine_out) return fail(c, MODIL_ERR_INVALID_ARG, "NULL pointer");
  if (c->prob.n_levels == 1) {
    HIP_OR_RETURN(c, hipMemcpyAsync(fine_out, theta, c->lay.fine_total * dtype_size(c->prob),
                                    hipMemcpyDeviceToDevice, c->stream),
                  "prolong copy");
    return MODIL_OK;
  }
  HIP_OR_RETURN(c, launch_horner(c, theta, fine_out, false), "prolong");
  return MODIL_OK;
}

int modil_prolong_noalloc(const modil_problem *p, const void *theta, void *fine_out, void *stream) {
  std::string msg;
  const int st = validate(p, msg);
  if (st) return fail_global(st, msg);
  if (!theta || !fine_out) return fail_global(MODIL_ERR_INVALID_ARG, "NULL pointer");
  modil_ctx c;  // host-side description only: no workspace, no measurements
  c.prob = *p;
  fill_layout(*p, c.lay);
  c.stream = (hipStream_t)stream;
  // the Horner intermediates w_l of levels 1 .. L-2 sit at their pack
  // offsets, so the scratch must hold the pack up to level L-1
  const size_t need = p->n_levels >= 3 ? (size_t)c.lay.level_offset[p->n_levels - 1] * dtype_size(*p) : 0;
  if (need > MODIL_NOALLOC_SCRATCH_BYTES)
    return fail_global(MODIL_ERR_SHAPE, "modil_prolong_noalloc: the intermediate levels need " +
                                            std::to_string(need) + " bytes of scratch, more than " +
                                            std::to_string((size_t)MODIL_NOALLOC_SCRATCH_BYTES));
  hipError_t e = hipGetDevice(&c.device);
  if (e == hipSuccess) e = scratch_address(c.device, &c.w_buf);
  if (e != hipSuccess) return fail_global(MODIL_ERR_HIP, std::string("prolong_noalloc: ") + hipGetErrorString(e));
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c.device) == hipSuccess && lds > 0)
    c.lds_budget = std::min<size_t>((size_t)lds, 160 * 1024);
  if (p->n_levels == 1)
    e = hipMemcpyAsync(fine_out, theta, c.lay.fine_total * dtype_size(*p), hipMemcpyDeviceToDevice, c.stream);
  else
    e = launch_horner(&c, theta, fine_out, false);
  if (e != hipSuccess) return fail_global(MODIL_ERR_HIP, std::string("prolong_noalloc: ") + hipGetErrorString(e));
  return MODIL_OK;
}

int modil_restrict_adjoint(modil_ctx *c, const void *fine_in, void *grad) {
  int st = ready(c);
  if (st) return st;
  if (!fine_in || !grad) return fail(c, MODIL_ERR_INVALID_ARG, "NULL pointer");
  HIP_OR_RETURN(c, hipMemcpyAsync(grad, fine_in, c->lay.fine_total * dtype_size(c->prob),
                                  hipMemcpyDeviceToDevice, c->stream),
                "restrict copy");
  HIP_OR_RETURN(c, launch_restrict_chain(c, grad, 0, nullptr, nullptr, nullptr, nullptr, nullptr),
                "restrict");
  return MODIL_OK;
}

int modil_loss(modil_ctx *c, const void *theta, double *terms) {
  int st = ready(c);
  if (st) return st;
  if (!theta || !terms) return fail(c, MODIL_ERR_INVALID_ARG, "NULL pointer");
  return evaluate(c, theta, nullptr, terms);
}

int modil_loss_grad(modil_ctx *c, const void *theta, void *grad, double *terms) {
  int st = ready(c);
  if (st) return st;
  if (!theta || !grad || !terms) return fail(c, MODIL_ERR_INVALID_ARG, "NULL pointer");
  return evaluate(c, theta, grad, terms);
}

static int check_hp(modil_ctx *c, const modil_adam_hp *hp, int64_t step) {
  if (!hp) return fail(c, MODIL_ERR_INVALID_ARG, "hyper-parameters are NULL");
  if (step < 1) return fail(c, MODIL_ERR_INVALID_ARG, "step must be >= 1");
  if (!(hp->beta1 >= 0.0 && hp->beta1 < 1.0 && hp->beta2 >= 0.0 && hp->beta2 < 1.0 &&
        hp->eps > 0.0 && std::isfinite(hp->lr)))
    return fail(c, MODIL_ERR_INVALID_ARG, "bad Adam hyper-parameters");
  return MODIL_OK;
}

// bias corrections of step t folded into the step size and the v scale (FP64 on the host)
static AdamHost adam_host(const modil_adam_hp *hp, int64_t step) {
  const double bc1 = 1.0 - std::pow(hp->beta1, (double)step);
  const double bc2 = 1.0 - std::pow(hp->beta2, (double)step);
  return AdamHost{hp->beta1, hp->beta2, hp->lr / bc1, 1.0 / std::sqrt(bc2), hp->eps};
}

int modil_adam(modil_ctx *c, const void *th_in, void *th_out, void *m, void *v, const void *g,
               const modil_adam_hp *hp, int64_t step) {
  if (!c) return fail_global(MODIL_ERR_INVALID_ARG, "ctx is NULL");
  int st = check_hp(c, hp, step);
  if (st) return st;
  if (!th_in || !th_out || !m || !v || !g) return fail(c, MODIL_ERR_INVALID_ARG, "NULL pointer");
  Timed t(c, 3);
  HIP_OR_RETURN(c, launch_adam(c, th_in, th_out, m, v, g, c->lay.total, adam_host(hp, step)), "adam");
  return MODIL_OK;
}

int modil_step(modil_ctx *c, const void *th_in, void *th_out, void *m, void *v,
               const modil_adam_hp *hp, int64_t step, double *terms) {
  int st = ready(c);
  if (st) return st;
  st = check_hp(c, hp, step);
  if (st) return st;
  if (!th_in || !th_out || !m || !v) return fail(c, MODIL_ERR_INVALID_ARG, "NULL pointer");
  if (th_in == th_out) return fail(c, MODIL_ERR_INVALID_ARG, "theta_out must differ from theta_in");
  const AdamHost ah = adam_host(hp, step);
  return evaluate(c, th_in, c->g_buf, terms ? terms : c->terms_tmp, &ah, th_out, m, v);
}

int modil_run(modil_ctx *c, void *th_a, void *th_b, void *m, void *v, const modil_adam_hp *hp,
              int64_t step0, int32_t n_steps, double *terms) {
  int st = ready(c);
  if (st) return st;
  if (n_steps < 1) return fail(c, MODIL_ERR_INVALID_ARG, "n_steps must be >= 1");
  st = check_hp(c, hp, step0);
  if (st) return st;
  if (!th_a || !th_b || !m || !v) return fail(c, MODIL_ERR_INVALID_ARG, "NULL pointer");
  if (th_a == th_b) return fail(c, MODIL_ERR_INVALID_ARG, "theta_b must differ from theta_a");
  // each iteration but the last has its restriction tail form the next
  // iteration's Horner tail (same values, one launch fewer)
  bool carried = false;
  for (int32_t k = 0; k < n_steps; ++k) {
    const AdamHost ah = adam_host(hp, step0 + k);
    void *in = (k & 1) ? th_b : th_a, *out = (k & 1) ? th_a : th_b;
    double *t = (k == n_steps - 1 && terms) ? terms : c->terms_tmp;
    bool next = false;
    st = evaluate(c, in, c->g_buf, t, &ah, out, m, v, carried, k + 1 < n_steps, &next);
    if (st) return st;
    carried = next;
  }
  return MODIL_OK;
}

int modil_residual_metric(modil_ctx *c, const void *theta, double *r) {
  int st = ready(c);
  if (st) return st;
  if (!theta || !r) return fail(c, MODIL_ERR_INVALID_ARG, "NULL pointer");
  st = evaluate(c, theta, nullptr, c->terms_tmp);
  if (st) return st;
  HIP_OR_RETURN(c, launch_metric(c, c->terms_tmp, r), "metric");
  return MODIL_OK;
}

int modil_set_option(modil_ctx *c, int32_t option, int64_t value) {
  if (!c) return fail_global(MODIL_ERR_INVALID_ARG, "ctx is NULL");
  if (option == MODIL_OPT_FUSED) {
    c->fused_enabled = value != 0;
    return MODIL_OK;
  }
  if (option == MODIL_OPT_MARCH) {
    c->march_enabled = value != 0;
    return MODIL_OK;
  }
  if (option == MODIL_OPT_TAIL) {
    c->tail_enabled = value != 0;
    return MODIL_OK;
  }
  if (option == MODIL_OPT_TILE) {
    c->tile_enabled = value != 0;
    return MODIL_OK;
  }
  if (option == MODIL_OPT_TWO_PASS) {
    c->two_pass_enabled = value != 0;
    return MODIL_OK;
  }
  if (option == MODIL_OPT_MARCH_TILE) {
    const int yr = (int)(value >> 6), zr = (int)(value & 63);
    const bool ok = value == 0 || (yr == 2 && (zr == 1 || zr == 2 || zr == 4 || zr == 8)) ||
                    (yr == 4 && (zr == 1 || zr == 2 || zr == 4 || zr == 8 || zr == 16)) ||
                    (yr == 8 && (zr == 4 || zr == 8));
    if (!ok || value < 0 || value > 1023) return fail(c, MODIL_ERR_INVALID_ARG, "unsupported tile");
    c->march_tile = (int)value;
    return MODIL_OK;
  }
  return fail(c, MODIL_ERR_INVALID_ARG, "unknown option");
}

int modil_fused_active(const modil_ctx *c) {
  if (!c) return fail_global(MODIL_ERR_INVALID_ARG, "ctx is NULL");
  return use_fused(c) ? 1 : 0;
}

int modil_check(modil_ctx *c) {
  if (!c) return fail_global(MODIL_ERR_INVALID_ARG, "ctx is NULL");
  HIP_OR_RETURN(c, hipStreamSynchronize(c->stream), "check");
  HIP_OR_RETURN(c, hipGetLastError(), "check");
  int32_t flag = 0;
  HIP_OR_RETURN(c, hipMemcpy(&flag, c->flag, 4, hipMemcpyDeviceToHost), "check");
  if (flag) {
    const int32_t zero = 0;
    HIP_OR_RETURN(c, hipMemcpy(c->flag, &zero, 4, hipMemcpyHostToDevice), "check");
    return fail(c, MODIL_ERR_NONFINITE, "a loss term was NaN or Inf");
  }
  return MODIL_OK;
}

int modil_profile(modil_ctx *c, int32_t enable) {
  if (!c) return fail_global(MODIL_ERR_INVALID_ARG, "ctx is NULL");
  c->profiling = enable != 0;
  return MODIL_OK;
}

int modil_profile_read(modil_ctx *c, int32_t cls, double *total_ms, int64_t *count) {
  if (!c) return fail_global(MODIL_ERR_INVALID_ARG, "ctx is NULL");
  if (cls < 0 || cls >= kProfileClasses || !total_ms || !count) return fail(c, MODIL_ERR_INVALID_ARG, "bad class");
  HIP_OR_RETURN(c, hipStreamSynchronize(c->stream), "profile");
  ProfileClass &pc = c->prof[cls];
  for (auto &ev : pc.pending) {
    float ms = 0.f;
    HIP_OR_RETURN(c, hipEventElapsedTime(&ms, ev.a, ev.b), "profile");
    pc.ms += ms;
    pc.count += 1;
    pc.pool.push_back(ev);
  }
  pc.pending.clear();
  *total_ms = pc.ms;
  *count = pc.count;
  pc.ms = 0.0;
  pc.count = 0;
  return MODIL_OK;
}

}  // extern "C"
