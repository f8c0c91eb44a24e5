// Fused finest-level pass of the 3-D channel-flow problem (Section 3.5).
//
// One pass over the finest grid does, per cell: the last Horner step
// u = theta_1 + T w_2 (prolongation fused into the read), the residuals of
// continuity and momentum and their FP64 loss partials, the measurement
// misfits, the exact adjoint gathered over the 7-point star (transposed
// stencils with the ghost maps folded back), and -- when Adam is fused --
// the Adam update of the finest level.  It writes the finest gradient for
// the restriction kernel that follows.
//
// Tiling: a block owns a 32 x 16 (x, y) tile of cells and marches along z
// through a chunk of planes.  Its 768 threads hold the tile with a 2-cell
// halo: 20 rows of 32 cache-line-aligned columns (the owned rows and the two
// halo rows on each side) and two more waves for the four halo columns.  Each
// thread keeps its column's last prolonged planes, three planes of residual
// seeds and its cell's own (centre) sensitivity in registers; the current
// planes of fields and seeds are staged in LDS for the xy neighbours.  Seeds
// are formed for the owned cells plus a 1-cell halo, the gradient for the
// owned cells.  The coarse plane
// interpolation is cached per column, so each coarse plane is read once per
// two fine planes.  Blocks are mapped to tiles so that every XCD works on one
// contiguous slab of z-chunks and neighbouring tiles share its L2.
//
// Node-based values (Section 2.2; NODE): the kernel marches over the
// interior nodes as its cells, with the boundary nodes as the halo slots
// across the walls: their values are imposed or copied from the interior
// node next to them (the node rules of the channel), so the ghost adjoint at
// an x or y wall is added explicitly to the cell next to it.  The boundary
// nodes carry no equation: each block gives those beyond its region a zero
// gradient (and Adam with it) in its epilogue.  The opt-in z-sum form (ZSUM)
// sums the finest gradient over the fine planes of each coarse plane instead
// of writing it; an assembly kernel finishes T^T in y and x.
//
// The kernel is built for FP32 fields (FP64 loss partials).  An FP64 build
// needs more registers than the 768-thread block allows and spills heavily;
// FP64 problems run on the generic engine.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.h"
#include "multigrid.h"
#include "ops.h"

namespace modil {

constexpr int NSO_X = 32, NSO_Y = 16;   // owned cells per block (x, y)
constexpr int NST_X = NSO_X + 4, NST_Y = NSO_Y + 4;  // tile with a 2-cell halo
constexpr int NS_MAIN = NSO_X * NST_Y;  // threads on the full-width rows
constexpr int NS_HALO = 4 * NST_Y;       // threads for the four halo columns
constexpr int NS_THREADS = NS_MAIN + (NS_HALO + 63) / 64 * 64;  // whole waves
constexpr int NS_XCD = 8;
constexpr long kComputeUnits = 256;  // compute units of the chip (32 per XCD)
constexpr int NF_MAX_COARSE = 5;  // unknown fields with a coarse hierarchy
static_assert(NS_THREADS - NS_MAIN >= NS_HALO, "every halo-column position needs a thread");
#ifndef NS_WAVES_PER_EU
#define NS_WAVES_PER_EU 3
#endif

template <typename T>
struct NS3DArgs {
  OpParams p;
  NSCoef<T> K;        // stencil coefficients (uniform: read from the kernel arguments)
  int nc[3];          // level-1 cells per axis (z, y, x); unused without coarse levels
  int has_coarse;
  int tz, nzt, ntx, nty;
  int tiles_per_xcd;  // ceil(nzt * ntx * nty / NS_XCD)
  int fsize, csize;   // cells of one field on level 0 / level 1
  const T *theta;     // level 0 of the theta pack
  int th_inst;        // instance stride on level 0
  const T *w1;        // level 1 of the prolonged coarse levels
  int w1_inst;
  T *g;               // level 0 of the gradient pack (written without Adam only)
  T *cpart;           // level-1 gradient partials of every tile (with coarse levels)
  int ncz, ncy, ncx;  // level-1 cells per axis
  const T *forcing[4];
  const T *chi;       // fixed chi, [instance][cells]
  const int32_t *mptr;      // [key + 1]: measurement records of (tile, plane)
  const FusedMeas *mrec;
  double *partials;
  int n_part_blocks;
  AdamArgs<T> adam;   // level-0 pointers of theta_in / theta_out / m / v
};

// Level-1 (coarse) window of a tile: the coarse cells that the xy
// interpolation of its 36 x 20 fine columns touches, 20 x 12 per field.
constexpr int NCT_X = NST_X / 2 + 2, NCT_Y = NST_Y / 2 + 2;
constexpr int NCT = NCT_X * NCT_Y;

// Restriction of the finest gradient to level 1 (T^T, Section 2.2): its z
// part is fused into the gradient write.  Each owned cell sums its column's
// gradient over the fine planes of each coarse plane (every fine plane adds
// to the two coarse planes of its row of T, in a ring of four LDS slots) and
// stores the sum once the plane is complete: a chunk writes the z sums of
// its coarse planes and of the one on each side (those take its fine planes
// next to the chunk ends), at fine (y, x) resolution.  The assembly kernel
// applies T^T in y and x and adds the two chunks' sums of the coarse planes
// at chunk ends, in a fixed order.
constexpr int NACC = 4;  // ring of z accumulators

// xy interpolation of one coarse plane of every field from its LDS window;
// lx, ly are window coordinates of the taps
template <typename T, int NF>
__device__ inline void coarse_xy(const T *cw, const int (&lx)[2], const T (&wx)[2],
                                 const int (&ly)[2], const T (&wy)[2], T (&W)[NF]) {
  for (int f = 0; f < NF; ++f) {
    const T *bf = cw + f * NCT;
    const T r0 = wx[0] * bf[ly[0] * NCT_X + lx[0]] + wx[1] * bf[ly[0] * NCT_X + lx[1]];
    const T r1 = wx[0] * bf[ly[1] * NCT_X + lx[0]] + wx[1] * bf[ly[1] * NCT_X + lx[1]];
    W[f] = wy[0] * r0 + wy[1] * r1;
  }
}

// Global accesses of the march: a base that is uniform over the block (an
// array and instance) plus a 32-bit byte offset, the column's offset in its
// field (per thread, fixed) plus the plane's (uniform, formed in the plane
// loop).  Formed in the loop, the offset stays 32-bit and the access takes the
// scalar-base + 32-bit-offset form: no 64-bit vector address arithmetic.
// Offsets are never formed for planes before the grid (no wrap-around).
template <typename T>
__device__ inline T ld_at(const T *base, uint32_t byte_off) {
  return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte_off);
}
template <typename T>
__device__ inline void st_at(T *base, uint32_t byte_off, T v) {
  *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + byte_off) = v;
}

// Adjoint of the residuals of a neighbour j across one face, added to g.
// at = {a_0, a_1 (1 - chi), a_2 (1 - chi), a_3 (1 - chi)} are j's residual
// seeds (continuity, then momentum scaled by 1 - chi: the momentum residual is
// (1 - chi) times the flow operator plus the body term), ukc is j's velocity
// component along the axis, sgi2h = side / (2 h) with side the direction from j
// to the cell receiving the sensitivity.  Convection u_kc d/da u_c, the
// viscous term, the pressure gradient and the stabilised continuity are the
// terms of j's residuals that read a neighbour along the axis.
template <typename T>
__device__ inline void face_add(const NSCoef<T> &K, int axis, T sgi2h, const T (&at)[4], T ukc,
                                T (&g)[4]) {
  const int kc = 2 - axis;  // velocity component along this axis
  const T coef = sgi2h * ukc - K.nu * K.ih2[axis];
#pragma unroll
  for (int c = 0; c < 3; ++c) g[c] += at[1 + c] * coef;
  g[kc] += sgi2h * at[0];
  g[3] += sgi2h * at[1 + kc] - K.tauh[axis] * at[0];
}

// Ghost value of field f (u, v, w, p) across face (axis, side) of a cell:
// b2 + c0 * (the cell's value).  Cell-based: the channel's ghost rules.
// Node-based (NODE): the boundary node itself, whose value the conditions
// impose (inlet u = (u_ref, 0, 0), outlet p = 0, zero normal velocity at the
// walls; c0 = 0) or take from the interior node next to it (c0 = 1).
template <bool NODE>
__host__ __device__ inline GhostRule channel_ghost(const OpParams &p, int f, int axis, int side) {
  if (!NODE) return ns_ghost<3>(p, f, axis, side);
  bool imposed;
  double val = 0.0;
  if (axis == 2) {
    imposed = side == 0 ? f < 3 : f == 3;
    if (side == 0 && f == 0) val = p.u_ref;
  } else {
    imposed = f == 2 - axis;
  }
  return imposed ? GhostRule{val, 0.0, 0.0} : GhostRule{0.0, 1.0, 0.0};
}

// CHI: 1 fixed chi array, 2 unknown chihat (field 4).  FORCING: some equation
// has a forcing array (compiled out otherwise: its pointers would hold scalar
// registers through the plane loop).
//
// The barriers of the plane loop order LDS traffic only (lds_barrier): global
// loads issued for later planes stay in flight across them, and the stores
// of the gather drain while the next plane is computed.  No thread reads
// global memory that another thread of the launch writes.
//
// Walls in x and y: a cell next to a wall writes into the halo slot across
// the wall (outside the grid, so no other cell owns it) the ghost values of
// its (u, v, w, p), which its stencil then reads like any neighbour, and, for
// the gather, seeds that make the neighbour formula give the ghost map's
// adjoint: with c_f the ghost rule's coefficient of field f (ghost = b + c_f
// u_f), the slot holds a_0 -c_k, a_c c_c (k the component normal to the
// wall) and normal velocity -u_k.  This relies on c_k = -c_p, which the host
// checks.  Walls in z are uniform over a plane and take a branch.
template <typename T, int CHI, bool ADAM, bool FORCING, bool ZSUM, bool NODE>
__global__ __launch_bounds__(NS_THREADS, NS_WAVES_PER_EU) void ns3d_fused_kernel(NS3DArgs<T> A) {
  constexpr int NF = (CHI == 2) ? 5 : 4;  // unknown fields
  constexpr int NA = 5;                   // per cell: seeds a_0, a_c (1 - chi), and u for x faces
  __shared__ T Ul[2][4][NST_Y][NST_X];
  __shared__ T Al[2][NA][NST_Y][NST_X];
  __shared__ T Dl[2][4][NST_Y][NST_X];  // data-term gradient, by plane parity
  __shared__ double red[NS_THREADS / 64][kTerms];
  static_assert(sizeof(T) == 4, "FP32 fields");
  // two coarse planes (coarse plane K in slot K & 1): the one a fine plane
  // interpolates from and the next; the next one is loaded a plane ahead
  static_assert(NF_MAX_COARSE * NCT <= 2 * NS_THREADS, "two coarse values per thread");
  __shared__ T Cw[2][NF_MAX_COARSE * NCT];
  // level-1 restriction: z sums per owned cell (ring of coarse planes), x-pass rows
  __shared__ T Acc[ZSUM ? NACC : 1][NF_MAX_COARSE][NSO_Y][NSO_X];

  const OpParams &p = A.p;
  const int tid = threadIdx.x;
  // block -> tile: consecutive blocks go to different XCDs, so the tiles of
  // XCD k are the contiguous range [k * tiles_per_xcd, (k + 1) * tiles_per_xcd)
  const int per_inst = NS_XCD * A.tiles_per_xcd;
  const int inst = blockIdx.x / per_inst;
  const int bl = blockIdx.x - inst * per_inst;
  const int tile = (bl % NS_XCD) * A.tiles_per_xcd + bl / NS_XCD;
  if (tile >= A.nzt * A.ntx * A.nty) return;  // whole block leaves together
  const int bx = tile % A.ntx, by = (tile / A.ntx) % A.nty, bz = tile / (A.ntx * A.nty);
  // position of this thread in the tile (X, Y), halo included
  int X = 0, Y = 0;
  bool active = true;
  if (tid < NS_MAIN) {
    X = 2 + (tid % NSO_X);
    Y = tid / NSO_X;
  } else if (tid < NS_MAIN + NS_HALO) {
    const int h = tid - NS_MAIN, c = h / NST_Y;
    X = c < 2 ? c : NSO_X + c;
    Y = h % NST_Y;
  } else {
    active = false;
  }
  const int nx = p.n[2], ny = p.n[1], nz = p.n[0];
  const int ox = bx * NSO_X - 2, oy = by * NSO_Y - 2;
  const int x = ox + X, y = oy + Y;
  const int z0 = bz * A.tz, z1 = min(z0 + A.tz, nz);
  const bool in_xy = active && x >= 0 && x < nx && y >= 0 && y < ny;
  const bool seed_xy = in_xy && X >= 1 && X <= NST_X - 2 && Y >= 1 && Y <= NST_Y - 2;
  const bool own_xy = in_xy && X >= 2 && X <= NST_X - 3 && Y >= 2 && Y <= NST_Y - 3;
  // walls next to a seed cell (its halo slot across the wall is in the tile)
  const bool wxm = seed_xy && x == 0, wxp = seed_xy && x == nx - 1;
  const bool wym = seed_xy && y == 0, wyp = seed_xy && y == ny - 1;
  // stored values per row and plane: cells, or the interior nodes and the two
  // boundary nodes of each axis (NODE)
  const int sx = NODE ? nx + 2 : nx;
  const int plane = sx * (NODE ? ny + 2 : ny);
  const int col = NODE ? (y + 1) * sx + (x + 1) : y * nx + x;
  const NSCoef<T> &K = A.K;
  const T wv = T(p.w_pde * p.V);
  const T *th_base = A.theta + inst * A.th_inst;
  // byte offset of this column in field f of plane 0 from the instance's
  // level-0 base (the host checks the largest offset used fits in 32 bits)
  const uint32_t plane_b = (uint32_t)plane * (uint32_t)sizeof(T);
  uint32_t fo[NF];
  for (int f = 0; f < NF; ++f)
    fo[f] = ((uint32_t)f * (uint32_t)A.fsize + (uint32_t)(in_xy ? col : 0)) * (uint32_t)sizeof(T);
  // byte offset of plane z (uniform); planes before the grid map to plane 0
  auto pofs = [&](int z) { return (uint32_t)(max(z, 0) + (NODE ? 1 : 0)) * plane_b; };
  const T *chi_base = CHI == 1 ? A.chi + inst * A.fsize : nullptr;

  // ---- z part of the level-1 restriction (with coarse levels): the owned
  // cell's sums sit in Acc[.][.][Y - 2][X - 2]; a chunk's sums are stored as
  // zsum[instance][chunk][field][plane][y][x] with plane = K - (z0 / 2 - 1)
  const int kz0 = z0 / 2 - 1, nkz = A.tz / 2 + 2;
  // first and last gather planes of this chunk adding to coarse plane K (the
  // first assigns, later ones add, the last stores): 2K - 1 .. 2K + 2 within
  // the chunk; fine plane 0 also reaches coarse plane 1, and fine plane
  // nz - 1 coarse plane ncz - 2
  auto first_plane = [&](int K) { return (K == 1 && z0 == 0) ? 0 : max(z0, 2 * K - 1); };
  auto last_plane = [&](int K) { return min(z1 - 1, K == A.ncz - 2 ? 2 * K + 3 : 2 * K + 2); };
  T *zs_base = A.cpart + ((long)inst * A.nzt + bz) * (long)NF * nkz * plane;
  const uint32_t zs_field_b = (uint32_t)nkz * plane_b;  // one field's planes, bytes

  // xy interpolation taps of this column from level 1
  int jx[2] = {0, 0}, jy[2] = {0, 0};
  T wx[2] = {T(0), T(0)}, wy[2] = {T(0), T(0)};
  if (A.has_coarse && in_xy) {
    if (NODE) {
      prolong_taps_node(x + 1, jx, wx);
      prolong_taps_node(y + 1, jy, wy);
    } else {
      prolong_taps(x, A.nc[2], jx, wx);
      prolong_taps(y, A.nc[1], jy, wy);
    }
  }
  T Wlo[NF], Whi[NF];
  for (int f = 0; f < NF; ++f) Wlo[f] = Whi[f] = T(0);
  int kmin_c = -1000;
  // coarse window origin (ox, oy are even) and the taps in window coordinates
  const int cxb = (ox >> 1) - 1, cyb = (oy >> 1) - 1;
  const int lx[2] = {jx[0] - cxb, jx[1] - cxb}, ly[2] = {jy[0] - cyb, jy[1] - cyb};
  // lower coarse plane of the interpolation of fine plane z (valid z)
  auto kbase = [&](int z) {
    if (NODE) return min((z + 1) >> 1, A.nc[0] - 2);  // coarse nodes of fine node z + 1
    if (z == 0) return 0;
    if (z == nz - 1) return A.nc[0] - 2;
    return (z & 1) ? z / 2 : z / 2 - 1;
  };
  // each thread moves two values of a coarse plane window: global -> registers -> LDS
  // the two window values this thread moves: byte offset within a coarse plane
  uint32_t co[2] = {0u, 0u};
  bool cin[2] = {false, false};
  for (int u = 0; u < 2; ++u) {
    const int e = tid + u * NS_THREADS;
    if (e < NF * NCT) {
      const int f = e / NCT, rem = e - f * NCT, j = rem / NCT_X, i = rem - j * NCT_X;
      const int cy = cyb + j, cx = cxb + i;
      cin[u] = cy >= 0 && cy < A.nc[1] && cx >= 0 && cx < A.nc[2];
      if (cin[u])
        co[u] = ((uint32_t)f * (uint32_t)A.csize + (uint32_t)(cy * A.nc[2] + cx)) * (uint32_t)sizeof(T);
    }
  }
  auto cload = [&](int Kc, T (&r)[2]) {
    const T *cb = A.w1 + inst * A.w1_inst + Kc * A.nc[1] * A.nc[2];
    for (int u = 0; u < 2; ++u) r[u] = cin[u] ? ld_at(cb, co[u]) : T(0);
  };
  auto cstore = [&](int Kc, const T (&r)[2]) {
    for (int u = 0; u < 2; ++u) {
      const int e = tid + u * NS_THREADS;
      if (e < NF * NCT) Cw[Kc & 1][e] = r[u];
    }
  };
  // planes resident in the two slots; prologue: the first fine plane's pair
  int res[2] = {-1, -1};
  if (A.has_coarse) {
    const int zf = max(z0 - 2, 0);
    const int k0 = kbase(zf);
    T r0[2], r1[2];
    cload(k0, r0);
    cload(k0 + 1, r1);
    cstore(k0, r0);
    cstore(k0 + 1, r1);
    res[k0 & 1] = k0;
    res[(k0 + 1) & 1] = k0 + 1;
    lds_barrier();
  }

  // planes pz-3 .. pz of this column: U0w is w at pz-3 (the gather's lower
  // z face), U1 (u, v, w, p) at pz-2, U2 and U3 all five values
  T U0w = T(0), U1[4], U2[5], U3[5];
  for (int f = 0; f < 4; ++f) U1[f] = T(0);
  for (int f = 0; f < 5; ++f) U2[f] = U3[f] = T(0);
  T A0[4], A1[4], A2[4];  // scaled seeds at planes pz-3 .. pz-1
  for (int e = 0; e < 4; ++e) A0[e] = A1[e] = A2[e] = T(0);
  // centre sensitivity of the cell at the gather plane, formed in its seed pass
  T Cq[5] = {T(0), T(0), T(0), T(0), T(0)};
  double part[kTerms] = {0.0, 0.0, 0.0, 0.0, 0.0};

  // ghost value of field f across face (axis a, side s) of a cell with value c
#define GB(f, a, s) T(channel_ghost<NODE>(p, f, a, s).b2)
#define GC0(f, a, s) T(channel_ghost<NODE>(p, f, a, s).c0)
#define GV(f, a, s, c) (GB(f, a, s) + GC0(f, a, s) * (c))

  const int key_base = (inst * A.nzt * A.ntx * A.nty + tile) * A.tz;

  // theta (and chi) of the next plane are loaded one iteration ahead; theta
  // of the two planes before is kept for the Adam update of the gather plane
  T thn[NF], chin = T(0), tA[NF], tB[NF];  // tA, tB: theta of the two planes below (without ZSUM)
  for (int f = 0; f < NF; ++f) thn[f] = tA[f] = tB[f] = T(0);
  if (in_xy && z0 - 2 >= 0) {
    const uint32_t zb = pofs(z0 - 2);
    for (int f = 0; f < NF; ++f) thn[f] = ld_at(th_base, fo[f] + zb);
    if (CHI == 1) chin = ld_at(chi_base, fo[0] + zb);
  }

  for (int pz = z0 - 2; pz <= z1 + 1; ++pz) {
    // ---- 0. issue the loads needed later: the coarse plane the next fine plane
    // adds (stored to LDS at the end of this iteration), theta of plane pz+1,
    // m and v of plane pz-2
    T cpre[2];
    int cnext = -1;
    if (A.has_coarse && pz + 1 <= z1 + 1 && pz + 1 >= 0 && pz + 1 < nz) {
      const int kn = kbase(pz + 1) + 1;
      if (res[kn & 1] != kn) {
        cnext = kn;
        cload(kn, cpre);
      }
    }
    T th[NF], chi_pz = chin;
    for (int f = 0; f < NF; ++f) th[f] = thn[f];
    if (in_xy && pz + 1 >= 0 && pz + 1 < nz) {
      const uint32_t zb = pofs(pz + 1);
      for (int f = 0; f < NF; ++f) thn[f] = ld_at(th_base, fo[f] + zb);
      if (CHI == 1) chin = ld_at(chi_base, fo[0] + zb);
    }
    T mq[NF], vq[NF], tq[NF];
    const int q = pz - 2, qb = q & 1;
    // the measurement records of plane pz-1 (read early: the loop waits on them)
    int mp0 = 0, mp1 = 0;
    if (pz - 1 >= z0 && pz - 1 < z1) {
      mp0 = A.mptr[key_base + (pz - 1 - z0)];
      mp1 = A.mptr[key_base + (pz - 1 - z0) + 1];
    }
    const bool gather = own_xy && q >= z0 && q < z1;
    const uint32_t qofs = pofs(q);
    if (ADAM && gather) {
      for (int f = 0; f < NF; ++f) {
        tq[f] = ZSUM ? ld_at(th_base, fo[f] + qofs) : tB[f];
        mq[f] = ld_at(A.adam.m + inst * A.th_inst, fo[f] + qofs);
        vq[f] = ld_at(A.adam.v + inst * A.th_inst, fo[f] + qofs);
      }
    }
    // ---- 1. prolong plane pz of this column
    T un[5];
    if (in_xy && pz >= 0 && pz < nz) {
      if (A.has_coarse) {
        int km;
        T wlo, whi;
        if (NODE) {  // fine node pz + 1: even copies coarse node (pz + 1) / 2, odd averages two
          const int n = pz + 1;
          km = kbase(pz);
          if (n & 1) { wlo = T(0.5); whi = T(0.5); }
          else if (n / 2 == km) { wlo = T(1); whi = T(0); }
          else { wlo = T(0); whi = T(1); }
        }
        else if (pz == 0) { km = 0; wlo = T(1.25); whi = T(-0.25); }
        else if (pz == nz - 1) { km = A.nc[0] - 2; wlo = T(-0.25); whi = T(1.25); }
        else if ((pz & 1) == 0) { km = pz / 2 - 1; wlo = T(0.25); whi = T(0.75); }
        else { km = pz / 2; wlo = T(0.75); whi = T(0.25); }
        if (km != kmin_c) {
          if (km == kmin_c + 1) {
            for (int f = 0; f < NF; ++f) Wlo[f] = Whi[f];
            coarse_xy<T, NF>(Cw[(km + 1) & 1], lx, wx, ly, wy, Whi);
          } else {
            coarse_xy<T, NF>(Cw[km & 1], lx, wx, ly, wy, Wlo);
            coarse_xy<T, NF>(Cw[(km + 1) & 1], lx, wx, ly, wy, Whi);
          }
          kmin_c = km;
        }
        for (int f = 0; f < NF; ++f) un[f] = th[f] + (wlo * Wlo[f] + whi * Whi[f]);
      } else {
        for (int f = 0; f < NF; ++f) un[f] = th[f];
      }
      if (CHI == 2) un[4] = sigmoid_stable(un[4] - T(p.chi_shift));
      else un[4] = chi_pz;
    } else {
      for (int f = 0; f < 5; ++f) un[f] = T(0);
    }
    U0w = U1[2];
    for (int f = 0; f < 4; ++f) U1[f] = U2[f];
    for (int f = 0; f < 5; ++f) { U2[f] = U3[f]; U3[f] = un[f]; }

    // ---- 2. stage plane pz-1 for the xy neighbours, with the wall ghosts;
    // clear the data seeds
    const int s = pz - 1, sb = s & 1;
    if (in_xy)
      for (int f = 0; f < 4; ++f) Ul[sb][f][Y][X] = U2[f];
    if (wxm) for (int f = 0; f < 4; ++f) Ul[sb][f][Y][X - 1] = GV(f, 2, 0, U2[f]);
    if (wxp) for (int f = 0; f < 4; ++f) Ul[sb][f][Y][X + 1] = GV(f, 2, 1, U2[f]);
    if (wym) for (int f = 0; f < 4; ++f) Ul[sb][f][Y - 1][X] = GV(f, 1, 0, U2[f]);
    if (wyp) for (int f = 0; f < 4; ++f) Ul[sb][f][Y + 1][X] = GV(f, 1, 1, U2[f]);
    for (int f = 0; f < 4; ++f) Dl[sb][f][Y][X] = T(0);
    lds_barrier();

    // ---- 3. residual and measurement seeds at plane s
    T an[4] = {T(0), T(0), T(0), T(0)};
    T Cs[5] = {T(0), T(0), T(0), T(0), T(0)};
    if (seed_xy && s >= 0 && s < nz && s >= z0 - 1 && s <= z1) {
      T Us[4][7];
      for (int f = 0; f < 4; ++f) {
        const T c = U2[f];
        Us[f][S_C] = c;
        Us[f][S_ZM] = s > 0 ? U1[f] : GV(f, 0, 0, c);
        Us[f][S_ZP] = s < nz - 1 ? U3[f] : GV(f, 0, 1, c);
        Us[f][S_YM] = Ul[sb][f][Y - 1][X];
        Us[f][S_YP] = Ul[sb][f][Y + 1][X];
        Us[f][S_XM] = Ul[sb][f][Y][X - 1];
        Us[f][S_XP] = Ul[sb][f][Y][X + 1];
      }
      NSLocal<3, T> L;
      ns_local<3>(K, Us, L);
      const T uc[3] = {U2[0], U2[1], U2[2]};
      const T chi = U2[4], omc = T(1) - chi;
      T r[4];
      ns_residual<3, true>(K, L, uc, chi, r);
      T a[4];
      for (int e = 0; e < 4; ++e) {
        if (FORCING && A.forcing[e]) r[e] -= ld_at(A.forcing[e] + inst * A.fsize, fo[0] + pofs(s));
        a[e] = T(2) * wv * r[e];
      }
      an[0] = a[0];
      for (int c = 0; c < 3; ++c) an[1 + c] = a[1 + c] * omc;
      for (int e = 0; e < 4; ++e) Al[sb][e][Y][X] = an[e];
      Al[sb][4][Y][X] = uc[0];
      // wall slots: seeds whose neighbour adjoint is the ghost map's
#define NS_WALL_SLOT(cond, axis, side, SY, SX)                                              \
      if (cond) {                                                                           \
        const int k = 2 - (axis);                                                           \
        if (NODE) {                                                                         \
          for (int e = 0; e < 5; ++e) Al[sb][e][SY][SX] = T(0);                             \
        } else {                                                                            \
          Al[sb][0][SY][SX] = -GC0(k, axis, side) * an[0];                                  \
          for (int c = 0; c < 3; ++c) Al[sb][1 + c][SY][SX] = GC0(c, axis, side) * an[1 + c]; \
          if ((axis) == 2) Al[sb][4][SY][SX] = -uc[0];                                      \
        }                                                                                   \
      }
      NS_WALL_SLOT(wxm, 2, 0, Y, X - 1)
      NS_WALL_SLOT(wxp, 2, 1, Y, X + 1)
      NS_WALL_SLOT(wym, 1, 0, Y - 1, X)
      NS_WALL_SLOT(wyp, 1, 1, Y + 1, X)
#undef NS_WALL_SLOT
      if (own_xy && s >= z0 && s < z1) {
        for (int e = 0; e < 4; ++e) part[MODIL_TERM_PDE] += (double)wv * (double)r[e] * (double)r[e];
        // the cell's own sensitivity (centre of its stencil), used by its
        // gather one plane later
        for (int f = 0; f < 3; ++f) {
          T v = T(2) * K.nu * K.ssum * an[1 + f] + K.lam * chi * a[1 + f];
          for (int c = 0; c < 3; ++c) v += an[1 + c] * L.du[c][f];
          Cs[f] = v;
        }
        Cs[3] = T(2) * K.tsum * a[0];
        if (CHI == 2) {
          T dchi = T(0);
          for (int c = 0; c < 3; ++c) dchi += a[1 + c] * (K.lam * uc[c] - L.body[c]);
          Cs[4] = dchi * chi * omc;
        }
      }
    }
    for (int e = 0; e < 4; ++e) { A0[e] = A1[e]; A1[e] = A2[e]; A2[e] = an[e]; }
    // measurements of plane s: their gradient is gathered one plane later
    if (s >= z0 && s < z1) {
      const int e0 = mp0, e1 = mp1;
      for (int e = e0 + tid; e < e1; e += NS_THREADS) {
        const FusedMeas me = A.mrec[e];
        const int f = me.field, k = me.cell;
        const T uv = Ul[sb][f][me.ly][me.lx];
        const double r = (double)uv - me.val;
        part[me.term] += me.w * r * r;
        if (e == e0 || A.mrec[e - 1].field != f || A.mrec[e - 1].cell != k) {
          double gs = 0.0;
          for (int j = e; j < e1 && A.mrec[j].field == f && A.mrec[j].cell == k; ++j)
            gs += 2.0 * A.mrec[j].w * ((double)uv - A.mrec[j].val);
          Dl[sb][f][me.ly][me.lx] = T(gs);
        }
      }
    }

    // ---- 4. gradient, and Adam, at plane q: it reads what the previous plane
    // wrote to LDS and its own column's seeds of plane s, so it shares the
    // phase of the seeds of plane s
    if (gather) {
      T g[4] = {Cq[0], Cq[1], Cq[2], Cq[3]};
      // z faces: the neighbours below and above, or the wall's ghost map
      if (q > 0) {
        face_add(K, 0, K.i2h[0], A0, U0w, g);
      } else {
        T fs[4] = {T(0), T(0), T(0), T(0)};
        face_add(K, 0, -K.i2h[0], A1, U1[2], fs);
        for (int f = 0; f < 4; ++f) g[f] += GC0(f, 0, 0) * fs[f];
      }
      if (q < nz - 1) {
        face_add(K, 0, -K.i2h[0], A2, U2[2], g);
      } else {
        T fs[4] = {T(0), T(0), T(0), T(0)};
        face_add(K, 0, K.i2h[0], A1, U1[2], fs);
        for (int f = 0; f < 4; ++f) g[f] += GC0(f, 0, 1) * fs[f];
      }
      // y and x faces: neighbours or wall slots alike
#define NS_XY_FACE(axis, sgn, SY, SX, UKC)                                                   \
      {                                                                                      \
        const T aj[4] = {Al[qb][0][SY][SX], Al[qb][1][SY][SX], Al[qb][2][SY][SX],           \
                         Al[qb][3][SY][SX]};                                                 \
        face_add(K, axis, (sgn) * K.i2h[axis], aj, UKC, g);                                  \
      }
      NS_XY_FACE(1, T(1), Y - 1, X, Ul[qb][1][Y - 1][X])
      NS_XY_FACE(1, T(-1), Y + 1, X, Ul[qb][1][Y + 1][X])
      NS_XY_FACE(2, T(1), Y, X - 1, Al[qb][4][Y][X - 1])
      NS_XY_FACE(2, T(-1), Y, X + 1, Al[qb][4][Y][X + 1])
#undef NS_XY_FACE
      if (NODE) {
        // the cell's own residuals read the boundary node across an x or y
        // wall, whose value is imposed or the cell's own (ghost = b + c u)
#define NS_NODE_WALL(cond, axis, side, sgn, UK)                                       \
        if (cond) {                                                                 \
          T fs[4] = {T(0), T(0), T(0), T(0)};                                       \
          face_add(K, axis, (sgn) * K.i2h[axis], A1, UK, fs);                       \
          for (int f = 0; f < 4; ++f) g[f] += GC0(f, axis, side) * fs[f];           \
        }
        NS_NODE_WALL(x == 0, 2, 0, T(-1), U1[0])
        NS_NODE_WALL(x == nx - 1, 2, 1, T(1), U1[0])
        NS_NODE_WALL(y == 0, 1, 0, T(-1), U1[1])
        NS_NODE_WALL(y == ny - 1, 1, 1, T(1), U1[1])
#undef NS_NODE_WALL
      }
      T gg[5];
      for (int f = 0; f < 4; ++f) gg[f] = g[f] + Dl[qb][f][Y][X];
      gg[4] = Cq[4];
      const int base = inst * A.th_inst;
      if (ZSUM && A.has_coarse) {
        // z sums: plane q adds to the two coarse planes of its row of T
        int kk[2];
        T ww[2];
        prolong_taps(q, A.ncz, kk, ww);
        for (int t = 0; t < 2; ++t) {
          T *acc = &Acc[kk[t] & (NACC - 1)][0][Y - 2][X - 2];
          const bool first = q == first_plane(kk[t]), last = q == last_plane(kk[t]);
          const uint32_t zb = (uint32_t)(kk[t] - kz0) * plane_b + fo[0];
          for (int f = 0; f < NF; ++f) {
            const T v = (first ? T(0) : acc[f * NSO_Y * NSO_X]) + ww[t] * gg[f];
            if (last) st_at(zs_base, zb + (uint32_t)f * zs_field_b, v);
            else acc[f * NSO_Y * NSO_X] = v;
          }
        }
      }
      for (int f = 0; f < NF; ++f) {
        if (!ADAM || !ZSUM) st_at(A.g + base, fo[f] + qofs, gg[f]);
        if (ADAM) {
          const T mm = A.adam.b1 * mq[f] + (T(1) - A.adam.b1) * gg[f];
          const T vv = A.adam.b2 * vq[f] + (T(1) - A.adam.b2) * gg[f] * gg[f];
          st_at(A.adam.m + base, fo[f] + qofs, mm);
          st_at(A.adam.v + base, fo[f] + qofs, vv);
          st_at(A.adam.th_out + base, fo[f] + qofs,
                adam_theta(tq[f], mm, vv, A.adam.step, A.adam.isb2, A.adam.eps));
        }
      }
    }
    if (!ZSUM)
      for (int f = 0; f < NF; ++f) { tB[f] = tA[f]; tA[f] = th[f]; }
    for (int f = 0; f < 5; ++f) Cq[f] = Cs[f];
    // the slot taken by the next coarse plane held the one below this fine
    // plane's pair, which nobody reads after step 1
    if (cnext >= 0) {
      cstore(cnext, cpre);
      res[cnext & 1] = cnext;
    }
    lds_barrier();
  }

#undef GV
#undef GC0
#undef GB
  // ---- node-based: the boundary nodes of this block's region carry no
  // equation and get a zero gradient (and, with Adam, the Adam update with
  // it).  The region in node coordinates: the nodes of its owned interior
  // cells, plus the boundary nodes beyond them where the tile or chunk ends
  // at the grid's boundary, so every boundary node belongs to one block.
  if (NODE) {
    const int Nx = nx + 1, Ny = ny + 1, Nz = nz + 1;  // last node index per axis
    const int lo[3] = {bz == 0 ? 0 : z0 + 1, by == 0 ? 0 : by * NSO_Y + 1, bx == 0 ? 0 : bx * NSO_X + 1};
    const int hi[3] = {bz == A.nzt - 1 ? Nz : z1, by == A.nty - 1 ? Ny : min(by * NSO_Y + NSO_Y, ny),
                       bx == A.ntx - 1 ? Nx : min(bx * NSO_X + NSO_X, nx)};
    const int last[3] = {Nz, Ny, Nx};
    const int ext[3] = {hi[0] - lo[0] + 1, hi[1] - lo[1] + 1, hi[2] - lo[2] + 1};
    const int base = inst * A.th_inst;
    // faces of the region on the grid's boundary; a node on several faces is
    // taken by the first of them (axis order z, y, x; low side first)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const int fixed = side ? last[a] : 0;
        if ((side ? hi[a] : lo[a]) != fixed) continue;
        const int b1 = (a + 1) % 3, b2 = (a + 2) % 3;
        const int n = ext[b1] * ext[b2];
        for (int e = tid; e < n; e += NS_THREADS) {
          int c[3];
          c[a] = fixed;
          c[b1] = lo[b1] + e / ext[b2];
          c[b2] = lo[b2] + e % ext[b2];
          bool earlier = false;  // on a face handled before this one
#pragma unroll
          for (int a2 = 0; a2 < a; ++a2) earlier = earlier || c[a2] == 0 || c[a2] == last[a2];
          if (earlier) continue;
          const uint32_t off = (uint32_t)(((c[0] * (ny + 2) + c[1]) * (nx + 2)) + c[2]) * (uint32_t)sizeof(T);
          const uint32_t fb = (uint32_t)A.fsize * (uint32_t)sizeof(T);
          T mo[NF], vo[NF], to[NF];  // every load issued before the first use
          if (ADAM)
            for (int f = 0; f < NF; ++f) {
              mo[f] = ld_at(A.adam.m + base, off + f * fb);
              vo[f] = ld_at(A.adam.v + base, off + f * fb);
              to[f] = ld_at(th_base, off + f * fb);
            }
          for (int f = 0; f < NF; ++f) {
            const uint32_t o = off + f * fb;
            st_at(A.g + base, o, T(0));
            if (ADAM) {
              const T mm = A.adam.b1 * mo[f], vv = A.adam.b2 * vo[f];
              st_at(A.adam.m + base, o, mm);
              st_at(A.adam.v + base, o, vv);
              st_at(A.adam.th_out + base, o, adam_theta(to[f], mm, vv, A.adam.step, A.adam.isb2, A.adam.eps));
            }
          }
        }
      }
  }
  // ---- block sum of the loss partials (fixed order: each wave's by
  // wave_sum, left in its lane 63, then the waves in order)
  for (int k = 0; k < kTerms; ++k) part[k] = wave_sum(part[k]);
  if ((tid & 63) == 63)
    for (int k = 0; k < kTerms; ++k) red[tid >> 6][k] = part[k];
  __syncthreads();
  if (tid < kTerms) {
    double sum = 0.0;
    for (int w = 0; w < NS_THREADS / 64; ++w) sum += red[w][tid];
    A.partials[((long)inst * A.n_part_blocks + tile) * kTerms + tid] = sum;
  }
}

// ------------------------------------------------------------------ host side
// the grid the fused kernel marches over: the cells, or the interior nodes
static void fused_grid(const modil_problem &P, int (&n)[3]) {
  for (int a = 0; a < 3; ++a) n[a] = P.dims[a] - (P.centering == MODIL_NODE ? 1 : 0);
}

void ns3d_tiles(const modil_problem &P, int &tz, int &nzt, int &ntx, int &nty, int &ox, int &oy) {
  int n[3];
  fused_grid(P, n);
  const int nz = n[0], ny = n[1], nx = n[2];
  ntx = (nx + NSO_X - 1) / NSO_X;
  nty = (ny + NSO_Y - 1) / NSO_Y;
  // z-chunk: the longest of 32, 16, 8, 4, 2 planes that still gives every
  // compute unit a block (one block fills a CU's LDS); a chunk marches 4 halo
  // planes besides its own, so shorter chunks cost more per output plane
  // (256^3: 32-plane chunks, 1024 blocks, 606 us against 640 with 16)
  const long xy = (long)ntx * nty * P.batch;
  tz = 32;
  while (tz > 2 && xy * ((nz + tz - 1) / tz) < kComputeUnits) tz /= 2;
  nzt = (nz + tz - 1) / tz;
  ox = NSO_X;
  oy = NSO_Y;
}

bool ns3d_offsets_fit(const modil_problem &P) {
  const unsigned long long e = P.centering == MODIL_NODE ? 1 : 0;
  const unsigned long long cells = (P.dims[0] + e) * (P.dims[1] + e) * (P.dims[2] + e);
  const unsigned long long ts = P.dtype == MODIL_F64 ? 8 : 4;
  return 5ull * cells * ts < (1ull << 32);  // fields of level 0; level 1 is smaller
}

template <typename T>
static hipError_t fused_t(modil_ctx *c, const void *theta, void *g, const AdamHost *ad,
                          const void *th_out, void *m, void *v) {
  const modil_problem &P = c->prob;
  NS3DArgs<T> A{};
  OpParams &p = A.p;
  p.ndim = 3;
  const bool node = P.centering == MODIL_NODE;
  fused_grid(P, p.n);
  for (int a = 0; a < 3; ++a) p.h[a] = P.lengths[a] / P.dims[a];
  p.V = p.h[0] * p.h[1] * p.h[2];
  p.w_pde = P.w_pde; p.w_reg = P.w_reg; p.w_bc = P.w_bc;
  p.re = P.re; p.diam = P.diam; p.lam = P.lambda_; p.chi_shift = P.chi_shift;
  p.tau_coef = P.tau_coef; p.u_ref = P.u_ref;
  p.inst_re = c->inst_re;
  // the kernel's wall slots rely on two properties of the x and y wall rules:
  // the normal velocity's ghost coefficient is minus the pressure's, and the
  // normal velocity at a y wall is mirrored (ghost -v)
  for (int side = 0; side < 2 && !node; ++side) {
    for (int axis = 1; axis <= 2; ++axis)
      if (ns_ghost<3>(p, 2 - axis, axis, side).c0 != -ns_ghost<3>(p, 3, axis, side).c0)
        return hipErrorInvalidValue;
    const GhostRule v = ns_ghost<3>(p, 1, 1, side);
    if (v.b2 != 0.0 || v.c0 != -1.0) return hipErrorInvalidValue;
  }
  int tox, toy;
  ns3d_tiles(P, A.tz, A.nzt, A.ntx, A.nty, tox, toy);
  A.tiles_per_xcd = (A.nzt * A.ntx * A.nty + NS_XCD - 1) / NS_XCD;
  for (int a = 0; a < 3; ++a) {
    A.K.i2h[a] = T(0.5 / p.h[a]);
    A.K.ih2[a] = T(1.0 / (p.h[a] * p.h[a]));
    A.K.tauh[a] = T(p.tau_coef / p.h[a]);
  }
  A.K.nu = T(P.diam / P.re);  // the fused path requires one Reynolds number for all instances
  A.K.lam = T(P.lambda_);
  A.K.ssum = A.K.ih2[0] + A.K.ih2[1] + A.K.ih2[2];
  A.K.tsum = A.K.tauh[0] + A.K.tauh[1] + A.K.tauh[2];
  A.has_coarse = P.n_levels > 1;
  A.fsize = (int)c->lay.fine_cells;
  A.th_inst = (int)c->lay.level_stride[0];
  A.theta = (const T *)theta;
  if (A.has_coarse) {
    for (int a = 0; a < 3; ++a) A.nc[a] = P.dims[a] / 2 + (node ? 1 : 0);  // cells or nodes
    A.ncz = A.nc[0];
    A.ncy = A.nc[1];
    A.ncx = A.nc[2];
    A.cpart = (T *)c->cpart;
    A.csize = A.nc[0] * A.nc[1] * A.nc[2];
    A.w1_inst = (int)c->lay.level_stride[1];
    // level 1 of the prolonged coarse fields: theta itself when it is the coarsest
    A.w1 = (P.n_levels == 2 ? (const T *)theta : (const T *)c->w_buf) + c->lay.level_offset[1];
  }
  A.g = (T *)g;
  for (int e = 0; e < 4; ++e) A.forcing[e] = (const T *)c->forcing[e];
  A.chi = (const T *)c->chi;
  A.mptr = c->fm_ptr;
  A.mrec = c->fm_rec;
  A.partials = c->partials;
  A.n_part_blocks = (int)c->n_part_blocks;
  if (ad) {
    A.adam.th_in = (const T *)theta; A.adam.th_out = (T *)th_out;
    A.adam.m = (T *)m; A.adam.v = (T *)v;
    A.adam.b1 = T(ad->b1); A.adam.b2 = T(ad->b2); A.adam.step = T(ad->step);
    A.adam.isb2 = T(ad->isb2); A.adam.eps = T(ad->eps);
  }
  const dim3 grid(NS_XCD * A.tiles_per_xcd * P.batch), block(NS_THREADS);
  const bool fixed = (P.flags & MODIL_FLAG_CHI_FIXED) != 0;
  const bool forcing = A.forcing[0] || A.forcing[1] || A.forcing[2] || A.forcing[3];
  auto go = [&](auto kernel) { kernel<<<grid, block, 0, c->stream>>>(A); };
  const bool zsum = A.has_coarse && (P.flags & MODIL_FLAG_FUSED_RESTRICT) != 0;
  auto pick = [&](auto chi_tag) {
    constexpr int C = decltype(chi_tag)::value;
    if (node) {
      if (ad) forcing ? go(ns3d_fused_kernel<T, C, true, true, false, true>) : go(ns3d_fused_kernel<T, C, true, false, false, true>);
      else forcing ? go(ns3d_fused_kernel<T, C, false, true, false, true>) : go(ns3d_fused_kernel<T, C, false, false, false, true>);
    } else if (zsum) {
      if (ad) forcing ? go(ns3d_fused_kernel<T, C, true, true, true, false>) : go(ns3d_fused_kernel<T, C, true, false, true, false>);
      else forcing ? go(ns3d_fused_kernel<T, C, false, true, true, false>) : go(ns3d_fused_kernel<T, C, false, false, true, false>);
    } else {
      if (ad) forcing ? go(ns3d_fused_kernel<T, C, true, true, false, false>) : go(ns3d_fused_kernel<T, C, true, false, false, false>);
      else forcing ? go(ns3d_fused_kernel<T, C, false, true, false, false>) : go(ns3d_fused_kernel<T, C, false, false, false, false>);
    }
  };
  if (fixed) pick(std::integral_constant<int, 1>{});
  else pick(std::integral_constant<int, 2>{});
  return hipGetLastError();
}

// Level-1 gradient from the chunks' z sums.  A block owns 32 x 8 level-1
// cells of one coarse plane, field and instance: it adds the (one or two)
// chunks' z sums of its fine region (the cells' rows and columns of T plus
// two on each side) into LDS, lower chunk first, applies T^T along x and then
// along y, writes the sums to the gradient pack and, with Adam, updates
// level 1.  Grid: (ncx / 32, ncy / 8, (instance * nf + field) * ncz + z).
constexpr int AS_X = 32, AS_Y = 8;                      // level-1 cells per block
constexpr int AS_FX = 2 * AS_X + 4, AS_FY = 2 * AS_Y + 4;  // fine region: two more each side

template <typename T>
struct AssembleArgs {
  const T *zsum;         // [instance][chunk][field][plane][fine y][fine x]
  T *g;                  // gradient pack (level 1 is written)
  int batch, nf, tz, nzt;
  int ncz, ncy, ncx;
  int off1, stride1;     // pack offset of level 1, its elements per instance
  AdamArgs<T> adam;      // pack bases
};

// One level-1 cell of T^T along an axis: coarse cell J (of n), v[0..3] the
// fine cells 2J - 1 .. 2J + 2 (zero outside the grid), v[-S] fine cell
// 2J - 2 and v[4S] fine cell 2J + 3.  Interior cells take 1/4, 3/4, 3/4,
// 1/4; the end rows of T (fine cells 0 and 2n - 1 extrapolate: 5/4 and -1/4)
// add to coarse cells 0, 1, n - 2 and n - 1.
template <typename T, int S>
__device__ inline T restrict_tap(const T *v, int J, int n) {
  T acc = T(0.25) * v[0] + T(0.75) * v[S] + T(0.75) * v[2 * S] + T(0.25) * v[3 * S];
  if (J <= 1 || J >= n - 2) {
    if (J == 0) acc += T(0.5) * v[S];          // fine 0: 5/4 instead of 3/4
    if (J == n - 1) acc += T(0.5) * v[2 * S];  // fine 2n - 1: 5/4 instead of 3/4
    if (J == 1) acc += T(-0.25) * v[-S];       // fine 0 reaches coarse 1
    if (J == n - 2) acc += T(-0.25) * v[4 * S];  // fine 2n - 1 reaches coarse n - 2
  }
  return acc;
}

template <typename T, bool ADAM>
__global__ __launch_bounds__(256) void fused_assemble_kernel(AssembleArgs<T> A) {
  __shared__ T F[AS_FY][AS_FX];  // fine region: row i is fine row 2 y0 - 2 + i
  __shared__ T Xs[AS_FY][AS_X];  // x sums of every fine row of the region
  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * AS_X, y0 = blockIdx.y * AS_Y;
  const int bz = blockIdx.z;
  const int z = bz % A.ncz, rest = bz / A.ncz;
  const int f = rest % A.nf, inst = rest / A.nf;
  const int hz = A.tz / 2, nkz = hz + 2;
  const int nx = 2 * A.ncx, ny = 2 * A.ncy;
  const long plane = (long)nx * ny;
  // the chunks holding z sums of coarse plane z (three when a chunk holds one
  // coarse plane): (chunk, plane slot), lower first
  int cz[3], sz[3], nc = 0;
  {
    const int c = z / hz, k = z - c * hz;
    if (k == 0 && c > 0) { cz[nc] = c - 1; sz[nc++] = hz + 1; }
    cz[nc] = c; sz[nc++] = k + 1;
    if (k == hz - 1 && c + 1 < A.nzt) { cz[nc] = c + 1; sz[nc++] = 0; }
  }
  // the level-1 state of this thread's cell, loaded early
  const int lx = tid % AS_X, ly = tid / AS_X;
  const int cx = x0 + lx, cy = y0 + ly;
  const bool mine = cx < A.ncx && cy < A.ncy;
  const long pe = (long)A.off1 + (long)inst * A.stride1 + ((long)f * A.ncz + z) * A.ncy * A.ncx +
                  (long)cy * A.ncx + cx;
  T th = T(0), mo = T(0), vo = T(0);
  if (ADAM && mine) { th = A.adam.th_in[pe]; mo = A.adam.m[pe]; vo = A.adam.v[pe]; }
  // fine region, chunks added in order (0 outside the grid)
  const int fy0 = 2 * y0 - 2, fx0 = 2 * x0 - 2;
  for (int e = tid; e < AS_FY * AS_FX; e += 256) {
    const int i = e / AS_FX, j = e - i * AS_FX;
    const int fy = fy0 + i, fx = fx0 + j;
    T v = T(0);
    if (fy >= 0 && fy < ny && fx >= 0 && fx < nx)
      for (int t = 0; t < nc; ++t)
        v += A.zsum[(((long)inst * A.nzt + cz[t]) * A.nf + f) * nkz * plane + sz[t] * plane +
                    (long)fy * nx + fx];
    F[i][j] = v;
  }
  __syncthreads();
  // x sums: fine row i, level-1 column x0 + c (fine columns 2(x0 + c) - 1 .. at F[i][2c + 1 ..])
  for (int e = tid; e < AS_FY * AS_X; e += 256) {
    const int i = e / AS_X, c = e - i * AS_X;
    Xs[i][c] = x0 + c < A.ncx ? restrict_tap<T, 1>(&F[i][2 * c + 1], x0 + c, A.ncx) : T(0);
  }
  __syncthreads();
  if (!mine) return;
  const T sum = restrict_tap<T, AS_X>(&Xs[2 * ly + 1][lx], cy, A.ncy);
  A.g[pe] = sum;
  if (ADAM) {
    const T mm = A.adam.b1 * mo + (T(1) - A.adam.b1) * sum;
    const T vv = A.adam.b2 * vo + (T(1) - A.adam.b2) * sum * sum;
    A.adam.m[pe] = mm;
    A.adam.v[pe] = vv;
    A.adam.th_out[pe] = adam_theta(th, mm, vv, A.adam.step, A.adam.isb2, A.adam.eps);
  }
}

size_t fused_partial_bytes(const modil_problem &P) {
  if (P.op != MODIL_OP_NS3D || P.centering != MODIL_CELL || P.dtype != MODIL_F32 || P.n_levels < 2 ||
      !(P.flags & MODIL_FLAG_FUSED_RESTRICT))
    return 0;
  int tz, nzt, ntx, nty, ox, oy;
  ns3d_tiles(P, tz, nzt, ntx, nty, ox, oy);
  const int nf = (P.flags & MODIL_FLAG_CHI_FIXED) ? 4 : 5;
  return (size_t)P.batch * nzt * nf * (tz / 2 + 2) * P.dims[1] * P.dims[2] * sizeof(float);
}

hipError_t launch_fused_assemble(modil_ctx *c, void *g, const AdamHost *ad, const void *th_in,
                                 void *th_out, void *m, void *v) {
  const modil_problem &P = c->prob;
  if (P.dtype != MODIL_F32 || P.n_levels < 2) return hipErrorInvalidValue;
  AssembleArgs<float> A{};
  int ox, oy, ntx, nty;
  ns3d_tiles(P, A.tz, A.nzt, ntx, nty, ox, oy);
  A.zsum = (const float *)c->cpart;
  A.g = (float *)g;
  A.batch = P.batch;
  A.nf = c->lay.n_fields;
  A.ncz = P.dims[0] / 2;
  A.ncy = P.dims[1] / 2;
  A.ncx = P.dims[2] / 2;
  A.off1 = (int)c->lay.level_offset[1];
  A.stride1 = (int)c->lay.level_stride[1];
  if (ad) {
    A.adam.th_in = (const float *)th_in; A.adam.th_out = (float *)th_out;
    A.adam.m = (float *)m; A.adam.v = (float *)v;
    A.adam.b1 = float(ad->b1); A.adam.b2 = float(ad->b2); A.adam.step = float(ad->step);
    A.adam.isb2 = float(ad->isb2); A.adam.eps = float(ad->eps);
  }
  const dim3 grid((unsigned)((A.ncx + AS_X - 1) / AS_X), (unsigned)((A.ncy + AS_Y - 1) / AS_Y),
                  (unsigned)(A.ncz * A.nf * A.batch)),
      block(256);
  if (grid.x > 65535 || grid.y > 65535 || grid.z > 65535) return hipErrorInvalidConfiguration;
  if (ad) fused_assemble_kernel<float, true><<<grid, block, 0, c->stream>>>(A);
  else fused_assemble_kernel<float, false><<<grid, block, 0, c->stream>>>(A);
  return hipGetLastError();
}

// FP32 only: the problem's FP64 channel flow runs on the generic engine
hipError_t launch_ns3d_fused(modil_ctx *c, const void *theta, void *g, const AdamHost *adam,
                             void *th_out, void *m, void *v) {
  if (c->prob.dtype != MODIL_F32) return hipErrorInvalidValue;
  return fused_t<float>(c, theta, g, adam, th_out, m, v);
}

}  // namespace modil
