// Residual operators of the mODIL problems and their local adjoints.
//
// Every operator is written for one cell j of the finest grid, in terms of
// the 7-point star of field values around it (slots below).  The values
// outside the grid are ghosts given by affine rules of the cell itself and
// of its opposite neighbour (value = b2 + c0 * u(j) + c1 * u(j - offset)),
// so that the adjoint of the ghost map can be folded back onto real cells by
// the stencil engine.
//
//   eval(): residual r_e of every equation e at j, its loss weight wv_e
//           (term weight times cell measure; 0 where the equation does not
//           apply) and the loss term it belongs to.
//   vjp():  s[f][slot] = d(sum_e a_e r_e) / d U[f][slot] for given seeds a_e.
//
// Discretisations (paper sections; readings where the paper is silent are
// the same as in the reference implementation used by the tests):
//   Poisson   Section 3.1: 3-point Laplacian per axis, u = 0 on the walls by
//             quadratic extrapolation, ghost = -2 u_0 + u_1 / 3.
//   Burgers   Section 3.2: implicit (u^n - u^{n-1})/dt plus the difference of
//             first-order upwind fluxes of u^2/2 (Murman-Roe form) on the
//             inner points; smoothing (u_{i+1} - u_i)/dx and
//             (u^{n+1} - u^n)/dt on inner faces.
//   Heat      Section 3.4 scheme with k = softplus(q(x)) and face
//             conductivity the mean of the adjacent cells; wall value by
//             quadratic extrapolation (15 u_0 - 10 u_1 + 3 u_2) / 8.
//   NS        Sections 3.3 and 3.5: collocated central differences,
//             continuity with pressure stabilisation tau_a = tau_coef h_a,
//             Brinkman penalisation (1 - chi)(...) + lambda chi u.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace modil {

enum Slot { S_C = 0, S_ZM = 1, S_ZP = 2, S_YM = 3, S_YP = 4, S_XM = 5, S_XP = 6 };
__host__ __device__ inline int slot_m(int a) { return 1 + 2 * a; }
__host__ __device__ inline int slot_p(int a) { return 2 + 2 * a; }

struct GhostRule {
  double b2, c0, c1;  // ghost = b2 + c0 * centre + c1 * opposite neighbour
};

template <typename T>
__device__ inline T sgn0(T x) {  // sign with sgn(0) = 0
  return x > T(0) ? T(1) : (x < T(0) ? T(-1) : T(0));
}

// ------------------------------------------------------------------ Poisson
struct OpPoisson {
  static constexpr int NF = 1, NE = 1;
  static constexpr bool kForcePdeOnly = false;
  __device__ static bool needs_nb(int) { return true; }
  __device__ static GhostRule ghost(const OpParams &, int, int, int) {
    return GhostRule{0.0, -2.0, 1.0 / 3.0};
  }
  template <typename T>
  __device__ static void eval(const OpParams &p, const int *, int, const T (&U)[NF][7],
                              T, T *r, T *wv, int *term) {
    T acc = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (a < 3 - p.ndim) continue;
      T ih2 = T(1.0 / (p.h[a] * p.h[a]));
      acc += (U[0][slot_p(a)] - T(2) * U[0][S_C] + U[0][slot_m(a)]) * ih2;
    }
    r[0] = acc;
    wv[0] = T(p.w_pde * p.V);
    term[0] = MODIL_TERM_PDE;
  }
  template <typename T>
  __device__ static void vjp(const OpParams &p, const int *, int, const T (&)[NF][7],
                             T, const T *a, T (&s)[NF][7]) {
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      if (ax < 3 - p.ndim) continue;
      T ih2 = T(1.0 / (p.h[ax] * p.h[ax]));
      s[0][slot_p(ax)] += a[0] * ih2;
      s[0][slot_m(ax)] += a[0] * ih2;
      s[0][S_C] -= T(2) * a[0] * ih2;
    }
  }
};

// Node-based Poisson (Section 3.1): values at the nodes; the zero Dirichlet
// condition is imposed on the boundary nodes directly, so a boundary node
// carries no equation and enters its interior neighbours' stencils as zero
// (whatever the prolonged field holds there), and the gradient there is zero.
// Interior nodes carry the finite-difference Laplacian minus the forcing.
struct OpPoissonNode {
  static constexpr int NF = 1, NE = 1;
  static constexpr bool kForcePdeOnly = true;
  __device__ static bool needs_nb(int) { return true; }
  __device__ static GhostRule ghost(const OpParams &, int, int, int) {
    return GhostRule{0.0, 0.0, 0.0};  // never used by an equation
  }
  __device__ static bool on_boundary(const OpParams &p, const int *j) {
    bool b = false;
    for (int a = 3 - p.ndim; a < 3; ++a) b |= j[a] == 0 || j[a] == p.n[a] - 1;
    return b;
  }
  template <typename T>
  __device__ static void eval(const OpParams &p, const int *j, int, const T (&U)[NF][7], T, T *r,
                              T *wv, int *term) {
    term[0] = MODIL_TERM_PDE;
    if (on_boundary(p, j)) {
      r[0] = T(0);
      wv[0] = T(0);
      return;
    }
    T acc = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (a < 3 - p.ndim) continue;
      const T ih2 = T(1.0 / (p.h[a] * p.h[a]));
      const T um = j[a] - 1 == 0 ? T(0) : U[0][slot_m(a)];
      const T up = j[a] + 1 == p.n[a] - 1 ? T(0) : U[0][slot_p(a)];
      acc += (up - T(2) * U[0][S_C] + um) * ih2;
    }
    r[0] = acc;
    wv[0] = T(p.w_pde * p.V);
  }
  template <typename T>
  __device__ static void vjp(const OpParams &p, const int *j, int, const T (&)[NF][7], T,
                             const T *a, T (&s)[NF][7]) {
    if (on_boundary(p, j)) return;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      if (ax < 3 - p.ndim) continue;
      const T ih2 = T(1.0 / (p.h[ax] * p.h[ax]));
      if (j[ax] + 1 != p.n[ax] - 1) s[0][slot_p(ax)] += a[0] * ih2;
      if (j[ax] - 1 != 0) s[0][slot_m(ax)] += a[0] * ih2;
      s[0][S_C] -= T(2) * a[0] * ih2;
    }
  }
};

// ------------------------------------------------------------------ Burgers
// grid axes: 1 = t (rows), 2 = x
struct OpBurgers {
  static constexpr int NF = 1, NE = 3;
  static constexpr bool kForcePdeOnly = false;
  __device__ static bool needs_nb(int) { return true; }
  __device__ static GhostRule ghost(const OpParams &, int, int, int) {
    return GhostRule{0.0, 0.0, 0.0};  // no equation reaches outside the grid
  }
  template <typename T>
  __device__ static T flux(T a, T b) {
    return T(0.25) * (a * a + b * b) - T(0.5) * fabs(T(0.5) * (a + b)) * (b - a);
  }
  template <typename T>
  __device__ static void dflux(T a, T b, T &da, T &db) {
    T m = T(0.5) * (a + b);
    T am = fabs(m), sm = sgn0(m);
    da = T(0.5) * a - T(0.25) * sm * (b - a) + T(0.5) * am;
    db = T(0.5) * b - T(0.25) * sm * (b - a) - T(0.5) * am;
  }
  template <typename T>
  __device__ static void eval(const OpParams &p, const int *i, int, const T (&U)[NF][7],
                              T, T *r, T *wv, int *term) {
    const int nt = p.n[1], nx = p.n[2], it = i[1], ix = i[2];
    const T idt = T(1.0 / p.h[1]), idx = T(1.0 / p.h[2]);
    const T c = U[0][S_C];
    const bool pde = it >= 1 && ix >= 1 && ix <= nx - 2;
    r[0] = pde ? (c - U[0][S_YM]) * idt + (flux(c, U[0][S_XP]) - flux(U[0][S_XM], c)) * idx : T(0);
    wv[0] = pde ? T(p.w_pde * p.V) : T(0);
    term[0] = MODIL_TERM_PDE;
    const bool rx = ix <= nx - 2;
    r[1] = rx ? (U[0][S_XP] - c) * idx : T(0);
    wv[1] = rx ? T(p.w_reg * p.V) : T(0);
    term[1] = MODIL_TERM_REG;
    const bool rt = it <= nt - 2;
    r[2] = rt ? (U[0][S_YP] - c) * idt : T(0);
    wv[2] = rt ? T(p.w_reg * p.V) : T(0);
    term[2] = MODIL_TERM_REG;
  }
  template <typename T>
  __device__ static void vjp(const OpParams &p, const int *, int, const T (&U)[NF][7],
                             T, const T *a, T (&s)[NF][7]) {
    const T idt = T(1.0 / p.h[1]), idx = T(1.0 / p.h[2]);
    const T c = U[0][S_C];
    T da1, db1, da2, db2;
    dflux(c, U[0][S_XP], da1, db1);       // F_{i+1/2}(c, right)
    dflux(U[0][S_XM], c, da2, db2);       // F_{i-1/2}(left, c)
    s[0][S_C] += a[0] * (idt + (da1 - db2) * idx);
    s[0][S_YM] -= a[0] * idt;
    s[0][S_XP] += a[0] * db1 * idx;
    s[0][S_XM] -= a[0] * da2 * idx;
    s[0][S_XP] += a[1] * idx;
    s[0][S_C] -= a[1] * idx;
    s[0][S_YP] += a[2] * idt;
    s[0][S_C] -= a[2] * idt;
  }
};

// --------------------------------------------------------------------- heat
// grid axes: 1 = t, 2 = x; field 0 = u [t][x], field 1 = q [x]
struct OpHeat {
  static constexpr int NF = 2, NE = 3;
  static constexpr bool kForcePdeOnly = false;
  __device__ static bool needs_nb(int) { return true; }
  __device__ static GhostRule ghost(const OpParams &, int, int, int) {
    return GhostRule{0.0, 0.0, 0.0};  // no equation reaches outside the grid
  }
  template <typename T>
  __device__ static T softplus(T q) {
    return q > T(0) ? q + log1p(exp(-q)) : log1p(exp(q));
  }
  template <typename T>
  __device__ static T sigmoid(T q) {
    return q >= T(0) ? T(1) / (T(1) + exp(-q)) : exp(q) / (T(1) + exp(q));
  }
  template <typename T>
  __device__ static void eval(const OpParams &p, const int *i, int, const T (&U)[NF][7],
                              T, T *r, T *wv, int *term) {
    const int nx = p.n[2], it = i[1], ix = i[2];
    const T idt = T(1.0 / p.h[1]), idx2 = T(1.0 / (p.h[2] * p.h[2]));
    const T c = U[0][S_C];
    const bool pde = it >= 1 && ix >= 1 && ix <= nx - 2;
    if (pde) {
      const T k0 = softplus(U[1][S_C]), kp = softplus(U[1][S_XP]), km = softplus(U[1][S_XM]);
      const T Kp = T(0.5) * (k0 + kp), Km = T(0.5) * (k0 + km);
      r[0] = (c - U[0][S_YM]) * idt - (Kp * (U[0][S_XP] - c) - Km * (c - U[0][S_XM])) * idx2;
    } else {
      r[0] = T(0);
    }
    wv[0] = pde ? T(p.w_pde * p.V) : T(0);
    term[0] = MODIL_TERM_PDE;
    const bool bl = it >= 1 && ix == 1;
    r[1] = bl ? (T(15) * U[0][S_XM] - T(10) * c + T(3) * U[0][S_XP]) * T(0.125) : T(0);
    wv[1] = bl ? T(p.w_bc * p.h[1]) : T(0);
    term[1] = MODIL_TERM_BC;
    const bool br = it >= 1 && ix == nx - 2;
    r[2] = br ? (T(15) * U[0][S_XP] - T(10) * c + T(3) * U[0][S_XM]) * T(0.125) : T(0);
    wv[2] = br ? T(p.w_bc * p.h[1]) : T(0);
    term[2] = MODIL_TERM_BC;
  }
  template <typename T>
  __device__ static void vjp(const OpParams &p, const int *, int, const T (&U)[NF][7],
                             T, const T *a, T (&s)[NF][7]) {
    const T idt = T(1.0 / p.h[1]), idx2 = T(1.0 / (p.h[2] * p.h[2]));
    const T c = U[0][S_C];
    if (a[0] != T(0)) {
      const T q0 = U[1][S_C], qp = U[1][S_XP], qm = U[1][S_XM];
      const T k0 = softplus(q0), kp = softplus(qp), km = softplus(qm);
      const T Kp = T(0.5) * (k0 + kp), Km = T(0.5) * (k0 + km);
      s[0][S_C] += a[0] * (idt + (Kp + Km) * idx2);
      s[0][S_YM] -= a[0] * idt;
      s[0][S_XP] -= a[0] * Kp * idx2;
      s[0][S_XM] -= a[0] * Km * idx2;
      const T dKp = -a[0] * (U[0][S_XP] - c) * idx2;   // d r / d Kp times a
      const T dKm = a[0] * (c - U[0][S_XM]) * idx2;    // d r / d Km times a
      s[1][S_C] += T(0.5) * (dKp + dKm) * sigmoid(q0);
      s[1][S_XP] += T(0.5) * dKp * sigmoid(qp);
      s[1][S_XM] += T(0.5) * dKm * sigmoid(qm);
    }
    s[0][S_XM] += a[1] * T(15.0 / 8.0);
    s[0][S_C] -= a[1] * T(10.0 / 8.0);
    s[0][S_XP] += a[1] * T(3.0 / 8.0);
    s[0][S_XP] += a[2] * T(15.0 / 8.0);
    s[0][S_C] -= a[2] * T(10.0 / 8.0);
    s[0][S_XM] += a[2] * T(3.0 / 8.0);
  }
};

// ------------------------------------------------------------ Navier-Stokes
// D = 3: channel [z][y][x], fields u (x), v (y), w (z), p, [chihat];
// D = 2: cavity [y][x], fields u (x), v (y), p.
// Velocity component c points along grid axis 2 - c.
// Equations: 0 continuity, 1 + c momentum of component c.
//
// The formulas are split into point functions shared by the generic stencil
// engine and the fused channel-flow kernel:
//   ns_residual     residuals at a cell from its star of (u.., p) and chi
//   ns_face_sens    sensitivity of sum_e a_e r_e(j) to the neighbour value of
//                   every (velocity, p) field across one face of j; it
//                   depends only on the seeds and centre values at j
//   ns_centre_sens  sensitivity to the centre values of j (needs the star)

template <int D>
__host__ __device__ inline double ns_nu(const OpParams &p, int inst) {
  const double re = p.inst_re ? p.inst_re[inst] : p.re;
  return (D == 3 ? p.diam : 1.0) / re;
}

// stencil coefficients in the working precision, computed once per thread
template <typename T>
struct NSCoef {
  T i2h[3];   // 1 / (2 h_a)
  T ih2[3];   // 1 / h_a^2
  T tauh[3];  // tau_coef / h_a (stabilisation tau_a / h_a^2 with tau_a = tau_coef h_a)
  T nu, lam, ssum, tsum;
};

template <int D, typename T>
__device__ inline NSCoef<T> ns_coef(const OpParams &p, int inst) {
  NSCoef<T> k;
  for (int a = 0; a < 3; ++a) {
    k.i2h[a] = T(0.5 / p.h[a]);
    k.ih2[a] = T(1.0 / (p.h[a] * p.h[a]));
    k.tauh[a] = T(p.tau_coef / p.h[a]);
  }
  k.nu = T(ns_nu<D>(p, inst));
  k.lam = T(p.lam);
  k.ssum = T(0);
  k.tsum = T(0);
  for (int a = 3 - D; a < 3; ++a) {
    k.ssum += k.ih2[a];
    k.tsum += k.tauh[a];
  }
  return k;
}

template <int D, typename T>
struct NSLocal {
  T du[D][D];  // du[c][k]: derivative of component c along the axis of component k
  T lap[D];
  T dp[D];
  T stab;
  T body[D];  // convection + pressure gradient - viscous term
};

// U: star values of the velocity components and p (fields 0..D), ghosts applied
template <int D, typename T, int NFU>
__device__ inline void ns_local(const NSCoef<T> &K, const T (&U)[NFU][7], NSLocal<D, T> &L) {
  for (int c = 0; c < D; ++c) {
    L.lap[c] = T(0);
    for (int k = 0; k < D; ++k) {
      const int ax = 2 - k;
      L.du[c][k] = (U[c][slot_p(ax)] - U[c][slot_m(ax)]) * K.i2h[ax];
      L.lap[c] += (U[c][slot_p(ax)] - T(2) * U[c][S_C] + U[c][slot_m(ax)]) * K.ih2[ax];
    }
  }
  L.stab = T(0);
  for (int k = 0; k < D; ++k) {
    const int ax = 2 - k;
    L.dp[k] = (U[D][slot_p(ax)] - U[D][slot_m(ax)]) * K.i2h[ax];
    L.stab += (U[D][slot_p(ax)] - T(2) * U[D][S_C] + U[D][slot_m(ax)]) * K.tauh[ax];
  }
  for (int c = 0; c < D; ++c) {
    T b = L.dp[c] - K.nu * L.lap[c];
    for (int k = 0; k < D; ++k) b += U[k][S_C] * L.du[c][k];
    L.body[c] = b;
  }
}

template <int D, bool HAS_CHI, typename T>
__device__ inline void ns_residual(const NSCoef<T> &K, const NSLocal<D, T> &L, const T *uc, T chi,
                                   T *r) {
  T cont = T(0);
  for (int c = 0; c < D; ++c) cont += L.du[c][c];
  r[0] = cont - L.stab;
  for (int c = 0; c < D; ++c)
    r[1 + c] = HAS_CHI ? (T(1) - chi) * L.body[c] + K.lam * chi * uc[c] : L.body[c];
}

// s[f], f = 0..D (velocity components, p): d(sum_e a_e r_e(j)) / d U_f(j + side * e_axis)
template <int D, bool HAS_CHI, typename T>
__device__ inline void ns_face_sens(const NSCoef<T> &K, int axis, int side, const T *a,
                                    const T *uc, T chi, T *s) {
  const T i2h = K.i2h[axis], ih2 = K.ih2[axis];
  const T sg = side > 0 ? T(1) : T(-1);
  const int kc = 2 - axis;  // component along this axis
  const T omc = HAS_CHI ? T(1) - chi : T(1);
  for (int c = 0; c < D; ++c) {
    const T A = a[1 + c] * omc;
    T v = A * (sg * uc[kc] * i2h - K.nu * ih2);
    if (c == kc) v += sg * a[0] * i2h;
    s[c] = v;
  }
  s[D] = -a[0] * K.tauh[axis] + sg * a[1 + kc] * omc * i2h;
}

// s[f], f = 0..D: sensitivity to the centre values; dchi = d(sum a r)/d chi
template <int D, bool HAS_CHI, typename T>
__device__ inline void ns_centre_sens(const NSCoef<T> &K, const NSLocal<D, T> &L, const T *a,
                                      const T *uc, T chi, T *s, T &dchi) {
  const T omc = HAS_CHI ? T(1) - chi : T(1);
  for (int f = 0; f < D; ++f) {
    T v = T(0);
    for (int c = 0; c < D; ++c) v += a[1 + c] * omc * L.du[c][f];
    v += T(2) * a[1 + f] * omc * K.nu * K.ssum;
    if (HAS_CHI) v += a[1 + f] * K.lam * chi;
    s[f] = v;
  }
  s[D] = T(2) * a[0] * K.tsum;
  dchi = T(0);
  if (HAS_CHI)
    for (int c = 0; c < D; ++c) dchi += a[1 + c] * (K.lam * uc[c] - L.body[c]);
}

template <typename T>
__device__ inline T sigmoid_stable(T z) {
  return z >= T(0) ? T(1) / (T(1) + exp(-z)) : exp(z) / (T(1) + exp(z));
}
// FP32: the hardware exponential and reciprocal (a few ulp, far inside the
// FP32 tolerance) instead of the correctly rounded library calls
template <>
__device__ inline float sigmoid_stable<float>(float z) {
  const float e = __expf(-fabsf(z));  // in (0, 1]
  const float r = __builtin_amdgcn_rcpf(1.0f + e);
  return z >= 0.0f ? r : e * r;
}

// Ghost rules of the channel (D = 3) and of the cavity (D = 2) for (velocity, p).
template <int D>
__host__ __device__ inline GhostRule ns_ghost(const OpParams &p, int f, int axis, int side) {
  const int P = D;
  if (D == 3) {
    if (axis == 2) {                      // inlet (side 0) / outlet (side 1)
      if (side == 0) {
        if (f == P) return GhostRule{0.0, 1.0, 0.0};              // dp/dn = 0
        return GhostRule{f == 0 ? 2.0 * p.u_ref : 0.0, -1.0, 0.0};  // u = (U, 0, 0)
      }
      if (f == P) return GhostRule{0.0, -1.0, 0.0};               // p = 0
      return GhostRule{0.0, 1.0, 0.0};                              // du/dn = 0
    }
    // free-slip walls: normal component zero, the rest Neumann
    const int normal = 2 - axis;
    if (f == normal) return GhostRule{0.0, -1.0, 0.0};
    return GhostRule{0.0, 1.0, 0.0};
  }
  // cavity: no-slip walls, lid (axis 1, side 1) moves with u = u_ref
  if (f == P) return GhostRule{0.0, 1.0, 0.0};
  if (axis == 1 && side == 1 && f == 0) return GhostRule{2.0 * p.u_ref, -1.0, 0.0};
  return GhostRule{0.0, -1.0, 0.0};
}

// CHI: 0 no body, 1 fixed chi array, 2 unknown chihat field.
template <int D, int CHI>
struct OpNS {
  static constexpr bool kForcePdeOnly = false;
  static constexpr int NF = D + 1 + (CHI == 2 ? 1 : 0);
  static constexpr int NE = D + 1;
  static constexpr int P = D;  // pressure field index

  __device__ static bool needs_nb(int f) { return f <= D; }
  __device__ static GhostRule ghost(const OpParams &p, int f, int axis, int side) {
    if (f > D) return GhostRule{0.0, 0.0, 0.0};
    return ns_ghost<D>(p, f, axis, side);
  }

  template <typename T>
  __device__ static T chi_of(const OpParams &p, const T (&U)[NF][7], T chi_fixed) {
    if (CHI == 1) return chi_fixed;
    if (CHI == 2) return sigmoid_stable(U[NF - 1][S_C] - T(p.chi_shift));
    return T(0);
  }

  template <typename T>
  __device__ static void eval(const OpParams &p, const int *, int inst, const T (&U)[NF][7],
                              T chi_fixed, T *r, T *wv, int *term) {
    const NSCoef<T> K = ns_coef<D, T>(p, inst);
    NSLocal<D, T> L;
    ns_local<D>(K, U, L);
    T uc[D];
    for (int c = 0; c < D; ++c) uc[c] = U[c][S_C];
    ns_residual<D, CHI != 0>(K, L, uc, chi_of(p, U, chi_fixed), r);
    for (int e = 0; e < NE; ++e) {
      wv[e] = T(p.w_pde * p.V);
      term[e] = MODIL_TERM_PDE;
    }
  }

  template <typename T>
  __device__ static void vjp(const OpParams &p, const int *, int inst, const T (&U)[NF][7],
                             T chi_fixed, const T *a, T (&s)[NF][7]) {
    const NSCoef<T> K = ns_coef<D, T>(p, inst);
    NSLocal<D, T> L;
    ns_local<D>(K, U, L);
    T uc[D];
    for (int c = 0; c < D; ++c) uc[c] = U[c][S_C];
    const T chi = chi_of(p, U, chi_fixed);
    T fs[D + 1];
    for (int k = 0; k < D; ++k) {
      const int ax = 2 - k;
      ns_face_sens<D, CHI != 0>(K, ax, 1, a, uc, chi, fs);
      for (int f = 0; f <= D; ++f) s[f][slot_p(ax)] += fs[f];
      ns_face_sens<D, CHI != 0>(K, ax, -1, a, uc, chi, fs);
      for (int f = 0; f <= D; ++f) s[f][slot_m(ax)] += fs[f];
    }
    T dchi;
    ns_centre_sens<D, CHI != 0>(K, L, a, uc, chi, fs, dchi);
    for (int f = 0; f <= D; ++f) s[f][S_C] += fs[f];
    if (CHI == 2) s[NF - 1][S_C] += dchi * chi * (T(1) - chi);
  }
};

// Node-based lid-driven cavity (Sections 2.2, 3.3): values at the nodes
// x_i = i h.  The no-slip condition is imposed on the wall nodes: their
// velocity is zero, except u = u_ref on the lid (axis 1, last row), whatever
// the prolonged field holds there.  The wall pressure equals that of the
// interior node next to it across the wall (zero normal derivative); for an
// interior node that neighbour is the node itself.  Wall nodes carry no
// equation; interior nodes carry the equations of OpNS<2, 0> evaluated on the
// star with these substitutions, so the adjoint drops the velocity wall slots
// and moves the pressure wall slots onto the centre.
struct OpCavityNode {
  using Base = OpNS<2, 0>;
  static constexpr bool kForcePdeOnly = false;
  static constexpr int NF = 3, NE = 3;

  __device__ static bool needs_nb(int) { return true; }
  __device__ static GhostRule ghost(const OpParams &, int, int, int) {
    return GhostRule{0.0, 0.0, 0.0};  // never used by an equation
  }
  __device__ static bool on_boundary(const OpParams &p, const int *j) {
    return j[1] == 0 || j[1] == p.n[1] - 1 || j[2] == 0 || j[2] == p.n[2] - 1;
  }
  // bit (2 a + side) set when the star's neighbour along axis a (1, 2) on that side is a wall node
  __device__ static int wall_mask(const OpParams &p, const int *j) {
    int m = 0;
    for (int a = 1; a < 3; ++a) {
      if (j[a] - 1 == 0) m |= 1 << (2 * a);
      if (j[a] + 1 == p.n[a] - 1) m |= 1 << (2 * a + 1);
    }
    return m;
  }
  template <typename T>
  __device__ static void impose(const OpParams &p, int m, const T (&U)[NF][7], T (&W)[NF][7]) {
    for (int f = 0; f < NF; ++f)
      for (int k = 0; k < 7; ++k) W[f][k] = U[f][k];
    for (int a = 1; a < 3; ++a)
      for (int side = 0; side < 2; ++side) {
        if (!(m >> (2 * a + side) & 1)) continue;
        const int k = side ? slot_p(a) : slot_m(a);
        W[0][k] = (a == 1 && side == 1) ? T(p.u_ref) : T(0);
        W[1][k] = T(0);
        W[2][k] = U[2][S_C];
      }
  }
  template <typename T>
  __device__ static void eval(const OpParams &p, const int *j, int inst, const T (&U)[NF][7],
                              T chi_fixed, T *r, T *wv, int *term) {
    if (on_boundary(p, j)) {
      for (int e = 0; e < NE; ++e) {
        r[e] = T(0);
        wv[e] = T(0);
        term[e] = MODIL_TERM_PDE;
      }
      return;
    }
    T W[NF][7];
    impose(p, wall_mask(p, j), U, W);
    Base::eval(p, j, inst, W, chi_fixed, r, wv, term);
  }
  template <typename T>
  __device__ static void vjp(const OpParams &p, const int *j, int inst, const T (&U)[NF][7],
                             T chi_fixed, const T *a, T (&s)[NF][7]) {
    if (on_boundary(p, j)) return;
    const int m = wall_mask(p, j);
    T W[NF][7], t[NF][7];
    impose(p, m, U, W);
    for (int f = 0; f < NF; ++f)
      for (int k = 0; k < 7; ++k) t[f][k] = T(0);
    Base::vjp(p, j, inst, W, chi_fixed, a, t);
    for (int ax = 1; ax < 3; ++ax)
      for (int side = 0; side < 2; ++side) {
        if (!(m >> (2 * ax + side) & 1)) continue;
        const int k = side ? slot_p(ax) : slot_m(ax);
        t[0][k] = T(0);
        t[1][k] = T(0);
        t[2][S_C] += t[2][k];
        t[2][k] = T(0);
      }
    for (int f = 0; f < NF; ++f)
      for (int k = 0; k < 7; ++k) s[f][k] += t[f][k];
  }
};

// Node-based channel flow past a body (Sections 2.2, 3.5): values at the
// nodes x_i = i h.  Boundary nodes carry no equation; the boundary conditions
// replace their values, whatever the prolonged field holds there:
//   inlet (axis 2, side 0)   u = (u_ref, 0, 0), p copied from the neighbouring
//                            interior node,
//   outlet (axis 2, side 1)  p = 0, the velocity copied,
//   free-slip walls (axes 0, 1)  the normal velocity component is zero, the
//                            other components and p are copied.
// For the interior node whose star reaches the boundary node, the copied
// neighbour is that node itself.  Nodes on an edge or a corner of the box lie
// in no interior star.  Interior nodes carry the equations of OpNS<3, CHI> on
// the star with these substitutions, so the adjoint drops the imposed slots
// and moves the copied slots onto the centre.
template <int CHI>
struct OpChannelNode {
  using Base = OpNS<3, CHI>;
  static constexpr bool kForcePdeOnly = false;
  static constexpr int NF = Base::NF, NE = Base::NE;

  __device__ static bool needs_nb(int f) { return f <= 3; }
  __device__ static GhostRule ghost(const OpParams &, int, int, int) {
    return GhostRule{0.0, 0.0, 0.0};  // never used by an equation
  }
  __device__ static bool on_boundary(const OpParams &p, const int *j) {
    bool b = false;
    for (int a = 0; a < 3; ++a) b = b || j[a] == 0 || j[a] == p.n[a] - 1;
    return b;
  }
  // bit (2 a + side) set when the star's neighbour along axis a on that side is a boundary node
  __device__ static int wall_mask(const OpParams &p, const int *j) {
    int m = 0;
    for (int a = 0; a < 3; ++a) {
      if (j[a] - 1 == 0) m |= 1 << (2 * a);
      if (j[a] + 1 == p.n[a] - 1) m |= 1 << (2 * a + 1);
    }
    return m;
  }
  // field f (u, v, w, p) on the boundary (axis a, side): imposed (true, value) or copied
  __device__ static bool imposed(const OpParams &p, int f, int a, int side, double &val) {
    val = 0.0;
    if (a == 2) {
      if (side == 0) {
        if (f == 0) val = p.u_ref;
        return f < 3;
      }
      return f == 3;
    }
    return f == 2 - a;
  }
  template <typename T>
  __device__ static void impose(const OpParams &p, int m, const T (&U)[NF][7], T (&W)[NF][7]) {
    for (int f = 0; f < NF; ++f)
      for (int k = 0; k < 7; ++k) W[f][k] = U[f][k];
    for (int a = 0; a < 3; ++a)
      for (int side = 0; side < 2; ++side) {
        if (!(m >> (2 * a + side) & 1)) continue;
        const int k = side ? slot_p(a) : slot_m(a);
        for (int f = 0; f < 4; ++f) {
          double val;
          W[f][k] = imposed(p, f, a, side, val) ? T(val) : U[f][S_C];
        }
      }
  }
  template <typename T>
  __device__ static void eval(const OpParams &p, const int *j, int inst, const T (&U)[NF][7],
                              T chi_fixed, T *r, T *wv, int *term) {
    if (on_boundary(p, j)) {
      for (int e = 0; e < NE; ++e) {
        r[e] = T(0);
        wv[e] = T(0);
        term[e] = MODIL_TERM_PDE;
      }
      return;
    }
    T W[NF][7];
    impose(p, wall_mask(p, j), U, W);
    Base::eval(p, j, inst, W, chi_fixed, r, wv, term);
  }
  template <typename T>
  __device__ static void vjp(const OpParams &p, const int *j, int inst, const T (&U)[NF][7],
                             T chi_fixed, const T *a, T (&s)[NF][7]) {
    if (on_boundary(p, j)) return;
    const int m = wall_mask(p, j);
    T W[NF][7], t[NF][7];
    impose(p, m, U, W);
    for (int f = 0; f < NF; ++f)
      for (int k = 0; k < 7; ++k) t[f][k] = T(0);
    Base::vjp(p, j, inst, W, chi_fixed, a, t);
    for (int ax = 0; ax < 3; ++ax)
      for (int side = 0; side < 2; ++side) {
        if (!(m >> (2 * ax + side) & 1)) continue;
        const int k = side ? slot_p(ax) : slot_m(ax);
        for (int f = 0; f < 4; ++f) {
          double val;
          if (!imposed(p, f, ax, side, val)) t[f][S_C] += t[f][k];
          t[f][k] = T(0);
        }
      }
    for (int f = 0; f < NF; ++f)
      for (int k = 0; k < 7; ++k) s[f][k] += t[f][k];
  }
};

}  // namespace modil
