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
  __device__ static bool needs_nb(int) { return true; }
  __device__ static GhostRule ghost(const OpParams &, int, int, int) {
    return GhostRule{0.0, -2.0, 1.0 / 3.0};
  }
  template <typename T>
  __device__ static void eval(const OpParams &p, const int *, int, const T (&U)[NF][7],
                              T, T *r, T *wv, int *term) {
    T acc = 0;
    for (int a = 3 - p.ndim; a < 3; ++a) {
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
    for (int ax = 3 - p.ndim; ax < 3; ++ax) {
      T ih2 = T(1.0 / (p.h[ax] * p.h[ax]));
      s[0][slot_p(ax)] += a[0] * ih2;
      s[0][slot_m(ax)] += a[0] * ih2;
      s[0][S_C] -= T(2) * a[0] * ih2;
    }
  }
};

// ------------------------------------------------------------------ Burgers
// grid axes: 1 = t (rows), 2 = x
struct OpBurgers {
  static constexpr int NF = 1, NE = 3;
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
// CHI: 0 no body, 1 fixed chi array, 2 unknown chihat field.
template <int D, int CHI>
struct OpNS {
  static constexpr int NF = D + 1 + (CHI == 2 ? 1 : 0);
  static constexpr int NE = D + 1;
  static constexpr int P = D;  // pressure field index

  __device__ static bool needs_nb(int f) { return f <= D; }
  __device__ static GhostRule ghost(const OpParams &p, int f, int axis, int side) {
    if (f > D) return GhostRule{0.0, 0.0, 0.0};
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

  template <typename T>
  struct Local {
    T du[D][D];  // du[c][k]: derivative of component c along the axis of component k
    T lap[D];
    T dp[D];
    T stab;
  };

  template <typename T>
  __device__ static void locals(const OpParams &p, const T (&U)[NF][7], Local<T> &L) {
    for (int c = 0; c < D; ++c) {
      L.lap[c] = T(0);
      for (int k = 0; k < D; ++k) {
        const int ax = 2 - k;
        const T i2h = T(0.5 / p.h[ax]), ih2 = T(1.0 / (p.h[ax] * p.h[ax]));
        L.du[c][k] = (U[c][slot_p(ax)] - U[c][slot_m(ax)]) * i2h;
        L.lap[c] += (U[c][slot_p(ax)] - T(2) * U[c][S_C] + U[c][slot_m(ax)]) * ih2;
      }
    }
    L.stab = T(0);
    for (int k = 0; k < D; ++k) {
      const int ax = 2 - k;
      L.dp[k] = (U[P][slot_p(ax)] - U[P][slot_m(ax)]) * T(0.5 / p.h[ax]);
      L.stab += (U[P][slot_p(ax)] - T(2) * U[P][S_C] + U[P][slot_m(ax)]) * T(p.tau_coef / p.h[ax]);
    }
  }

  template <typename T>
  __device__ static T nu_of(const OpParams &p, int inst) {
    const double re = p.inst_re ? p.inst_re[inst] : p.re;
    return T((D == 3 ? p.diam : 1.0) / re);
  }

  template <typename T>
  __device__ static T chi_of(const OpParams &p, const T (&U)[NF][7], T chi_fixed) {
    if (CHI == 1) return chi_fixed;
    if (CHI == 2) {
      const T z = U[NF - 1][S_C] - T(p.chi_shift);
      return z >= T(0) ? T(1) / (T(1) + exp(-z)) : exp(z) / (T(1) + exp(z));
    }
    return T(0);
  }

  template <typename T>
  __device__ static void eval(const OpParams &p, const int *, int inst, const T (&U)[NF][7],
                              T chi_fixed, T *r, T *wv, int *term) {
    Local<T> L;
    locals(p, U, L);
    const T nu = nu_of<T>(p, inst);
    T cont = T(0);
    for (int c = 0; c < D; ++c) cont += L.du[c][c];
    r[0] = cont - L.stab;
    const T chi = chi_of(p, U, chi_fixed);
    for (int c = 0; c < D; ++c) {
      T body = L.dp[c] - nu * L.lap[c];
      for (int k = 0; k < D; ++k) body += U[k][S_C] * L.du[c][k];
      r[1 + c] = CHI ? (T(1) - chi) * body + T(p.lam) * chi * U[c][S_C] : body;
    }
    for (int e = 0; e < NE; ++e) {
      wv[e] = T(p.w_pde * p.V);
      term[e] = MODIL_TERM_PDE;
    }
  }

  template <typename T>
  __device__ static void vjp(const OpParams &p, const int *, int inst, const T (&U)[NF][7],
                             T chi_fixed, const T *a, T (&s)[NF][7]) {
    Local<T> L;
    locals(p, U, L);
    const T nu = nu_of<T>(p, inst);
    const T chi = chi_of(p, U, chi_fixed);
    // continuity
    for (int c = 0; c < D; ++c) {
      const int ax = 2 - c;
      const T i2h = T(0.5 / p.h[ax]);
      s[c][slot_p(ax)] += a[0] * i2h;
      s[c][slot_m(ax)] -= a[0] * i2h;
      const T t = a[0] * T(p.tau_coef / p.h[ax]);
      s[P][slot_p(ax)] -= t;
      s[P][slot_m(ax)] -= t;
      s[P][S_C] += T(2) * t;
    }
    // momentum
    for (int c = 0; c < D; ++c) {
      const T A = CHI ? a[1 + c] * (T(1) - chi) : a[1 + c];
      T body = L.dp[c] - nu * L.lap[c];
      for (int k = 0; k < D; ++k) {
        const int ax = 2 - k;
        const T i2h = T(0.5 / p.h[ax]), ih2 = T(1.0 / (p.h[ax] * p.h[ax]));
        body += U[k][S_C] * L.du[c][k];
        s[k][S_C] += A * L.du[c][k];
        const T cv = A * U[k][S_C] * i2h;
        const T vs = A * nu * ih2;
        s[c][slot_p(ax)] += cv - vs;
        s[c][slot_m(ax)] -= cv + vs;
        s[c][S_C] += T(2) * vs;
      }
      const int axc = 2 - c;
      s[P][slot_p(axc)] += A * T(0.5 / p.h[axc]);
      s[P][slot_m(axc)] -= A * T(0.5 / p.h[axc]);
      if (CHI) s[c][S_C] += a[1 + c] * T(p.lam) * chi;
      if (CHI == 2)
        s[NF - 1][S_C] += a[1 + c] * (T(p.lam) * U[c][S_C] - body) * chi * (T(1) - chi);
    }
  }
};

}  // namespace modil
