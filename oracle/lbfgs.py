"""Limited-memory BFGS with a strong-Wolfe line search (test infrastructure only).

The paper minimises the discrete loss with SciPy's L-BFGS-B (Section 2.1;
a history of 50 pairs in the Poisson study of Section 3.1).  Without bounds
that method is limited-memory BFGS.  This module writes the textbook method
out in FP64 (Nocedal & Wright, Numerical Optimization, 2nd ed.):

  direction   d = -H g by the two-loop recursion (their Algorithm 7.4), with
              the initial matrix gamma I, gamma = s^T y / y^T y of the newest
              pair (their eq. 7.20); d = -g while no pair is stored
  step        a line search that brackets a step satisfying the strong Wolfe
              conditions and zooms into the bracket (their Algorithms 3.5 and
              3.6), trial steps by safeguarded cubic interpolation (eq. 3.59)
  memory      the pair s = alpha d, y = g_new - g is stored when s^T y > eps y^T y
              (eps the FP64 unit roundoff); beyond m pairs the oldest is dropped

Readings where the paper is silent (it names the SciPy routine only): the
Wolfe constants c1 = 1e-4, c2 = 0.9; the first trial step is
min(1, 1 / ||d||_2) while no pair is stored and 1 afterwards; the bracketing
phase doubles the step; a cubic trial point outside the middle 80 % of the
bracket is replaced by its midpoint; a line search ends after 20 evaluations
with the best point that satisfies the sufficient-decrease condition, if any.
A direction that is not a descent direction resets the memory.

Vectors are flat numpy arrays; the objective is a callable x -> (f, g).
"""
import math

import numpy as np

EPS = np.finfo(np.float64).eps


def two_loop(g, S, Y):
    """H g for the L-BFGS matrix of the pairs (S[i], Y[i]), oldest first."""
    q = np.array(g, dtype=np.float64, copy=True)
    k = len(S)
    if k == 0:
        return q
    rho = [1.0 / float(np.dot(Y[i], S[i])) for i in range(k)]
    alpha = [0.0] * k
    for i in range(k - 1, -1, -1):
        alpha[i] = rho[i] * float(np.dot(S[i], q))
        q -= alpha[i] * Y[i]
    gamma = float(np.dot(S[-1], Y[-1])) / float(np.dot(Y[-1], Y[-1]))
    r = gamma * q
    for i in range(k):
        beta = rho[i] * float(np.dot(Y[i], r))
        r += (alpha[i] - beta) * S[i]
    return r


def cubic_step(a, fa, da, b, fb, db):
    """Minimiser of the cubic through (a, fa, da) and (b, fb, db), or None."""
    if not all(math.isfinite(v) for v in (a, fa, da, b, fb, db)) or a == b:
        return None
    d1 = da + db - 3.0 * (fa - fb) / (a - b)
    disc = d1 * d1 - da * db
    if disc < 0.0:
        return None
    d2 = math.copysign(math.sqrt(disc), b - a)
    den = db - da + 2.0 * d2
    if den == 0.0:
        return None
    return b - (b - a) * (db + d2 - d1) / den


def _trial(lo, flo, dlo, hi, fhi, dhi):
    lo_b, hi_b = min(lo, hi), max(lo, hi)
    width = hi_b - lo_b
    t = cubic_step(lo, flo, dlo, hi, fhi, dhi)
    if t is None or not (lo_b + 0.1 * width <= t <= hi_b - 0.1 * width):
        t = 0.5 * (lo + hi)
    return t


class LineSearchResult:
    def __init__(self, alpha, f, g, dphi, evals, status):
        self.alpha, self.f, self.g, self.dphi = alpha, f, g, dphi
        self.evals, self.status = evals, status  # status 0: strong Wolfe, 1: decrease only, 2: failed


def line_search(fg, x, d, f0, dphi0, alpha1, c1=1e-4, c2=0.9, max_evals=20):
    """Strong-Wolfe line search along d from x; phi(a) = f(x + a d)."""
    evals = 0
    cache = {}

    def phi(a):
        nonlocal evals
        evals += 1
        f, g = fg(x + a * d)
        dphi = float(np.dot(g, d))
        cache[a] = (f, g, dphi)
        return f, dphi

    def ok_decrease(a, fa):
        return math.isfinite(fa) and fa <= f0 + c1 * a * dphi0

    def finish(a, status):
        f, g, dphi = cache[a]
        return LineSearchResult(a, f, g, dphi, evals, status)

    def zoom(lo, flo, dlo, hi, fhi, dhi):
        while evals < max_evals:
            a = _trial(lo, flo, dlo, hi, fhi, dhi)
            fa, da = phi(a)
            if not ok_decrease(a, fa) or fa >= flo:
                hi, fhi, dhi = a, fa, da
            else:
                if abs(da) <= -c2 * dphi0:
                    return finish(a, 0)
                if da * (hi - lo) >= 0.0:
                    hi, fhi, dhi = lo, flo, dlo
                lo, flo, dlo = a, fa, da
        if lo > 0.0:
            return finish(lo, 1)
        return LineSearchResult(0.0, f0, None, dphi0, evals, 2)

    a_prev, f_prev, d_prev = 0.0, f0, dphi0
    a = alpha1
    first = True
    while evals < max_evals:
        fa, da = phi(a)
        if not ok_decrease(a, fa) or (not first and fa >= f_prev):
            return zoom(a_prev, f_prev, d_prev, a, fa, da)
        if abs(da) <= -c2 * dphi0:
            return finish(a, 0)
        if da >= 0.0:
            return zoom(a, fa, da, a_prev, f_prev, d_prev)
        a_prev, f_prev, d_prev = a, fa, da
        a = 2.0 * a
        first = False
    if a_prev > 0.0:
        return finish(a_prev, 1)
    return LineSearchResult(0.0, f0, None, dphi0, evals, 2)


class LBFGS:
    """State of the iteration: x, f(x), g(x) and the stored pairs (oldest first)."""

    def __init__(self, fg, x0, m=50, c1=1e-4, c2=0.9, max_evals=20):
        self.fg, self.m, self.c1, self.c2, self.max_evals = fg, m, c1, c2, max_evals
        self.x = np.array(x0, dtype=np.float64, copy=True)
        self.f, self.g = fg(self.x)
        self.g = np.asarray(self.g, dtype=np.float64)
        self.evals = 1
        self.S, self.Y = [], []

    def direction(self):
        return -two_loop(self.g, self.S, self.Y)

    def step(self):
        """One iteration; returns the line-search result (alpha 0 if it failed)."""
        d = self.direction()
        dphi0 = float(np.dot(self.g, d))
        if not dphi0 < 0.0:
            self.S, self.Y = [], []
            d = -self.g
            dphi0 = float(np.dot(self.g, d))
        if self.S:
            alpha1 = 1.0
        else:
            alpha1 = min(1.0, 1.0 / float(np.linalg.norm(d)))
        ls = line_search(self.fg, self.x, d, self.f, dphi0, alpha1, self.c1, self.c2, self.max_evals)
        self.evals += ls.evals
        if ls.status == 2:
            self.S, self.Y = [], []
            return ls
        s = ls.alpha * d
        g_new = np.asarray(ls.g, dtype=np.float64)
        y = g_new - self.g
        self.x = self.x + ls.alpha * d
        self.f, self.g = ls.f, g_new
        if float(np.dot(s, y)) > EPS * float(np.dot(y, y)):
            self.S.append(s)
            self.Y.append(y)
            if len(self.S) > self.m:
                self.S.pop(0)
                self.Y.pop(0)
        return ls
