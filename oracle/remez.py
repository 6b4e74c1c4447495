"""Remez exchange for minimax polynomials and rationals, FP64 (oracle; test
infrastructure only).

Sec. 3.1 names the Remez exchange algorithm and the Chebyshev (max-norm)
criterion but gives no steps.  This is the textbook algorithm:

  1. start from a reference of N = n + m + 2 points (Chebyshev extrema of the
     interval);
  2. levelled solve: find p (degree n), q (degree m) and E with
     p(x_i) - (f(x_i) + (-1)^i E) q(x_i) = 0 at every reference point.  For
     m = 0 this is a linear system; for m > 0 it is the generalised
     eigenproblem A c = E B c, and the eigenvalue of smallest |E| whose q has
     no root in [a, b] is taken;
  3. locate every local extremum of the error e = p/q - f on the interval
     (dense sampling, then bounded scalar refinement), endpoints included;
  4. exchange: keep one point per run of equal sign (the largest |e|) and cut
     the alternating sequence down to N points holding the global maximum;
  5. stop when the largest error and the smallest reference error agree to a
     relative tolerance.

A positive weight w(x) turns the criterion into max |w (p/q - f)| (weighted
Chebyshev approximation): the levelled equations become
p(x_i) - (f(x_i) + (-1)^i E / w(x_i)) q(x_i) = 0 and the extrema are those of
w e.  With w = 1 (the default) this is the plain minimax of Sec. 3.1.

Coefficients are solved in the Chebyshev basis on [a, b] and returned as
monomial coefficients in x, lowest degree first, with q[0] = 1.

``lp_minimax`` is an independent route to the same optimum on a discrete
grid (linear programming; bisection on the level for rationals), used by the
tests as a cross-check.
"""
import numpy as np
from numpy.polynomial import chebyshev as C
from numpy.polynomial import polynomial as Pm
import scipy.linalg
import scipy.optimize


class Fit:
    def __init__(self, p, q, eps, alt, iters, converged, a, b):
        self.p = np.asarray(p, dtype=np.float64)
        self.q = np.asarray(q, dtype=np.float64)
        self.eps = float(eps)
        self.alt = np.asarray(alt, dtype=np.float64)
        self.iters = int(iters)
        self.converged = bool(converged)
        self.a, self.b = float(a), float(b)

    def __call__(self, x):
        x = np.asarray(x, dtype=np.float64)
        return Pm.polyval(x, self.p) / Pm.polyval(x, self.q)

    def __repr__(self):
        return "Fit(n=%d, m=%d, eps=%.6e, iters=%d, converged=%s)" % (
            len(self.p) - 1, len(self.q) - 1, self.eps, self.iters, self.converged)


def _to_s(x, a, b):
    return (2.0 * np.asarray(x, dtype=np.float64) - (a + b)) / (b - a)


def _cheb_to_monomial_x(c, a, b):
    """Chebyshev series in s = (2x - a - b)/(b - a) -> monomial coefficients in x."""
    c = np.asarray(c, dtype=np.float64)
    ms = C.cheb2poly(c)  # monomial in s
    lin = np.array([-(a + b) / (b - a), 2.0 / (b - a)])
    out = np.zeros(len(c))
    power = np.array([1.0])
    for k, ck in enumerate(ms):
        if k > 0:
            power = Pm.polymul(power, lin)
        out[:len(power)] += ck * power
    return out


def _dense_grid(a, b, ref, n_cheb=1 << 16, per_gap=64):
    k = np.arange(n_cheb)
    g = 0.5 * (a + b) - 0.5 * (b - a) * np.cos(np.pi * k / (n_cheb - 1))
    gaps = [np.linspace(ref[i], ref[i + 1], per_gap + 2)[1:-1] for i in range(len(ref) - 1)]
    g = np.concatenate([g] + gaps + [[a, b]])
    g = np.unique(np.clip(g, a, b))
    return g


def _local_extrema(err, a, b, ref):
    """Local extrema of err on [a, b] (endpoints included): one candidate per
    run of equal sign on a dense grid (the largest |e| in the run), each then
    refined by bounded scalar search."""
    g = _dense_grid(a, b, ref)
    e = err(g)
    d = np.diff(e)
    turn = (d[:-1] * d[1:] <= 0) & ~((d[:-1] == 0) & (d[1:] == 0))
    idx = np.array([0] + (np.nonzero(turn)[0] + 1).tolist() + [len(g) - 1])
    # one candidate per run of equal sign
    sg = np.sign(e[idx])
    keep = []
    for i, s_ in zip(idx, sg):
        if keep and np.sign(e[keep[-1]]) == s_:
            if abs(e[i]) > abs(e[keep[-1]]):
                keep[-1] = i
        else:
            keep.append(i)
    xs, es = [], []
    for i in keep:
        if i == 0 or i == len(g) - 1:
            xs.append(g[i])
            es.append(e[i])
            continue
        sgn = 1.0 if e[i] >= 0 else -1.0
        lo, hi = g[i - 1], g[i + 1]
        r = scipy.optimize.minimize_scalar(lambda t: -sgn * float(err(np.array([t]))[0]),
                                           bounds=(lo, hi), method="bounded",
                                           options={"xatol": 1e-15 * max(1.0, abs(g[i]))})
        xr = float(r.x)
        er = float(err(np.array([xr]))[0])
        if sgn * er < sgn * e[i]:
            xr, er = g[i], e[i]
        xs.append(xr)
        es.append(er)
    order = np.argsort(xs)
    return np.asarray(xs)[order], np.asarray(es)[order]


def _exchange(xs, es, N):
    """Alternating subsequence of N extrema containing the global maximum."""
    # one point per run of equal sign, the largest |e| in the run
    keep_x, keep_e = [], []
    for x, e in zip(xs, es):
        if e == 0:
            continue
        if keep_e and np.sign(e) == np.sign(keep_e[-1]):
            if abs(e) > abs(keep_e[-1]):
                keep_x[-1], keep_e[-1] = x, e
        else:
            keep_x.append(x)
            keep_e.append(e)
    if len(keep_x) < N:
        return None
    keep_x = list(keep_x)
    keep_e = list(keep_e)
    while len(keep_x) > N:
        gmax = int(np.argmax(np.abs(keep_e)))
        # drop the smaller end unless it holds the global maximum
        if (abs(keep_e[0]) <= abs(keep_e[-1]) and gmax != 0) or gmax == len(keep_e) - 1:
            keep_x.pop(0)
            keep_e.pop(0)
        else:
            keep_x.pop()
            keep_e.pop()
    return np.asarray(keep_x)


def _solve_level(f, n, m, a, b, ref, w=None):
    """Levelled solve on the reference: Chebyshev coefficients of p, q and E
    (E is the level of the weighted error w e)."""
    s = _to_s(ref, a, b)
    fi = f(ref)
    N = len(ref)
    sig = (-1.0) ** np.arange(N)
    if w is not None:
        sig = sig / w(ref)
    Tn = C.chebvander(s, n)
    if m == 0:
        A = np.hstack([Tn, sig[:, None]])
        sol = np.linalg.solve(A, fi)
        return sol[:n + 1], np.array([1.0]), sol[n + 1]
    Tm = C.chebvander(s, m)
    A = np.hstack([Tn, -fi[:, None] * Tm])
    B = np.hstack([np.zeros((N, n + 1)), sig[:, None] * Tm])
    w, V = scipy.linalg.eig(A, B)
    probe = np.linspace(-1.0, 1.0, 4001)
    best = None
    for k in range(len(w)):
        if not np.isfinite(w[k]) or abs(w[k].imag) > 1e-9 * max(1.0, abs(w[k].real)):
            continue
        v = V[:, k].real
        if np.max(np.abs(V[:, k].imag)) > 1e-6 * np.max(np.abs(v)):
            continue
        cq = v[n + 1:]
        qv = C.chebval(probe, cq)
        if not (np.all(qv > 0) or np.all(qv < 0)):
            continue
        E = w[k].real
        if best is None or abs(E) < abs(best[2]):
            if qv[0] < 0:
                v = -v
            best = (v[:n + 1], v[n + 1:], E)
    if best is None:
        raise np.linalg.LinAlgError("no pole-free levelled solution on this reference")
    return best


def remez(f, n, m, a, b, tol=1e-8, maxit=100, ref=None, w=None):
    """Minimax approximation of f by p/q, deg p = n, deg q = m, on [a, b].

    Returns a Fit (monomial p, q with q[0] = 1, eps = max |p/q - f| on the
    interval, the final reference, the iteration count, the convergence flag).
    With a weight w (a callable, positive on [a, b]) the fit minimises
    max |w (p/q - f)| and eps is that weighted maximum.
    """
    wf = (lambda x: np.ones_like(np.asarray(x, dtype=np.float64))) if w is None else w
    N = n + m + 2
    if ref is None:
        ref = 0.5 * (a + b) - 0.5 * (b - a) * np.cos(np.pi * np.arange(N) / (N - 1))
    ref = np.asarray(ref, dtype=np.float64)
    converged = False
    eps = np.inf
    it = 0
    for it in range(1, maxit + 1):
        cp, cq, E = _solve_level(f, n, m, a, b, ref, w)

        def err(x, cp=cp, cq=cq):
            s = _to_s(x, a, b)
            return wf(x) * (C.chebval(s, cp) / C.chebval(s, cq) - f(x))

        xs, es = _local_extrema(err, a, b, ref)
        eps = float(np.max(np.abs(es)))
        new = _exchange(xs, es, N)
        if new is None:
            break
        ref_err = np.abs(err(new))
        ref = new
        if (eps - np.min(ref_err)) <= tol * eps:
            converged = True
            break
    p = _cheb_to_monomial_x(cp, a, b)
    q = _cheb_to_monomial_x(cq, a, b)
    p, q = p / q[0], q / q[0]
    fit = Fit(p, q, 0.0, ref, it, converged, a, b)
    fit.eps = max_error(fit, f, a, b, w=w)
    return fit


def max_error(g, f, a, b, n_pts=1 << 18, w=None):
    """Max |g - f| (max |w (g - f)| with a weight) on [a, b]: dense Chebyshev
    sampling then local refinement around the largest samples."""
    wf = (lambda x: np.ones_like(x)) if w is None else w
    k = np.arange(n_pts)
    x = np.unique(np.clip(0.5 * (a + b) - 0.5 * (b - a) * np.cos(np.pi * k / (n_pts - 1)), a, b))
    e = np.abs(wf(x) * (g(x) - f(x)))
    best = float(np.max(e))
    for i in np.argsort(e)[-8:]:
        lo, hi = x[max(i - 1, 0)], x[min(i + 1, len(x) - 1)]
        if hi <= lo:
            continue

        def neg(t):
            tt = np.array([t])
            return -abs(float(wf(tt)[0] * (g(tt)[0] - f(tt)[0])))
        r = scipy.optimize.minimize_scalar(neg, bounds=(lo, hi), method="bounded")
        best = max(best, -float(r.fun))
    return best


def lp_minimax(f, n, m, a, b, n_grid=3001, rel_tol=1e-7, w=None):
    """Discrete minimax of f by p/q on n_grid Chebyshev points of [a, b] by
    linear programming: directly for m = 0; for m > 0 by bisection on the
    level d with the feasibility problem |p(x_i) - f(x_i) q(x_i)| <= d q(x_i),
    q(x_i) >= 1.  Returns (p, q, eps on the grid), monomial in x, q[0] = 1.
    With a weight w the bound at x_i is d / w(x_i) (and eps is weighted)."""
    k = np.arange(n_grid)
    x = 0.5 * (a + b) - 0.5 * (b - a) * np.cos(np.pi * k / (n_grid - 1))
    s = _to_s(x, a, b)
    fx = f(x)
    wx = np.ones_like(x) if w is None else w(x)
    Tn = C.chebvander(s, n)
    if m == 0:
        # variables: c (n+1), d ; minimise d s.t. +-w (Tn c - f) <= d
        col = -np.ones((n_grid, 1))
        A = np.vstack([np.hstack([wx[:, None] * Tn, col]), np.hstack([-wx[:, None] * Tn, col])])
        rhs = np.concatenate([wx * fx, -wx * fx])
        cost = np.zeros(n + 2)
        cost[-1] = 1.0
        r = scipy.optimize.linprog(cost, A_ub=A, b_ub=rhs, bounds=[(None, None)] * (n + 2), method="highs")
        cp = r.x[:n + 1]
        p = _cheb_to_monomial_x(cp, a, b)
        return p, np.array([1.0]), float(np.max(np.abs(wx * (Pm.polyval(x, p) - fx))))
    Tm = C.chebvander(s, m)
    nv = n + 1 + m + 1

    def feasible(d):
        # p - f q <= d q  ->  Tn cp - (f + d) Tm cq <= 0 ; -(p - f q) <= d q -> -Tn cp + (f - d) Tm cq <= 0
        A1 = np.hstack([Tn, -(fx + d / wx)[:, None] * Tm])
        A2 = np.hstack([-Tn, (fx - d / wx)[:, None] * Tm])
        A3 = np.hstack([np.zeros((n_grid, n + 1)), -Tm])  # q >= 1
        A = np.vstack([A1, A2, A3])
        rhs = np.concatenate([np.zeros(2 * n_grid), -np.ones(n_grid)])
        r = scipy.optimize.linprog(np.zeros(nv), A_ub=A, b_ub=rhs, bounds=[(-1e6, 1e6)] * nv, method="highs")
        return r.x if r.status == 0 else None

    lo, hi = 0.0, float(np.max(np.abs(wx * fx))) + float(np.max(wx))
    sol = feasible(hi)
    while hi - lo > rel_tol * hi:
        mid = 0.5 * (lo + hi)
        v = feasible(mid)
        if v is None:
            lo = mid
        else:
            hi, sol = mid, v
    p = _cheb_to_monomial_x(sol[:n + 1], a, b)
    q = _cheb_to_monomial_x(sol[n + 1:], a, b)
    p, q = p / q[0], q / q[0]
    return p, q, float(np.max(np.abs(wx * (Pm.polyval(x, p) / Pm.polyval(x, q) - fx))))
