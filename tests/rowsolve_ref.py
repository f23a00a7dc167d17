"""An independent NumPy statement of the PQNR reading for one row subproblem,
used only by the oracle's pins (vectorised, written from the definitions:
the row objective f(b) = sum(b) - sum_k x_k log(b . pi_k) over b >= 0, its
gradient 1 - phi, the L-BFGS two-loop recursion of Nocedal & Wright
(Numerical Optimization, Algorithm 7.4) restricted to the free variables, and
a projected backtracking search with a sufficient-decrease test)."""
import numpy as np


def objective_change(b, delta, xs, P, eps=1e-10):
    """f(b + delta) - f(b), or +inf when a model value above eps would reach eps."""
    m = P @ b
    dm = P @ delta
    if np.any((m > eps) & (m + dm <= eps)):
        return np.inf
    return float(delta.sum() - np.sum(xs * np.log1p(dm / m)))


def gradient(b, xs, P, eps=1e-10):
    return 1.0 - (xs / np.maximum(P @ b, eps)) @ P


def two_loop(g, pairs, free):
    """-H g on the free set from the (s, y) pairs (oldest first); pairs whose
    free-set curvature s.y is not positive are skipped; H0 = gamma I with gamma
    = s.y / y.y of the newest usable pair. None when no pair is usable."""
    q = np.where(free, g, 0.0)
    used, alphas = [], []
    for s, y in reversed(pairs):
        sy = float(np.dot(s[free], y[free]))
        if sy <= 0.0:
            continue
        a = float(np.dot(s[free], q[free])) / sy
        q[free] -= a * y[free]
        used.append((s, y, sy))
        alphas.append(a)
    if not used:
        return None
    s0, y0, sy0 = used[0]
    yy = float(np.dot(y0[free], y0[free]))
    gamma = sy0 / yy if yy > 0.0 else 0.0
    if not gamma > 0.0:
        return None
    q *= gamma
    for (s, y, sy), a in zip(reversed(used), reversed(alphas)):
        beta = float(np.dot(y[free], q[free])) / sy
        q[free] += (a - beta) * s[free]
    return np.where(free, -q, 0.0)


def pqnr_row(xs, P, b0, steps, trials=4, sigma=1e-4, mem=3, curv=1e-10, keep_pairs_on_fail=False, log=None):
    """Iterates b_0 .. b_steps of the reading: the scaled gradient -b*g at the
    first step and whenever the quasi-Newton direction is unusable or not a
    descent direction; `trials` backtracking trials alpha = 1, 1/2, ...; with
    none acceptable the MU step b*phi and the pairs dropped (kept when
    keep_pairs_on_fail, a variant for the pins to tell apart)."""
    b = np.array(b0, dtype=np.float64)
    pairs, s_last, g_prev = [], None, None
    its = [b.copy()]
    for step in range(steps):
        g = gradient(b, xs, P)
        if step > 0:
            y = g - g_prev
            if np.dot(s_last, y) > curv * np.sqrt(np.dot(s_last, s_last) * np.dot(y, y)):
                pairs = (pairs + [(s_last, y)])[-mem:]
        free = ~((b == 0.0) & (g > 0.0))
        d = two_loop(g, pairs, free) if pairs else None
        if d is None or not np.dot(g, d) < 0.0:
            d = -b * g
        step_taken, alpha = None, 1.0
        for _ in range(trials):
            delta = np.maximum(b + alpha * d, 0.0) - b
            gd = float(np.dot(g, delta))
            if gd < 0.0 and objective_change(b, delta, xs, P) <= sigma * gd:
                step_taken = delta
                break
            alpha *= 0.5
        if log is not None:
            log.append(dict(b=b.copy(), g=g, d=d, npairs=len(pairs), accepted=step_taken is not None))
        if step_taken is None:
            step_taken = b * (1.0 - g) - b  # the MU step b*phi, as a change of b
            if not keep_pairs_on_fail:
                pairs = []
        s_last, g_prev = step_taken, g
        b = b + step_taken
        its.append(b.copy())
    return its
