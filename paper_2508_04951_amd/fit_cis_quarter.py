"""Fit the float32 coefficients of cis_quarter (csrc/fft.hip): cos and sin of pi w / 2 for
|w| <= 1/2, the remainder of the dispersive phase after whole quarter turns.

In u = w^2 on [0, 1/4]: sin(pi w / 2) = w S(u) and cos(pi w / 2) = 1 + u C(u), S and C cubics.
Each is a weighted minimax (Remez exchange) fit of the absolute error in w, |w| |S - sin/w| and
u |C - (cos - 1)/u|.  The coefficients are then rounded to float32 one at a time, from the
constant term up, each time refitting the remaining ones to the rounding of those fixed so far.

    python -m paper_2508_04951_amd.fit_cis_quarter      # prints the coefficients and errors
"""
from __future__ import annotations

import numpy as np

U_LO, U_HI = 1e-8, 0.25
GRID = np.linspace(U_LO, U_HI, 200001)


def _remez(g, wt, free: list[int], fixed: dict[int, float], iters: int = 40):
    """Minimise max wt(u) |sum_j c_j u^j - g(u)| over the free powers, the fixed ones held."""
    n = len(free)
    k = np.arange(n + 1)
    u = (U_LO + U_HI) / 2 + (U_HI - U_LO) / 2 * np.cos(np.pi * (n - k) / n)

    def rest(x):
        return g(x) - sum(c * x ** j for j, c in fixed.items())

    c = np.zeros(n)
    for _ in range(iters):
        M = np.hstack([np.stack([u ** j for j in free], 1), ((-1.0) ** k / wt(u))[:, None]])
        sol = np.linalg.solve(M, rest(u))
        c = sol[:n]
        err = wt(GRID) * (np.stack([GRID ** j for j in free], 1) @ c - rest(GRID))
        s = np.sign(err)
        starts = np.concatenate([[0], np.nonzero(np.diff(s) != 0)[0] + 1, [GRID.size]])
        idx = np.array([i0 + np.argmax(np.abs(err[i0:i1])) for i0, i1 in zip(starts[:-1], starts[1:])])
        if idx.size > n + 1:
            j = max(range(idx.size - n), key=lambda q: np.abs(err[idx[q:q + n + 1]]).min())
            idx = idx[j:j + n + 1]
        if idx.size < n + 1:
            break
        u = GRID[idx]
    return dict(zip(free, c))


def fit(g, wt, degree: int = 3) -> list[float]:
    fixed: dict[int, float] = {}
    for j in range(degree + 1):
        sol = _remez(g, wt, list(range(j, degree + 1)), fixed)
        fixed[j] = float(np.float32(sol[j]))
    return [fixed[j] for j in range(degree + 1)]


def sin_over_w(u):
    w = np.sqrt(u)
    return np.sin(np.pi * w / 2) / w


def cos_minus_one_over_u(u):
    w = np.sqrt(u)
    return (np.cos(np.pi * w / 2) - 1) / u


def coefficients() -> tuple[list[float], list[float]]:
    """(S, C): float32 coefficients of S(u) and C(u), constant term first."""
    return fit(sin_over_w, np.sqrt), fit(cos_minus_one_over_u, lambda u: u)


def errors(S, C, w=None) -> tuple[float, float]:
    """Largest absolute error of w S(w^2) and 1 + w^2 C(w^2) over |w| <= 1/2 (float64 arithmetic)."""
    w = np.linspace(-0.5, 0.5, 400001) if w is None else w
    u = w * w
    s = w * sum(c * u ** j for j, c in enumerate(S))
    c = 1 + u * sum(q * u ** j for j, q in enumerate(C))
    return float(np.abs(s - np.sin(np.pi * w / 2)).max()), float(np.abs(c - np.cos(np.pi * w / 2)).max())


if __name__ == "__main__":
    S, C = coefficients()
    print("S:", [float(v).hex() for v in S])
    print("C:", [float(v).hex() for v in C])
    print("max abs error sin %.3e cos %.3e" % errors(S, C))
