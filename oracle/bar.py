"""Bennett acceptance ratio free-energy estimators on per-window energy samples (Sec.
"Hydration free energies", eqs. PIBAR1-PIBAR2, and the appendix "Single-bead PI-BAR
Estimator"). TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Notation as in the paper: states A and B, Delta F_AB = beta^-1 ln(Z_A / Z_B), the Fermi
function f(x) = 1 / (1 + exp(beta x)), and

    Delta F_AB = C + beta^-1 ln( <f(U_A - U_B + C)>_B / <f(U_B - U_A - C)>_A ),
    C = Delta F_AB + beta^-1 ln(n_B / n_A),

a self-consistent pair of equations. Substituting the second into the first, the pair
holds exactly when sum_B f(C - du) = sum_A f(du - C) (a reading: the paper says only that
the set is solved iteratively). The left side falls and the right side rises with C, so
the root is unique; it is found here by bisection, which converges whatever the overlap of
the two samples (plain fixed-point iteration of the pair can stall when it is poor).
The inputs are the energy differences sampled in each state:
``du_a[k] = U_B(x_k) - U_A(x_k)`` for configurations x_k of state A and
``du_b[k] = U_B(x_k) - U_A(x_k)`` for configurations of state B (the same sign
convention for both). PI-BAR takes U = the bead-averaged potential U_P = (1/P) sum_b
V(x_b) (eq. PI_potential); the single-bead estimator takes V at one bead instead.
"""
import numpy as np


def fermi(x, beta):
    """f(x) = 1 / (1 + exp(beta x)), evaluated without overflow and with full relative
    accuracy in both tails: exp(-y) / (1 + exp(-y)) for y = beta x > 0, else 1 / (1 + e^y)."""
    y = beta * np.asarray(x, dtype=np.float64)
    e = np.exp(-np.abs(y))
    return np.where(y > 0, e / (1.0 + e), 1.0 / (1.0 + e))


def bar(du_a, du_b, beta, max_iter=400):
    """Delta F_AB from the two samples (see the module docstring) -> (dF, iterations)."""
    du_a = np.asarray(du_a, dtype=np.float64)
    du_b = np.asarray(du_b, dtype=np.float64)
    n_a, n_b = len(du_a), len(du_b)

    def h(C):                      # decreasing in C; zero at the self-consistent C
        return np.sum(fermi(C - du_b, beta)) - np.sum(fermi(du_a - C, beta))

    lo = min(du_a.min(), du_b.min()) - 40.0 / beta
    hi = max(du_a.max(), du_b.max()) + 40.0 / beta
    it = 0
    for it in range(1, max_iter + 1):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if h(mid) > 0:
            lo = mid
        else:
            hi = mid
    C = 0.5 * (lo + hi)
    return C - np.log(n_b / n_a) / beta, it


def window_differences(E_a_at_a, E_b_at_a, E_a_at_b, E_b_at_b, estimator="pi"):
    """Energy differences for ``bar`` from per-sample, per-bead potentials [n][P]:
    E_x_at_y = V of state x at the configurations sampled in state y. ``pi``: the
    bead-averaged U_P; ``single``: bead 0 only."""
    def U(E):
        E = np.asarray(E, dtype=np.float64)
        return E.mean(axis=1) if estimator == "pi" else E[:, 0]
    return U(E_b_at_a) - U(E_a_at_a), U(E_b_at_b) - U(E_a_at_b)
