"""Right-hand-side evaluation counts of the paper's performance model.

Part of the test oracle (test infrastructure only).

Paper: section "Performance Model", eq. (perf_RK4), eq. (perf_AB) and
eq. (speedup).  Right-hand-side evaluations are taken to dominate the cost and
every integrator runs at its own largest stable step.  Classic RK4 evaluates
the right-hand side four times per step on every point; an AB or MRAB scheme
evaluates it once per (micro-)step, the fast grid SR times per macrostep and
the slow grid once.  An AB integrator's macrostep is r_RK4 times the RK4 step
(r_RK4 = dt / dt_RK4, the ratio of the stable steps, section "Stability
Results").
"""


def rhs_evals_rk4(t: float, dt_rk4: float, n_f: int, n_s: int) -> float:
    """Point right-hand-side evaluations of RK4 up to time t (eq. perf_RK4)."""
    return 4.0 * (t / dt_rk4) * (n_f + n_s)


def rhs_evals_ab(t: float, dt_rk4: float, r_rk4: float, sr: int, n_f: int, n_s: int) -> float:
    """Point right-hand-side evaluations of AB/MRAB with step ratio sr up to
    time t, macrostep r_rk4 * dt_rk4 (eq. perf_AB; sr = 1 is single-rate)."""
    return (t / (dt_rk4 * r_rk4)) * (sr * n_f + n_s)


def speedup(t: float, dt_rk4: float, r_rk4: float, sr: int, n_f: int, n_s: int) -> float:
    """SU = RK4 evaluations / AB evaluations (eq. speedup)."""
    return rhs_evals_rk4(t, dt_rk4, n_f, n_s) / rhs_evals_ab(t, dt_rk4, r_rk4, sr, n_f, n_s)


def rhs_evals_per_macrostep(rates, points) -> int:
    """Point right-hand-side evaluations of one MRAB macrostep with any number
    of levels: level l evaluates r_l times on its N_l points (the two-level
    count SR * n_f + n_s of eq. perf_AB, generalised)."""
    return int(sum(int(r) * int(n) for r, n in zip(rates, points)))
