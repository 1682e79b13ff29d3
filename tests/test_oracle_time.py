"""Time integrators of the oracle: SSP-RK3 (Shu-Osher), Heun's RK2 and the five-stage
fourth-order LSERK in 2N-storage form.  On a uniform state the DG right-hand side is the
one-step source alone, so one element integrates the reactor ODE
dY/dt = -K Y exp(-E_a / T), T = (gamma - 1)(e - q Y), with the scheme; the error against a
tight-tolerance ODE solution falls as dt^p with the scheme's order p."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from workloads import gen

GAMMA, Q, EA, K = 1.4, 1.0, 10.0, 1.0e4
RHO, P0, Y0 = 1.0, 1.0, 1.0
T_END = 1.0


def reactor_reference():
    e = P0 / ((GAMMA - 1.0) * RHO) + Q * Y0          # internal + chemical energy per mass (constant)

    def f(t, y):
        T = (GAMMA - 1.0) * (e - Q * y[0])
        return [-K * y[0] * np.exp(-EA / T)]

    sol = solve_ivp(f, (0.0, T_END), [Y0], method="DOP853", rtol=1e-13, atol=1e-15)
    return sol.y[0, -1]


def reactor_run(orc, rk, n_steps):
    case, _ = gen.case_c0(E=1, n_pe=1, mode="sync")
    case["physics"].update(gamma=GAMMA, q_heat=Q, e_act=EA, k_pre=K)
    case["disc"].update(rk=rk, dt=T_END / n_steps)
    w0 = np.zeros((1, 5, 3))
    w0[0, :, 0] = gen.onestep_conserved(np.array([RHO]), 0.0, np.array([P0]), Y0, case["physics"])[:, 0]
    w0 = gen._fix_density_modes(w0)
    s = orc.OracleSolver(case, w0, n_steps + 1)
    s.step(n_steps)
    w = s.state()
    return w[0, 3, 0] / w[0, 0, 0]


@pytest.mark.parametrize("rk,order", [("rk2", 2), ("ssprk3", 3), ("lserk4", 4)])
def test_integrator_order_on_the_reactor_ode(orc, rk, order):
    ref = reactor_reference()
    errs = [abs(reactor_run(orc, rk, n) - ref) for n in (10, 20, 40)]
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    print(rk, errs, rates)
    assert abs(rates[-1] - order) < 0.3, (rk, errs, rates)
    assert errs[-1] < 1e-2


def test_rk2_is_heun(orc):
    """Two stages of the 2N form with A = (0, -1), B = (1, 1/2) are Heun's method, checked on
    one step of the reactor ODE by hand."""
    e = P0 / ((GAMMA - 1.0) * RHO) + Q * Y0
    f = lambda y: -K * y * np.exp(-EA / ((GAMMA - 1.0) * (e - Q * y)))
    dt = T_END / 5
    y1 = Y0 + dt * f(Y0)
    heun = 0.5 * (Y0 + y1 + dt * f(y1))
    assert abs(reactor_run_steps(orc, "rk2", dt, 1) - heun) < 1e-14


def reactor_run_steps(orc, rk, dt, steps):
    case, _ = gen.case_c0(E=1, n_pe=1, mode="sync")
    case["physics"].update(gamma=GAMMA, q_heat=Q, e_act=EA, k_pre=K)
    case["disc"].update(rk=rk, dt=dt)
    w0 = np.zeros((1, 5, 3))
    w0[0, :, 0] = gen.onestep_conserved(np.array([RHO]), 0.0, np.array([P0]), Y0, case["physics"])[:, 0]
    w0 = gen._fix_density_modes(w0)
    s = orc.OracleSolver(case, w0, steps + 1)
    s.step(steps)
    w = s.state()
    return w[0, 3, 0] / w[0, 0, 0]
