"""Pins of the oracle's limiter (Sec. 3.3, Eq. (9)-(11)) against mathematics it must satisfy."""
import numpy as np
import pytest
from numpy.polynomial import legendre as L

from workloads import gen


def onestep_cfg(orc, order_p=3, gamma=1.2, q=50.0):
    case, _ = gen.case_c2(E=16, order_p=order_p, length=16.0, shock_x=4.0, n_pe=2, k_pre=1.0)
    case["physics"]["gamma"] = gamma
    case["physics"]["q_heat"] = q
    return orc.Config(case)


@pytest.mark.parametrize("np_", [1, 2, 3, 4])
def test_beta_matrix_against_polynomial_integration(orc, np_):
    """Eq. (10) mapped to xi: B_ab = sum_s 2^(2s-1) int P_a^(s) P_b^(s); integrate with numpy."""
    M = np_ + 1
    B = np.zeros(M * M)
    orc.lib().or_beta_matrix(np_, orc._dptr(B))
    B = B.reshape(M, M)
    ref = np.zeros((M, M))
    for a in range(M):
        for b in range(M):
            for s in range(1, np_ + 1):
                pa = L.legder(np.eye(M)[a], s)
                pb = L.legder(np.eye(M)[b], s)
                prod = L.legmul(pa, pb)
                anti = L.legint(prod)
                ref[a, b] += 2.0 ** (2 * s - 1) * (L.legval(1.0, anti) - L.legval(-1.0, anti))
    np.testing.assert_allclose(B, ref, rtol=1e-13, atol=1e-15 * np.abs(ref).max())


@pytest.mark.parametrize("np_", [1, 2, 3, 4])
@pytest.mark.parametrize("side", [-1, 1])
def test_translation_matrix(orc, np_, side):
    """The neighbour polynomial re-expanded in the cell: evaluate both forms at random points."""
    M = np_ + 1
    T = np.zeros(M * M)
    orc.lib().or_translation(np_, side, orc._dptr(T))
    T = T.reshape(M, M)
    rng = np.random.default_rng(3)
    c = rng.normal(size=M)
    xi = rng.uniform(-1, 1, size=7)
    direct = L.legval(xi - 2.0 * side, c)
    moved = L.legval(xi, T @ c)
    np.testing.assert_allclose(moved, direct, rtol=1e-12, atol=1e-12)


def flux_jacobian_fd(orc, cfg, w, h=1e-6):
    V = len(w)
    A = np.zeros((V, V))
    for j in range(V):
        dw = np.zeros(V)
        dw[j] = h * max(1.0, abs(w[j]))
        fp = orc.call_vec("or_conv_flux", cfg, w + dw, nout=V)
        fm = orc.call_vec("or_conv_flux", cfg, w - dw, nout=V)
        A[:, j] = (fp - fm) / (2 * dw[j])
    return A


@pytest.mark.parametrize("seed", range(4))
def test_eigenvectors_diagonalise_the_flux_jacobian(orc, seed):
    """L A R = diag(u-a, u, u, u, u+a) with A from finite differences of f^c; L R = I."""
    cfg = onestep_cfg(orc)
    rng = np.random.default_rng(seed)
    rho, u, p, yr = rng.uniform(0.5, 8), rng.uniform(-3, 6), rng.uniform(0.5, 40), rng.uniform(0, 1)
    w = np.array(gen.onestep_conserved(np.array(rho), np.array(u), np.array(p), np.array(yr),
                                       {"gamma": 1.2, "q_heat": 50.0}), dtype=float)
    V = 5
    Lm = np.zeros(V * V)
    Rm = np.zeros(V * V)
    rc = orc.lib().or_char_matrices(cfg.ref(), orc._dptr(w), orc._dptr(Lm), orc._dptr(Rm))
    assert rc == 0
    Lm, Rm = Lm.reshape(V, V), Rm.reshape(V, V)
    np.testing.assert_allclose(Lm @ Rm, np.eye(V), atol=1e-12)
    A = flux_jacobian_fd(orc, cfg, w)
    a = np.sqrt(1.2 * p / rho)
    lam = np.diag([u - a, u, u, u, u + a])
    scale = abs(u) + a
    np.testing.assert_allclose(Lm @ A @ Rm, lam, atol=1e-6 * scale)


def run_limiter_once(orc, case, w0):
    """Run one step with dt = 0 so only the limiter acts (three times, once per stage)."""
    case = dict(case)
    case["disc"] = dict(case["disc"], dt=0.0)
    s = orc.OracleSolver(case, w0, 4)
    s.step(1)
    return s.state(), s.flags(), s.total_flags()


def test_limiter_preserves_means_and_flags_the_jump(orc):
    case, w0 = gen.case_c2(E=64, order_p=3, length=8.0, shock_x=4.0, n_pe=4, k_pre=0.0, mode="sync")
    rng = np.random.default_rng(1)
    w0 = w0 * (1 + 0.01 * rng.uniform(size=w0.shape) * (np.arange(4) > 0))  # some wiggles
    w0 = gen._fix_density_modes(w0)
    w, flags, total = run_limiter_once(orc, case, w0)
    assert flags[31] or flags[32], "cells next to the jump must be troubled"
    assert total > 0
    np.testing.assert_allclose(w[:, :, 0], w0[:, :, 0], rtol=1e-13, atol=1e-13)
    # sum_i rho Y_i = rho survives the characteristic limiting, mode by mode
    np.testing.assert_allclose(w[:, 3:, :].sum(1), w[:, 0, :], rtol=1e-12, atol=1e-12)


def test_limiter_is_identity_on_smooth_data(orc):
    case, w0 = gen.case_c0(E=64, order_p=3)
    case["disc"]["limiter"] = 1
    case["disc"]["bc"] = "periodic"
    case["async"]["mode"] = "sync"
    w, flags, total = run_limiter_once(orc, case, w0)
    assert total == 0
    np.testing.assert_allclose(w, w0, rtol=4e-16, atol=4e-16 * np.abs(w0).max())  # dt = 0: RK weights only


def test_weno_reproduces_a_global_polynomial(orc):
    """If the three stencil polynomials are one global polynomial, the WENO result is that polynomial."""
    E, np_ = 12, 3
    case, _ = gen.case_c0(E=E, order_p=np_)
    case["disc"].update(limiter=1, bc="periodic", x_right=float(E))
    case["async"]["mode"] = "sync"
    phys = case["physics"]

    def fn(x):
        rho = 2.0 + 0.01 * x + 0.002 * x**2
        return gen.onestep_conserved(rho, 0.5, 1.0 + 0.001 * x**3 / 100.0, 0.7, phys)

    w0 = gen._fix_density_modes(gen.project(fn, E, np_, 0.0, float(E)))
    # force every interior cell to be limited: use the WENO routine on each stencil directly
    cfg = orc.Config(case)
    V, M = 5, np_ + 1
    for e in range(1, E - 1):
        out = np.zeros(V * M)
        args = [np.ascontiguousarray(w0[e + d]) for d in (-1, 0, 1)]
        rc = orc.lib().or_weno_cell(cfg.ref(), *[orc._dptr(a) for a in args], orc._dptr(out))
        assert rc == 0
        np.testing.assert_allclose(out.reshape(V, M), w0[e], rtol=1e-11, atol=1e-11)


# ---- the TVB minmod indicator (the TVD slope-limiter test of Sec. 3.3 when M = 0)

def minmod_case(E, fn, order_p=2, tvb_m=0.0, bc="transmissive"):
    case, _ = gen.case_c0(E=E, order_p=order_p)
    case["disc"].update(limiter=1, bc=bc, indicator="minmod", tvb_m=tvb_m, x_left=0.0, x_right=1.0, flux="hllc")
    case["async"].update(mode="sync", n_pe=1)
    w0 = gen._fix_density_modes(gen.project(fn, E, order_p, 0.0, 1.0))
    return case, w0


def test_minmod_passes_linear_data(orc):
    """A global linear state: every face deviation is half of both mean differences."""
    phys = gen.case_c0()[0]["physics"]
    case, w0 = minmod_case(40, lambda x: gen.onestep_conserved(1.0 + 0.5 * x, 0.3 + 0.2 * x, 1.0 + x, 0.8, phys))
    _, flags, _ = run_limiter_once(orc, case, w0)
    assert not flags[1:-1].any()      # the ends see a ghost with their own mean (no slope allowed)


def test_minmod_flags_a_jump_and_smooth_extrema_only_when_tvd(orc):
    phys = gen.case_c0()[0]["physics"]
    # a jump inside cell 20 (a jump on a face between two constant cells is already monotone)
    case, w0 = minmod_case(40, lambda x: gen.onestep_conserved(np.where(x < 0.512, 2.0, 1.0), 0.0, 1.0, 1.0, phys))
    _, flags, total = run_limiter_once(orc, case, w0)
    assert total > 0            # troubled in the first stage; limited, it passes the later ones
    # a smooth periodic wave: with M = 0 the cells around its extrema are troubled (TVD clips them),
    # with a large M none is
    wave = lambda x: gen.onestep_conserved(1.0 + 0.2 * np.sin(2 * np.pi * x), 1.0, 1.0, 1.0, phys)
    case, w0 = minmod_case(64, wave, bc="periodic")
    _, flags, total = run_limiter_once(orc, case, w0)
    assert flags[15] or flags[16]      # the maximum sits at x = 0.25 (between cells 15 and 16)
    assert flags[47] or flags[48]      # the minimum at x = 0.75
    assert not flags[30:34].any()      # no cell near the zero crossing at x = 0.5 (monotone there)
    case, w0 = minmod_case(64, wave, bc="periodic", tvb_m=1e4)
    _, flags, total = run_limiter_once(orc, case, w0)
    assert total == 0


def _kxrcf_cfg(orc, order_p, E=64):
    case, _ = gen.case_c0(E=E, order_p=order_p, n_pe=1, mode="sync")
    case["disc"]["limiter"] = 1
    case["disc"]["indicator"] = "kxrcf"
    return orc.Config(case)


def _cell(rho_modes, u, p, gamma=1.4, q=1.0):
    """Modal block [V][M] of a one-step state with the given density modes, constant u and p."""
    rho = np.asarray(rho_modes, dtype=float)
    M = len(rho)
    w = np.zeros((5, M))
    w[0] = rho
    w[1] = rho * u
    w[2] = 0.5 * rho * u * u
    w[2, 0] += p / (gamma - 1.0) + q * rho[0]
    w[2, 1:] += q * rho[1:]
    w[3] = rho
    return w


def _flag(orc, cfg, nbL, we, nbR):
    f = orc.lib().or_indicator(cfg.ref(), orc.vec(nbL.ravel()), orc.vec(we.ravel()), orc.vec(nbR.ravel()), 0, 0)
    assert f in (0, 1)
    return f


@pytest.mark.parametrize("order_p", [1, 2, 3])
@pytest.mark.parametrize("u", [0.7, -0.7])
@pytest.mark.parametrize("target", [0.9, 1.1])
def test_kxrcf_threshold_exponent_and_inflow_face(orc, order_p, u, target):
    """KXRCF (config of the detonation workload): I = |jump at the inflow face| / (h^((N_p+1)/2) max_q |w_e(xi_q)|)
    on rho (and rho E); troubled when I > 1.  The cell has a slope, so the normaliser is the largest value at
    the Gauss nodes, not the mean.  A jump of I = target at the inflow face decides the flag; a jump ten times
    larger at the outflow face changes nothing."""
    E = 64
    h = 1.0 / E
    cfg = _kxrcf_cfg(orc, order_p, E)
    M = order_p + 1
    c0, c1 = 2.0, 0.4
    rho_e = np.zeros(M)
    rho_e[0], rho_e[1] = c0, c1
    xq, _ = np.polynomial.legendre.leggauss(M)
    norm = np.max(np.abs(c0 + c1 * xq))
    we = _cell(rho_e, u, 1.0)
    delta = target * h ** (0.5 * (order_p + 1)) * norm
    inflow_left = u > 0
    trace = c0 - c1 if inflow_left else c0 + c1       # the cell's density at its inflow face
    out_trace = c0 + c1 if inflow_left else c0 - c1
    # neighbours: constant states; the inflow neighbour's density differs by delta at the face, its
    # energy equals the cell's trace there (no rho E jump), the outflow neighbour jumps by 10 delta
    w_in = _cell([trace - delta] + [0.0] * (M - 1), u, 1.0)
    w_out = _cell([out_trace + 10 * delta] + [0.0] * (M - 1), u, 1.0)
    e_trace = np.sum(we[2] * (np.array([(-1.0) ** j for j in range(M)]) if inflow_left else np.ones(M)))
    w_in[2, 0] = e_trace
    w_out[2, 0] = np.sum(we[2] * (np.ones(M) if inflow_left else np.array([(-1.0) ** j for j in range(M)])))
    nbL, nbR = (w_in, w_out) if inflow_left else (w_out, w_in)
    assert _flag(orc, cfg, nbL, we, nbR) == (1 if target > 1 else 0)


@pytest.mark.parametrize("target", [0.9, 1.1])
def test_kxrcf_energy_jump(orc, target):
    """The same test on rho E alone: no density jump, an energy jump of I = target (normalised by the
    largest |rho E| at the Gauss nodes)."""
    order_p, E, u = 2, 64, 0.5
    h = 1.0 / E
    cfg = _kxrcf_cfg(orc, order_p, E)
    M = order_p + 1
    we = _cell([1.5, 0.0, 0.0], u, 1.0)
    norm = abs(we[2, 0])
    delta = target * h ** 1.5 * norm
    nbL = we.copy()
    nbL[2, 0] -= delta
    nbR = we.copy()
    assert _flag(orc, cfg, nbL, we, nbR) == (1 if target > 1 else 0)
