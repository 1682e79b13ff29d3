"""adg_create_noalloc (the solver in the library's static device scratch, for callers that cannot
allocate) against adg_create with a workspace: two calls in a row, the second on a smaller problem,
through the C ABI; bitwise equal states, step counts and flags."""
import numpy as np
import pytest

from workloads import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def adg():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_01747_amd import adg as lib

    return lib


def run(adg, case, w0, steps, noalloc):
    s = adg.Solver(case, noalloc=noalloc)
    s.set_state(w0)
    s.step(steps)
    w = s.state()
    n = s.step_count()
    flags = s.flags() if case["disc"].get("limiter") else None
    s.close()
    return w, n, flags


@pytest.mark.parametrize("kind", ["onestep", "limited", "detailed"])
def test_noalloc_equals_workspace_solver(adg, kind):
    mech = gen.c1_mechanism() if kind == "detailed" else None
    if kind == "onestep":
        cases = [gen.case_c0(E=700, n_pe=7, mode="saa"), gen.case_c0(E=130, n_pe=3, mode="caa")]
    elif kind == "limited":
        cases = [gen.case_shock(512, 3, n_pe=16), gen.case_shock(160, 2, n_pe=5)]
    else:
        cases = [gen.case_c1(E=200, n_pe=8, mech=mech, Lx=0.01 * 200 / 2048),
                 gen.case_c1(E=40, order_p=2, n_pe=4, mech=mech, cfl=0.08, Lx=0.01 * 40 / 2048)]
    for call, (case, w0) in enumerate(cases):
        print(f"[noalloc] {kind} call {call}: E={case['disc']['n_elem']} Np={case['disc']['order_p']}", flush=True)
        steps = 9 + call
        ref, n_ref, f_ref = run(adg, case, w0, steps, noalloc=False)
        got, n_got, f_got = run(adg, case, w0, steps, noalloc=True)
        assert n_got == n_ref == steps
        np.testing.assert_array_equal(got, ref)
        if f_ref is not None:
            assert np.array_equal(f_got[0], f_ref[0]) and f_got[1] == f_ref[1]


def test_noalloc_limits(adg):
    """One static solver per device at a time, and problems beyond the scratch are refused."""
    case, w0 = gen.case_c0(E=100, n_pe=4)
    a = adg.Solver(case, noalloc=True)
    with pytest.raises(adg.AdgError) as ei:
        adg.Solver(case, noalloc=True)
    assert ei.value.code == adg.ADG_ERR_STATE
    a.close()
    b = adg.Solver(case, noalloc=True)   # free again after destroy
    b.close()
    big, _ = gen.case_c0(E=600_000, n_pe=4)
    with pytest.raises(adg.AdgError) as ei:
        adg.Solver(big, noalloc=True)
    assert ei.value.code == adg.ADG_ERR_NOMEM and "static scratch" in str(ei.value)
