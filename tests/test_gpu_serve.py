"""Served stream on the GPU: requests of both models, all orders and different sizes arrive
while others run; each served result equals the same request solved alone (bitwise, same
precision), and admission waits when the workspace is full."""
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


def small_stream(n=16, rate=None):
    from paper_2501_01747_amd.serve import Request

    reqs = []
    for r in gen.c4_requests(n, rate, e_range=(256, 640), steps_range=(8, 30)):
        reqs.append(Request(r["rid"], r["case"], r["w0"], r["steps"], r["arrival"]))
    return reqs


@pytest.mark.parametrize("precision,graph_steps", [("mixed", 0), ("fp64", 0), ("mixed", 2)])
def test_served_equals_alone(adg, precision, graph_steps):
    """With graph_steps = 2 the rounds replay captured two-step graphs of the batch, captured
    again whenever an admission or a retirement changes its composition."""
    from paper_2501_01747_amd.serve import Server, summarize

    reqs = small_stream()
    foot = [adg.Batch.instance_bytes(r.case) for r in reqs]
    # every request arrives at t = 0 and there is room for about a third of them at once
    b = adg.Batch(8, 1 << 20, sum(foot) // 3, precision=precision)
    srv = Server(b, chunk=6, keep_states=True, graph_steps=graph_steps)
    res = srv.run(reqs)
    b.close()
    s = summarize(res)
    print(f"[serve] {precision} graph {graph_steps} {s} rounds={srv.rounds} max_active={srv.max_active}", flush=True)
    assert s["failed"] == 0 and 1 < srv.max_active < len(reqs)
    assert any(r.admitted > r.arrival for r in res[3:])           # all arrive at once: some wait for space
    for q, r in zip(reqs, res):
        alone = adg.Batch(1, q.case["disc"]["n_elem"], adg.Batch.instance_bytes(q.case), precision=precision)
        sl = alone.add(q.case, q.w0, n_steps=q.steps)
        alone.step(q.steps + 3)
        w = alone.state(sl)
        st, _ = alone.poll()
        alone.close()
        assert st[sl] == q.steps
        np.testing.assert_array_equal(r.state, w, err_msg=f"request {q.rid} ({q.case['name']})")


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_served_against_oracle(adg, orc, precision):
    """One request of every (model, order) of the served stream, served together with continuous
    batching (half of them fit at once, so admissions wait for retirements), each result against
    the FP64 oracle run of the same request: shocks (always FP64) and FP64 ignition to 1e-10,
    mixed-precision ignition to the mixed path's stated 1e-8 per variable."""
    from _parity import check, species_floor, var_errors
    from paper_2501_01747_amd.serve import Request, Server

    mech = gen.c1_mechanism()
    reqs = []
    for k, (kind, P) in enumerate([(kd, p) for p in (1, 2, 3, 4) for kd in ("ignition", "shock")]):
        E = 96 + 16 * k if kind == "ignition" else 256
        steps = 24 + 3 * k
        case, w0 = gen.c4_request(kind, E, P, steps, (2505 << 20) + k, mech=mech, phase=0.4 * k)
        reqs.append(Request(k, case, w0, steps, 0.0))
    foot = [adg.Batch.instance_bytes(r.case) for r in reqs]
    b = adg.Batch(8, 1 << 20, sum(foot) // 2, precision=precision)
    srv = Server(b, chunk=5, keep_states=True)
    res = srv.run(reqs)
    b.close()
    assert all(r.ok for r in res) and any(r.admitted > r.arrival for r in res)
    for q, r in zip(reqs, res):
        ref = orc.run(q.case, q.w0, q.steps)
        err = float(np.max(var_errors(r.state, ref, species_floor(q.case))))
        print(f"[serve-oracle] {precision} {q.case['name']} Np={q.case['disc']['order_p']} "
              f"E={q.case['disc']['n_elem']} steps={q.steps} err {err:.2e}", flush=True)
        if precision == "fp64" or q.case["physics"]["model"] == "onestep":
            check(r.state, ref, q.case, 1e-10, f"request {q.rid}")
        else:
            assert err < 1e-8, (q.rid, err)
