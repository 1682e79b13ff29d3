"""Host-side parts of bench.py (no GPU): the one-GPU refusal and the algorithmic units the
roofline divides by."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_euler_stage_bytes():
    """Stage 1 reads w^(s) and writes (16 B per scalar DOF), stages 2 and 3 also read w^n
    (24 B): 64/3 B per DOF per launch, plus one flag byte per element with the limiter."""
    import bench
    from workloads import gen

    case, _ = gen.case_c0(E=512)
    dof = 512 * 3 * 5
    assert gen.dof(case) == dof
    assert abs(bench.euler_stage_bytes(case) - dof * 64.0 / 3.0) < 1e-6
    case2, _ = gen.case_c2(E=256, order_p=3, length=8.0, shock_x=1.0, n_pe=4)
    dof2 = 256 * 4 * 5
    assert abs(bench.euler_stage_bytes(case2) - (dof2 * 64.0 / 3.0 + 256)) < 1e-6


def test_detailed_stage_flops_of_the_ignition_workload():
    """The per-element operation count (Sec. 4 formula in bench.detailed_stage_flops) for
    N_s = 9, N_r = 21, N_p = 3, summed over 2048 elements."""
    import bench

    case, _ = bench.workload("c1")
    ns, nr, M = 9, 21, 4
    V = 3 + ns
    point = 80 * ns + (10 + 4 * ns) + (30 + 8 * ns) + (4 + ns)
    chem = 14 * ns + 14 * nr + 2 * nr * ns
    elem = 2 * M * (M + 2) * V + 4 * M * M * V + 2 * M * M * (V + ns) + 8 * M * V
    face = 8 * V + 8
    per_elem = (M + 2) * point + M * chem + elem + face
    assert bench.detailed_stage_flops(case) == 2048.0 * per_elem
    assert 22.0e6 < bench.detailed_stage_flops(case) < 23.0e6
