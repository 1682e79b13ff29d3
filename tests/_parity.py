"""Error measures of the GPU parity tests (GPU result against the oracle's, same inputs)."""
import numpy as np


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def pe_interface_elements(case):
    """The elements on both sides of every PE interface (the periodic wrap face included)."""
    E, P = case["disc"]["n_elem"], case["async"]["n_pe"]
    off = case["async"].get("pe_offsets") or [(p * E) // P for p in range(P + 1)]
    periodic = case["disc"].get("bc", "periodic") == "periodic"
    faces = off[:P] if periodic else off[1:P]
    out = set()
    for f in faces:
        out.add((f - 1) % E if periodic else f - 1)
        out.add(f % E)
    return sorted(out)


def element_errors(a, b, elems=None):
    """Largest |difference| of each listed element's modal data over that element's largest |value|."""
    idx = np.arange(a.shape[0]) if elems is None else np.asarray(elems, dtype=int)
    d = np.abs(a[idx] - b[idx]).reshape(len(idx), -1).max(axis=1)
    s = np.abs(b[idx]).reshape(len(idx), -1).max(axis=1)
    return d / s


def var_errors(a, b, floor=1e-6):
    """L2 error of each conserved variable against that variable's own scale: ||rho|| for rho,
    ||rho E|| for the energy, sqrt(||rho|| ||rho E||) for the momentum (near zero in quiescent
    states), and for every partial density its own norm, floored at `floor` ||rho|| (radicals at
    mole fractions of 1e-4 are then checked to their own size, not the mixture's)."""
    V = a.shape[1]
    num = np.linalg.norm((a - b).transpose(1, 0, 2).reshape(V, -1), axis=1)
    nrm = np.linalg.norm(b.transpose(1, 0, 2).reshape(V, -1), axis=1)
    scale = np.maximum(nrm, floor * nrm[0])
    scale[0] = nrm[0]
    scale[1] = np.sqrt(nrm[0] * nrm[2])
    scale[2] = nrm[2]
    return num / scale


def species_floor(case):
    """Smallest scale of a partial density, relative to ||rho||.  With the limiter, w = R v mixes
    every variable at the density's scale, so a partial density carries rounding errors of order
    eps ||rho|| whatever its own size (the one-step product is 1e-6 ||rho|| and less ahead of a
    front); it is checked against 1e-3 ||rho|| there, else against 1e-6 ||rho||."""
    return 1e-3 if case["disc"].get("limiter") else 1e-6


def element_tol(case, tol):
    """Bound of the element-by-element check.  Smooth runs: the parity tolerance itself.  Limited
    runs: 100 x it, since near a front the limiter's nonlinear weights and the flow amplify
    differences of a few ulps of the AT extrapolation element by element (measured: 7e-10 in one
    PE-interface element of the detonation workload after 60 steps, with the relative L2 at 5e-11);
    a mistake at a PE interface shows at 1e-4 and more."""
    return tol * (100.0 if case["disc"].get("limiter") else 1.0)


def check(a, b, case, tol=1e-10, what=""):
    """Relative L2 over the state, each variable against its own scale, and element by element at
    the PE interfaces; returns the worst of the three (the element errors scaled to the tolerance)."""
    r = rel_l2(a, b)
    ve = var_errors(a, b, species_floor(case))
    pe = pe_interface_elements(case)
    ee = element_errors(a, b, pe).max() if pe else 0.0
    etol = element_tol(case, tol)
    worst = max(r, float(ve.max()), float(ee) * tol / etol)
    if worst >= tol:
        print(f"[parity] {what} rel L2 {r:.2e} per variable {np.array2string(ve, precision=2)} "
              f"PE-interface elements {ee:.2e} (bound {etol:.0e})", flush=True)
    assert r < tol and ve.max() < tol and ee < etol, (what, r, ve.max(), ee)
    return worst
