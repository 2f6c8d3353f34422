"""Orbital alignment (the convergence aid at the end of Sec. 2) through the
C ABI against the oracle's SVD-based Procrustes solution."""
import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
from paper_1801_09263_amd import lace  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def unitary(rng, n):
    z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def orthonormal_rows(x):
    q, _ = np.linalg.qr(x.T)
    return np.ascontiguousarray(q.T)


def run_align(cell, new, old, prec=lace.LACE_FP64):
    plan = lace.lace_plan_create([cell], prec)
    n = new.shape[0]
    ws = torch.empty(lace.lace_workspace_size(plan, 0, n, n), dtype=torch.uint8,
                     device="cuda")
    tn = torch.tensor(new, device="cuda")
    to = torch.tensor(old, device="cuda")
    out = torch.empty_like(tn)
    resid = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    lace.lace_align(plan, 0, tn, to, n, out, resid, ws)
    torch.cuda.synchronize()
    plan.close()
    return out.cpu().numpy(), resid.item()


@pytest.fixture(scope="module")
def small():
    inp = synth.make_inputs("plain-ace-24")
    return dict(L=inp["L"], n=inp["n"], miller=inp["miller"]), inp["coeffs"]


def test_align_recovers_rotation(small):
    cell, old = small
    new = unitary(np.random.default_rng(31), old.shape[0]).T @ old
    out, resid = run_align(cell, new, old)
    say(f"rotation: resid {resid:.2e} err {np.abs(out - old).max():.2e}")
    assert resid <= 1e-13
    assert np.abs(out - old).max() <= 1e-12


@pytest.mark.parametrize("noise", [1e-3, 0.3])
def test_align_matches_oracle(small, noise):
    cell, old = small
    rng = np.random.default_rng(32)
    new = orthonormal_rows(unitary(rng, old.shape[0]).T @ old + noise * (
        rng.standard_normal(old.shape) + 1j * rng.standard_normal(old.shape)))
    out, resid = run_align(cell, new, old)
    ref = O.align_orbitals(new, old)
    say(f"noise {noise}: resid {resid:.2e} rel {rel(out, ref):.2e}")
    assert resid <= 1e-12
    assert rel(out, ref) <= 1e-12


def test_align_unrelated_orbital_sets(small):
    """Two unrelated orthonormal sets: the singular values of new^H old are
    small and spread; the iteration still converges to the oracle's U."""
    cell, _ = small
    m = cell["miller"]
    old = synth.random_orbitals(m, cell["L"], 8, synth.rng_for(33))
    new = synth.random_orbitals(m, cell["L"], 8, synth.rng_for(34))
    out, resid = run_align(cell, new, old)
    ref = O.align_orbitals(new, old)
    say(f"unrelated: resid {resid:.2e} rel {rel(out, ref):.2e}")
    assert resid <= 1e-10
    assert rel(out, ref) <= 1e-9


def test_align_full_size_perturbed_localized_orbitals():
    """256 localized orbitals at 120^3 against those of a perturbed outer
    step (centres and widths moved), as in the serving jobs."""
    L, ecut = 23.5, 40.0
    m = synth.miller_sphere(L, ecut)
    rng = synth.rng_for(2, 0, 0, 0, 0)
    pos, wid = synth.gaussian_params(L, 256, 128, rng)
    old = synth.orbitals_from_params(m, L, pos, wid)
    p2, w2 = synth.perturb_gaussian_params(pos, wid, synth.rng_for(2, 0, 0, 1))
    new = synth.orbitals_from_params(m, L, p2, w2)
    # a mixing of the new set, as an eigensolver would return it
    new = unitary(np.random.default_rng(35), 256).T @ new
    out, resid = run_align(dict(L=L, n=120, miller=m), new, old,
                           prec=lace.LACE_FP32)
    ref = O.align_orbitals(new, old)
    say(f"full size: resid {resid:.2e} rel {rel(out, ref):.2e}")
    assert resid <= 1e-12
    assert rel(out, ref) <= 1e-10
    assert np.linalg.norm(out - old) < np.linalg.norm(new - old)


def test_align_rejects_aliased_output(small):
    cell, old = small
    plan = lace.lace_plan_create([cell], lace.LACE_FP64)
    n = old.shape[0]
    ws = torch.empty(lace.lace_workspace_size(plan, 0, n, n), dtype=torch.uint8,
                     device="cuda")
    t = torch.tensor(old, device="cuda")
    with pytest.raises(lace.LaceError):
        lace.lace_align(plan, 0, t, t.clone(), n, t, None, ws)
    plan.close()
