"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Tolerances are relative Frobenius norms against the FP64 oracle.  FP64 path:
rounding-order differences only.  FP32 path: pair densities, FFTs and W in
FP32 (unit roundoff 6e-8, grown by ~log2(N_g) FFT stages and the sum over
orbitals) with FP64 energies, M, Cholesky and xi; the exchange energy must
meet 1e-5 relative.
"""
import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
from paper_1801_09263_amd import lace  # noqa: E402
from paper_1801_09263_amd.session import CellSession  # noqa: E402

pytestmark = pytest.mark.gpu

FP64, FP32 = lace.LACE_FP64, lace.LACE_FP32
TOL = {
    FP64: dict(fft=1e-13, w=1e-11, m=1e-11, ex=1e-12, xi=1e-10, ace=1e-11,
               s=1e-12),
    FP32: dict(fft=2e-6, w=1e-5, m=1e-5, ex=1e-5, xi=1e-4, ace=1e-5, s=1e-6),
}
NAMES = {FP64: "fp64", FP32: "fp32"}


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def say(*a):
    print(*a, flush=True)


# ------------------------------------------------------------------ FFT
def brute_dft3(a, sign):
    n = a.shape[-1]
    k = np.arange(n)
    f = np.exp(sign * 2j * np.pi * np.outer(k, k) / n)
    return np.einsum("az,by,cx,...zyx->...abc", f, f, f, a, optimize=True)


def set_schedule(plan, mode):
    """Select an xy schedule (0 pencils, 1 whole plane, 2 half planes) on
    cell 0; False where the whole plane does not fit LDS."""
    ppb = lace.lace_get_tuning(plan, 0)[0]
    try:
        lace.lace_set_tuning(plan, 0, ppb, mode)
    except lace.LaceError:
        assert mode == 1
        return False
    return True


@pytest.mark.parametrize("mode", [0, 1, 2], ids=["pencil", "plane", "half"])
@pytest.mark.parametrize("prec", [FP64, FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("n", [8, 12, 16, 24, 32, 48, 64, 80, 96, 120])
def test_fft3d_against_definition(n, prec, mode):
    say(f"fft3d n={n} prec={NAMES[prec]} mode={mode}")
    cell = dict(L=7.0, n=n, miller=np.zeros((1, 3), np.int32))
    plan = lace.lace_plan_create([cell], prec)
    if not set_schedule(plan, mode):
        plan.close()
        pytest.skip("xy plane does not fit LDS")
    count = 3
    rng = np.random.default_rng(n)
    x = (rng.standard_normal((count, n, n, n))
         + 1j * rng.standard_normal((count, n, n, n)))
    cdt = torch.complex128 if prec == FP64 else torch.complex64
    for direction in (-1, +1):
        t = torch.tensor(x, dtype=cdt, device="cuda")
        lace.lace_fft3d(plan, 0, direction, t, count)
        got = t.cpu().numpy().astype(np.complex128)
        if n <= 12:
            ref = brute_dft3(x, direction)
        elif direction < 0:
            ref = np.fft.fftn(x, axes=(1, 2, 3))
        else:
            ref = np.fft.ifftn(x, axes=(1, 2, 3)) * n ** 3
        assert rel(got, ref) <= TOL[prec]["fft"], (n, direction)
    plan.close()


# ------------------------------------------------------- dense kernels
@pytest.mark.parametrize("n_orb,n_pw", [(8, 2777), (37, 1001), (70, 5003)])
def test_exchange_matrix_gemm(n_orb, n_pw):
    """M = psi^H W for arbitrary inputs (MFMA split-K GEMM), ragged sizes."""
    say(f"gemm psi^H W n_orb={n_orb} n_pw={n_pw}")
    rng = np.random.default_rng(n_orb)
    miller = synth.miller_sphere(40.0, 30.0)[:n_pw]
    cell = dict(L=40.0, n=120, miller=miller)
    s = CellSession(cell, n_orb, FP64, n_vec=n_orb)
    a = rng.standard_normal((n_orb, n_pw)) + 1j * rng.standard_normal((n_orb, n_pw))
    b = rng.standard_normal((n_orb, n_pw)) + 1j * rng.standard_normal((n_orb, n_pw))
    s.psi.copy_(torch.tensor(a))
    s.w.copy_(torch.tensor(b))
    s.build_ace("avg")
    torch.cuda.synchronize()
    ref = np.conj(a) @ b.T
    err = rel(s.m.cpu().numpy(), ref)
    say("  rel err", err)
    assert err <= 1e-13
    assert s.ex_tr.item() == pytest.approx(0.5 * np.trace(ref).real, rel=1e-12)
    s.close()


@pytest.mark.parametrize("n_orb,n_vec,n_pw", [(8, 3, 2777), (37, 70, 1001)])
def test_ace_application_gemms(n_orb, n_vec, n_pw):
    """y = -xi (xi^H x) for arbitrary xi, x (split-K GEMM + tall GEMM)."""
    say(f"apply_ace n_orb={n_orb} n_vec={n_vec} n_pw={n_pw}")
    rng = np.random.default_rng(n_vec)
    miller = synth.miller_sphere(40.0, 30.0)[:n_pw]
    cell = dict(L=40.0, n=120, miller=miller)
    s = CellSession(cell, n_orb, FP64, n_vec=n_vec)
    xi = rng.standard_normal((n_orb, n_pw)) + 1j * rng.standard_normal((n_orb, n_pw))
    x = rng.standard_normal((n_vec, n_pw)) + 1j * rng.standard_normal((n_vec, n_pw))
    s.xi.copy_(torch.tensor(xi))
    y = s.apply_ace(torch.tensor(x, device="cuda")).cpu().numpy()
    err = rel(y, O.apply_ace(xi, x))
    say("  rel err", err)
    assert err <= 1e-13
    s.close()


def test_cholesky_and_projector_on_known_matrix():
    """psi orthonormal, W = -psi A with A Hermitian positive definite:
    M = -A, L = chol(A), xi = W L^{-H}."""
    say("cholesky + projector on a known matrix")
    rng = np.random.default_rng(11)
    n_orb, n_pw = 40, 3001
    miller = synth.miller_sphere(40.0, 30.0)[:n_pw]
    cell = dict(L=40.0, n=120, miller=miller)
    q, _ = np.linalg.qr(rng.standard_normal((n_pw, n_orb))
                        + 1j * rng.standard_normal((n_pw, n_orb)))
    psi = q.T.copy()
    z = rng.standard_normal((n_orb, n_orb)) + 1j * rng.standard_normal((n_orb, n_orb))
    a = z @ z.conj().T + n_orb * np.eye(n_orb)
    w = -(a.T @ psi)                   # column j of W = -sum_k psi_k A_kj
    s = CellSession(cell, n_orb, FP64)
    s.psi.copy_(torch.tensor(psi))
    s.w.copy_(torch.tensor(w))
    s.build_ace("avg")
    torch.cuda.synchronize()
    m = s.m.cpu().numpy()
    say("  M err", rel(m, -a))
    assert rel(m, -a) <= 1e-13
    assert s.info() == 0
    res_l = O.cholesky_neg(O.symmetrize(m))
    xi_ref = O.projector(w, res_l)
    say("  xi err", rel(s.xi.cpu().numpy(), xi_ref))
    assert rel(s.xi.cpu().numpy(), xi_ref) <= 1e-12
    s.close()


# --------------------------------------------------- 24^3 plain ACE (c0)
@pytest.fixture(scope="module")
def c0():
    inp = synth.make_inputs("plain-ace-24")
    res = O.run_path(inp["coeffs"], inp["miller"], inp["L"], inp["n"])
    return inp, res


@pytest.mark.parametrize("prec", [FP64, FP32], ids=["fp64", "fp32"])
def test_plain_ace_24(c0, prec):
    inp, res = c0
    say(f"plain ACE 24^3 N=8 prec={NAMES[prec]}")
    tol = TOL[prec]
    n_orb = inp["coeffs"].shape[0]
    s = CellSession(inp, n_orb, prec, n_vec=4)
    s.set_orbitals(inp["coeffs"])
    s.apply_exchange(0.0)
    torch.cuda.synchronize()
    say("  W rel err", rel(s.w.cpu().numpy(), res["W_pw"]),
        "E_x", s.e_x.item(), res["ex_pairs"])
    assert s.n_kept == n_orb * (n_orb + 1) // 2
    assert rel(s.w.cpu().numpy(), res["W_pw"]) <= tol["w"]
    assert abs(s.e_x.item() - res["ex_pairs"]) <= tol["ex"] * abs(res["ex_pairs"])
    s.build_ace("avg")
    torch.cuda.synchronize()
    say("  M rel err", rel(s.m.cpu().numpy(), res["M"]))
    assert rel(s.m.cpu().numpy(), res["M"]) <= tol["m"]
    assert abs(s.ex_tr.item() - res["ex_trace"]) <= tol["ex"] * abs(res["ex_trace"])
    assert s.info() == 0
    assert rel(s.xi.cpu().numpy(), res["xi"]) <= tol["xi"]
    # ACE on its build set and on random functions
    y = s.apply_ace(s.psi).cpu().numpy()
    assert rel(y, res["W_pw"]) <= tol["ace"]
    rng = np.random.default_rng(5)
    x = (rng.standard_normal((3, s.n_pw)) + 1j * rng.standard_normal((3, s.n_pw)))
    yx = s.apply_ace(torch.tensor(x, device="cuda")).cpu().numpy()
    assert rel(yx, O.apply_ace(res["xi"], x)) <= tol["ace"]
    s.close()


# ----------------------------------- ragged multi-tile case, several sizes
@pytest.mark.parametrize("prec", [FP64, FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("L,n,ecut,n_orb", [(9.0, 16, 6.0, 5),
                                            (12.0, 48, 20.0, 19),
                                            (16.0, 80, 30.0, 7)])
def test_plain_ace_sizes(L, n, ecut, n_orb, prec):
    say(f"plain ACE n={n} N={n_orb} prec={NAMES[prec]}")
    tol = TOL[prec]
    miller = synth.miller_sphere(L, ecut)
    assert np.abs(miller).max() < n / 2
    coeffs = synth.random_orbitals(miller, L, n_orb, synth.rng_for(77, n))
    res = O.run_path(coeffs, miller, L, n)
    cell = dict(L=L, n=n, miller=miller)
    s = CellSession(cell, n_orb, prec)
    s.set_orbitals(coeffs)
    s.apply_exchange(0.0)
    s.build_ace("avg")
    torch.cuda.synchronize()
    assert s.info() == 0
    assert rel(s.w.cpu().numpy(), res["W_pw"]) <= tol["w"]
    assert rel(s.m.cpu().numpy(), res["M"]) <= tol["m"]
    assert rel(s.xi.cpu().numpy(), res["xi"]) <= tol["xi"]
    assert abs(s.e_x.item() - res["ex_pairs"]) <= tol["ex"] * abs(res["ex_pairs"])
    s.close()


# ------------------------------------------- screened (L-ACE) small case
@pytest.fixture(scope="module")
def localized():
    L, n, ecut = 16.0, 32, 15.0
    miller = synth.miller_sphere(L, ecut)
    coeffs = synth.gaussian_orbitals(miller, L, 16, 8, synth.rng_for(90))
    psi = O.orbitals_on_grid(coeffs, miller, L, n)
    S = O.overlap_of_moduli(psi, L)
    return dict(L=L, n=n, miller=miller, coeffs=coeffs, S=S)


@pytest.mark.parametrize("prec", [FP64, FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("s_thr", [2e-3, 5e-3])
def test_screened_lace_small(localized, prec, s_thr):
    loc = localized
    say(f"L-ACE 32^3 N=16 s_thr={s_thr} prec={NAMES[prec]}")
    tol = TOL[prec]
    cell = dict(L=loc["L"], n=loc["n"], miller=loc["miller"])
    s = CellSession(cell, 16, prec, n_vec=16)
    s.set_orbitals(loc["coeffs"])
    S = s.screen().cpu().numpy()
    assert rel(S, loc["S"]) <= tol["s"]
    pairs = O.kept_pairs(loc["S"], s_thr)
    # screening decision: identical unless an S_ij sits within rounding of
    # the threshold
    margin = np.abs(loc["S"] - s_thr).min() / s_thr
    s.apply_exchange(s_thr)
    if margin > 1e-6:
        assert s.n_kept == len(pairs)
    # parity of W', M', xi with the oracle's own pair list
    s.apply_exchange(s_thr, pairs=np.array(pairs))
    assert s.n_kept == len(pairs)
    for sym in ("avg", "upper", "lower"):
        res = O.run_path(loc["coeffs"], loc["miller"], loc["L"], loc["n"],
                         pairs=pairs, sym=sym)
        s.build_ace(sym)
        torch.cuda.synchronize()
        assert s.info() == 0
        assert rel(s.w.cpu().numpy(), res["W_pw"]) <= tol["w"]
        assert rel(s.m.cpu().numpy(), res["M"]) <= tol["m"]
        assert rel(s.xi.cpu().numpy(), res["xi"]) <= tol["xi"]
        assert abs(s.e_x.item() - res["ex_pairs"]) <= tol["ex"] * abs(
            res["ex_pairs"])
    s.close()


def test_cholesky_failure_sets_info(c0):
    """A non-positive-definite -M_s (here: W replaced by +W, so M is
    positive) is reported through the info word, not by a fault."""
    inp, res = c0
    say("cholesky failure path")
    s = CellSession(inp, 8, FP64)
    s.set_orbitals(inp["coeffs"])
    s.w.copy_(torch.tensor(-res["W_pw"], device="cuda"))
    s.build_ace("avg")
    torch.cuda.synchronize()
    assert s.info() == 1
    s.close()


def test_explicit_pairs_checked(c0):
    """Host pair lists are checked by the binding (i > j, out of range,
    repeats).  Device lists reach the library unchecked: the device drops
    the bad entries and runs a repeat once, which n_kept shows, and W is the
    oracle's for the pairs that remain."""
    inp, _ = c0
    s = CellSession(inp, 8, FP64)
    s.set_orbitals(inp["coeffs"])
    for bad in ([[1, 0]], [[0, 8]], [[0, 1], [0, 1]], [[-1, 2]]):
        with pytest.raises(ValueError):
            s.apply_exchange(0.0, pairs=np.array(bad))
    pi = torch.tensor([0, 1, 0, 0, 3, -1], dtype=torch.int32, device="cuda")
    pj = torch.tensor([1, 0, 1, 8, 3, 2], dtype=torch.int32, device="cuda")
    s.apply_exchange(0.0, pairs=(pi, pj))
    torch.cuda.synchronize()
    assert s.n_kept == 2
    psi = O.orbitals_on_grid(inp["coeffs"], inp["miller"], inp["L"], inp["n"])
    w_pw = O.grid_to_pw(O.apply_exchange(psi, O.coulomb_kernel(inp["L"], inp["n"]),
                                         [(0, 1), (3, 3)]), inp["miller"], inp["L"])
    assert rel(s.w.cpu().numpy(), w_pw) <= TOL[FP64]["w"]
    with pytest.raises(lace.LaceError):
        s.apply_exchange(1.5)
    s.close()


@pytest.mark.parametrize("prec", [FP32, lace.LACE_FP32_GAMMA],
                         ids=["fp32", "fp32g"])
def test_argument_errors(prec):
    """Short workspaces, thresholds outside [0, 1), a cell that does not
    exist and an empty orbital set are rejected before any device work; the
    session stays usable and then gives the oracle's W (real orbitals, so
    that both the complex and the real-orbital plans apply)."""
    L, n, n_orb = 10.0, 24, 8
    miller = synth.miller_sphere(L, 15.0)
    coeffs = synth.virtual_orbitals(
        miller, L, np.zeros((0, miller.shape[0]), complex), n_orb,
        synth.rng_for(82, n))
    res = O.run_path(coeffs, miller, L, n)
    inp = dict(L=L, n=n, miller=miller, coeffs=coeffs)
    s = CellSession(inp, n_orb, prec, n_vec=4)
    s.set_orbitals(inp["coeffs"])
    short = s.ws[: s.ws.numel() // 2]

    def code_of(call):
        with pytest.raises(lace.LaceError) as ei:
            call()
        return ei.value.code

    y = torch.empty((4, s.n_pw), dtype=torch.complex128, device="cuda")
    assert code_of(lambda: lace.lace_apply_exchange(
        s.plan, 0, s.psi, n_orb, 0.0, None, s.w, s.e_x, short)) == lace.LACE_ENOMEM
    assert code_of(lambda: lace.lace_build_ace(
        s.plan, 0, s.psi, s.w, n_orb, "avg", s.xi, s.m, s.ex_tr, short)) == lace.LACE_ENOMEM
    assert code_of(lambda: lace.lace_apply_ace(
        s.plan, 0, s.xi, n_orb, s.psi[:4], 4, y, short)) == lace.LACE_ENOMEM
    assert code_of(lambda: lace.lace_screen(
        s.plan, 0, s.psi, n_orb, s.s, short)) == lace.LACE_ENOMEM
    for bad in (-0.1, 1.0, float("nan")):
        assert code_of(lambda: s.apply_exchange(bad)) == lace.LACE_EINVAL
    assert code_of(lambda: lace.lace_apply_exchange(
        s.plan, 1, s.psi, n_orb, 0.0, None, s.w, s.e_x, s.ws)) == lace.LACE_EINVAL
    assert code_of(lambda: lace.lace_apply_exchange(
        s.plan, 0, s.psi, 0, 0.0, None, s.w, s.e_x, s.ws)) == lace.LACE_EINVAL
    # after the rejections the same session still computes the right W
    s.apply_exchange(0.0)
    torch.cuda.synchronize()
    assert rel(s.w.cpu().numpy(), res["W_pw"]) <= TOL[FP32]["w"]
    s.close()


def test_deterministic_repeat(c0):
    """Same inputs, same schedule: bitwise identical W and E_x."""
    inp, _ = c0
    s = CellSession(inp, 8, FP32)
    s.set_orbitals(inp["coeffs"])
    s.apply_exchange(0.0)
    w1, e1 = s.w.clone(), s.e_x.clone()
    s.apply_exchange(0.0)
    assert torch.equal(w1, s.w) and torch.equal(e1, s.e_x)
    s.close()


# ----------------------------------------- real (Gamma-point) orbitals
FP64G, FP32G = lace.LACE_FP64_GAMMA, lace.LACE_FP32_GAMMA
TOL[FP64G] = TOL[FP64]
TOL[FP32G] = TOL[FP32]


@pytest.mark.parametrize("prec", [FP64G, FP32G], ids=["fp64g", "fp32g"])
@pytest.mark.parametrize("s_thr,n_orb", [(0.0, 16), (5e-3, 16), (2e-3, 15)])
def test_gamma_packed_real_orbitals(prec, s_thr, n_orb):
    """Real orbitals with two pair densities per complex transform (and an
    odd orbital count: one orbital transformed alone) against the oracle,
    which treats them as general complex orbitals."""
    say(f"gamma packing n_orb={n_orb} s_thr={s_thr} prec={prec}")
    tol = TOL[prec]
    L, n, ecut = 16.0, 32, 15.0
    miller = synth.miller_sphere(L, ecut)
    coeffs = synth.gaussian_orbitals(miller, L, n_orb, 8, synth.rng_for(90))
    psi = O.orbitals_on_grid(coeffs, miller, L, n)
    S = O.overlap_of_moduli(psi, L)
    pairs = O.kept_pairs(S, s_thr)
    cell = dict(L=L, n=n, miller=miller)
    s = CellSession(cell, n_orb, prec, n_vec=n_orb)
    s.set_orbitals(coeffs)
    assert s.check_real() <= 1e-14
    assert rel(s.screen().cpu().numpy(), S) <= tol["s"]
    s.apply_exchange(s_thr, pairs=np.array(pairs))
    assert s.n_kept == len(pairs)
    for sym in ("avg", "upper", "lower"):
        res = O.run_path(coeffs, miller, L, n, pairs=pairs, sym=sym)
        s.build_ace(sym)
        torch.cuda.synchronize()
        assert s.info() == 0
        assert rel(s.w.cpu().numpy(), res["W_pw"]) <= tol["w"]
        assert rel(s.m.cpu().numpy(), res["M"]) <= tol["m"]
        assert rel(s.xi.cpu().numpy(), res["xi"]) <= tol["xi"]
        assert abs(s.e_x.item() - res["ex_pairs"]) <= tol["ex"] * abs(
            res["ex_pairs"])
    s.close()


def test_gamma_check_flags_complex_orbitals(c0):
    inp, _ = c0
    s = CellSession(inp, 8, FP32G)
    s.set_orbitals(inp["coeffs"])
    dev = s.check_real()
    say("  deviation of random complex orbitals", dev)
    assert dev > 0.5
    s.close()


def test_gamma_plan_needs_symmetric_sphere():
    m = synth.miller_sphere(10.0, 15.0)
    half = m[(m[:, 2] > 0) | ((m[:, 2] == 0) & (m[:, 1] > 0))]
    with pytest.raises(lace.LaceError) as ei:
        lace.lace_plan_create([dict(L=10.0, n=24, miller=half)], FP32G)
    assert ei.value.code == lace.LACE_EINVAL


# ------------------------------- the three xy schedules of the pair passes
@pytest.mark.parametrize("mode", [0, 1, 2], ids=["pencil", "plane", "half"])
@pytest.mark.parametrize("prec", [FP64, FP32, FP64G, FP32G],
                         ids=["fp64", "fp32", "fp64g", "fp32g"])
@pytest.mark.parametrize("L,n,ecut,n_orb", [(10.0, 24, 15.0, 7),
                                            (12.0, 48, 20.0, 11)])
def test_pair_passes_every_schedule(L, n, ecut, n_orb, prec, mode):
    """Pencil, whole-plane and half-plane xy passes, on complex and on
    packed real orbitals (odd count), give the oracle's W and E_x."""
    say(f"schedule mode={mode} n={n} N={n_orb} prec={prec}")
    tol = TOL[prec]
    miller = synth.miller_sphere(L, ecut)
    coeffs = synth.gaussian_orbitals(miller, L, n_orb, (n_orb + 1) // 2,
                                     synth.rng_for(78, n))
    res = O.run_path(coeffs, miller, L, n)
    s = CellSession(dict(L=L, n=n, miller=miller), n_orb, prec)
    assert set_schedule(s.plan, mode)
    s.set_orbitals(coeffs)
    s.apply_exchange(0.0)
    torch.cuda.synchronize()
    assert rel(s.w.cpu().numpy(), res["W_pw"]) <= tol["w"]
    assert abs(s.e_x.item() - res["ex_pairs"]) <= tol["ex"] * abs(
        res["ex_pairs"])
    s.close()


# ------------------------------------ every supported grid size, pair passes
_EVERY_SIZE = {}


def _every_size_case(n):
    """Cell of L = n/2 bohr, Ecut 4.5 Ha (sphere radius about n/4 grid
    points), five real orthonormal orbitals; the oracle's plain-ACE path."""
    if n not in _EVERY_SIZE:
        L = n / 2.0
        miller = synth.miller_sphere(L, 4.5)
        assert np.abs(miller).max() < n / 2
        coeffs = synth.virtual_orbitals(
            miller, L, np.zeros((0, miller.shape[0]), complex), 5,
            synth.rng_for(79, n))
        _EVERY_SIZE[n] = (L, miller, coeffs, O.run_path(coeffs, miller, L, n))
    return _EVERY_SIZE[n]


@pytest.mark.parametrize("sched", ["auto", "half"])
@pytest.mark.parametrize("prec", [FP32G, FP32, FP64G],
                         ids=["fp32g", "fp32", "fp64g"])
@pytest.mark.parametrize("n", [8, 12, 16, 24, 32, 48, 64, 80, 96, 120])
def test_pair_pipeline_every_grid_size(n, prec, sched):
    """Every supported grid through the pair passes against the oracle:
    single-stage radix plans (8, 12), two-stage plans with the prime-factor
    radices (48 = 4 x 12, 60 = 4 x 15, 80 = 8 x 10, 96 = 8 x 12,
    120 = 8 x 15), and the z pass whose middle stage runs in registers;
    complex and packed real orbitals (an odd count).  "half" forces the
    half-plane schedule, whose forward xy pass splits the plane in time and
    whose z pass combines the halves over paired tiles, at every size."""
    L, miller, coeffs, res = _every_size_case(n)
    say(f"every size n={n} prec={prec} sched={sched}")
    tol = TOL[prec]
    s = CellSession(dict(L=L, n=n, miller=miller), coeffs.shape[0], prec)
    if sched == "half":
        assert set_schedule(s.plan, 2)
    s.set_orbitals(coeffs)
    s.apply_exchange(0.0)
    torch.cuda.synchronize()
    assert rel(s.w.cpu().numpy(), res["W_pw"]) <= tol["w"]
    assert abs(s.e_x.item() - res["ex_pairs"]) <= tol["ex"] * abs(
        res["ex_pairs"])
    s.close()


@pytest.mark.parametrize("variant", [(1, 0), (2, 0), (0, 1), (2, 1)],
                         ids=["ztile-half", "ztile-twice", "radix-rev",
                              "ztile-twice-radix-rev"])
@pytest.mark.parametrize("sched", [0, 1, 2], ids=["pencil", "plane", "half"])
@pytest.mark.parametrize("prec", [FP32G, FP64], ids=["fp32g", "fp64"])
@pytest.mark.parametrize("n", [12, 24, 48, 96, 120])
def test_pair_pipeline_tuning_variants(n, prec, sched, variant):
    """The autotuner's other instantiations against the oracle: the z pass
    with tiles half and twice as wide (where the plane divides into them)
    and every transform with its radices in reverse order (60 = 15 x 4,
    120 = 15 x 8, ...), under each xy schedule."""
    zt, ro = variant
    L, miller, coeffs, res = _every_size_case(n)
    say(f"tuning variant n={n} prec={prec} sched={sched} z_tile={zt} radix={ro}")
    tol = TOL[prec]
    s = CellSession(dict(L=L, n=n, miller=miller), coeffs.shape[0], prec)
    ppb = lace.lace_get_tuning(s.plan, 0)[0]
    try:
        lace.lace_set_tuning(s.plan, 0, ppb, sched, zt, ro)
    except lace.LaceError:
        assert sched == 1    # the whole plane does not fit LDS
        s.close()
        return
    s.set_orbitals(coeffs)
    s.apply_exchange(0.0)
    torch.cuda.synchronize()
    assert rel(s.w.cpu().numpy(), res["W_pw"]) <= tol["w"]
    assert abs(s.e_x.item() - res["ex_pairs"]) <= tol["ex"] * abs(
        res["ex_pairs"])
    s.close()


# ---------------------- screening product over several (ragged) tiles
@pytest.mark.parametrize("prec", [FP64, FP32, FP64G, FP32G],
                         ids=["fp64", "fp32", "fp64g", "fp32g"])
def test_screening_matrix_ragged_tiles(prec):
    """S = dV |psi|^T |psi| with 150 orbitals: three 64-wide tiles per side,
    the last one ragged, of which only those on and above the diagonal are
    computed and the rest mirrored; complex and real grids."""
    L, n, n_orb = 10.0, 24, 150
    miller = synth.miller_sphere(L, 15.0)
    rng = synth.rng_for(81, n)
    if prec in (FP64G, FP32G):
        coeffs = synth.virtual_orbitals(
            miller, L, np.zeros((0, miller.shape[0]), complex), n_orb, rng)
    else:
        coeffs = synth.random_orbitals(miller, L, n_orb, rng)
    psi = O.orbitals_on_grid(coeffs, miller, L, n)
    ref = O.overlap_of_moduli(psi, L)
    say(f"screening n_orb={n_orb} prec={prec}")
    sess = CellSession(dict(L=L, n=n, miller=miller), n_orb, prec)
    sess.set_orbitals(coeffs)
    got = sess.screen().cpu().numpy()
    torch.cuda.synchronize()
    sess.close()
    assert np.array_equal(got, got.T)
    assert rel(got, ref) <= TOL[prec]["s"]


# ------------------------- two-stream batch pipeline = one stream, bitwise
@pytest.mark.parametrize("prec", [FP32, FP32G, FP64G], ids=["fp32", "fp32g", "fp64g"])
def test_overlapped_batches_match_one_stream(prec):
    """An exchange call overlaps consecutive batches on two internal streams
    (pass C ordered across them by events); with the pass profiler on it runs
    every launch on the caller's stream.  W and E_x agree bitwise."""
    say(f"overlap vs one stream prec={prec}")
    L, n, ecut, n_orb = 12.0, 48, 20.0, 26
    miller = synth.miller_sphere(L, ecut)
    coeffs = synth.gaussian_orbitals(miller, L, n_orb, 13, synth.rng_for(79))
    s = CellSession(dict(L=L, n=n, miller=miller), n_orb, prec)
    lace.lace_set_tuning(s.plan, 0, 8, 2)     # many small batches
    s.set_orbitals(coeffs)
    s.apply_exchange(2e-3)
    torch.cuda.synchronize()
    w_ov, e_ov = s.w.clone(), s.e_x.clone()
    lace.lace_profile_enable(s.plan, True)
    s.apply_exchange(2e-3)
    torch.cuda.synchronize()
    prof = lace.lace_profile_read(s.plan)
    lace.lace_profile_enable(s.plan, False)
    assert prof["launches"][0] > 8
    assert torch.equal(w_ov, s.w) and torch.equal(e_ov, s.e_x)
    # and a second overlapped call reproduces the first
    s.apply_exchange(2e-3)
    torch.cuda.synchronize()
    assert torch.equal(w_ov, s.w) and torch.equal(e_ov, s.e_x)
    s.close()


# --------------------------------------------------------------- edge cases
@pytest.mark.parametrize("prec", [FP64, FP64G], ids=["fp64", "fp64g"])
@pytest.mark.parametrize("n_orb", [1, 2, 3])
def test_few_orbitals(c0, prec, n_orb):
    """One, two and three orbitals: a lone diagonal pair, a packed slot with
    a single pair left over."""
    inp, _ = c0
    coeffs = synth.gaussian_orbitals(inp["miller"], inp["L"], n_orb,
                                     max(1, n_orb - 1), synth.rng_for(60, n_orb))
    res = O.run_path(coeffs, inp["miller"], inp["L"], inp["n"])
    s = CellSession(inp, n_orb, prec)
    s.set_orbitals(coeffs)
    s.apply_exchange(0.0)
    s.build_ace("avg")
    torch.cuda.synchronize()
    assert s.n_kept == n_orb * (n_orb + 1) // 2
    assert s.info() == 0
    assert rel(s.w.cpu().numpy(), res["W_pw"]) <= 1e-11
    assert rel(s.xi.cpu().numpy(), res["xi"]) <= 1e-10
    assert abs(s.e_x.item() - res["ex_pairs"]) <= 1e-12 * abs(res["ex_pairs"])
    s.close()


@pytest.mark.parametrize("prec", [FP32, FP32G], ids=["fp32", "fp32g"])
def test_threshold_keeping_only_diagonal_pairs(localized, prec):
    """S_ii = 1 and every S_ij < 1 off the diagonal: a threshold just below 1
    keeps exactly the diagonal pairs."""
    inp = localized
    nb = inp["coeffs"].shape[0]
    s_thr = 0.999
    assert (inp["S"][~np.eye(nb, dtype=bool)] < s_thr).all()
    res = O.run_path(inp["coeffs"], inp["miller"], inp["L"], inp["n"],
                     pairs=[(i, i) for i in range(nb)])
    s = CellSession(dict(L=inp["L"], n=inp["n"], miller=inp["miller"]), nb, prec)
    s.set_orbitals(inp["coeffs"])
    s.apply_exchange(s_thr)
    torch.cuda.synchronize()
    assert s.n_kept == nb
    assert rel(s.w.cpu().numpy(), res["W_pw"]) <= TOL[prec]["w"]
    assert abs(s.e_x.item() - res["ex_pairs"]) <= TOL[prec]["ex"] * abs(
        res["ex_pairs"])
    s.close()


@pytest.mark.parametrize("prec", [FP32, FP32G], ids=["fp32", "fp32g"])
def test_empty_pair_list(c0, prec):
    """An explicit empty pair list runs no pair: W = 0 and E_x = 0."""
    inp, _ = c0
    s = CellSession(inp, 8, prec)
    s.set_orbitals(inp["coeffs"])
    s.w.fill_(1.0)
    s.e_x.fill_(1.0)
    s.apply_exchange(0.0, pairs=np.zeros((0, 2), np.int32))
    torch.cuda.synchronize()
    assert s.n_kept == 0
    assert float(s.w.abs().max()) == 0.0 and s.e_x.item() == 0.0
    s.close()


# ---------------------------------------- screened (HSE-type) interaction
@pytest.mark.parametrize("prec", [FP64, FP32, FP64G, FP32G],
                         ids=["fp64", "fp32", "fp64g", "fp32g"])
def test_screened_interaction(localized, prec):
    """omega > 0 in the cell: the short-range erfc(omega r) / r kernel
    (HSE's omega = 0.106 bohr^-1), screened pairs, whole ACE build."""
    inp = localized
    omega, s_thr = 0.106, 2e-3
    tol = TOL[prec]
    res = O.run_path(inp["coeffs"], inp["miller"], inp["L"], inp["n"],
                     s_thr=s_thr, omega=omega)
    cell = dict(L=inp["L"], n=inp["n"], miller=inp["miller"], omega=omega)
    nb = inp["coeffs"].shape[0]
    s = CellSession(cell, nb, prec)
    s.set_orbitals(inp["coeffs"])
    s.apply_exchange(s_thr, pairs=np.array(res["pairs"]))
    s.build_ace("avg")
    torch.cuda.synchronize()
    assert s.info() == 0
    assert rel(s.w.cpu().numpy(), res["W_pw"]) <= tol["w"]
    assert rel(s.xi.cpu().numpy(), res["xi"]) <= tol["xi"]
    assert abs(s.e_x.item() - res["ex_pairs"]) <= tol["ex"] * abs(res["ex_pairs"])
    s.close()


def test_negative_omega_rejected(localized):
    cell = dict(L=localized["L"], n=localized["n"], miller=localized["miller"],
                omega=-1.0)
    with pytest.raises(lace.LaceError):
        lace.lace_plan_create([cell], FP32)
