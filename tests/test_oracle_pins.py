"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test states what it pins.  None re-types an oracle formula: brute-force
DFTs, closed forms of Gaussian and plane-wave integrals, lattice-point
counts and operator identities are written independently here.
"""
import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# ----------------------------------------------------------------- helpers
def dft_matrix(n, sign):
    k = np.arange(n)
    return np.exp(sign * 2j * np.pi * np.outer(k, k) / n)


def brute_dft3(a, sign):
    """Unscaled 3D DFT by dense matrices along each axis."""
    n = a.shape[0]
    f = dft_matrix(n, sign)
    return np.einsum("az,by,cx,zyx->abc", f, f, f, a, optimize=True)


def signed(k, n):
    return np.where(k < (n + 1) // 2, k, k - n)


def kernel_direct(L, n, rc):
    """v(G) = 4 pi (1 - cos(|G| Rc)) / |G|^2, v(0) = 2 pi Rc^2 at each
    integer grid frequency (the cosine form, written out point by point)."""
    v = np.empty((n, n, n))
    for a in range(n):
        for b in range(n):
            for c in range(n):
                g = 2 * np.pi / L * np.array(
                    [signed(c, n), signed(b, n), signed(a, n)], dtype=float)
                gg = np.sqrt(g @ g)
                v[a, b, c] = (2 * np.pi * rc * rc if gg == 0 else
                              4 * np.pi * (1 - np.cos(gg * rc)) / gg ** 2)
    return v


def gaussian_coeffs(miller, L, center, sigma):
    g = 2 * np.pi / L * miller.astype(float)
    c = np.exp(-0.5 * np.sum(g * g, 1) * sigma ** 2) * np.exp(-1j * g @ center)
    return c / np.sqrt(np.vdot(c, c).real)


def gauss_self_coulomb(tau, rc):
    """Truncated-Coulomb self-energy of a normalized 3D Gaussian density
    (2 pi tau^2)^{-3/2} exp(-r^2 / (2 tau^2)) with kernel 1/r for r < rc:
    the separation r - r' is Gaussian with variance 2 tau^2 per axis, and
    integral_0^rc 4 pi u^2 (1/u) p(u) du gives the closed form below."""
    return (1.0 - np.exp(-rc * rc / (4 * tau * tau))) / (tau * np.sqrt(np.pi))


@pytest.fixture(scope="module")
def c0():
    inp = synth.make_inputs("plain-ace-24")
    res = O.run_path(inp["coeffs"], inp["miller"], inp["L"], inp["n"],
                     want_grid=True)
    return inp, res


@pytest.fixture(scope="module")
def localized():
    """Small localized case: 16 Gaussians on 8 centres in a 16 bohr cell."""
    L, n, ecut = 16.0, 32, 15.0
    miller = synth.miller_sphere(L, ecut)
    rng = synth.rng_for(90, 0, 0, 0, 0)
    coeffs = synth.gaussian_orbitals(miller, L, 16, 8, rng)
    psi = O.orbitals_on_grid(coeffs, miller, L, n)
    v = O.coulomb_kernel(L, n)
    s = O.overlap_of_moduli(psi, L)
    return dict(L=L, n=n, miller=miller, coeffs=coeffs, psi=psi, v=v, S=s)


# ------------------------------------------------------------ T0 the basis
def test_sphere_lattice_counts():
    """Lattice points with |m|^2 <= R^2 in a ball: 7 (R^2 = 1), 19 (2),
    27 (3), 33 (4), 57 (5)."""
    L = 2 * np.pi   # G = m
    for r2, count in ((1, 7), (2, 19), (3, 27), (4, 33), (5, 57)):
        assert len(O.sphere_miller(L, 0.5 * r2)) == count


def test_generator_sphere_matches_oracle_basis():
    for L, ecut in ((10.0, 15.0), (12.0, 40.0)):
        gen = synth.miller_sphere(L, ecut)
        assert {tuple(m) for m in gen} == O.sphere_miller(L, ecut)
        assert len(gen) == len(set(map(tuple, gen)))


# ---------------------------------------------------------- T1 transforms
@pytest.mark.parametrize("n,L,ecut", [(4, 4.0, 0.6), (5, 5.0, 1.0),
                                      (6, 6.0, 1.5), (8, 8.0, 2.0),
                                      (10, 10.0, 2.2), (12, 9.0, 3.0)])
def test_orbitals_and_back_vs_brute_dft(n, L, ecut):
    miller = synth.miller_sphere(L, ecut)
    assert np.abs(miller).max() < n / 2
    rng = np.random.default_rng(n)
    c = rng.standard_normal((2, len(miller))) + 1j * rng.standard_normal(
        (2, len(miller)))
    psi = O.orbitals_on_grid(c, miller, L, n)
    # direct plane-wave sum at each grid point r_p = L p / n
    p = np.arange(n)
    pz, py, px = np.meshgrid(p, p, p, indexing="ij")
    for j in range(2):
        ref = np.zeros((n, n, n), complex)
        for m, cm in zip(miller, c[j]):
            ref += cm * np.exp(2j * np.pi * (m[0] * px + m[1] * py + m[2] * pz)
                               / n)
        ref /= np.sqrt(L ** 3)
        assert np.abs(psi[j] - ref).max() <= 1e-13 * np.abs(ref).max()
    # and back: <G_m|psi_j> recovers the coefficients (Parseval on the grid)
    back = O.grid_to_pw(psi, miller, L)
    assert np.abs(back - c).max() <= 1e-13 * np.abs(c).max()


@pytest.mark.parametrize("n", [3, 4, 5, 6])
def test_pair_potential_vs_brute_dft(n):
    L, rc = 7.0, 3.5
    rng = np.random.default_rng(10 + n)
    a = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
    b = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
    v = O.coulomb_kernel(L, n, rc)
    assert np.allclose(v, kernel_direct(L, n, rc), rtol=1e-14, atol=1e-14)
    rho = np.conj(a) * b
    ref = brute_dft3(kernel_direct(L, n, rc) * brute_dft3(rho, -1), +1) / n**3
    got = O.pair_potential(a, b, v)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


# --------------------------------------------------------------- T2 kernel
def test_kernel_table_properties(c0):
    inp, _ = c0
    L, n = inp["L"], inp["n"]
    rc = L / 2
    v = O.coulomb_kernel(L, n)
    assert v[0, 0, 0] == pytest.approx(2 * np.pi * rc * rc, rel=1e-15)
    # G -> 0 limit of 4 pi (1 - cos G Rc)/G^2 is 2 pi Rc^2
    g = 1e-5
    lim = 8 * np.pi * np.sin(0.5 * g * rc) ** 2 / g ** 2
    assert lim == pytest.approx(2 * np.pi * rc * rc, rel=1e-9)
    assert (v >= 0).all()
    # exact zeros where |G| Rc = pi |m| is a multiple of 2 pi: |m| even
    f = signed(np.arange(n), n)
    mz, my, mx = np.meshgrid(f, f, f, indexing="ij")
    m2 = mx * mx + my * my + mz * mz
    root = np.sqrt(m2)
    even = (np.abs(root - np.round(root)) < 1e-12) & (np.round(root) % 2 == 0) \
        & (m2 > 0)
    assert even.sum() > 0
    assert np.abs(v[even]).max() <= 1e-14 * v.max()
    assert (v[~even] > 0).all()
    # the cancellation-free form agrees with the cosine form
    assert np.allclose(v, kernel_direct(L, n, rc), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n", [8, 12, 60, 120])
@pytest.mark.parametrize("omega", [0.0, 0.2])
def test_kernel_table_octant_determines_it(n, omega):
    """In a cubic cell v depends on |G| only, so the table is unchanged,
    bit for bit, under k -> n - k along each axis: the octant
    0 <= kx, ky, kz <= n/2, (n/2 + 1)^3 values, determines the whole table
    (the device keeps only that octant)."""
    v = O.coulomb_kernel(9.0, n, omega=omega)
    fold = np.minimum(np.arange(n), n - np.arange(n))
    assert fold.max() == n // 2
    octant = v[: n // 2 + 1, : n // 2 + 1, : n // 2 + 1]
    rebuilt = octant[np.ix_(fold, fold, fold)]
    assert np.array_equal(rebuilt, v)
    assert np.array_equal(rebuilt.astype(np.float32), v.astype(np.float32))


# --------------------------------------------------- T3 plane-wave orbitals
def test_plane_wave_orbitals_closed_form():
    """psi_j = Omega^{-1/2} exp(i G_j r): V_ij = v(G_j - G_i) rho_ij, so
    K psi_j = -(1/Omega) sum_i v(G_j - G_i) psi_j and M is diagonal with
    M_jj = -(1/Omega) sum_i v(G_j - G_i), frequency differences folded onto
    the grid."""
    L, n, ecut = 8.0, 12, 4.0
    miller = synth.miller_sphere(L, ecut)
    rng = np.random.default_rng(3)
    pick = rng.choice(len(miller), size=5, replace=False)
    coeffs = np.zeros((5, len(miller)), complex)
    coeffs[np.arange(5), pick] = 1.0
    res = O.run_path(coeffs, miller, L, n)
    omega = L ** 3
    rc = L / 2
    m = miller[pick]
    expect = np.zeros(5)
    for j in range(5):
        for i in range(5):
            d = signed(np.mod(m[j] - m[i], n), n)
            gg = 2 * np.pi / L * np.sqrt(float(d @ d))
            vv = (2 * np.pi * rc * rc if gg == 0 else
                  4 * np.pi * (1 - np.cos(gg * rc)) / gg ** 2)
            expect[j] -= vv / omega
    assert np.abs(res["M"] - np.diag(expect)).max() <= 1e-13 * np.abs(
        expect).max()
    assert res["ex_trace"] == pytest.approx(0.5 * expect.sum(), rel=1e-13)
    assert res["ex_pairs"] == pytest.approx(0.5 * expect.sum(), rel=1e-13)


# ---------------------------------------------------- T4 unitary invariance
def test_unitary_invariance(c0):
    inp, res = c0
    rng = np.random.default_rng(4)
    nb = inp["coeffs"].shape[0]
    z = rng.standard_normal((nb, nb)) + 1j * rng.standard_normal((nb, nb))
    u, _ = np.linalg.qr(z)
    rot = u.T @ inp["coeffs"]            # orbital b = sum_a c_a U_ab
    r2 = O.run_path(rot, inp["miller"], inp["L"], inp["n"])
    assert r2["ex_trace"] == pytest.approx(res["ex_trace"], rel=1e-13)
    assert np.abs(r2["W_pw"] - u.T @ res["W_pw"]).max() <= 1e-13
    assert np.abs(r2["M"] - u.conj().T @ res["M"] @ u).max() <= 1e-13
    x = rng.standard_normal((3, len(inp["miller"]))) + 0j
    assert np.abs(O.apply_ace(r2["xi"], x) - O.apply_ace(res["xi"], x)
                  ).max() <= 1e-12 * np.abs(O.apply_ace(res["xi"], x)).max()


# ------------------------------------------------ T5-T7 ACE properties
def test_ace_exact_on_build_set(c0):
    """ACE equals the exchange operator on the functions it was built from
    (Sec. 2): -xi xi^H psi = K psi."""
    inp, res = c0
    y = O.apply_ace(res["xi"], inp["coeffs"])
    err = np.linalg.norm(y - res["W_pw"]) / np.linalg.norm(res["W_pw"])
    assert err <= 1e-12


def test_ace_bound_schur(c0):
    """x^H (K_ace - K) x >= 0 for any x, = 0 on span(psi): ACE expectation
    values lie above those of K (the bound of Sec. 2 in the K = -V_X sign)."""
    inp, res = c0
    L, n, miller = inp["L"], inp["n"], inp["miller"]
    rng = np.random.default_rng(6)
    x = (rng.standard_normal((3, len(miller)))
         + 1j * rng.standard_normal((3, len(miller))))
    x[2] = inp["coeffs"].T @ (rng.standard_normal(8) + 0j)   # in span(psi)
    xg = O.orbitals_on_grid(x, miller, L, n)
    kx = O.grid_to_pw(O.apply_exchange_to(res["psi"], xg, res["v"]), miller, L)
    kace = O.apply_ace(res["xi"], x)
    for b in range(3):
        q_k = np.vdot(x[b], kx[b]).real
        q_ace = np.vdot(x[b], kace[b]).real
        assert q_k < 0
        assert q_ace - q_k >= -1e-13 * abs(q_k)
    assert q_ace - q_k == pytest.approx(0.0, abs=1e-12 * abs(q_k))
    assert np.vdot(x[0], kace[0]).real - np.vdot(x[0], kx[0]).real > 1e-6


def test_m_hermitian_negative_semidefinite(c0):
    _, res = c0
    m = res["M"]
    assert np.linalg.norm(m - m.conj().T) <= 1e-13 * np.linalg.norm(m)
    assert np.linalg.eigvalsh(0.5 * (m + m.conj().T)).max() < 0


# ------------------------------------------------- T8/T9 Gaussian integrals
def test_gaussian_self_exchange_closed_form():
    """One normalized Gaussian orbital (sigma = 1): |psi|^2 is a normalized
    Gaussian of width sigma / sqrt(2), so E_x = -(1/2)(11|11) with the
    truncated-Coulomb self-energy of that density."""
    L, n, ecut, sigma = 20.0, 64, 40.0, 1.0
    miller = synth.miller_sphere(L, ecut)
    assert np.abs(miller).max() < n / 2
    c = gaussian_coeffs(miller, L, np.array([7.3, 9.1, 11.7]), sigma)[None]
    res = O.run_path(c, miller, L, n)
    expect = -0.5 * gauss_self_coulomb(sigma / np.sqrt(2), L / 2)
    assert res["ex_trace"] == pytest.approx(expect, rel=1e-10)
    assert res["ex_pairs"] == pytest.approx(expect, rel=1e-10)


def test_two_gaussian_cross_integral_closed_form():
    """(ab|ba) for Gaussians of widths sa, sb at A, B: the pair density is a
    Gaussian of width tau = sa sb / sqrt(sa^2 + sb^2) with weight
    Q = Na Nb exp(-|A-B|^2 / (2 (sa^2 + sb^2))) (2 pi tau^2)^{3/2}."""
    L, n, ecut = 20.0, 64, 40.0
    sa, sb = 0.9, 1.2
    A, B = np.array([9.0, 10.0, 10.5]), np.array([10.2, 10.6, 11.1])
    miller = synth.miller_sphere(L, ecut)
    c = np.stack([gaussian_coeffs(miller, L, A, sa),
                  gaussian_coeffs(miller, L, B, sb)])
    psi = O.orbitals_on_grid(c, miller, L, n)
    v = O.coulomb_kernel(L, n)
    na, nb = (np.pi * sa * sa) ** -0.75, (np.pi * sb * sb) ** -0.75
    d2 = np.sum((A - B) ** 2)
    tau = sa * sb / np.sqrt(sa * sa + sb * sb)
    q = na * nb * np.exp(-d2 / (2 * (sa * sa + sb * sb))) * (
        2 * np.pi * tau * tau) ** 1.5
    expect = q * q * gauss_self_coulomb(tau, L / 2)
    got = O.pair_energy(psi[0], psi[1], v, L)
    assert got == pytest.approx(expect, rel=1e-9)
    # the full path with both orbitals: off-diagonal ordered pairs counted
    # twice, diagonal once each
    e_aa = gauss_self_coulomb(sa / np.sqrt(2), L / 2)
    e_bb = gauss_self_coulomb(sb / np.sqrt(2), L / 2)
    ex = O.exchange_energy_pairs(psi, v, L)
    assert ex == pytest.approx(-0.5 * (e_aa + e_bb + 2 * expect), rel=1e-9)


# ------------------------------------------------- T10/T11 identities
def test_symmetric_pair_identity(c0):
    """V_ji = conj(V_ij): v is real and even in G."""
    inp, res = c0
    psi, v = res["psi"], res["v"]
    for i, j in ((0, 1), (2, 5), (7, 3)):
        vij = O.pair_potential(psi[i], psi[j], v)
        vji = O.pair_potential(psi[j], psi[i], v)
        assert np.abs(vji - np.conj(vij)).max() <= 1e-14 * np.abs(vij).max()


def test_parseval_real_space_matches_pw(c0):
    inp, res = c0
    n, L = inp["n"], inp["L"]
    dv = L ** 3 / n ** 3
    psi = res["psi"].reshape(8, -1)
    w = res["W"].reshape(8, -1)
    m_real = dv * np.conj(psi) @ w.T
    assert np.abs(m_real - res["M"]).max() <= 1e-13 * np.abs(res["M"]).max()


# ------------------------------------------------ T12-T15 screening (L-ACE)
def test_zero_threshold_keeps_every_pair(c0):
    inp, res = c0
    assert len(res["pairs"]) == 8 * 9 // 2
    assert np.allclose(np.diag(res["S"]), 1.0, rtol=1e-13)
    r2 = O.run_path(inp["coeffs"], inp["miller"], inp["L"], inp["n"],
                    pairs=[(i, j) for j in range(8) for i in range(j + 1)])
    assert np.array_equal(r2["W_pw"], res["W_pw"])


def test_energy_routes_agree(c0, localized):
    _, res = c0
    assert res["ex_trace"] == pytest.approx(res["ex_pairs"], rel=1e-13)
    loc = localized
    pairs = O.kept_pairs(loc["S"], 2e-3)
    w = O.apply_exchange(loc["psi"], loc["v"], pairs)
    m = O.exchange_matrix(loc["coeffs"], O.grid_to_pw(w, loc["miller"],
                                                      loc["L"]))
    assert O.exchange_energy_trace(m) == pytest.approx(
        O.exchange_energy_pairs(loc["psi"], loc["v"], loc["L"], pairs),
        rel=1e-12)


def test_overlap_of_moduli_brute(localized):
    """S_ik against a direct double loop over grid points for a few pairs."""
    loc = localized
    psi, L, n = loc["psi"], loc["L"], loc["n"]
    dv = L ** 3 / n ** 3
    for i, k in ((0, 0), (0, 1), (3, 12), (15, 2)):
        a = psi[i].ravel()
        b = psi[k].ravel()
        tot = 0.0
        for p in range(0, a.size, 4096):
            tot += float(np.sum(np.sqrt(a[p:p + 4096].real ** 2 + a[p:p + 4096].imag ** 2)
                                * np.sqrt(b[p:p + 4096].real ** 2 + b[p:p + 4096].imag ** 2)))
        assert loc["S"][i, k] == pytest.approx(dv * tot, rel=1e-12)


def test_truncation_energy_identity(localized):
    """E'_x - E_x = (1/2) sum over discarded ordered pairs of (ij|ji) >= 0,
    each discarded integral computed with a brute-force DFT."""
    loc = localized
    L, n, psi, v = loc["L"], loc["n"], loc["psi"], loc["v"]
    s_thr = 5e-3
    pairs = O.kept_pairs(loc["S"], s_thr)
    kept = set(pairs)
    disc = [(i, j) for j in range(16) for i in range(j + 1)
            if (i, j) not in kept]
    assert 0 < len(disc) < 136
    full = O.exchange_energy_trace(O.exchange_matrix(
        loc["coeffs"], O.grid_to_pw(O.apply_exchange(psi, v), loc["miller"],
                                    L)))
    trunc = O.exchange_energy_trace(O.exchange_matrix(
        loc["coeffs"], O.grid_to_pw(O.apply_exchange(psi, v, pairs),
                                    loc["miller"], L)))
    vd = kernel_direct(L, n, L / 2) if n <= 8 else v
    f = dft_matrix(n, -1)
    extra = 0.0
    for i, j in disc:
        rho = np.conj(psi[i]) * psi[j]
        rg = np.einsum("az,by,cx,zyx->abc", f, f, f, rho, optimize=True) / n**3
        eij = L ** 3 * np.sum(vd * np.abs(rg) ** 2)
        extra += eij * (1 if i == j else 2)
    assert trunc - full == pytest.approx(0.5 * extra, rel=1e-10)
    assert trunc - full > 0


@pytest.mark.parametrize("s_thr", [1e-3, 2e-3, 5e-3])
def test_truncated_matrix_positive_definite_all_symmetrizations(
        localized, s_thr):
    """-sym(M') admits a Cholesky factor for thresholds in the paper's
    working range (0, 0.005], for each of the three symmetrizations, and
    xi xi^H then acts on the build set as W' M_s^{-1} W'^H."""
    loc = localized
    pairs = O.kept_pairs(loc["S"], s_thr)
    w_pw = O.grid_to_pw(O.apply_exchange(loc["psi"], loc["v"], pairs),
                        loc["miller"], loc["L"])
    m = O.exchange_matrix(loc["coeffs"], w_pw)
    assert np.linalg.norm(m - m.conj().T) > 0      # M' is not Hermitian
    traces = []
    for mode in ("avg", "upper", "lower"):
        ms = O.symmetrize(m, mode)
        assert np.array_equal(ms, ms.conj().T)
        chol = O.cholesky_neg(ms)
        assert np.allclose(chol @ chol.conj().T, -ms, atol=1e-13)
        xi = O.projector(w_pw, chol)
        y = O.apply_ace(xi, loc["coeffs"])
        # K_ace psi = W' M_s^{-1} (W'^H psi), and W'^H psi = M'^H
        t = np.linalg.solve(ms, m.conj().T)
        assert np.abs(y - t.T @ w_pw).max() <= 1e-11 * np.abs(w_pw).max()
        traces.append(np.trace(ms).real)
    assert traces[0] == pytest.approx(traces[1]) == pytest.approx(traces[2])


def test_cholesky_failure_is_reported():
    m = np.diag([-1.0, 0.5, -2.0]).astype(complex)
    with pytest.raises(O.NotPositiveDefinite):
        O.cholesky_neg(O.symmetrize(m))


def test_symmetrizations_agree_on_hermitian(c0):
    _, res = c0
    m = res["M"]
    a = O.symmetrize(m, "avg")
    for mode in ("upper", "lower"):
        assert np.abs(O.symmetrize(m, mode) - a).max() <= 1e-15 * np.abs(m).max()


def test_symmetrization_keeps_the_named_triangle():
    """Sec. 2, text after Eq. (10): 'upper' copies the upper triangle of M'
    (entries M'_jk = <psi_j|K|psi_k> with j < k) into the lower one, 'lower'
    the lower triangle into the upper one, 'avg' averages M' with its
    adjoint.  On a non-Hermitian complex M' the kept triangle must come back
    unchanged, the other one as its mirror image, and the diagonal real."""
    rng = np.random.default_rng(31)
    n = 7
    m = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    iu = np.triu_indices(n, 1)
    il = np.tril_indices(n, -1)
    up = O.symmetrize(m, "upper")
    assert np.array_equal(up[iu], m[iu])
    assert np.array_equal(up.T[iu], np.conj(m[iu]))
    lo = O.symmetrize(m, "lower")
    assert np.array_equal(lo[il], m[il])
    assert np.array_equal(lo.T[il], np.conj(m[il]))
    # the two modes disagree off the diagonal when M' is not Hermitian
    assert np.abs(up - lo).max() > 0.1
    av = O.symmetrize(m, "avg")
    for a in range(n):
        for b in range(n):
            if a != b:
                want = 0.5 * (m[a, b] + np.conj(m[b, a]))
                assert abs(av[a, b] - want) <= 1e-15 * abs(want) + 1e-300
    for out in (up, lo, av):
        assert np.array_equal(np.diag(out), np.diag(m).real.astype(complex))


def test_scdm_orbitals_are_the_loewdin_polar_factor(localized):
    """The SCDM orbitals are the density-matrix columns Loewdin-
    orthonormalized: with D_k = P(., r_k) = sum_n psi_n conj(psi_n(r_k))
    (built here by a plain loop over the orbitals) and Phi the returned set,
    D = Phi H with H = Phi^H D Hermitian positive definite (the polar
    decomposition, unique for full-rank D), so no other orthonormal set is
    closer to D in the Frobenius norm: Gram-Schmidt (QR) of D and random
    unitary mixes of Phi all lie further away."""
    L, n, miller = localized["L"], localized["n"], localized["miller"]
    coeffs = localized["coeffs"]
    psi = localized["psi"]
    nb = coeffs.shape[0]
    pts = O.scdm_points(psi)
    phi = O.scdm_given_points(coeffs, psi, pts)
    flat = psi.reshape(nb, -1)
    d = np.zeros_like(coeffs)
    for k, r in enumerate(pts):
        for m in range(nb):
            d[k] += coeffs[m] * np.conj(flat[m, r])
    assert np.abs(np.conj(phi) @ phi.T - np.eye(nb)).max() <= 1e-12
    h = np.conj(phi) @ d.T             # h[a, b] = <phi_a | D_b>
    assert np.abs(h - h.conj().T).max() <= 1e-12 * np.abs(h).max()
    assert np.linalg.eigvalsh(0.5 * (h + h.conj().T)).min() > 0
    assert np.abs(phi.T @ h - d.T).max() <= 1e-12 * np.abs(d).max()
    best = np.linalg.norm(phi - d)
    q, _ = np.linalg.qr(d.T)
    assert np.linalg.norm(q.T - d) > best * (1 + 1e-6)
    rng = np.random.default_rng(73)
    for _ in range(20):
        z = rng.standard_normal((nb, nb)) + 1j * rng.standard_normal((nb, nb))
        u, _ = np.linalg.qr(z)
        u = np.linalg.qr(np.eye(nb) + 0.05 * (u - np.eye(nb)))[0]
        assert np.linalg.norm(u.T @ phi - d) > best


def test_exchange_integral_columns_sum_to_the_energy(localized):
    """The per-column integral sums of the screened energy add up to
    -2 E_x of the kept ordered pairs."""
    loc = localized
    pairs = O.kept_pairs(loc["S"], 2e-3)
    cols = O.exchange_integrals_columns(loc["psi"], loc["v"], loc["L"], pairs,
                                        range(loc["psi"].shape[0]))
    ex = O.exchange_energy_pairs(loc["psi"], loc["v"], loc["L"], pairs)
    assert -0.5 * cols.sum() == pytest.approx(ex, rel=1e-13)
    assert np.all(cols > 0)


def test_localized_generator_orthonormal_real(localized):
    c = localized["coeffs"]
    assert np.abs(c.conj() @ c.T - np.eye(16)).max() < 1e-12
    psi = localized["psi"]
    assert np.abs(psi.imag).max() <= 1e-10 * np.abs(psi.real).max()


# ------------------------------------------------- planted mistakes bite
def _c0_small():
    inp = synth.make_inputs("plain-ace-24")
    return inp["coeffs"][:4], inp["miller"], inp["L"], inp["n"]


def test_planted_missing_conjugate_breaks_hermiticity(monkeypatch):
    """Plant rho = psi_i psi_j (no conjugate) in the oracle: M stops being
    Hermitian, so the Hermiticity pin catches it."""
    import oracle.lace_oracle as mod

    def bad(pi, pj, v):
        return np.fft.ifftn(v * np.fft.fftn(pi * pj))
    c, miller, L, n = _c0_small()
    good = O.run_path(c, miller, L, n)["M"]
    assert np.linalg.norm(good - good.conj().T) <= 1e-13 * np.linalg.norm(good)
    monkeypatch.setattr(mod, "pair_potential", bad)
    psi = O.orbitals_on_grid(c, miller, L, n)
    w = O.apply_exchange(psi, O.coulomb_kernel(L, n))
    m = O.exchange_matrix(c, O.grid_to_pw(w, miller, L))
    assert np.linalg.norm(m - m.conj().T) > 1e-3 * np.linalg.norm(m)


def test_planted_bare_kernel_breaks_gaussian_pin(monkeypatch):
    """Plant the untruncated 4 pi / G^2 kernel (G = 0 dropped): the Gaussian
    closed form no longer holds."""
    import oracle.lace_oracle as mod
    real = mod.coulomb_kernel

    def bare(L, n, rc=None, omega=0.0):
        v = real(L, n, rc, omega)
        f = np.fft.fftfreq(n, d=1.0 / n) * 2 * np.pi / L
        gz, gy, gx = np.meshgrid(f, f, f, indexing="ij")
        g2 = gx ** 2 + gy ** 2 + gz ** 2
        g2[0, 0, 0] = 1.0
        out = 4 * np.pi / g2
        out[0, 0, 0] = 0.0
        return out + 0 * v
    monkeypatch.setattr(mod, "coulomb_kernel", bare)
    L, n, ecut, sigma = 20.0, 64, 40.0, 1.0
    miller = synth.miller_sphere(L, ecut)
    c = gaussian_coeffs(miller, L, np.array([7.3, 9.1, 11.7]), sigma)[None]
    res = O.run_path(c, miller, L, n)
    expect = -0.5 * gauss_self_coulomb(sigma / np.sqrt(2), L / 2)
    assert abs(res["ex_trace"] - expect) > 1e-3 * abs(expect)


def test_planted_scale_error_breaks_plane_wave_pin(monkeypatch):
    """Plant a missing Omega^{1/2} in the back-transform: the plane-wave
    closed form for M fails."""
    import oracle.lace_oracle as mod
    real = mod.grid_to_pw

    def bad(w, miller, L):
        return real(w, miller, L) / np.sqrt(L ** 3)
    monkeypatch.setattr(mod, "grid_to_pw", bad)
    L, n, ecut = 8.0, 12, 4.0
    miller = synth.miller_sphere(L, ecut)
    coeffs = np.zeros((2, len(miller)), complex)
    coeffs[0, 3] = coeffs[1, 17] = 1.0
    res = O.run_path(coeffs, miller, L, n)
    assert res["ex_trace"] != pytest.approx(res["ex_pairs"], rel=1e-3)


# ---------------------------------------------- virtual orbitals (Sec. 4.1)
def test_virtual_plane_wave_closed_form():
    """Occupied plane waves a, virtual plane waves b: K psi_b =
    -(1/Omega) sum_a v(G_b - G_a) psi_b (the occupied sum only), so M is
    diagonal over the whole projection space and E_x counts the occupied
    block only."""
    L, n, ecut = 8.0, 12, 4.0
    miller = synth.miller_sphere(L, ecut)
    rng = np.random.default_rng(13)
    n_occ, n_virt = 4, 3
    pick = rng.choice(len(miller), size=n_occ + n_virt, replace=False)
    coeffs = np.zeros((n_occ + n_virt, len(miller)), complex)
    coeffs[np.arange(n_occ + n_virt), pick] = 1.0
    res = O.run_path_virtual(coeffs, n_occ, miller, L, n)
    omega, rc = L ** 3, L / 2
    m = miller[pick]
    expect = np.zeros(n_occ + n_virt)
    for b in range(n_occ + n_virt):
        for a in range(n_occ):
            d = signed(np.mod(m[b] - m[a], n), n)
            gg = 2 * np.pi / L * np.sqrt(float(d @ d))
            vv = (2 * np.pi * rc * rc if gg == 0 else
                  4 * np.pi * (1 - np.cos(gg * rc)) / gg ** 2)
            expect[b] -= vv / omega
    assert np.abs(res["M"] - np.diag(expect)).max() <= 1e-13 * np.abs(
        expect).max()
    assert np.abs(res["W_pw"] - expect[:, None] * coeffs).max() <= 1e-13
    assert res["ex_pairs"] == pytest.approx(0.5 * expect[:n_occ].sum(),
                                            rel=1e-13)


def test_virtual_ace_exact_on_projection_space(localized):
    """Unscreened, ACE built on occupied + virtual orbitals reproduces K on
    every one of them and lies above K elsewhere; the occupied block of M
    is the occupied-only M; M is Hermitian negative definite."""
    L, n, miller = localized["L"], localized["n"], localized["miller"]
    occ = localized["coeffs"][:10]
    virt = synth.virtual_orbitals(miller, L, occ, 4, synth.rng_for(91))
    coeffs = np.concatenate([occ, virt])
    res = O.run_path_virtual(coeffs, 10, miller, L, n)
    y = O.apply_ace(res["xi"], coeffs)
    assert np.linalg.norm(y - res["W_pw"]) <= 1e-12 * np.linalg.norm(
        res["W_pw"])
    m = res["M"]
    assert np.abs(m - m.conj().T).max() <= 1e-13 * np.abs(m).max()
    assert np.linalg.eigvalsh(0.5 * (m + m.conj().T)).max() < 0
    occ_only = O.run_path(occ, miller, L, n)
    assert np.abs(m[:10, :10] - occ_only["M"]).max() <= 1e-13 * np.abs(m).max()
    assert res["ex_pairs"] == pytest.approx(occ_only["ex_pairs"], rel=1e-13)
    # a function outside the projection space: ACE above K (Schur bound)
    x = synth.virtual_orbitals(miller, L, coeffs, 1, synth.rng_for(92))
    xg = O.orbitals_on_grid(x, miller, L, n)
    kx = O.grid_to_pw(O.apply_exchange_to(res["psi"][:10], xg, res["v"]),
                      miller, L)
    gap = np.vdot(x[0], O.apply_ace(res["xi"], x)[0]).real - np.vdot(
        x[0], kx[0]).real
    assert gap > 1e-8


def test_virtual_screening_keeps_every_virtual_integral(localized):
    """With a threshold that drops occupied pairs, the virtual columns are
    still the full K applied to them, and the occupied columns are those of
    the screened occupied-only run."""
    L, n, miller = localized["L"], localized["n"], localized["miller"]
    occ = localized["coeffs"][:10]
    virt = synth.virtual_orbitals(miller, L, occ, 2, synth.rng_for(93))
    coeffs = np.concatenate([occ, virt])
    s_thr = 5e-3
    scr = O.run_path_virtual(coeffs, 10, miller, L, n, s_thr=s_thr)
    full = O.run_path_virtual(coeffs, 10, miller, L, n)
    occ_scr = O.run_path(occ, miller, L, n, s_thr=s_thr)
    assert len(occ_scr["pairs"]) < 55
    assert np.abs(scr["W_pw"][10:] - full["W_pw"][10:]).max() <= 1e-14
    assert np.abs(scr["W_pw"][:10] - occ_scr["W_pw"]).max() <= 1e-14


# ------------------------------------------------ alignment (end of Sec. 2)
def _random_unitary(rng, n, real=False):
    z = rng.standard_normal((n, n))
    if not real:
        z = z + 1j * rng.standard_normal((n, n))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def test_align_recovers_a_rotation(c0):
    """new = old rotated by a unitary: aligning gives old back."""
    inp, _ = c0
    old = inp["coeffs"]
    rot = _random_unitary(np.random.default_rng(21), old.shape[0])
    new = rot.T @ old                     # new_a = sum_b rot[b, a] old_b
    assert np.abs(O.align_orbitals(new, old) - old).max() <= 1e-13


def test_align_is_the_closest_unitary_mix(c0):
    """Procrustes optimality against random unitary mixes and the identity;
    the result spans the space of new and is orthonormal."""
    inp, _ = c0
    old = inp["coeffs"]
    rng = np.random.default_rng(22)
    n = old.shape[0]
    noise = 0.05 * (rng.standard_normal(old.shape)
                    + 1j * rng.standard_normal(old.shape))
    new, _ = np.linalg.qr((_random_unitary(rng, n).T @ old + noise).T)
    new = new.T
    out = O.align_orbitals(new, old)
    best = np.linalg.norm(out - old)
    for q in [np.eye(n)] + [_random_unitary(rng, n) for _ in range(20)]:
        assert best <= np.linalg.norm(q.T @ new - old) + 1e-12
    assert np.abs(np.conj(out) @ out.T - np.eye(n)).max() <= 1e-13
    proj = np.conj(new) @ out.T           # out lies in span(new)
    assert np.abs(proj.T @ new - out).max() <= 1e-12


def test_align_keeps_real_orbitals_real(localized):
    """Real orbitals rotated by a real orthogonal matrix align back with a
    real orthogonal U (C_{-G} = conj(C_G) kept)."""
    old = localized["coeffs"]
    rng = np.random.default_rng(23)
    rot = _random_unitary(rng, old.shape[0], real=True)
    new = rot.T @ old + 1e-3 * (rot.T @ old)[::-1]
    out = O.align_orbitals(new, old)
    a = np.conj(new) @ old.T
    assert np.abs(a.imag).max() <= 1e-13
    miller = localized["miller"]
    where = {tuple(m): k for k, m in enumerate(miller.tolist())}
    neg = np.array([where[(-x, -y, -z)] for x, y, z in miller.tolist()])
    assert np.abs(out[:, neg] - np.conj(out)).max() <= 1e-13


# -------------------------------------------- SCDM localization (Sec. 2)
def _greedy_points_brute(psi):
    """Greedy picks by their definition: at each step the point whose column
    conj(psi(r)) has the largest residual after least-squares projection on
    the columns already picked."""
    nb = psi.shape[0]
    a = np.conj(psi.reshape(nb, -1))
    picks = []
    for _ in range(nb):
        if picks:
            b = a[:, picks]
            coef, *_ = np.linalg.lstsq(b, a, rcond=None)
            res = a - b @ coef
        else:
            res = a
        norms = np.einsum("ij,ij->j", np.conj(res), res).real
        norms[picks] = -1.0
        picks.append(int(np.argmax(norms)))
    return np.array(picks)


def test_scdm_points_are_the_greedy_picks():
    L, n, ecut = 8.0, 12, 4.0
    miller = synth.miller_sphere(L, ecut)
    coeffs = synth.random_orbitals(miller, L, 5, synth.rng_for(70))
    psi = O.orbitals_on_grid(coeffs, miller, L, n)
    assert list(O.scdm_points(psi)) == list(_greedy_points_brute(psi))


def test_scdm_is_gauge_invariant(localized):
    """Mixing the orbitals by any unitary changes neither the points nor the
    localized orbitals (they depend on the density matrix only)."""
    L, n, miller = localized["L"], localized["n"], localized["miller"]
    coeffs = localized["coeffs"]
    rng = np.random.default_rng(71)
    z = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    v, _ = np.linalg.qr(z)
    phi1, p1 = O.scdm(coeffs, miller, L, n)
    phi2, p2 = O.scdm(v.T @ coeffs, miller, L, n)
    assert list(p1) == list(p2)
    assert np.abs(phi1 - phi2).max() <= 1e-12


def test_scdm_localizes_mixed_localized_orbitals(localized):
    """Localized orbitals mixed by a random rotation are delocalized (every
    pair survives the screening); SCDM makes them local again, orthonormal
    and spanning the same space."""
    L, n, miller = localized["L"], localized["n"], localized["miller"]
    coeffs = localized["coeffs"]
    rng = np.random.default_rng(72)
    v, _ = np.linalg.qr(rng.standard_normal((16, 16)))
    mixed = v.T @ coeffs
    s_thr = 5e-3
    def kept(c):
        return len(O.kept_pairs(O.overlap_of_moduli(
            O.orbitals_on_grid(c, miller, L, n), L), s_thr))
    k_loc, k_mix = kept(coeffs), kept(mixed)
    phi, _ = O.scdm(mixed, miller, L, n)
    k_scdm = kept(phi)
    assert k_mix == 16 * 17 // 2
    assert k_scdm < 0.8 * k_mix
    assert abs(k_scdm - k_loc) <= 0.35 * k_loc
    assert np.abs(np.conj(phi) @ phi.T - np.eye(16)).max() <= 1e-13
    proj = np.conj(coeffs) @ phi.T
    assert np.abs(proj.T @ coeffs - phi).max() <= 1e-12


# ------------------------------- screened (HSE-type) kernel, closed form
def test_screened_gaussian_self_exchange_closed_form():
    """The short-range interaction erfc(omega r) / r: for one normalized
    Gaussian orbital the self-energy of its density (width tau) is the bare
    1 / (tau sqrt(pi)) minus the long-range part, the potential at its
    centre of a Gaussian charge of variance 2 tau^2 + 1 / (2 omega^2)
    (erf(omega r) / r is the potential of a Gaussian charge of variance
    1 / (2 omega^2)).  Periodic images are below 1e-40 at omega = 0.5."""
    L, n, ecut, sigma, omega = 20.0, 64, 40.0, 1.0, 0.5
    miller = synth.miller_sphere(L, ecut)
    c = gaussian_coeffs(miller, L, np.array([7.3, 9.1, 11.7]), sigma)[None]
    res = O.run_path(c, miller, L, n, omega=omega)
    tau = sigma / np.sqrt(2)
    self_sr = 1.0 / (tau * np.sqrt(np.pi)) - np.sqrt(2.0 / np.pi) / np.sqrt(
        2 * tau * tau + 1.0 / (2 * omega * omega))
    assert res["ex_trace"] == pytest.approx(-0.5 * self_sr, rel=1e-10)
    assert res["ex_pairs"] == pytest.approx(-0.5 * self_sr, rel=1e-10)
    # screening only removes interaction: weaker than the bare kernel
    bare = O.run_path(c, miller, L, n, rc=L / 2)
    assert abs(res["ex_trace"]) < abs(bare["ex_trace"])
