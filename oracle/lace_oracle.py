"""Plain CPU FP64 oracle of the L-ACE exchange path.

TEST INFRASTRUCTURE ONLY: used by ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py``; never by the library.

Written from Carnimeo, Baroni, Giannozzi, "Fast hybrid density-functional
computations using plane-wave basis sets" (arXiv:1801.09263), Sec. 2.
Everything is double precision.  FFTs are numpy's ``fftn`` (no scale) and
``ifftn`` (1/N_g scale), used as library primitives; there is no blocking,
fusion or reordering beyond the definitions below.

Conventions (readings of the paper, each pinned by a test):

* Hartree atomic units, e^2 = 1.  The paper's V_X is positive (Sec. 2, text
  after Eq. (1)); here K = -V_X is applied, so W = K psi, M = psi^H K psi is
  negative semidefinite and -M = L L^H.  xi = W L^{-H} is -1 times the
  paper's xi of Eq. (5) and xi xi^H is unchanged.
* Complex orbitals: the paper's real-orbital transposes (L^{-T}, (M'+M'^T)/2)
  are read as adjoints (L^{-H}, (M'+M'^H)/2).
* One spin channel, occupation 1 per orbital, no hybrid weight alpha.
* Cubic cell of side L, volume Omega = L^3, grid n^3 with r_p = L p / n,
  dV = Omega / N_g.  Plane-wave basis: all G = 2 pi m / L with
  |G|^2 / 2 <= Ecut.  Grid arrays are indexed [z, y, x] (x fastest).
* Coulomb interaction: the spherically truncated kernel
  v(G) = 4 pi (1 - cos(|G| R_c)) / |G|^2, v(0) = 2 pi R_c^2, evaluated on
  every grid frequency; the paper's bare 1/|r - r'| (Eq. (2)) states no
  G = 0 rule for a periodic cell.
* Screening keeps a pair when S_ij >= S_thr (the paper discards S < S_thr,
  Eq. (6)); S_ii = 1 so diagonal pairs are always kept for S_thr < 1.

Functions with "parity unpinned": none.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

__all__ = [
    "cell_volume", "sphere_miller", "grid_index", "orbitals_on_grid",
    "coulomb_kernel", "overlap_of_moduli", "kept_pairs", "pair_potential",
    "pair_energy", "apply_exchange", "apply_exchange_columns",
    "apply_exchange_to", "grid_to_pw", "exchange_matrix",
    "exchange_energy_trace", "exchange_energy_pairs",
    "exchange_integrals_columns", "symmetrize",
    "cholesky_neg", "NotPositiveDefinite", "projector", "apply_ace",
    "run_path", "apply_exchange_virtual", "run_path_virtual",
    "align_orbitals", "scdm_points", "scdm_given_points", "scdm",
]


class NotPositiveDefinite(Exception):
    """-M_s is not positive definite (the L-ACE Cholesky of Eq. (4) fails)."""


def cell_volume(L: float) -> float:
    return float(L) ** 3


def sphere_miller(L: float, ecut: float) -> set:
    """Plane-wave basis as a set of Miller triples (m_x, m_y, m_z):
    every G = 2 pi m / L with kinetic energy |G|^2 / 2 <= Ecut (the orbital
    cutoff of Sec. 3)."""
    out = set()
    mmax = int(np.ceil(np.sqrt(2.0 * ecut) * L / (2.0 * np.pi)))
    for mz in range(-mmax, mmax + 1):
        for my in range(-mmax, mmax + 1):
            for mx in range(-mmax, mmax + 1):
                g2 = (2.0 * np.pi / L) ** 2 * (mx * mx + my * my + mz * mz)
                if 0.5 * g2 <= ecut:
                    out.add((mx, my, mz))
    return out


def grid_index(miller: np.ndarray, n: int):
    """FFT-array position of each Miller triple: (m_z mod n, m_y mod n,
    m_x mod n)."""
    m = np.asarray(miller)
    return (np.mod(m[:, 2], n), np.mod(m[:, 1], n), np.mod(m[:, 0], n))


def orbitals_on_grid(coeffs: np.ndarray, miller: np.ndarray, L: float,
                     n: int) -> np.ndarray:
    """psi_j(r_p) = Omega^{-1/2} sum_m C_mj exp(i G_m . r_p) on the n^3 grid.

    The plane-wave representation of the orbitals (Sec. 2, text after
    Eq. (2)).  ``coeffs`` is (n_orb, n_pw); returns (n_orb, n, n, n).
    """
    omega = cell_volume(L)
    ng = n ** 3
    iz, iy, ix = grid_index(miller, n)
    out = np.empty((coeffs.shape[0], n, n, n), dtype=np.complex128)
    for j in range(coeffs.shape[0]):
        g = np.zeros((n, n, n), dtype=np.complex128)
        g[iz, iy, ix] = coeffs[j]
        # numpy's ifftn carries 1/N_g and the + sign: undo the scale.
        out[j] = (ng / np.sqrt(omega)) * np.fft.ifftn(g)
    return out


def coulomb_kernel(L: float, n: int, rc: float | None = None,
                   omega: float = 0.0) -> np.ndarray:
    """v(G) on every frequency of the n^3 grid, indexed [z, y, x].

    Fourier transform of the Coulomb interaction e^2 / |r - r'| of Eq. (2)
    cut off at |r - r'| = R_c (default L / 2):
    v(G) = 8 pi sin^2(|G| R_c / 2) / |G|^2 (the same as
    4 pi (1 - cos |G| R_c) / |G|^2 without cancellation), v(0) = 2 pi R_c^2.
    With omega > 0, the short-range part erfc(omega r) / r of the screened
    hybrids (HSE, named in Sec. 3; Heyd, Scuseria and Ernzerhof's
    definition), summed over all periodic images:
    v(G) = 4 pi (1 - exp(-|G|^2 / (4 omega^2))) / |G|^2, v(0) = pi / omega^2.
    """
    rc = L / 2.0 if rc is None else float(rc)
    f = np.fft.fftfreq(n, d=1.0 / n)          # signed integer frequencies
    g1 = (2.0 * np.pi / L) * f
    gz, gy, gx = np.meshgrid(g1, g1, g1, indexing="ij")
    gg = np.sqrt(gx * gx + gy * gy + gz * gz)
    v = np.empty_like(gg)
    nz = gg > 0
    if omega > 0.0:
        g2 = gg[nz] ** 2
        v[nz] = -4.0 * np.pi * np.expm1(-g2 / (4.0 * omega * omega)) / g2
        v[~nz] = np.pi / (omega * omega)
        return v
    v[nz] = 8.0 * np.pi * np.sin(0.5 * gg[nz] * rc) ** 2 / gg[nz] ** 2
    v[~nz] = 2.0 * np.pi * rc * rc
    return v


def overlap_of_moduli(psi: np.ndarray, L: float) -> np.ndarray:
    """S_ik = integral |w_i(r)| |w_k(r)| dr on the grid (Eq. (6))."""
    n = psi.shape[1]
    dv = cell_volume(L) / n ** 3
    a = np.abs(psi).reshape(psi.shape[0], -1)
    nb = a.shape[0]
    s = np.empty((nb, nb))
    for i in range(nb):
        for k in range(i, nb):
            s[i, k] = dv * np.sum(a[i] * a[k])
            s[k, i] = s[i, k]
    return s


def kept_pairs(s: np.ndarray, s_thr: float) -> list:
    """Unordered pairs (i, j), i <= j, whose integral is retained:
    S_ij >= S_thr (Eq. (6) discards S_ij < S_thr).  Sorted by (j, i)."""
    nb = s.shape[0]
    out = []
    for j in range(nb):
        for i in range(j + 1):
            if s[i, j] >= s_thr:
                out.append((i, j))
    return out


def pair_potential(psi_i: np.ndarray, psi_j: np.ndarray,
                   v: np.ndarray) -> np.ndarray:
    """V_ij(r) = integral v(r - r') psi_i^*(r') psi_j(r') dr', solved in
    reciprocal space: ifftn(v * fftn(conj(psi_i) psi_j)) (Eq. (2))."""
    rho = np.conj(psi_i) * psi_j
    return np.fft.ifftn(v * np.fft.fftn(rho))


def pair_energy(psi_i: np.ndarray, psi_j: np.ndarray, v: np.ndarray,
                L: float) -> float:
    """(ij|ji) = integral rho_ij^* V_ij = Omega sum_G v(G) |rho_ij(G)|^2,
    rho_ij(G) = fftn(rho_ij) / N_g (the exchange integral of Eq. (2))."""
    ng = v.size
    rho_g = np.fft.fftn(np.conj(psi_i) * psi_j) / ng
    return float(cell_volume(L) * np.sum(v * np.abs(rho_g) ** 2))


def _kept_lookup(pairs, nb):
    keep = np.zeros((nb, nb), dtype=bool)
    for i, j in pairs:
        keep[i, j] = keep[j, i] = True
    return keep


def apply_exchange(psi: np.ndarray, v: np.ndarray, pairs=None) -> np.ndarray:
    """W_j = K psi_j = -sum_{i : (i, j) kept} psi_i V_ij.

    Eq. (2) with the sign of K = -V_X, truncated to the kept pairs as in
    Eqs. (7)-(8): a discarded unordered pair removes both of its ordered
    terms.  Loops over every ordered pair; each V_ij is its own Poisson
    solve (no use of V_ji = conj(V_ij)).  ``pairs=None`` keeps all pairs.
    """
    return apply_exchange_columns(psi, v, pairs, range(psi.shape[0]))


def apply_exchange_columns(psi, v, pairs, cols) -> np.ndarray:
    """W_j of ``apply_exchange`` for the listed columns j only."""
    nb = psi.shape[0]
    keep = (np.ones((nb, nb), dtype=bool) if pairs is None
            else _kept_lookup(pairs, nb))
    cols = list(cols)
    w = np.zeros((len(cols),) + psi.shape[1:], dtype=np.complex128)
    for c, j in enumerate(cols):
        for i in range(nb):
            if keep[i, j]:
                w[c] -= psi[i] * pair_potential(psi[i], psi[j], v)
    return w


def apply_exchange_to(psi_occ: np.ndarray, x: np.ndarray,
                      v: np.ndarray) -> np.ndarray:
    """K x = -sum_i psi_i V[psi_i^* x] for arbitrary grid functions x
    (Eq. (2) applied to a generic function)."""
    out = np.zeros_like(x, dtype=np.complex128)
    for b in range(x.shape[0]):
        for i in range(psi_occ.shape[0]):
            out[b] -= psi_occ[i] * pair_potential(psi_occ[i], x[b], v)
    return out


def grid_to_pw(w: np.ndarray, miller: np.ndarray, L: float) -> np.ndarray:
    """What_mj = <G_m | W_j> = Omega^{-1/2} integral exp(-i G_m.r) W_j(r) dr
    = Omega^{1/2} / N_g * fftn(W_j)[m]: W as the N_P x N_PW matrix of the
    paper's reciprocal-space representation (Sec. 2).  Returns
    (n_orb, n_pw)."""
    n = w.shape[1]
    ng = n ** 3
    iz, iy, ix = grid_index(miller, n)
    scale = np.sqrt(cell_volume(L)) / ng
    out = np.empty((w.shape[0], miller.shape[0]), dtype=np.complex128)
    for j in range(w.shape[0]):
        out[j] = scale * np.fft.fftn(w[j])[iz, iy, ix]
    return out


def exchange_matrix(coeffs: np.ndarray, w_pw: np.ndarray) -> np.ndarray:
    """M_kj = <psi_k | K | psi_j> = sum_m conj(C_mk) What_mj (Eq. (3); the
    truncated M' of Eq. (9) when What comes from a screened W)."""
    return np.conj(coeffs) @ w_pw.T


def exchange_energy_trace(m: np.ndarray) -> float:
    """E_x = (1/2) Re tr M = (1/2) sum_j <psi_j|K|psi_j>, one spin channel,
    occupation 1 (energy of the density matrix, Sec. 2)."""
    return 0.5 * float(np.real(np.trace(m)))


def exchange_energy_pairs(psi: np.ndarray, v: np.ndarray, L: float,
                          pairs=None) -> float:
    """E_x = -(1/2) sum over kept ordered pairs of (ij|ji), each integral
    computed from its own pair density."""
    nb = psi.shape[0]
    keep = (np.ones((nb, nb), dtype=bool) if pairs is None
            else _kept_lookup(pairs, nb))
    e = 0.0
    for j in range(nb):
        for i in range(nb):
            if keep[i, j]:
                e += pair_energy(psi[i], psi[j], v, L)
    return -0.5 * e


def exchange_integrals_columns(psi: np.ndarray, v: np.ndarray, L: float,
                               pairs, cols) -> np.ndarray:
    """For each listed column j: sum over i with (i, j) kept of (ij|ji),
    every integral from its own pair density (the terms of
    ``exchange_energy_pairs``, grouped by column so that columns can be
    computed apart).  E_x = -(1/2) times the sum over all columns."""
    nb = psi.shape[0]
    keep = (np.ones((nb, nb), dtype=bool) if pairs is None
            else _kept_lookup(pairs, nb))
    cols = list(cols)
    out = np.zeros(len(cols))
    for c, j in enumerate(cols):
        for i in range(nb):
            if keep[i, j]:
                out[c] += pair_energy(psi[i], psi[j], v, L)
    return out


def symmetrize(m: np.ndarray, mode: str = "avg") -> np.ndarray:
    """The three symmetrizations of the non-Hermitian M' (Sec. 2, after
    Eq. (10)): 'avg' = (M + M^H)/2, 'upper' = upper triangle mirrored into
    the lower, 'lower' = lower triangle mirrored into the upper.  The
    diagonal is Re(M_jj) in every mode."""
    d = np.diag(np.real(np.diag(m)))
    if mode == "avg":
        out = 0.5 * (m + m.conj().T)
        np.fill_diagonal(out, np.real(np.diag(m)))
        return out
    if mode == "upper":
        u = np.triu(m, 1)
        return u + u.conj().T + d
    if mode == "lower":
        lo = np.tril(m, -1)
        return lo + lo.conj().T + d
    raise ValueError(mode)


def cholesky_neg(ms: np.ndarray) -> np.ndarray:
    """Lower-triangular L with positive real diagonal and -M_s = L L^H
    (the Cholesky factorization of Sec. 2, Eq. (4)-(5))."""
    try:
        return np.linalg.cholesky(-ms)
    except np.linalg.LinAlgError as exc:
        raise NotPositiveDefinite(str(exc)) from exc


def projector(w_pw: np.ndarray, chol: np.ndarray) -> np.ndarray:
    """xi = What L^{-H} (Eq. (5), adjoint reading).  With orbital-major
    arrays (row j = column j of the matrix) this is xi^T = conj(L)^{-1}
    What^T, a lower-triangular solve."""
    return scipy.linalg.solve_triangular(chol.conj(), w_pw, lower=True)


def apply_ace(xi: np.ndarray, x: np.ndarray) -> np.ndarray:
    """K_ace x = -xi (xi^H x): N_P scalar products per function, then a
    combination of the xi columns (Sec. 2, after Eq. (5)).  ``xi`` is
    (n_orb, n_pw), ``x`` is (n_vec, n_pw); returns (n_vec, n_pw)."""
    t = np.conj(xi) @ x.T          # (n_orb, n_vec) = xi^H x
    return -(t.T @ xi)


def run_path(coeffs, miller, L, n, s_thr=0.0, rc=None, sym="avg",
             pairs=None, want_grid=False, omega=0.0):
    """The whole path on one cell: grid orbitals, screening, exchange,
    What, M, E_x (both routes), Cholesky, xi.  ``pairs`` overrides the
    screening decision when given."""
    psi = orbitals_on_grid(coeffs, miller, L, n)
    v = coulomb_kernel(L, n, rc, omega)
    s = overlap_of_moduli(psi, L)
    if pairs is None:
        pairs = kept_pairs(s, s_thr)
    w = apply_exchange(psi, v, pairs)
    w_pw = grid_to_pw(w, miller, L)
    m = exchange_matrix(coeffs, w_pw)
    ex_trace = exchange_energy_trace(m)
    ex_pairs = exchange_energy_pairs(psi, v, L, pairs)
    ms = symmetrize(m, sym)
    chol = cholesky_neg(ms)
    xi = projector(w_pw, chol)
    out = dict(S=s, pairs=pairs, W_pw=w_pw, M=m, Ms=ms, L=chol, xi=xi,
               ex_trace=ex_trace, ex_pairs=ex_pairs)
    if want_grid:
        out.update(psi=psi, W=w, v=v)
    return out


def apply_exchange_virtual(psi: np.ndarray, v: np.ndarray, n_occ: int,
                           pairs=None) -> np.ndarray:
    """W for the occupied orbitals psi[:n_occ] and the virtual ones after
    them (the projection space of the band-gap runs in Sec. 4.1).  K sums
    over the occupied orbitals only (Eq. (2)).  Occupied columns keep the
    screened occupied pairs (Eqs. (7)-(8)); every integral that involves a
    virtual orbital is evaluated, so a virtual column is K applied to that
    function."""
    w_occ = apply_exchange(psi[:n_occ], v, pairs)
    w_virt = apply_exchange_to(psi[:n_occ], psi[n_occ:], v)
    return np.concatenate([w_occ, w_virt])


def run_path_virtual(coeffs, n_occ, miller, L, n, s_thr=0.0, rc=None,
                     sym="avg"):
    """``run_path`` on occupied plus virtual orbitals (occupied first):
    screening among the occupied orbitals, W of all of them, M, Cholesky
    and xi over the whole projection space; E_x from the occupied pairs."""
    psi = orbitals_on_grid(coeffs, miller, L, n)
    v = coulomb_kernel(L, n, rc)
    s = overlap_of_moduli(psi[:n_occ], L)
    pairs = kept_pairs(s, s_thr)
    w = apply_exchange_virtual(psi, v, n_occ, pairs)
    w_pw = grid_to_pw(w, miller, L)
    m = exchange_matrix(coeffs, w_pw)
    ex_pairs = exchange_energy_pairs(psi[:n_occ], v, L, pairs)
    ms = symmetrize(m, sym)
    chol = cholesky_neg(ms)
    xi = projector(w_pw, chol)
    return dict(S=s, pairs=pairs, W_pw=w_pw, M=m, Ms=ms, L=chol, xi=xi,
                ex_pairs=ex_pairs, psi=psi, v=v)


def align_orbitals(new: np.ndarray, old: np.ndarray) -> np.ndarray:
    """Align orbitals to those of the previous iteration (the convergence
    aid at the end of Sec. 2).  Reading: new U with U the unitary that
    minimizes ||new U - old||_F, the polar factor of A = new^H old, taken
    from the singular value decomposition A = P diag(s) Q^H as U = P Q^H.
    Rows are orbitals; returns the aligned rows."""
    a = np.conj(new) @ old.T              # a[x, y] = <new_x | old_y>
    p, _, qh = np.linalg.svd(a)
    u = p @ qh
    return u.T @ new


def scdm_points(psi: np.ndarray) -> np.ndarray:
    """The grid points of the SCDM localization (Sec. 2, the cited selected
    columns of the density matrix): the first N pivots of column-pivoted QR
    (LAPACK's, through scipy) of Psi^H, whose column at point r is
    conj(psi(r)).  Flat grid indices, in pivot order."""
    nb = psi.shape[0]
    a = np.conj(psi.reshape(nb, -1))
    _, piv = scipy.linalg.qr(a, mode="r", pivoting=True)
    return piv[:nb]


def scdm_given_points(coeffs: np.ndarray, psi: np.ndarray,
                      points) -> np.ndarray:
    """Localized orbitals for given points: the density matrix columns
    P(., r_k) = sum_n psi_n conj(psi_n(r_k)), Loewdin-orthonormalized, i.e.
    psi U with U the polar factor (from an SVD) of A[n, k] =
    conj(psi_n(r_k)).  Returns plane-wave coefficient rows."""
    nb = psi.shape[0]
    a = np.conj(psi.reshape(nb, -1)[:, np.asarray(points)])
    p, _, qh = np.linalg.svd(a)
    return (p @ qh).T @ coeffs


def scdm(coeffs, miller, L, n):
    """SCDM localization of the orbitals ``coeffs``: (coefficients, points)."""
    psi = orbitals_on_grid(coeffs, miller, L, n)
    pts = scdm_points(psi)
    return scdm_given_points(coeffs, psi, pts), pts
