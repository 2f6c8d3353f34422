"""Seeded generators for the synthetic workloads.

Every random draw goes through ``rng_for(stream, cell, job, step, seed)`` so
that a given (stream, cell, job, step, seed) tuple always yields the same
arrays.  Coefficient arrays are returned orbital-major: shape
``(n_orb, n_pw)``, C-contiguous complex128, i.e. the column-major
``n_pw x n_orb`` matrix whose column ``j`` holds orbital ``j``.

The workloads stand in for the paper's condensed-phase systems (amorphous
silica cells of 18.7-38.6 bohr with an 80 Ry orbital cutoff, Sec. 4.1), which
are not available here:

* random delocalized orbitals (canonical-orbital-like, unscreened ACE),
* Gaussians, two per random centre, Loewdin-orthonormalized (localized
  orbitals as produced by a localization step, the L-ACE case).
"""
from __future__ import annotations

import numpy as np

# Single-cell workloads by name (sizes in bohr / Hartree); `stream` selects
# the workload's own random stream.
WORKLOADS = {
    "plain-ace-24": dict(stream=0, L=10.0, n=24, ecut=15.0, n_orb=8,
                         kind="random", s_thr=0.0),
    "plain-ace-120": dict(stream=1, L=23.5, n=120, ecut=40.0, n_orb=256,
                          kind="random", s_thr=0.0),
    "lace-120": dict(stream=2, L=23.5, n=120, ecut=40.0, n_orb=256,
                     kind="gaussian", n_centers=128, s_thr=1e-3),
}
# Batched multi-cell workload: (L, n, n_orb); 4 cells of each class.
BATCH_CLASSES = [(12.0, 48, 32), (16.0, 64, 64), (20.0, 80, 96), (24.0, 96, 128)]
BATCH_ECUT = 40.0
BATCH_S_THR = 1e-3


def rng_for(stream: int, cell: int = 0, job: int = 0, step: int = 0,
            seed: int = 0) -> np.random.Generator:
    """Independent stream per (stream, cell, job, step, seed)."""
    return np.random.default_rng(
        np.random.SeedSequence([int(stream), int(cell), int(job), int(step),
                                int(seed)]))


def miller_sphere(L: float, ecut: float) -> np.ndarray:
    """Integer triples m with 0.5*|2*pi*m/L|^2 <= ecut.

    Returned as int32 array (n_pw, 3) holding (m_x, m_y, m_z), ordered
    lexicographically in (m_z, m_y, m_x).
    """
    mmax = int(np.floor(np.sqrt(2.0 * ecut) * L / (2.0 * np.pi))) + 1
    r = np.arange(-mmax, mmax + 1)
    mz, my, mx = np.meshgrid(r, r, r, indexing="ij")
    kin = 0.5 * (2.0 * np.pi / L) ** 2 * (mx * mx + my * my + mz * mz)
    keep = kin <= ecut
    return np.stack([mx[keep], my[keep], mz[keep]], axis=1).astype(np.int32)


def _g_vectors(miller: np.ndarray, L: float) -> np.ndarray:
    return (2.0 * np.pi / L) * miller.astype(np.float64)


def random_orbitals(miller: np.ndarray, L: float, n_orb: int,
                    rng: np.random.Generator) -> np.ndarray:
    """Delocalized orthonormal orbitals.

    C_mj = (a + i b) exp(-|G_m|^2 / 8) with a, b ~ N(0, 1), followed by a
    reduced Householder QR; the Q factor is returned (orbital-major).
    """
    g = _g_vectors(miller, L)
    damp = np.exp(-np.einsum("ij,ij->i", g, g) / 8.0)
    n_pw = miller.shape[0]
    a = rng.standard_normal((n_pw, n_orb))
    b = rng.standard_normal((n_pw, n_orb))
    c = (a + 1j * b) * damp[:, None]
    q, _ = np.linalg.qr(c)
    return np.ascontiguousarray(q.T)


def _sample_centers(n_centers: int, L: float, min_sep: float,
                    rng: np.random.Generator, max_tries: int = 200000):
    """Uniform centres in the cubic cell, sequential rejection sampling
    with a periodic minimum-image separation of at least ``min_sep``."""
    pts = []
    tries = 0
    while len(pts) < n_centers:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place centres with the requested "
                               "minimum separation")
        p = rng.uniform(0.0, L, size=3)
        ok = True
        for q in pts:
            d = p - q
            d -= L * np.round(d / L)
            if np.dot(d, d) < min_sep * min_sep:
                ok = False
                break
        if ok:
            pts.append(p)
    return np.array(pts)


def gaussian_params(L: float, n_orb: int, n_centers: int,
                    rng: np.random.Generator, min_sep: float = 2.5,
                    wmin: float = 0.8, wmax: float = 1.6):
    """Centres (n_centers, 3) and widths (n_orb,) for Gaussian orbitals;
    orbital o sits on centre o // 2 when n_orb == 2 * n_centers."""
    centers = _sample_centers(n_centers, L, min_sep, rng)
    widths = rng.uniform(wmin, wmax, size=n_orb)
    owner = (np.arange(n_orb) * n_centers) // n_orb
    return centers[owner], widths


def orbitals_from_params(miller: np.ndarray, L: float, pos: np.ndarray,
                         widths: np.ndarray) -> np.ndarray:
    """Periodic Gaussians exp(-|r - R|^2 / (2 sigma^2)) written analytically
    in the plane-wave basis (c_G ~ exp(-G^2 sigma^2 / 2) exp(-i G.R)),
    normalized, then Loewdin-orthonormalized: C <- C S^{-1/2}, S = C^H C."""
    g = _g_vectors(miller, L)
    g2 = np.einsum("ij,ij->i", g, g)
    n_orb = widths.shape[0]
    c = np.empty((n_orb, miller.shape[0]), dtype=np.complex128)
    for o in range(n_orb):
        amp = np.exp(-0.5 * g2 * widths[o] ** 2)
        ph = np.exp(-1j * (g @ pos[o]))
        row = amp * ph
        row /= np.sqrt(np.vdot(row, row).real)
        c[o] = row
    # Two Loewdin passes: the second removes the ~kappa(S) * eps residue
    # left by the first when two widths on one centre nearly coincide.  The
    # orbitals are real functions, so S is real: its real part is used,
    # which keeps C_{-G} = conj(C_G) exact through the transformation.
    for _ in range(2):
        s = (c.conj() @ c.T).real     # s[a, b] = <c_a | c_b>
        s = 0.5 * (s + s.T)
        w, u = np.linalg.eigh(s)
        s_inv_half = (u * (1.0 / np.sqrt(w))) @ u.T
        # new orbital b = sum_a c_a (S^{-1/2})_{ab}
        c = s_inv_half.T @ c
    return np.ascontiguousarray(c)


def gaussian_orbitals(miller: np.ndarray, L: float, n_orb: int,
                      n_centers: int, rng: np.random.Generator) -> np.ndarray:
    pos, widths = gaussian_params(L, n_orb, n_centers, rng)
    return orbitals_from_params(miller, L, pos, widths)


def virtual_orbitals(miller: np.ndarray, L: float, occ: np.ndarray,
                     n_virt: int, rng: np.random.Generator,
                     real: bool = True) -> np.ndarray:
    """Delocalized functions orthonormal to each other and to the rows of
    ``occ`` (n_occ, n_pw): random coefficients under the envelope
    exp(-|G|^2 / 8), real functions (C_{-G} = conj(C_G)) when ``real``,
    then twice: project out the occupied rows, Loewdin-orthonormalize."""
    g = _g_vectors(miller, L)
    env = np.exp(-np.einsum("ij,ij->i", g, g) / 8.0)
    c = (rng.standard_normal((n_virt, miller.shape[0]))
         + 1j * rng.standard_normal((n_virt, miller.shape[0]))) * env
    if real:
        where = {tuple(m): k for k, m in enumerate(miller.tolist())}
        neg = np.array([where[(-a, -b, -d)] for a, b, d in miller.tolist()])
        c = 0.5 * (c + np.conj(c[:, neg]))
    for _ in range(2):
        o = occ.conj() @ c.T                # o[a, v] = <occ_a | c_v>
        if real:
            o = o.real
        c = c - o.T @ occ
        s = c.conj() @ c.T
        if real:
            s = s.real
        s = 0.5 * (s + s.conj().T)
        w, u = np.linalg.eigh(s)
        c = ((u * (1.0 / np.sqrt(w))) @ u.conj().T).T @ c
    return np.ascontiguousarray(c)


def perturb_gaussian_params(pos: np.ndarray, widths: np.ndarray,
                            rng: np.random.Generator):
    """One synthetic outer-iteration update: centres move by 0.02 z bohr and
    widths scale by (1 + 0.01 z), z ~ N(0, 1)."""
    dp = 0.02 * rng.standard_normal(pos.shape)
    dw = 1.0 + 0.01 * rng.standard_normal(widths.shape)
    return pos + dp, widths * dw


def make_inputs(name: str, seed: int = 0, cell: int = 0):
    """Inputs of the single-cell workload `name` (a key of WORKLOADS): dict
    with name, L, n, ecut, miller, coeffs (n_orb, n_pw), s_thr, rc."""
    cfg = WORKLOADS[name]
    L, n, ecut = cfg["L"], cfg["n"], cfg["ecut"]
    miller = miller_sphere(L, ecut)
    rng = rng_for(cfg["stream"], cell, 0, 0, seed)
    if cfg["kind"] == "random":
        coeffs = random_orbitals(miller, L, cfg["n_orb"], rng)
    else:
        coeffs = gaussian_orbitals(miller, L, cfg["n_orb"], cfg["n_centers"],
                                   rng)
    return dict(name=name, L=L, n=n, ecut=ecut, miller=miller,
                coeffs=coeffs, s_thr=cfg["s_thr"], rc=L / 2.0)


def make_batch_cells(seed: int = 0, classes=None, cells_per_class: int = 4):
    """The 16-cell batched workload: cell c has class c % 4."""
    classes = BATCH_CLASSES if classes is None else classes
    out = []
    for c in range(len(classes) * cells_per_class):
        L, n, n_orb = classes[c % len(classes)]
        miller = miller_sphere(L, BATCH_ECUT)
        rng = rng_for(3, c, 0, 0, seed)
        coeffs = gaussian_orbitals(miller, L, n_orb, n_orb // 2, rng)
        out.append(dict(name=f"batch-{int(L)}-{n}-{n_orb}", L=L, n=n,
                        ecut=BATCH_ECUT, miller=miller, coeffs=coeffs,
                        s_thr=BATCH_S_THR, rc=L / 2.0))
    return out


def poisson_arrivals(rate: float, n_jobs: int, rng: np.random.Generator):
    """Arrival times (s) of a Poisson stream: cumulative exponential gaps."""
    return np.cumsum(rng.exponential(1.0 / rate, size=n_jobs))


# Serving stream: the four batched cell classes plus the localized 120^3 cell.
SERVE_RATE = 40.0
SERVE_STEPS = 4
SERVE_LARGE_FRACTION = 0.05


def serving_classes(seed: int = 0, n_variants: int = 4,
                    n_variants_large: int = 2, include_large: bool = True,
                    specs=None):
    """Size classes of the serving stream.  Each class holds a few orbital
    sets that follow one another as synthetic outer iterations: Gaussian
    centres move by 0.02 z bohr and widths scale by (1 + 0.01 z) from one
    set to the next, then Loewdin.  Returns dicts with the cell fields and
    `variants` (list of (n_orb, n_pw) arrays)."""
    if specs is None:
        specs = [(L, n, n_orb) for (L, n, n_orb) in BATCH_CLASSES]
        if include_large:
            specs.append((23.5, 120, 256))
    out = []
    for k, (L, n, n_orb) in enumerate(specs):
        miller = miller_sphere(L, BATCH_ECUT)
        pos, widths = gaussian_params(L, n_orb, n_orb // 2,
                                      rng_for(4, k, 0, 0, seed))
        nv = n_variants_large if n == 120 else n_variants
        variants = []
        for v in range(nv):
            if v > 0:
                pos, widths = perturb_gaussian_params(
                    pos, widths, rng_for(4, k, 0, v, seed))
            variants.append(orbitals_from_params(miller, L, pos, widths))
        out.append(dict(name=f"serve-{int(L)}-{n}-{n_orb}", L=L, n=n,
                        ecut=BATCH_ECUT, miller=miller, s_thr=BATCH_S_THR,
                        rc=L / 2.0, n_orb=n_orb, variants=variants))
    return out


def serving_stream(n_jobs: int, n_small_classes: int, n_variants,
                   rate: float = SERVE_RATE, n_steps: int = SERVE_STEPS,
                   large_fraction: float = SERVE_LARGE_FRACTION,
                   seed: int = 0):
    """Job list of a Poisson stream: (job id, arrival s, class, variant of
    each outer step).  A fraction `large_fraction` of the jobs use class
    `n_small_classes` (the large cell), the rest a uniform small class.
    `n_variants[c]` is the number of orbital sets of class c."""
    rng = rng_for(4, 99, 0, 0, seed)
    arrivals = poisson_arrivals(rate, n_jobs, rng)
    jobs = []
    for j in range(n_jobs):
        large = large_fraction > 0 and rng.random() < large_fraction
        cls = n_small_classes if large else int(rng.integers(n_small_classes))
        nv = n_variants[cls]
        start = int(rng.integers(nv))
        jobs.append((j, float(arrivals[j]), cls,
                     [(start + s) % nv for s in range(n_steps)]))
    return jobs
