/*
 * lace.h - C ABI of liblace, the MI355X (gfx950) implementation of the
 * L-ACE exact-exchange path of Carnimeo, Baroni, Giannozzi,
 * "Fast hybrid density-functional computations using plane-wave basis sets"
 * (arXiv:1801.09263).
 *
 * Three operations follow the paper's statement of the problem (Sec. 2):
 *   lace_apply_exchange  W = K psi over the screened orbital pairs
 *                        (Eq. (2); truncated as in Eqs. (6)-(8)),
 *   lace_build_ace       M = psi^H W, symmetrize, -M_s = L L^H,
 *                        xi = W L^{-H} (Eqs. (3)-(5), (9); symmetrizations
 *                        of the text after Eq. (10)),
 *   lace_apply_ace       y = -xi (xi^H x) (text after Eq. (5)).
 *
 * Conventions.  Hartree atomic units, e^2 = 1.  K = -V_X (the paper's V_X
 * is made positive, Sec. 2), so M is negative semidefinite and xi is -1
 * times the paper's xi; xi xi^H is the same.  One spin channel, occupation
 * 1.  Cubic cell of side L, n^3 FFT grid, Omega = L^3.  Coulomb kernel
 * truncated at R_c: v(G) = 4 pi (1 - cos |G| R_c) / |G|^2, v(0) = 2 pi R_c^2.
 *
 * Plane-wave arrays (psi_g, w_g, xi_g, x_g, y_g) are complex128 (interleaved
 * re, im doubles), column-major n_pw x n_cols: column j is contiguous and
 * holds orbital/function j in the order of the Miller list given at plan
 * creation.  Matrices M and S are n_orb x n_orb, row-major, M[a][b] =
 * <psi_a|K|psi_b>.
 *
 * Ownership.  All data buffers and the workspace belong to the caller; the
 * library keeps no pointer to them after a call returns.  The plan owns its
 * own tables (sphere-to-grid map, kernel table, twiddles) in device memory.
 *
 * Errors.  Every call returns an int status: LACE_OK (0) or a negative code.
 * Argument, shape and workspace errors are detected on the host before any
 * device work is enqueued.  A failed Cholesky factorization (M_s not
 * negative definite) is a device-side event recorded in an info word that
 * belongs to the call (a device int32 the caller passes, else the first
 * word of the call's workspace, read with lace_get_info).  HIP runtime
 * errors map to LACE_EHIP.
 *
 * Streams.  Work is enqueued on the given stream (0 = null stream) and is
 * asynchronous, except where a call says it synchronizes.  A plan must be
 * used by one host thread at a time.
 */
#ifndef LACE_H
#define LACE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* lace_stream_t; /* a hipStream_t */

enum {
  LACE_OK = 0,
  LACE_EINVAL = -1,      /* bad argument (null pointer, out-of-range value) */
  LACE_ENOMEM = -2,      /* workspace too small, or a plan allocation failed */
  LACE_ENOTPD = -3,      /* -M_s not positive definite (via lace_get_info) */
  LACE_EUNSUPPORTED = -4,/* grid size not supported, or sphere exceeds grid */
  LACE_EHIP = -5         /* HIP runtime error */
};

typedef enum {
  LACE_FP64 = 0,  /* grids, FFTs and pair products in FP64 */
  LACE_FP32 = 1,  /* grids, FFTs and pair products in FP32; screening sums,
                     exchange-energy sums, M, Cholesky, xi in FP64 */
  /* Real orbitals (Gamma point: C_{-G} = conj(C_G) for every orbital; the
   * caller guarantees it, lace_check_real measures it).  Orbitals and W are
   * stored as real grids and two pair densities of the same kind share one
   * complex transform (rho_ij + i rho_kl: the potentials come back as real
   * and imaginary parts), halving the transforms and the grid traffic. */
  LACE_FP64_GAMMA = 2,
  LACE_FP32_GAMMA = 3
} lace_precision;

typedef enum {
  LACE_SYM_AVG = 0,   /* M_s = (M + M^H) / 2 */
  LACE_SYM_UPPER = 1, /* upper triangle of M mirrored into the lower */
  LACE_SYM_LOWER = 2  /* lower triangle of M mirrored into the upper */
} lace_sym;

typedef struct {
  double L;              /* cubic cell side (bohr), > 0 */
  int32_t n;             /* FFT grid points per axis; one of the supported
                            sizes 8 12 16 24 32 48 64 80 96 120 */
  double rc;             /* Coulomb truncation radius; <= 0 selects L / 2 */
  int64_t n_pw;          /* number of plane waves, >= 1 */
  const int32_t* miller; /* host, n_pw x 3 int32 (m_x, m_y, m_z) per plane
                            wave; every |m_d| < n / 2 and no duplicates */
  double omega;          /* 0: the Coulomb interaction of Eq. (2), truncated
                            at rc.  > 0: its short-range part
                            erfc(omega r) / r, the screened exchange of the
                            HSE functionals named in Sec. 3 (definition of
                            Heyd, Scuseria and Ernzerhof, J. Chem. Phys. 118,
                            8207 (2003)): v(G) = 4 pi (1 - exp(-|G|^2 /
                            (4 omega^2))) / |G|^2, v(0) = pi / omega^2, no
                            truncation (rc unused).  < 0 is EINVAL. */
} lace_cell_desc;

typedef struct lace_plan lace_plan; /* opaque */

/* Create a plan for n_cells cells.  Builds on the current device the
 * sphere-to-grid map, the kernel table v(G) (evaluated in FP64, stored in
 * the plan precision) and FFT twiddles.  Synchronous.  *out is set only on
 * success.  Errors: EINVAL (null pointers, n_cells < 1, L <= 0, n_pw < 1,
 * duplicate Miller triples; for the Gamma precisions, a triple m whose -m
 * is not in the list), EUNSUPPORTED (grid size, sphere outside the grid),
 * ENOMEM, EHIP. */
int lace_plan_create(const lace_cell_desc* cells, int n_cells,
                     lace_precision prec, lace_plan** out);

/* Free the plan's device tables.  Synchronizes the device.  NULL is OK. */
int lace_plan_destroy(lace_plan* plan);

/* Workspace bytes needed by lace_apply_exchange, lace_build_ace and
 * lace_apply_ace on this cell for up to n_orb orbitals and n_vec functions
 * per lace_apply_ace call.  One workspace of this size serves all three. */
int lace_workspace_size(const lace_plan* plan, int cell, int n_orb, int n_vec,
                        size_t* bytes);

/* Screening matrix S_ij = integral |psi_i(r)| |psi_j(r)| dr (Eq. (6)),
 * computed from the orbitals on the grid in the plan precision and summed
 * in FP64.  psi_g: device, n_pw x n_orb complex128.  s_out: device,
 * n_orb x n_orb double, row-major.  Also leaves the grid orbitals in the
 * workspace.  Asynchronous. */
int lace_screen(lace_plan* plan, int cell, const void* psi_g, int n_orb,
                double* s_out, void* ws, size_t ws_bytes,
                lace_stream_t stream);

/* W = K psi restricted to the kept pairs (Eq. (2) truncated by
 * Eqs. (6)-(8)).
 *   psi_g   device, n_pw x n_orb complex128, orthonormal orbitals
 *           (1 <= n_orb <= 4096; also for the virtual, batched and
 *           autotuning calls).
 *   s_thr   screening threshold in [0, 1): an unordered pair (i, j) is kept
 *           when S_ij >= s_thr (Eq. (6)); s_thr = 0 keeps every pair (plain
 *           ACE).
 *   pair_i, pair_j  optional device int32 arrays of n_pairs unordered pairs
 *           (0 <= i <= j < n_orb) that replace the screening; pass
 *           NULL/NULL/0 to screen with s_thr.  A pair out of range or with
 *           i > j is dropped and a repeat runs once (n_kept then differs
 *           from n_pairs).
 *   w_g     device, n_pw x n_orb complex128 output (K psi on the sphere).
 *   e_x     device double output (may be NULL): exchange energy
 *           -(1/2) sum over kept ordered pairs of (ij|ji), summed in FP64
 *           from the pair densities.
 *   n_kept  device int64 output (may be NULL): unordered pairs run.
 *   kept    device int32 output (may be NULL; written only when the call
 *           screens, pair_i == NULL), room for n_orb (n_orb + 1) int32:
 *           the kept pairs (i, j), i <= j, as consecutive int32 couples,
 *           column by column (j ascending), i ascending within a column;
 *           n_kept of them.
 * The screening decision, the pair list and the batch schedule are made on
 * the device; the call is asynchronous (it enqueues as many pipeline
 * launches as a schedule of any pair set can need; those past the end of
 * this schedule return at once).  Errors: EINVAL, ENOMEM (workspace),
 * EHIP. */
int lace_apply_exchange(lace_plan* plan, int cell, const void* psi_g,
                        int n_orb, double s_thr, const int32_t* pair_i,
                        const int32_t* pair_j, int64_t n_pairs, void* w_g,
                        double* e_x, int64_t* n_kept, int32_t* kept, void* ws,
                        size_t ws_bytes, lace_stream_t stream);

/* W = K psi for occupied plus virtual orbitals (the band-gap setting of the
 * silica results in Sec. 4.1: the projection space holds the occupied
 * orbitals and a few virtual ones).  The exchange operator sums over the
 * occupied orbitals only (Eq. (2)); the occupied pairs are screened with
 * s_thr among themselves (Eq. (6)), and every integral that involves a
 * virtual orbital is evaluated.  An occupied x virtual pair (i, v) adds
 * -psi_i V_iv to W_v only and nothing to E_x.
 *   psi_g   device, n_pw x (n_occ + n_virt) complex128, orthonormal, the
 *           n_occ occupied orbitals first.
 *   w_g     device, n_pw x (n_occ + n_virt) complex128 output.
 *   e_x     device double (may be NULL): the exchange energy of the
 *           occupied orbitals, as for lace_apply_exchange.
 *   n_kept  device int64 (may be NULL): pair transforms run (kept occupied
 *           pairs + n_occ n_virt).
 * The workspace is that of n_orb = n_occ + n_virt.  lace_build_ace with
 * n_orb = n_occ + n_virt then builds ACE on the whole projection space
 * (its ex_tr then includes the virtual diagonal and is not E_x).
 * Asynchronous, like lace_apply_exchange.  Errors: EINVAL (n_occ < 1,
 * n_virt < 0, ...), ENOMEM, EHIP. */
int lace_apply_exchange_virtual(lace_plan* plan, int cell, const void* psi_g,
                                int n_occ, int n_virt, double s_thr,
                                void* w_g, double* e_x, int64_t* n_kept,
                                void* ws, size_t ws_bytes,
                                lace_stream_t stream);

/* Orbital alignment, the aid to tight SCF convergence at the end of Sec. 2
 * (align the orbitals of one iteration to those of the previous one).
 * Reading: the unitary U that minimizes ||psi_new U - psi_old||_F (the
 * orthogonal Procrustes problem) is the polar factor of
 * A = psi_new^H psi_old; psi_out = psi_new U spans the space of psi_new.
 * U is computed on the device by 30 Newton-Schulz steps
 * X <- X (3 I - X^H X) / 2 from X_0 = A / b, b^2 >= the largest eigenvalue
 * of A^H A (Gershgorin); singular values of A below ~1e-4 of the largest
 * are not resolved (resid then stays large).
 *   psi_new, psi_old  device, n_pw x n_orb complex128.
 *   psi_out  device, n_pw x n_orb complex128, distinct from both inputs.
 *   resid    device double (may be NULL): ||U^H U - I||_F / sqrt(n_orb).
 * Workspace of n_orb.  Asynchronous.  Errors: EINVAL, ENOMEM, EHIP. */
int lace_align(lace_plan* plan, int cell, const void* psi_new,
               const void* psi_old, int n_orb, void* psi_out, double* resid,
               void* ws, size_t ws_bytes, lace_stream_t stream);

/* Localization by selected columns of the density matrix (SCDM; Sec. 2
 * localizes the occupied manifold this way before screening; its modified
 * version is not described, so this is the cited method itself).  The
 * n_orb grid points r_k are picked greedily by column-pivoted QR of
 * Psi^H on the grid (each pick maximizes the part of conj(psi(r)) outside
 * the span of the earlier picks); the localized orbitals are the density
 * matrix columns P(., r_k), Loewdin-orthonormalized:
 * phi = psi U, U the polar factor of A, A[n][k] = conj(psi_n(r_k)).
 * Picks use the plan's grids (FP32 or FP64) with FP64 sums; U comes from
 * the Newton-Schulz iteration of lace_align.
 *   psi_g   device, n_pw x n_orb complex128, orthonormal.
 *   phi_g   device, n_pw x n_orb complex128 output (not psi_g).
 *   points  device int32 [n_orb] (may be NULL): the picks in order, as flat
 *           grid indices (z n + y) n + x.
 *   resid   device double (may be NULL): ||U^H U - I||_F / sqrt(n_orb).
 * n_orb <= 3072.  Workspace of n_orb.  Asynchronous (n_orb steps, each a
 * pass over the orbital grids).  Errors: EINVAL, ENOMEM, EHIP. */
int lace_scdm(lace_plan* plan, int cell, const void* psi_g, int n_orb,
              void* phi_g, int32_t* points, double* resid, void* ws,
              size_t ws_bytes, lace_stream_t stream);

/* ACE projector from psi and W = K psi (Eqs. (3)-(5), (9)).
 *   m_out   device n_orb x n_orb complex128 (may be NULL): M = psi^H W.
 *   xi_g    device n_pw x n_orb complex128 output: xi = W L^{-H} with
 *           -M_s = L L^H, L lower triangular with positive diagonal.
 *   ex_tr   device double (may be NULL): (1/2) Re tr M.
 *   info    device int32 (may be NULL): 0 when the Cholesky factorization
 *           succeeds, else k + 1 for the first non-positive pivot k; xi is
 *           then undefined.  NULL writes the word into the workspace
 *           instead (its first 4 bytes), where lace_get_info reads it.
 *           Each call clears and sets only its own word, so builds on
 *           different streams with different workspaces (or info words)
 *           never see each other's failures.
 * Asynchronous. */
int lace_build_ace(lace_plan* plan, int cell, const void* psi_g,
                   const void* w_g, int n_orb, lace_sym sym, void* xi_g,
                   void* m_out, double* ex_tr, int32_t* info, void* ws,
                   size_t ws_bytes, lace_stream_t stream);

/* y = -xi (xi^H x): the compressed exchange applied to n_vec functions.
 * xi_g device n_pw x n_orb, x_g device n_pw x n_vec, y_g device
 * n_pw x n_vec (complex128; y_g must not alias x_g).  Asynchronous. */
int lace_apply_ace(lace_plan* plan, int cell, const void* xi_g, int n_orb,
                   const void* x_g, int n_vec, void* y_g, void* ws,
                   size_t ws_bytes, lace_stream_t stream);

/* lace_apply_ace without a workspace, for callers that cannot allocate
 * device memory or pass one: code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation.  Arguments, layouts and the
 * result are those of lace_apply_ace (the same kernels, bit for bit).
 * The intermediate xi^H x and its split-K partials live in one fixed
 * 96 MiB array per GPU that the library holds until the process ends;
 * the call allocates nothing.  A problem whose n_orb x n_vec product and
 * partials need more than that returns LACE_ENOMEM before any work is
 * enqueued (n_orb = n_vec = 1024 fits at any n_pw).  Every call on a GPU
 * shares that GPU's array: calls that overlap in time on one GPU
 * (different streams, or different host threads) race, and the caller
 * must order them.
 * The plan must have been created on the current device.  Asynchronous. */
int lace_apply_ace_noalloc(lace_plan* plan, int cell, const void* xi_g,
                           int n_orb, const void* x_g, int n_vec, void* y_g,
                           lace_stream_t stream);

/* One job of lace_apply_exchange_batched: the exchange (and optionally the
 * ACE build) of one set of orbitals on one cell of the plan.  Fields are as
 * in lace_apply_exchange / lace_build_ace; each job brings its own
 * workspace (sized by lace_workspace_size for its cell and n_orb) because
 * jobs run concurrently. */
typedef struct {
  int32_t cell;
  const void* psi_g;     /* device n_pw x n_orb complex128 */
  int32_t n_orb;
  double s_thr;          /* [0, 1) */
  void* w_g;             /* device n_pw x n_orb complex128, output */
  double* e_x;           /* device, may be NULL */
  int64_t* n_kept;       /* device int64, may be NULL: pairs run */
  int32_t sym;           /* lace_sym, used when xi_g != NULL */
  void* xi_g;            /* device n_pw x n_orb, or NULL: no ACE build */
  void* m_out;           /* device n_orb x n_orb complex128, may be NULL */
  double* ex_tr;         /* device, may be NULL */
  int32_t* info;         /* device int32, may be NULL (then the job's
                            workspace word): Cholesky info of the ACE build */
  void* ws;              /* device workspace of this job */
  size_t ws_bytes;
} lace_job;

#define LACE_BATCH_GRAPH 1  /* capture the device work in one HIP graph */

/* Several independent exchange applications (and ACE builds) at once, on
 * cells of any supported sizes: the multi-cell batching of the same method.
 * Jobs are spread over the plan's internal streams (forked from and joined
 * back to `stream`), so small cells overlap on the device.  Every step of
 * every job (grid orbitals, screening, pair list and schedule, pair
 * pipeline, W back-transform, ACE build) runs on the device; the call is
 * asynchronous.  With LACE_BATCH_GRAPH all of it is captured in one HIP
 * graph, cached on the plan and replayed while the jobs' buffers, counts,
 * thresholds and the plan's tuning stay the same (a replay screens the
 * orbitals the buffers then hold).  Results are identical to running each
 * job alone (same kernels, same schedule, same summation order).  Errors:
 * EINVAL (a bad job, two jobs sharing a workspace, W or info word),
 * ENOMEM (a job workspace too small), EHIP. */
int lace_apply_exchange_batched(lace_plan* plan, lace_job* jobs, int n_jobs,
                                int flags, lace_stream_t stream);

/* Per-cell tuning of the pair pipeline (the Poisson solves of Eq. (2) by
 * FFT), host only:
 *   pairs_per_batch  1..64; real-orbital plans 1..128 (two pairs per slot)
 *   use_plane  the xy schedule: 1, fused xy-plane passes (where the plane
 *              fits LDS); 2, the xy plane in two halves of N/2 rows after a
 *              radix-2 split along y (half the LDS, two workgroups per CU);
 *              0, separate x and y pencil passes
 *   z_tile     the z pass's tile of the flattened xy plane per z row: 0,
 *              256 bytes (32 FP32 or 16 FP64 complex points); 1, half as
 *              wide; 2, twice as wide (where the plane divides into such
 *              tiles, else the default)
 *   radix_order  0, the radices of each transform length in the listed
 *              order (e.g. 120 = 8 x 15, 60 = 4 x 15); 1, reversed
 * EINVAL for values out of range, EUNSUPPORTED for use_plane = 1 where the
 * plane does not fit LDS. */
int lace_set_tuning(lace_plan* plan, int cell, int pairs_per_batch,
                    int use_plane, int z_tile, int radix_order);
int lace_get_tuning(const lace_plan* plan, int cell, int* pairs_per_batch,
                    int* use_plane, int* z_tile, int* radix_order);

/* Autotuner: times the pair pipeline of this cell on the given orbitals
 * and the pairs that S keeps at s_thr (Eq. (6); 0 keeps every pair), on
 * two internal streams as the exchange runs it, each candidate with its
 * own schedule of those pairs.  Stage 1: every pairs per batch (8, 16, 32,
 * 64, and 128 for real-orbital plans) with every xy schedule that exists
 * (half-plane, plane, pencil), timed on its first batches holding at
 * least 2048 pairs; the three fastest again over their whole schedules as
 * the exchange runs them (the batches past the schedule's end included).
 * Stage 2, for the fastest of those: the z tiles half and twice as wide
 * and the reversed radix order, where they differ from the default, over
 * the whole schedule.  Every time includes its pairs' share of the time
 * the device takes to build that candidate's schedule.  Keeps the fastest
 * whole-schedule time with lace_set_tuning.  Writes up to *n_cand
 * candidates (cand_ppb, cand_plane, cand_ztile, cand_radix,
 * cand_us_per_pair: the whole-schedule time where it was taken, else the
 * first batches'; host arrays, may be NULL) and sets *n_cand to the number
 * timed.  Synchronizes the stream.  The workspace is the one of
 * lace_workspace_size (W is overwritten). */
int lace_autotune(lace_plan* plan, int cell, const void* psi_g, int n_orb,
                  double s_thr, void* ws, size_t ws_bytes, lace_stream_t stream,
                  int* cand_ppb, int* cand_plane, int* cand_ztile,
                  int* cand_radix, double* cand_us_per_pair, int* n_cand);

/* In-place 3D FFT of `count` n^3 grids stored back to back in the plan
 * precision (complex64 or complex128, x fastest).  direction -1: forward
 * (exp(-i G.r)), +1: backward; both unscaled.  Exposed so the transform
 * itself can be tested.  Asynchronous. */
int lace_fft3d(lace_plan* plan, int cell, int direction, void* grids,
               int count, lace_stream_t stream);

/* Info word kept in a workspace: that of the last lace_build_ace (or
 * batched job) that used workspace `ws` with info == NULL: 0 if the
 * Cholesky factorization succeeded, else k + 1 for the first non-positive
 * pivot k.  Synchronizes `stream` (the stream of that call) only, then
 * copies the word.  Returns LACE_OK when the word is 0 and LACE_ENOTPD when
 * it is not (*info_host is filled in both cases); EINVAL for NULL
 * pointers, EHIP. */
int lace_get_info(const void* ws, lace_stream_t stream, int32_t* info_host);

/* Host only, no device work: the batch schedule that lace_apply_exchange
 * builds on the device for plans of complex orbitals, computed the same way
 * on the host (the results are identical).  The n_pairs unordered pairs
 * (host arrays, 0 <= i <= j < n_orb <= 4096, no repeats) are grouped into
 * batches of at most per_batch (1..64) pairs in which no orbital appears
 * twice; batch_of[k] (host, n_pairs int32) receives the batch of pair k and
 * *n_batches the number of batches.  Pairs are taken round by round of a
 * round-robin tournament over the orbitals (every round a set of disjoint
 * pairs); the list is cut into sections of whole rounds, each section is
 * placed first-fit into a window of eight open batches, and the pairs of
 * the batches that did not fill are placed first-fit once more.  Should
 * that take more batches than the round robin does (one batch per round,
 * or several of per_batch pairs, and the diagonal pairs), the round-robin
 * batches are used instead. */
int lace_schedule_pairs(const int32_t* pair_i, const int32_t* pair_j,
                        int64_t n_pairs, int n_orb, int per_batch,
                        int32_t* batch_of, int64_t* n_batches);

/* Host only, no device work: the schedule lace_apply_exchange builds on the
 * device for plans of real orbitals (LACE_*_GAMMA), where two pair
 * densities share one complex transform, a slot; computed the same way on
 * the host.  Same arguments as lace_schedule_pairs, plus slot_of[k] (host,
 * n_pairs int32), the slot of pair k within its batch.  A slot holds one or
 * two pairs of the same kind (both diagonal or both off-diagonal); two
 * off-diagonal pairs of a slot share an orbital where the pair set allows
 * it (a star slot), so the slot reads and updates three orbital grids
 * instead of four (the pair products are those inside the integrals of
 * Eqs. (2) and (8)).  Stars come from the cycle that two consecutive rounds
 * of the round robin form, then from left-over pairs meeting at an orbital.
 * The slots are packed like the pairs of lace_schedule_pairs (sections of
 * whole cycles, then the unfilled batches once more); the round-robin
 * batches (two pairs of one round per slot, no stars) replace them only
 * when they would number more than the round robin's count b plus
 * max(4, b / 64), since star slots move fewer bytes than a few extra
 * batches cost.  No orbital appears in two slots of one batch; a batch
 * holds at most per_batch pairs (1..128) and (per_batch + 1) / 2 slots. */
int lace_schedule_slots(const int32_t* pair_i, const int32_t* pair_j,
                        int64_t n_pairs, int n_orb, int per_batch,
                        int32_t* batch_of, int32_t* slot_of,
                        int64_t* n_batches);

/* The schedule the last exchange call on workspace `ws` (cell, n_orb of
 * that call) built on the device, read back: for each of the n_pairs given
 * unordered pairs (host arrays) its batch and slot (-1 when the schedule
 * does not hold it), and the number of batches.  Synchronizes `stream`.
 * For tests and inspection.  Errors: EINVAL, EHIP. */
int lace_read_schedule(const lace_plan* plan, int cell, int n_orb,
                       const void* ws, lace_stream_t stream,
                       const int32_t* pair_i, const int32_t* pair_j,
                       int64_t n_pairs, int32_t* batch_of, int32_t* slot_of,
                       int64_t* n_batches);

/* Kernel timing of the pair pipeline of lace_apply_exchange, for
 * roofline measurement.  While enabled, every batch of the pipeline is
 * bracketed by HIP events on the call's stream, one interval per pass:
 *   0  pass A: pair product + forward transform along x and y,
 *   1  pass B: forward z transform, kernel multiply, backward z transform,
 *   2  pass C: backward transform along y and x + accumulation into W.
 * While enabled, an exchange call reads its schedule back (synchronizing
 * the stream) and launches only the batches it holds, one at a time on the
 * call's stream.  lace_profile_enable(plan, 1) clears the totals and starts
 * recording, (plan, 0) stops.  lace_profile_read synchronizes the device and returns
 * per pass: total milliseconds ms[3], launches (batches) launches[3], pairs
 * processed pairs[3], and algorithmic HBM bytes alg_bytes[3].  With U the
 * bytes of one complex grid, G those of one orbital grid (U, or U/2 for
 * real orbitals) and o the distinct orbitals of a transform slot, a slot
 * moves o G + U in pass A (read the orbitals, write the pair buffer), 2 U
 * in pass B, and U + 3 o G in pass C (read the buffer and the orbitals,
 * read and write their W).  Arrays are host memory of 3 elements; any may
 * be NULL. */
int lace_profile_enable(lace_plan* plan, int enable);
int lace_profile_read(lace_plan* plan, double* ms, int64_t* launches,
                      int64_t* pairs, double* alg_bytes);

/* Reality of the orbitals for the Gamma precisions: returns in *rel_dev
 * sqrt(sum |C_m - conj(C_{-m})|^2 / sum |C_m|^2) over all orbitals (0 for
 * real orbitals up to rounding).  Synchronizes the stream.  EINVAL if the
 * plan is not a Gamma plan. */
int lace_check_real(lace_plan* plan, int cell, const void* psi_g, int n_orb,
                    void* ws, size_t ws_bytes, lace_stream_t stream,
                    double* rel_dev);

/* Static text for a status code. */
const char* lace_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif /* LACE_H */
