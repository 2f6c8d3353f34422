// internal.hpp - launchers shared between the C-ABI layer and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

namespace lace {

// First-launch guard.  Before a kernel is launched for the first time on a
// device, the runtime loads the library's code object and looks the kernel
// up.  resolve_kernel does that lookup (hipFuncGetAttributes) under one
// process-wide mutex and marks the kernel resolved on the current device,
// so first launches from several host threads (one plan per thread) never
// run the lookup concurrently; later launches only test a bit.
hipError_t resolve_kernel(const void* kernel, std::atomic<uint64_t>& done);
template <auto K> struct KernelOnce {
  static inline std::atomic<uint64_t> done{0};   // bit d: resolved on device d
};
template <auto K> inline hipError_t resolved() {
  return resolve_kernel(reinterpret_cast<const void*>(K), KernelOnce<K>::done);
}

// A batch holds at most SMAX slots (one bit per slot in 64-bit masks) and
// PMAX pairs: one pair per slot for complex orbitals, up to two for real
// orbitals.
constexpr int SMAX = 64;
constexpr int PMAX = 128;

// One batch of the pair pipeline as the kernels read it from device memory.
// Slot q: complex orbitals hold one pair (i[q], j[q]); real orbitals pack
// two pair densities rho_ij + i rho_kl in one transform (k = l = -1: a
// single pair; k = i: a star slot, whose two pairs share orbital i).  No
// orbital appears in two slots.  Batches past the end of a schedule have
// n = 0, and every kernel of such a batch returns at once.
struct BatchDev {
  int32_t n;          // slots
  int32_t star;       // 1: every slot is a star slot (real orbitals)
  int32_t npairs;     // pairs in the batch
  int32_t pad;
  uint64_t one_sided; // bit q: slot q holds one-sided pairs (no energy)
  uint64_t skip[4];   // bit q: W_i, W_j, W_k, W_l of slot q not updated
  int32_t i[SMAX], j[SMAX], k[SMAX], l[SMAX];
};

// Geometry and device tables of one cell, shared by all launchers.
struct CellDev {
  int n;              // grid points per axis
  int64_t ng;         // n^3
  int64_t n_pw;
  double L, rc, omega;
  const int32_t* gidx;  // n_pw linear grid indices (x + n (y + n z))
  const void* vtab;     // v(G) / ng in the plan precision for one octant,
                        // 0 <= kx, ky, kz <= n/2, index (kz (n/2+1) + ky)
                        // (n/2+1) + kx (v depends on |G| only; cubic cell)
  const void* tw;       // n twiddles exp(-2 pi i m / n), plan precision
  const int32_t* negidx;  // n_pw: position of -m in the Miller list (Gamma)
  int ppb;              // pairs per batch (1..PMAX; complex orbitals 1..SMAX)
  int use_plane;        // 1: fused xy-plane passes where the plane fits LDS
  int ztile;            // z-pass tile: 0 default, 1 half as wide, 2 twice
  int radix;            // radix order of the pair passes' transforms: 0, 1
                        // reversed
};

bool grid_supported(int n);
// Whether the fused xy-plane pass fits LDS for this size and precision.
bool plane_fits(int n, bool fp64);

// All launchers enqueue on `st` and return hipSuccess or the launch error.
// Grids are `count` n^3 arrays back to back, x fastest.
hipError_t launch_fft3d(const CellDev& c, bool fp64, int sign, void* grids,
                        int count, hipStream_t st);
// psi grids <- Omega^{-1/2} B[scatter(C)], C device complex128 n_pw x n_orb.
hipError_t launch_orbitals_to_grid(const CellDev& c, bool fp64,
                                   const void* coeffs, int n_orb, void* psi,
                                   hipStream_t st);
// What <- Omega^{1/2}/ng * F[W] gathered on the sphere; W grids destroyed.
hipError_t launch_grid_to_pw(const CellDev& c, bool fp64, void* w, int n_orb,
                             void* w_pw, hipStream_t st);
// One batch of pairs (no orbital used twice): forward, kernel multiply,
// backward, accumulate into W; adds per-tile energy partials.
// Cross-stream order of pass C: wait for wait_c before it, record done_c
// after it (either may be null).
struct BatchSync {
  hipEvent_t wait_c;
  hipEvent_t done_c;
};
// bt: the batch in device memory; cap: its slot capacity (the launch
// grids are sized for cap slots; the kernels read the batch's own count).
// ev (may be null): ev[0..3] recorded before pass A, between the passes and
// after pass C.
hipError_t launch_pair_batch(const CellDev& c, bool fp64, const BatchDev* bt,
                             int cap, const void* psi, void* w, void* tmp,
                             double* epart, hipStream_t st, hipEvent_t* ev,
                             const BatchSync* sy = nullptr);
// ---- real (Gamma-point) orbitals: real grids, packed complex transforms
// psi_real (n_orb real grids) <- real parts of Omega^{-1/2} B[C]; two
// orbitals per complex transform.  psi_real must hold ceil(n_orb/2) complex
// grids (it first receives the packed coefficients); the transform passes
// through `scratch` (as many complex grids, apart from psi_real).
hipError_t launch_orbitals_to_grid_real(const CellDev& c, bool fp64,
                                        const void* coeffs, int n_orb,
                                        void* psi_real, void* scratch,
                                        hipStream_t st);
// What <- Omega^{1/2}/ng F[W] on the sphere for real W grids, two per
// complex transform in `scratch`; W is left intact.
hipError_t launch_grid_to_pw_real(const CellDev& c, bool fp64,
                                  const void* w_real, int n_orb, void* scratch,
                                  void* w_pw, hipStream_t st);
// One batch of packed pair slots of real orbitals (no orbital twice).
hipError_t launch_quad_batch(const CellDev& c, bool fp64, const BatchDev* bt,
                             int cap, const void* psi_real, void* w_real,
                             void* tmp, double* epart, hipStream_t st,
                             hipEvent_t* ev, const BatchSync* sy = nullptr);
// Sum over orbitals of sum_m |C_m - conj(C_{-m})|^2 and sum_m |C_m|^2 into
// part[2 * nblocks] (host reduces); returns the number of blocks used.
hipError_t launch_real_check(const CellDev& c, const void* coeffs, int n_orb,
                             double* part, int* nblocks, hipStream_t st);
// S from real grids (float or double per fp64).
hipError_t launch_gemm_ip_abs_real(bool fp64, const void* A, int64_t lda,
                                   int na, int64_t K, double scale,
                                   double* out, void* part, int64_t part_bytes,
                                   hipStream_t st);

// Number of energy partial slots per pair slot (tiles of the z pass).
int64_t energy_tiles(int n, bool fp64);
// z-pass tile width (points of the flattened xy plane per z row) of tile
// option z (0 default, 1 half, 2 twice) at grid size n.
int ztile_points(int n, bool fp64, int z);
// The two radix orders of the pair passes' transforms (lengths n and n/2)
// differ at grid size n.
bool radix_orders_differ(int n);
hipError_t launch_zero(void* p, int64_t bytes, hipStream_t st);
// out = factor * sum(part[0..count)), fixed summation order.
hipError_t launch_reduce_sum(const double* part, int64_t count, double factor,
                             double* out, hipStream_t st);

// ---- dense linear algebra (FP64, MFMA) ----
// out[a][b] (+ split-K partials in `part`) = scale * sum_k conj(A[a][k]) B[b][k]
// A: na rows of K complex128 (row stride lda), B: nb rows (ldb).
hipError_t launch_gemm_ip_c128(const void* A, int64_t lda, int na,
                               const void* B, int64_t ldb, int nb, int64_t K,
                               double scale, void* out, void* part,
                               int64_t part_bytes, hipStream_t st);
// S[a][b] = scale * sum_k |A[a][k]| |A[b][k]| over K grid values (float2 or
// double2 per fp64), real output.
hipError_t launch_gemm_ip_abs(bool fp64, const void* A, int64_t lda, int na,
                              int64_t K, double scale, double* out, void* part,
                              int64_t part_bytes, hipStream_t st);
int64_t gemm_ip_part_bytes(int na, int nb, int64_t K, bool complex_out);
// Y[b][m] = sum_k X[k][m] Z[k][b]: X nk rows of M complex128 (ldx), Z nk x nb
// row-major complex128, Y nb rows (ldy).
hipError_t launch_gemm_tall(const void* X, int64_t ldx, int64_t M, int nk,
                            const void* Z, int nb, void* Y, int64_t ldy,
                            hipStream_t st);
// A <- -sym(M) (mode 0 avg, 1 upper, 2 lower), n x n complex128 row-major.
hipError_t launch_neg_sym(const void* M, int n, int mode, void* A,
                          hipStream_t st);
// In-place Cholesky A = L L^H (lower), info <- 0 or the first failing
// pivot + 1.  tmp: (n - 64)^2 complex128 scratch; part: split-K
// scratch of the trailing-update GEMMs.
hipError_t launch_cholesky(void* A, int n, int32_t* info, void* tmp,
                           void* part, int64_t part_bytes, hipStream_t st);
// Z <- (L^{-1})^H, upper triangular, n x n row-major.
hipError_t launch_trinv_adj(const void* L, int n, void* Z, hipStream_t st);
// out <- factor * Re tr(M)
hipError_t launch_trace_re(const void* M, int n, double factor, double* out,
                           hipStream_t st);

// Polar-iteration helpers, n x n complex128 row-major.  elem: 0 conj,
// 1 scale by *s, 2 (3 I - in) / 2, 3 transpose (out distinct from in).
// norm: 0 Gershgorin scale 1 / sqrt(max row sum |B|), 1 ||B - I||_F / sqrt n.
hipError_t launch_polar_elem(int mode, const void* in, int n, const double* s,
                             void* out, hipStream_t st);
hipError_t launch_polar_norm(int mode, const void* B, int n, double* out,
                             hipStream_t st);

// ---- screening decision and batch schedule on the device ----
// Kept pairs of Eq. (6) from S (n x n, device): pairs (2 int32 each) column
// by column, *total their count; s == nullptr lists every pair.  cnt: n
// int32, off: n + 1 int64 scratch.
hipError_t launch_kept_pairs(const double* s, int n, double thr, int32_t* cnt,
                             int64_t* off, int32_t* pairs, int64_t* total,
                             hipStream_t st);
// Schedule of the pair pipeline into a batch table (device), from S and a
// threshold or from an explicit device pair list.
struct SchedDesc {
  int n_orb;               // orbitals (occupied first)
  int n_occ;               // n_occ < n_orb: pairs (i < n_occ <= j) are one-sided
  int ppb;                 // pairs per batch
  bool gamma;              // real orbitals: two pairs per slot, stars
  bool force_fallback;     // build the round-robin schedule directly
  int64_t max_batches;     // table entries (the host launches this many)
  const double* s;         // S (device, s_n x s_n) or nullptr: every pair
  int s_n;                 // orbitals with two-sided pairs (S's size)
  double s_thr;
  const int32_t* pair_i;   // explicit list (device) instead of S, or nullptr
  const int32_t* pair_j;
  int64_t n_pairs;
  BatchDev* table;         // device, max_batches entries
  int32_t* n_batches;      // device: batches used
  int64_t* n_kept;         // device: pairs scheduled (may be null)
  int32_t* bad;            // device: bit 0 set for a bad explicit list (may be null)
  void* scratch;           // sched_scratch_bytes(n_orb)
};
int64_t sched_scratch_bytes(int n_orb);
hipError_t launch_schedule(const SchedDesc& d, hipStream_t st);
// First-fit sections of the schedule for n_orb orbitals, and the bound on
// its slots (the host form of the schedule uses the same).
int sched_sections(int n_orb);
int64_t sched_slot_bound(int n_orb);

// SCDM point selection on the workspace orbital grids (complex or real,
// FP32 or FP64): n_orb greedy picks of column-pivoted QR of Psi^H into
// points (device int32), then Y[k][n] = conj(psi_n(points[k])) (n_orb x n_orb
// complex128 row-major).  d: ng doubles; scratch: scdm_scratch_bytes.
int64_t scdm_scratch_bytes(int n_orb);
hipError_t launch_scdm(bool fp64, bool real, const void* psi, int n_orb,
                       int64_t ng, double* d, void* scratch, int32_t* points,
                       void* Y, hipStream_t st);

}  // namespace lace

// Every kernel launch of the library: the first-launch guard, then the
// launch.  Used inside functions that return hipError_t (a failed guard
// returns its error).
#define LACE_LAUNCH(K, ...)                                        \
  do {                                                             \
    const hipError_t lace_resolve_err_ = ::lace::resolved<K>();    \
    if (lace_resolve_err_ != hipSuccess) return lace_resolve_err_; \
    hipLaunchKernelGGL(K, __VA_ARGS__);                            \
  } while (0)
