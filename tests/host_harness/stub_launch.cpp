// Stand-ins for the kernel launchers of internal.hpp: no arithmetic, but
// every launcher writes (or reads) the whole extent of the buffers the real
// kernels write (read), so that the address sanitizer checks the host
// layer's pointers and sizes against the allocations they come from.
#include <cmath>
#include <cstring>
#include <initializer_list>

#include "internal.hpp"

namespace lace {

static void touch(void* p, int64_t bytes) {
  if (bytes > 0) std::memset(p, 0x3c, (size_t)bytes);
}
static unsigned char peek(const void* p, int64_t bytes) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  return bytes > 0 ? (unsigned char)(c[0] ^ c[bytes - 1]) : 0;
}
static int64_t gb(bool fp64) { return fp64 ? 16 : 8; }
static thread_local volatile unsigned char sink;

bool grid_supported(int n) {
  for (int v : {8, 12, 16, 24, 32, 48, 64, 80, 96, 120})
    if (n == v) return true;
  return false;
}
bool plane_fits(int n, bool fp64) { return (int64_t)n * n * gb(fp64) <= 150 * 1024; }
int64_t energy_tiles(int n, bool fp64) { return (int64_t)n * n / (256 / gb(fp64)) + 1; }
int64_t gemm_ip_part_bytes(int na, int nb, int64_t K, bool complex_out) {
  return 2 * (int64_t)na * nb * (complex_out ? 16 : 8) + (K & 7);
}
int64_t scdm_scratch_bytes(int n_orb) { return 4096 * 16 + 16 * (int64_t)n_orb * (n_orb + 1); }

hipError_t launch_fft3d(const CellDev& c, bool fp64, int, void* grids, int count,
                        hipStream_t) {
  touch(grids, count * c.ng * gb(fp64));
  return hipSuccess;
}
hipError_t launch_orbitals_to_grid(const CellDev& c, bool fp64, const void* coeffs,
                                   int n_orb, void* psi, hipStream_t) {
  sink = peek(coeffs, c.n_pw * n_orb * 16);
  touch(psi, n_orb * c.ng * gb(fp64));
  return hipSuccess;
}
hipError_t launch_grid_to_pw(const CellDev& c, bool fp64, void* w, int n_orb,
                             void* w_pw, hipStream_t) {
  touch(w, n_orb * c.ng * gb(fp64));
  touch(w_pw, c.n_pw * n_orb * 16);
  return hipSuccess;
}
static hipError_t batch(const CellDev& c, bool fp64, bool real,
                        const BatchDev* bt, int cap, const void* psi, void* w,
                        void* tmp, double* epart, hipEvent_t* ev) {
  if (cap < 1 || cap > SMAX || bt->n < 0 || bt->n > cap)
    return hipErrorInvalidValue;
  if (ev)
    for (int k = 0; k < 4; ++k)
      if (!ev[k]) return hipErrorInvalidValue;
  const int64_t g = c.ng * gb(fp64) / (real ? 2 : 1);
  for (int q = 0; q < bt->n; ++q)
    for (int o : {bt->i[q], bt->j[q], bt->k[q], bt->l[q]}) {
      if (o < 0) continue;
      sink = peek(static_cast<const char*>(psi) + o * g, g);
      touch(static_cast<char*>(w) + o * g, g);
    }
  touch(tmp, cap * c.ng * gb(fp64));
  touch(epart, cap * energy_tiles(c.n, fp64) * (int64_t)sizeof(double));
  return hipSuccess;
}
hipError_t launch_pair_batch(const CellDev& c, bool fp64, const BatchDev* bt,
                             int cap, const void* psi, void* w, void* tmp,
                             double* epart, hipStream_t, hipEvent_t* ev,
                             const BatchSync*) {
  return batch(c, fp64, false, bt, cap, psi, w, tmp, epart, ev);
}
hipError_t launch_orbitals_to_grid_real(const CellDev& c, bool fp64,
                                        const void* coeffs, int n_orb,
                                        void* psi_real, void* scratch, hipStream_t) {
  sink = peek(coeffs, c.n_pw * n_orb * 16);
  touch(psi_real, (n_orb + 1) / 2 * c.ng * gb(fp64));
  touch(scratch, (n_orb + 1) / 2 * c.ng * gb(fp64));
  return hipSuccess;
}
hipError_t launch_grid_to_pw_real(const CellDev& c, bool fp64, const void* w_real,
                                  int n_orb, void* scratch, void* w_pw, hipStream_t) {
  sink = peek(w_real, n_orb * c.ng * gb(fp64) / 2);
  touch(scratch, (n_orb + 1) / 2 * c.ng * gb(fp64));
  touch(w_pw, c.n_pw * n_orb * 16);
  return hipSuccess;
}
hipError_t launch_quad_batch(const CellDev& c, bool fp64, const BatchDev* bt,
                             int cap, const void* psi_real, void* w_real,
                             void* tmp, double* epart, hipStream_t,
                             hipEvent_t* ev, const BatchSync*) {
  return batch(c, fp64, true, bt, cap, psi_real, w_real, tmp, epart, ev);
}
hipError_t launch_real_check(const CellDev& c, const void* coeffs, int n_orb,
                             double* part, int* nblocks, hipStream_t) {
  sink = peek(coeffs, c.n_pw * n_orb * 16);
  part[0] = 0.0;
  part[1] = 1.0;
  *nblocks = 1;
  return hipSuccess;
}
// A screening matrix with a band of large overlaps: S_ab = exp(-|a - b| / 3)
static void fake_s(int na, double* out) {
  for (int a = 0; a < na; ++a)
    for (int b = 0; b < na; ++b) out[(int64_t)a * na + b] = std::exp(-std::abs(a - b) / 3.0);
}
hipError_t launch_gemm_ip_abs_real(bool fp64, const void* A, int64_t lda, int na,
                                   int64_t K, double, double* out, void* part,
                                   int64_t part_bytes, hipStream_t) {
  if (gemm_ip_part_bytes(na, na, K, false) > part_bytes) return hipErrorInvalidValue;
  sink = peek(A, (na - 1) * lda * gb(fp64) / 2 + K * gb(fp64) / 2);
  touch(part, part_bytes);
  fake_s(na, out);
  return hipSuccess;
}
hipError_t launch_gemm_ip_abs(bool fp64, const void* A, int64_t lda, int na,
                              int64_t K, double, double* out, void* part,
                              int64_t part_bytes, hipStream_t) {
  if (gemm_ip_part_bytes(na, na, K, false) > part_bytes) return hipErrorInvalidValue;
  sink = peek(A, ((na - 1) * lda + K) * gb(fp64));
  touch(part, part_bytes);
  fake_s(na, out);
  return hipSuccess;
}
hipError_t launch_zero(void* p, int64_t bytes, hipStream_t) {
  if (bytes > 0) std::memset(p, 0, (size_t)bytes);
  return hipSuccess;
}
hipError_t launch_reduce_sum(const double* part, int64_t count, double factor,
                             double* out, hipStream_t) {
  double t = 0.0;
  for (int64_t k = 0; k < count; ++k) t += part[k] != part[k] ? 0.0 : 1e-300;
  *out = factor * t;
  return hipSuccess;
}
hipError_t launch_gemm_ip_c128(const void* A, int64_t lda, int na, const void* B,
                               int64_t ldb, int nb, int64_t K, double, void* out,
                               void* part, int64_t part_bytes, hipStream_t) {
  if (gemm_ip_part_bytes(na, nb, K, true) > part_bytes) return hipErrorInvalidValue;
  sink = peek(A, ((na - 1) * lda + K) * 16);
  sink = peek(B, ((nb - 1) * ldb + K) * 16);
  touch(part, part_bytes);
  touch(out, (int64_t)na * nb * 16);
  return hipSuccess;
}
hipError_t launch_gemm_tall(const void* X, int64_t ldx, int64_t M, int nk,
                            const void* Z, int nb, void* Y, int64_t ldy, hipStream_t) {
  sink = peek(X, ((nk - 1) * ldx + M) * 16);
  sink = peek(Z, (int64_t)nk * nb * 16);
  touch(Y, ((nb - 1) * ldy + M) * 16);
  return hipSuccess;
}
hipError_t launch_neg_sym(const void* M, int n, int mode, void* A, hipStream_t) {
  if (mode < 0 || mode > 2) return hipErrorInvalidValue;
  sink = peek(M, (int64_t)n * n * 16);
  touch(A, (int64_t)n * n * 16);
  return hipSuccess;
}
hipError_t launch_cholesky(void* A, int n, int32_t* info, void* tmp, void* part,
                           int64_t part_bytes, hipStream_t) {
  touch(A, (int64_t)n * n * 16);
  if (n > 64) touch(tmp, (int64_t)(n - 64) * (n - 64) * 16);
  if (n > 64 && gemm_ip_part_bytes(n - 64, n - 64, 64, true) > part_bytes)
    return hipErrorInvalidValue;
  *info = 0;
  return hipSuccess;
}
hipError_t launch_trinv_adj(const void* L, int n, void* Z, hipStream_t) {
  sink = peek(L, (int64_t)n * n * 16);
  touch(Z, (int64_t)n * n * 16);
  return hipSuccess;
}
hipError_t launch_trace_re(const void* M, int n, double factor, double* out,
                           hipStream_t) {
  sink = peek(M, (int64_t)n * n * 16);
  *out = factor;
  return hipSuccess;
}
hipError_t launch_polar_elem(int, const void* in, int n, const double*, void* out,
                             hipStream_t) {
  sink = peek(in, (int64_t)n * n * 16);
  touch(out, (int64_t)n * n * 16);
  return hipSuccess;
}
hipError_t launch_polar_norm(int, const void* B, int n, double* out, hipStream_t) {
  sink = peek(B, (int64_t)n * n * 16);
  *out = 1.0;
  return hipSuccess;
}
int64_t sched_scratch_bytes(int n_orb) { return 4096 + 64 * (int64_t)n_orb * n_orb; }
int ztile_points(int n, bool fp64, int z) {
  const int def = fp64 ? 16 : 32;
  const int tx = z == 1 ? def / 2 : z == 2 ? def * 2 : def;
  return (n * n) % tx == 0 ? tx : def;
}
bool radix_orders_differ(int n) { return n != 8 && n != 12 && n != 16 && n != 64; }
int sched_sections(int n_orb) {
  const int64_t s = (int64_t)n_orb * n_orb / 4096;
  return s < 1 ? 1 : s > 16 ? 16 : (int)s;
}
int64_t sched_slot_bound(int n_orb) {
  return (int64_t)n_orb * (n_orb + 1) / 2 + (int64_t)n_orb * n_orb / 4 + n_orb + 8;
}
// A schedule of the diagonal pairs, one per batch, written where the device
// scheduler writes its table; the scratch is touched whole.
hipError_t launch_schedule(const SchedDesc& d, hipStream_t) {
  if (d.n_orb < 1 || d.ppb < 1 || d.ppb > PMAX || d.max_batches < 1) return hipErrorInvalidValue;
  if (!d.pair_i && d.s && d.s_n < 1) return hipErrorInvalidValue;
  if (d.s) sink = peek(d.s, 8 * (int64_t)d.s_n * d.s_n);
  if (d.pair_i) {
    sink = peek(d.pair_i, 4 * d.n_pairs);
    sink = peek(d.pair_j, 4 * d.n_pairs);
  }
  touch(d.scratch, sched_scratch_bytes(d.n_orb));
  const int64_t nb = d.max_batches < d.n_orb ? d.max_batches : d.n_orb;
  for (int64_t b = 0; b < d.max_batches; ++b) {
    BatchDev& t = d.table[b];
    std::memset(&t, 0, sizeof(t));
    if (b < nb) { t.n = 1; t.npairs = 1; t.i[0] = t.j[0] = (int)b; t.k[0] = t.l[0] = -1; }
  }
  *d.n_batches = (int32_t)nb;
  if (d.n_kept) *d.n_kept = nb;
  if (d.bad) *d.bad = 0;
  return hipSuccess;
}
hipError_t launch_kept_pairs(const double* s, int n, double, int32_t* cnt,
                             int64_t* off, int32_t* pairs, int64_t* total,
                             hipStream_t) {
  if (s) sink = peek(s, 8 * (int64_t)n * n);
  touch(cnt, 4 * (int64_t)n);
  touch(off, 8 * ((int64_t)n + 1));
  touch(pairs, 4 * (int64_t)n * (n + 1));
  if (total) *total = (int64_t)n * (n + 1) / 2;
  return hipSuccess;
}

hipError_t launch_scdm(bool fp64, bool real, const void* psi, int n_orb,
                       int64_t ng, double* d, void* scratch, int32_t* points,
                       void* Y, hipStream_t) {
  sink = peek(psi, n_orb * ng * gb(fp64) / (real ? 2 : 1));
  touch(d, ng * (int64_t)sizeof(double));
  touch(scratch, scdm_scratch_bytes(n_orb));
  for (int k = 0; k < n_orb; ++k) points[k] = k;
  touch(Y, (int64_t)n_orb * n_orb * 16);
  return hipSuccess;
}

}  // namespace lace
