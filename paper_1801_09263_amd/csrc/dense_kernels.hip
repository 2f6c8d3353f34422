// dense_kernels.hip - FP64 dense linear algebra of the ACE construction.
//
//   M   = psi^H W          (Eq. (3); M' of Eq. (9) when W is truncated)
//   S   = |psi|^T |psi| dV (Eq. (6), screening)
//   T   = xi^H x,  y = -xi T  (ACE application)
//   -M_s = L L^H, Z = L^{-H}, xi = W Z  (Eqs. (4)-(5))
//
// The contractions run on the FP64 matrix cores with
// v_mfma_f64_16x16x4_f64: per wave D(16x16) += A(16x4) B(4x16), where
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and holds
// D[l / 16 + 4 e][l % 16] in accumulator element e (rows interleaved; the
// layout was confirmed with a one-wave probe on gfx950).
#include <hip/hip_runtime.h>
#include <cmath>

#include "internal.hpp"

namespace lace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ inline d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------------
// Inner-product GEMM with split K:
//   part[z][a][b] = sum_{k in chunk z} op(A[a][k]) op(B[b][k])
// MODE 0: complex, op(A) = conj(A), op(B) = B (complex128 inputs)
// MODE 1: real, op = |.| of float2 inputs (computed in FP64)
// MODE 2: real, op = |.| of double2 inputs
// MODE 3, 4: real, op = |.| of float / double inputs (real grids)
// (the screening product of FP32 grids, modes 1 and 3, runs on the FP32
// matrix cores in k_gemm_ip_f32 below)
// Workgroup: 256 threads = 4 waves in a 2 x 2 arrangement, 64 x 64 output,
// each wave a 32 x 32 block (2 x 2 MFMA tiles).  K is staged through LDS
// in chunks of KC (32 real, 16 complex) with coalesced row loads; the
// next chunk's loads are issued before the current chunk's MFMAs, so
// their latency hides behind the matrix work.  SYM (A = B): only the
// tiles on and above the diagonal are computed; the reduction mirrors.
// ------------------------------------------------------------------
constexpr int IP_T = 64;
template <int MODE> struct IpKc { static constexpr int value = MODE == 0 ? 16 : 32; };
constexpr int IP_KC_MAX = 32;

// Element loads: load() fetches the raw element (zero when out of range)
// and conv() turns it into the operand, so a prefetched element is not
// waited for until it is converted, at its LDS store.
template <int MODE> struct IpLoad;
template <> struct IpLoad<0> {
  using Raw = double2;
  __device__ static inline Raw load(const void* p, int64_t off) {
    return static_cast<const double2*>(p)[off];
  }
  __device__ static inline Raw zero() { return make_double2(0.0, 0.0); }
  __device__ static inline void conv(Raw v, double& re, double& im) {
    re = v.x; im = v.y;
  }
};
template <> struct IpLoad<1> {
  using Raw = float2;
  __device__ static inline Raw load(const void* p, int64_t off) {
    return static_cast<const float2*>(p)[off];
  }
  __device__ static inline Raw zero() { return make_float2(0.f, 0.f); }
  __device__ static inline void conv(Raw v, double& re, double& im) {
    const double x = v.x, y = v.y;
    re = sqrt(x * x + y * y); im = 0.0;
  }
};
template <> struct IpLoad<2> {
  using Raw = double2;
  __device__ static inline Raw load(const void* p, int64_t off) {
    return static_cast<const double2*>(p)[off];
  }
  __device__ static inline Raw zero() { return make_double2(0.0, 0.0); }
  __device__ static inline void conv(Raw v, double& re, double& im) {
    re = sqrt(v.x * v.x + v.y * v.y); im = 0.0;
  }
};
template <> struct IpLoad<3> {
  using Raw = float;
  __device__ static inline Raw load(const void* p, int64_t off) {
    return static_cast<const float*>(p)[off];
  }
  __device__ static inline Raw zero() { return 0.f; }
  __device__ static inline void conv(Raw v, double& re, double& im) {
    re = fabs(double(v)); im = 0.0;
  }
};
template <> struct IpLoad<4> {
  using Raw = double;
  __device__ static inline Raw load(const void* p, int64_t off) {
    return static_cast<const double*>(p)[off];
  }
  __device__ static inline Raw zero() { return 0.0; }
  __device__ static inline void conv(Raw v, double& re, double& im) {
    re = fabs(v); im = 0.0;
  }
};

template <int MODE, bool SYM>
__global__ __launch_bounds__(256) void k_gemm_ip(const void* A, int64_t lda,
                                                 int na, const void* B,
                                                 int64_t ldb, int nb,
                                                 int64_t K, int64_t kchunk,
                                                 double* part) {
  constexpr bool CPLX = (MODE == 0);
  constexpr int KC = IpKc<MODE>::value;
  constexpr int PT = IP_T * KC / 256;   // elements per thread and matrix
  __shared__ double sAr[IP_T][KC + 1];
  __shared__ double sBr[IP_T][KC + 1];
  __shared__ double sAi[CPLX ? IP_T : 1][KC + 1];
  __shared__ double sBi[CPLX ? IP_T : 1][KC + 1];
  const int tid = threadIdx.x, lane = tid % 64, w = tid / 64;
  const int wa = w % 2, wb = w / 2;
  int ta = blockIdx.x, tb = blockIdx.y;
  if (SYM) {   // blockIdx.x enumerates the tile pairs ta <= tb, column by column
    ta = blockIdx.x;
    tb = 0;
    while (ta > tb) { ta -= tb + 1; ++tb; }
  }
  const int a0 = ta * IP_T, b0 = tb * IP_T;
  const int64_t kb = blockIdx.z * kchunk;
  int64_t ke = kb + kchunk;
  if (ke > K) ke = K;

  d4 accR[2][2], accI[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      accR[p][q] = d4{0, 0, 0, 0};
      accI[p][q] = d4{0, 0, 0, 0};
    }

  using L = IpLoad<MODE>;
  typename L::Raw xa[PT], xb[PT];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < PT; ++e) {
      const int idx = tid + e * 256;
      const int r = idx / KC, kk = idx % KC;
      const int64_t k = k0 + kk;
      xa[e] = (a0 + r < na && k < ke) ? L::load(A, (a0 + r) * lda + k) : L::zero();
      xb[e] = (b0 + r < nb && k < ke) ? L::load(B, (b0 + r) * ldb + k) : L::zero();
    }
  };
  fetch(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += KC) {
#pragma unroll
    for (int e = 0; e < PT; ++e) {
      const int idx = tid + e * 256;
      const int r = idx / KC, kk = idx % KC;
      double re, im;
      L::conv(xa[e], re, im);
      sAr[r][kk] = re;
      if (CPLX) sAi[r][kk] = im;
      L::conv(xb[e], re, im);
      sBr[r][kk] = re;
      if (CPLX) sBi[r][kk] = im;
    }
    __syncthreads();
    if (k0 + KC < ke) fetch(k0 + KC);
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      const int kk = ks * 4 + lane / 16;
      double ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const int rra = wa * 32 + p * 16 + lane % 16;
        const int rrb = wb * 32 + p * 16 + lane % 16;
        ar[p] = sAr[rra][kk];
        br[p] = sBr[rrb][kk];
        if (CPLX) {
          ai[p] = sAi[rra][kk];
          bi[p] = sBi[rrb][kk];
        }
      }
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          accR[p][q] = mfma(ar[p], br[q], accR[p][q]);
          if (CPLX) {
            // conj(a) b = (ar br + ai bi) + i (ar bi - ai br)
            accR[p][q] = mfma(ai[p], bi[q], accR[p][q]);
            accI[p][q] = mfma(ar[p], bi[q], accI[p][q]);
            accI[p][q] = mfma(-ai[p], br[q], accI[p][q]);
          }
        }
    }
    __syncthreads();
  }
  double* out = part + (int64_t)blockIdx.z * na * nb * (CPLX ? 2 : 1);
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int a = a0 + wa * 32 + p * 16 + lane / 16 + 4 * e;
        const int b = b0 + wb * 32 + q * 16 + lane % 16;
        if (a < na && b < nb) {
          if (CPLX) {
            out[2 * ((int64_t)a * nb + b)] = accR[p][q][e];
            out[2 * ((int64_t)a * nb + b) + 1] = accI[p][q][e];
          } else {
            out[(int64_t)a * nb + b] = accR[p][q][e];
          }
        }
      }
}

// The screening product S = |A|^T |B| of FP32 grids on the FP32 matrix
// cores: MODE 3 real grids (|x|), MODE 1 complex grids (|z| in FP32).  The
// same tiling as k_gemm_ip (64 x 64 per workgroup, 2 x 2 waves of 2 x 2
// v_mfma_f32_16x16x4f32 tiles) with K staged in chunks of 64; each chunk's
// FP32 sums are added into FP64 accumulators, so FP32 rounding acts on
// 64-term sums only.  Partials in FP64 as k_gemm_ip's.
typedef float f4 __attribute__((ext_vector_type(4)));

template <int MODE> struct IpLoad32;
template <> struct IpLoad32<1> {
  using Raw = float2;
  __device__ static inline Raw load(const void* p, int64_t off) {
    return static_cast<const float2*>(p)[off];
  }
  __device__ static inline Raw zero() { return make_float2(0.f, 0.f); }
  __device__ static inline float conv(Raw v) { return sqrtf(v.x * v.x + v.y * v.y); }
};
template <> struct IpLoad32<3> {
  using Raw = float;
  __device__ static inline Raw load(const void* p, int64_t off) {
    return static_cast<const float*>(p)[off];
  }
  __device__ static inline Raw zero() { return 0.f; }
  __device__ static inline float conv(Raw v) { return fabsf(v); }
};

template <int MODE, bool SYM>
__global__ __launch_bounds__(256) void k_gemm_ip_f32(const void* A, int64_t lda,
                                                     int na, const void* B,
                                                     int64_t ldb, int nb,
                                                     int64_t K, int64_t kchunk,
                                                     double* part) {
  constexpr int KC = 64;
  constexpr int PT = IP_T * KC / 256;   // elements per thread and matrix
  __shared__ float sA[IP_T][KC + 1];
  __shared__ float sB[IP_T][KC + 1];
  const int tid = threadIdx.x, lane = tid % 64, w = tid / 64;
  const int wa = w % 2, wb = w / 2;
  int ta = blockIdx.x, tb = blockIdx.y;
  if (SYM) {   // blockIdx.x enumerates the tile pairs ta <= tb, column by column
    ta = blockIdx.x;
    tb = 0;
    while (ta > tb) { ta -= tb + 1; ++tb; }
  }
  const int a0 = ta * IP_T, b0 = tb * IP_T;
  const int64_t kb = blockIdx.z * kchunk;
  int64_t ke = kb + kchunk;
  if (ke > K) ke = K;

  d4 acc[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[p][q] = d4{0, 0, 0, 0};

  using L = IpLoad32<MODE>;
  typename L::Raw xa[PT], xb[PT];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < PT; ++e) {
      const int idx = tid + e * 256;
      const int r = idx / KC, kk = idx % KC;
      const int64_t k = k0 + kk;
      xa[e] = (a0 + r < na && k < ke) ? L::load(A, (a0 + r) * lda + k) : L::zero();
      xb[e] = (b0 + r < nb && k < ke) ? L::load(B, (b0 + r) * ldb + k) : L::zero();
    }
  };
  fetch(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += KC) {
#pragma unroll
    for (int e = 0; e < PT; ++e) {
      const int idx = tid + e * 256;
      const int r = idx / KC, kk = idx % KC;
      sA[r][kk] = L::conv(xa[e]);
      sB[r][kk] = L::conv(xb[e]);
    }
    __syncthreads();
    if (k0 + KC < ke) fetch(k0 + KC);
    f4 c[2][2];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q) c[p][q] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      const int kk = ks * 4 + lane / 16;
      float av[2], bv[2];
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        av[p] = sA[wa * 32 + p * 16 + lane % 16][kk];
        bv[p] = sB[wb * 32 + p * 16 + lane % 16][kk];
      }
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
          c[p][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[p], bv[q], c[p][q], 0, 0, 0);
    }
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[p][q][e] += (double)c[p][q][e];
    __syncthreads();
  }
  double* out = part + (int64_t)blockIdx.z * na * nb;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        // v_mfma_f32_16x16x4f32 holds D[4 (l / 16) + e][l % 16] in lane l
        const int a = a0 + wa * 32 + p * 16 + 4 * (lane / 16) + e;
        const int b = b0 + wb * 32 + q * 16 + lane % 16;
        if (a < na && b < nb) out[(int64_t)a * nb + b] = acc[p][q][e];
      }
}

// out[e] = scale * sum_z part[z][e].  A workgroup takes 16 elements at a
// time; lane group g (of 16) sums z = g, g + 16, ... in increasing order,
// then the 16 group sums are added in group order: one fixed order for any
// grid, so results repeat bitwise.  sym_nb > 0: a real sym_nb x sym_nb
// result of which only the tiles on and above the diagonal were computed;
// an element below reads its mirror.
constexpr int RED_E = 16, RED_G = 16;
__global__ __launch_bounds__(RED_E * RED_G) void k_splitk_reduce(
    const double* part, int64_t nel, int nsplit, double scale, double* out,
    int sym_nb) {
  __shared__ double red[RED_G][RED_E + 1];
  const int el = threadIdx.x % RED_E, g = threadIdx.x / RED_E;
  for (int64_t e0 = (int64_t)blockIdx.x * RED_E; e0 < nel;
       e0 += (int64_t)gridDim.x * RED_E) {
    const int64_t e = e0 + el;
    double t = 0.0;
    if (e < nel) {
      int64_t src = e;
      if (sym_nb > 0) {
        const int64_t a = e / sym_nb, b = e % sym_nb;
        if (a / IP_T > b / IP_T) src = b * sym_nb + a;
      }
      constexpr int U = 8;   // loads in flight; the additions stay in order
      int z = g;
      for (; z + (U - 1) * RED_G < nsplit; z += U * RED_G) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = part[(int64_t)(z + u * RED_G) * nel + src];
#pragma unroll
        for (int u = 0; u < U; ++u) t += v[u];
      }
      for (; z < nsplit; z += RED_G) t += part[(int64_t)z * nel + src];
    }
    red[g][el] = t;
    __syncthreads();
    if (g == 0 && e < nel) {
      double u = 0.0;
      for (int q = 0; q < RED_G; ++q) u += red[q][el];
      out[e] = scale * u;
    }
    __syncthreads();
  }
}

static hipError_t launch_splitk_reduce(const double* part, int64_t nel,
                                       int nsplit, double scale, double* out,
                                       int sym_nb, hipStream_t st) {
  int64_t blocks = (nel + RED_E - 1) / RED_E;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  LACE_LAUNCH(k_splitk_reduce, dim3((unsigned)blocks), dim3(RED_E * RED_G), 0,
              st, part, nel, nsplit, scale, out, sym_nb);
  return hipGetLastError();
}

struct SplitPlan {
  int nsplit;
  int64_t kchunk;
};

// Split K so that about 1024 workgroups run.  The chunk is a multiple of
// the largest KC, which keeps the partial layout the same for every mode.
static SplitPlan split_plan(int na, int nb, int64_t K) {
  const int64_t tiles = (int64_t)((na + IP_T - 1) / IP_T) * ((nb + IP_T - 1) / IP_T);
  int64_t want = (1024 + tiles - 1) / tiles;
  const int64_t maxs = (K + IP_KC_MAX - 1) / IP_KC_MAX;
  if (want > maxs) want = maxs;
  if (want < 1) want = 1;
  int64_t chunk = (K + want - 1) / want;
  chunk = ((chunk + IP_KC_MAX - 1) / IP_KC_MAX) * IP_KC_MAX;
  if (chunk < IP_KC_MAX) chunk = IP_KC_MAX;
  SplitPlan sp;
  sp.kchunk = chunk;
  sp.nsplit = (int)((K + chunk - 1) / chunk);
  if (sp.nsplit < 1) sp.nsplit = 1;
  return sp;
}

int64_t gemm_ip_part_bytes(int na, int nb, int64_t K, bool complex_out) {
  const SplitPlan sp = split_plan(na, nb, K);
  return (int64_t)sp.nsplit * na * nb * (complex_out ? 16 : 8);
}

// SYM: B is A (na = nb), the result is symmetric.
template <int MODE, bool SYM = false>
static hipError_t gemm_ip(const void* A, int64_t lda, int na, const void* B,
                          int64_t ldb, int nb, int64_t K, double scale,
                          double* out, void* part, int64_t part_bytes,
                          hipStream_t st) {
  static_assert(!SYM || MODE != 0, "symmetric only for real results");
  const SplitPlan sp = split_plan(na, nb, K);
  const bool cplx = (MODE == 0);
  if ((int64_t)sp.nsplit * na * nb * (cplx ? 16 : 8) > part_bytes)
    return hipErrorInvalidValue;
  if (SYM && (A != B || na != nb || lda != ldb)) return hipErrorInvalidValue;
  const int ta = (na + IP_T - 1) / IP_T, tb = (nb + IP_T - 1) / IP_T;
  dim3 grid(SYM ? ta * (ta + 1) / 2 : ta, SYM ? 1 : tb, sp.nsplit);
  LACE_LAUNCH((k_gemm_ip<MODE, SYM>), grid, dim3(256), 0, st, A, lda,
                     na, B, ldb, nb, K, sp.kchunk, static_cast<double*>(part));
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  const int64_t nel = (int64_t)na * nb * (cplx ? 2 : 1);
  return launch_splitk_reduce(static_cast<const double*>(part), nel, sp.nsplit,
                              scale, out, SYM ? nb : 0, st);
}

// S of FP32 grids: FP32 products on the matrix cores, FP64 sums.
template <int MODE>
static hipError_t gemm_ip_abs_f32(const void* A, int64_t lda, int na,
                                  int64_t K, double scale, double* out,
                                  void* part, int64_t part_bytes, hipStream_t st) {
  const SplitPlan sp = split_plan(na, na, K);
  if ((int64_t)sp.nsplit * na * na * 8 > part_bytes) return hipErrorInvalidValue;
  const int ta = (na + IP_T - 1) / IP_T;
  dim3 grid(ta * (ta + 1) / 2, 1, sp.nsplit);
  LACE_LAUNCH((k_gemm_ip_f32<MODE, true>), grid, dim3(256), 0, st, A, lda, na,
              A, lda, na, K, sp.kchunk, static_cast<double*>(part));
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  return launch_splitk_reduce(static_cast<const double*>(part), (int64_t)na * na,
                              sp.nsplit, scale, out, na, st);
}

hipError_t launch_gemm_ip_c128(const void* A, int64_t lda, int na,
                               const void* B, int64_t ldb, int nb, int64_t K,
                               double scale, void* out, void* part,
                               int64_t part_bytes, hipStream_t st) {
  return gemm_ip<0>(A, lda, na, B, ldb, nb, K, scale,
                    static_cast<double*>(out), part, part_bytes, st);
}

hipError_t launch_gemm_ip_abs(bool fp64, const void* A, int64_t lda, int na,
                              int64_t K, double scale, double* out, void* part,
                              int64_t part_bytes, hipStream_t st) {
  return fp64 ? gemm_ip<2, true>(A, lda, na, A, lda, na, K, scale, out, part,
                                 part_bytes, st)
              : gemm_ip_abs_f32<1>(A, lda, na, K, scale, out, part, part_bytes, st);
}

hipError_t launch_gemm_ip_abs_real(bool fp64, const void* A, int64_t lda,
                                   int na, int64_t K, double scale,
                                   double* out, void* part, int64_t part_bytes,
                                   hipStream_t st) {
  return fp64 ? gemm_ip<4, true>(A, lda, na, A, lda, na, K, scale, out, part,
                                 part_bytes, st)
              : gemm_ip_abs_f32<3>(A, lda, na, K, scale, out, part, part_bytes, st);
}

// ------------------------------------------------------------------
// Tall GEMM  Y[b][m] = sum_k X[k][m] Z[k][b]  (complex, no conjugation).
// Workgroup 256 threads: 64 rows m (one 16-row block per wave) x 64
// columns b (4 MFMA tiles per wave).  X is read straight from global
// memory (16 consecutive m per k row per wave); the workgroup's columns of
// Z are staged through LDS in chunks of TALL_KC k, read once per
// workgroup instead of once per wave.  The next chunk's X and Z are
// loaded before the current chunk's MFMAs.  The flat workgroup id is remapped so that the column
// blocks of one row block run back to back on one XCD and share its
// rows of X in that XCD's L2.
// ------------------------------------------------------------------
constexpr int TALL_KC = 16;
__global__ __launch_bounds__(256) void k_gemm_tall(const double2* X,
                                                   int64_t ldx, int64_t M,
                                                   int nk, const double2* Z,
                                                   int nb, double2* Y,
                                                   int64_t ldy, int nbb) {
  // Z chunk [TALL_KC][64] in LDS, rows padded by one element
  __shared__ double2 zs[TALL_KC][64 + 1];
  const int tid = threadIdx.x, lane = tid % 64, w = tid / 64;
  // XCD-aware remap of the flat id: XCD x (ids x, x + 8, ...) takes the
  // logical range [x per, (x + 1) per); a ragged tail keeps its id
  const int total = gridDim.x, per = total / 8;
  const int bid = blockIdx.x;
  const int lg = bid < per * 8 ? (bid % 8) * per + bid / 8 : bid;
  const int64_t m0 = (int64_t)(lg / nbb) * 64 + w * 16;
  const int b0 = (lg % nbb) * 64;
  d4 accR[4], accI[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    accR[q] = d4{0, 0, 0, 0};
    accI[q] = d4{0, 0, 0, 0};
  }
  const int64_t m = m0 + lane % 16;
  constexpr int ZPT = TALL_KC * 64 / 256;   // Z elements per thread and chunk
  double2 xn[TALL_KC / 4], zn[ZPT];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int s4 = 0; s4 < TALL_KC / 4; ++s4) {
      const int k = k0 + s4 * 4 + lane / 16;
      xn[s4] = make_double2(0.0, 0.0);
      if (k < nk && m < M) xn[s4] = X[(int64_t)k * ldx + m];
    }
#pragma unroll
    for (int e = 0; e < ZPT; ++e) {
      const int idx = tid + e * 256, kk = idx / 64, bb = idx % 64;
      const int k = k0 + kk, b = b0 + bb;
      zn[e] = make_double2(0.0, 0.0);
      if (k < nk && b < nb) zn[e] = Z[(int64_t)k * nb + b];
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < nk; k0 += TALL_KC) {
    double2 x[TALL_KC / 4];
#pragma unroll
    for (int s4 = 0; s4 < TALL_KC / 4; ++s4) x[s4] = xn[s4];
#pragma unroll
    for (int e = 0; e < ZPT; ++e) {
      const int idx = tid + e * 256;
      zs[idx / 64][idx % 64] = zn[e];
    }
    __syncthreads();
    if (k0 + TALL_KC < nk) fetch(k0 + TALL_KC);
#pragma unroll
    for (int s4 = 0; s4 < TALL_KC / 4; ++s4) {
      const int kk = s4 * 4 + lane / 16;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double2 z = zs[kk][q * 16 + lane % 16];
        accR[q] = mfma(x[s4].x, z.x, accR[q]);
        accR[q] = mfma(-x[s4].y, z.y, accR[q]);
        accI[q] = mfma(x[s4].x, z.y, accI[q]);
        accI[q] = mfma(x[s4].y, z.x, accI[q]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int b = b0 + q * 16 + lane % 16;
    if (b >= nb) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t mm = m0 + lane / 16 + 4 * e;
      if (mm < M) Y[(int64_t)b * ldy + mm] = make_double2(accR[q][e], accI[q][e]);
    }
  }
}

hipError_t launch_gemm_tall(const void* X, int64_t ldx, int64_t M, int nk,
                            const void* Z, int nb, void* Y, int64_t ldy,
                            hipStream_t st) {
  const int nbb = (nb + 63) / 64;
  const int64_t blocks = ((M + 63) / 64) * nbb;
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  LACE_LAUNCH(k_gemm_tall, dim3((unsigned)blocks), dim3(256), 0, st,
                     static_cast<const double2*>(X), ldx, M, nk,
                     static_cast<const double2*>(Z), nb,
                     static_cast<double2*>(Y), ldy, nbb);
  return hipGetLastError();
}

// ------------------------------------------------------------------
// A = -sym(M): mode 0 (M + M^H)/2, 1 upper mirrored, 2 lower mirrored;
// the diagonal is -Re(M_aa) in every mode.
// ------------------------------------------------------------------
__global__ void k_neg_sym(const double2* M, int n, int mode, double2* A) {
  const int64_t total = (int64_t)n * n;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < total;
       e += stride) {
    const int a = (int)(e / n), b = (int)(e % n);
    double2 r;
    if (a == b) {
      r = make_double2(-M[e].x, 0.0);
    } else {
      const double2 u = M[(int64_t)a * n + b];
      const double2 v = M[(int64_t)b * n + a];
      if (mode == 0) {
        r = make_double2(-0.5 * (u.x + v.x), -0.5 * (u.y - v.y));
      } else if ((mode == 1) == (a < b)) {
        r = make_double2(-u.x, -u.y);           // take own triangle
      } else {
        r = make_double2(-v.x, v.y);            // mirror: -conj(M[b][a])
      }
    }
    A[e] = r;
  }
}

hipError_t launch_neg_sym(const void* M, int n, int mode, void* A,
                          hipStream_t st) {
  const int64_t total = (int64_t)n * n;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  LACE_LAUNCH(k_neg_sym, dim3((unsigned)blocks), dim3(256), 0, st,
                     static_cast<const double2*>(M), n, mode,
                     static_cast<double2*>(A));
  return hipGetLastError();
}

// ------------------------------------------------------------------
// Right-looking Cholesky A = L L^H in one workgroup (n <= a few thousand).
// A is row-major complex128, overwritten by L (strict upper zeroed).
// ------------------------------------------------------------------
// Blocked right-looking Cholesky, panels of CB columns: factor the diagonal
// block in LDS (one workgroup), solve the panel below it (one thread per
// row), subtract the panel's outer product from the trailing matrix (an
// MFMA GEMM into tmp, then a lower-triangle update).  The first failing
// pivot is kept in info; later blocks see it and do nothing.
constexpr int CB = 64;

__global__ __launch_bounds__(256) void k_chol_diag(double2* A, int n, int k0,
                                                   int kb, int32_t* info) {
  __shared__ double2 a[CB][CB + 1];
  __shared__ int fail;
  const int tid = threadIdx.x;
  for (int e = tid; e < kb * kb; e += 256) {
    const int i = e / kb, j = e % kb;
    a[i][j] = A[(int64_t)(k0 + i) * n + k0 + j];
  }
  if (tid == 0) fail = (*info != 0) ? -1 : 0;
  __syncthreads();
  if (fail) return;
  for (int k = 0; k < kb; ++k) {
    if (tid == 0) {
      const double d = a[k][k].x;
      if (!(d > 0.0)) fail = k0 + k + 1;
      else a[k][k] = make_double2(sqrt(d), 0.0);
    }
    __syncthreads();
    if (fail) break;
    const double inv = 1.0 / a[k][k].x;
    for (int i = k + 1 + tid; i < kb; i += 256)
      a[i][k] = make_double2(a[i][k].x * inv, a[i][k].y * inv);
    __syncthreads();
    const int m = kb - k - 1;
    for (int e = tid; e < m * m; e += 256) {
      const int i = k + 1 + e / m, j = k + 1 + e % m;
      if (j > i) continue;
      const double2 li = a[i][k], lj = a[j][k];
      a[i][j].x -= li.x * lj.x + li.y * lj.y;
      a[i][j].y -= li.y * lj.x - li.x * lj.y;
    }
    __syncthreads();
  }
  if (fail) {
    if (tid == 0) *info = fail;
    return;
  }
  for (int e = tid; e < kb * kb; e += 256) {
    const int i = e / kb, j = e % kb;
    if (j <= i) A[(int64_t)(k0 + i) * n + k0 + j] = a[i][j];
  }
}

// Rows i >= k0 + kb of the panel: x L_kk^H = a, i.e. forward substitution
// x_j = (a_j - sum_{m<j} x_m conj(L_jm)) / L_jj; one thread per row, 64 rows
// per workgroup, the rows' solutions in LDS.
constexpr int CP_ROWS = 64;
__global__ __launch_bounds__(CP_ROWS) void k_chol_panel(double2* A, int n, int k0,
                                                        int kb, const int32_t* info) {
  __shared__ double2 l[CB][CB + 1];
  __shared__ double2 xs[CP_ROWS][CB + 1];
  for (int e = threadIdx.x; e < kb * kb; e += CP_ROWS) {
    const int i = e / kb, j = e % kb;
    l[i][j] = A[(int64_t)(k0 + i) * n + k0 + j];
  }
  __syncthreads();
  if (*info != 0) return;
  const int t = threadIdx.x;
  const int i = k0 + kb + blockIdx.x * CP_ROWS + t;
  if (i >= n) return;
  double2* row = A + (int64_t)i * n + k0;
  for (int j = 0; j < kb; ++j) {
    double2 s = row[j];
    for (int m = 0; m < j; ++m) {
      const double2 L = l[j][m], x = xs[t][m];   // s -= x_m conj(L_jm)
      s.x -= x.x * L.x + x.y * L.y;
      s.y -= x.y * L.x - x.x * L.y;
    }
    const double inv = 1.0 / l[j][j].x;
    xs[t][j] = make_double2(s.x * inv, s.y * inv);
  }
  for (int j = 0; j < kb; ++j) row[j] = xs[t][j];
}

__global__ void k_set_zero(int32_t* v) { *v = 0; }

// A[i][j] -= T[j - off][i - off] for off <= j <= i < n (T = the GEMM output,
// m x m with m = n - off).
__global__ void k_chol_update(double2* A, int n, int off, const double2* T,
                              const int32_t* info) {
  if (*info != 0) return;
  const int m = n - off;
  const int64_t total = (int64_t)m * m;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < total;
       e += stride) {
    const int i = (int)(e / m), j = (int)(e % m);
    if (j > i) continue;
    const double2 t = T[(int64_t)j * m + i];
    double2& a = A[(int64_t)(off + i) * n + off + j];
    a.x -= t.x;
    a.y -= t.y;
  }
}

__global__ void k_zero_upper(double2* A, int n) {
  const int64_t total = (int64_t)n * n;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < total;
       e += stride)
    if ((int)(e % n) > (int)(e / n)) A[e] = make_double2(0.0, 0.0);
}

hipError_t launch_cholesky(void* Av, int n, int32_t* info, void* tmp,
                           void* part, int64_t part_bytes, hipStream_t st) {
  double2* A = static_cast<double2*>(Av);
  LACE_LAUNCH(k_set_zero, dim3(1), dim3(1), 0, st, info);
  hipError_t e = hipGetLastError();
  for (int k0 = 0; k0 < n && e == hipSuccess; k0 += CB) {
    const int kb = n - k0 < CB ? n - k0 : CB;
    LACE_LAUNCH(k_chol_diag, dim3(1), dim3(256), 0, st, A, n, k0, kb, info);
    e = hipGetLastError();
    const int off = k0 + kb, m = n - off;
    if (e != hipSuccess || m <= 0) continue;
    LACE_LAUNCH(k_chol_panel, dim3((m + CP_ROWS - 1) / CP_ROWS),
                       dim3(CP_ROWS), 0, st, A, n, k0, kb, info);
    e = hipGetLastError();
    // T[a][b] = sum_t conj(L[off + a][k0 + t]) L[off + b][k0 + t]
    if (e == hipSuccess)
      e = launch_gemm_ip_c128(A + (int64_t)off * n + k0, n, m,
                              A + (int64_t)off * n + k0, n, m, kb, 1.0, tmp,
                              part, part_bytes, st);
    if (e == hipSuccess) {
      int64_t blocks = ((int64_t)m * m + 255) / 256;
      if (blocks > 2048) blocks = 2048;
      LACE_LAUNCH(k_chol_update, dim3((unsigned)blocks), dim3(256), 0,
                         st, A, n, off, static_cast<const double2*>(tmp), info);
      e = hipGetLastError();
    }
  }
  if (e == hipSuccess) {
    int64_t blocks = ((int64_t)n * n + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    LACE_LAUNCH(k_zero_upper, dim3((unsigned)blocks), dim3(256), 0, st,
                       A, n);
    e = hipGetLastError();
  }
  return e;
}

// ------------------------------------------------------------------
// Z = (L^{-1})^H.  Workgroup c (one wave) solves L x = e_c by forward
// substitution with x in LDS, then writes row c of Z: Z[c][i] = conj(x_i).
// ------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_trinv_adj(const double2* L, int n,
                                                  double2* Z) {
  extern __shared__ double2 x[];
  const int c = blockIdx.x, l = threadIdx.x;
  for (int i = l; i < n; i += 64) x[i] = make_double2(0.0, 0.0);
  __syncthreads();
  if (l == 0) x[c] = make_double2(1.0 / L[(int64_t)c * n + c].x, 0.0);
  __syncthreads();
  for (int i = c + 1; i < n; ++i) {
    double sr = 0.0, si = 0.0;
    const double2* row = L + (int64_t)i * n;
    for (int m = c + l; m < i; m += 64) {
      const double2 a = row[m], b = x[m];
      sr += a.x * b.x - a.y * b.y;
      si += a.x * b.y + a.y * b.x;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      sr += __shfl_xor(sr, o, 64);
      si += __shfl_xor(si, o, 64);
    }
    if (l == 0) {
      const double d = 1.0 / row[i].x;
      x[i] = make_double2(-sr * d, -si * d);
    }
    __syncthreads();
  }
  for (int i = l; i < n; i += 64) {
    const double2 v = x[i];
    Z[(int64_t)c * n + i] = (i >= c) ? make_double2(v.x, -v.y)
                                     : make_double2(0.0, 0.0);
  }
}

hipError_t launch_trinv_adj(const void* L, int n, void* Z, hipStream_t st) {
  LACE_LAUNCH(k_trinv_adj, dim3(n), dim3(64), n * sizeof(double2), st,
                     static_cast<const double2*>(L), n,
                     static_cast<double2*>(Z));
  return hipGetLastError();
}

__global__ void k_trace_re(const double2* M, int n, double factor,
                           double* out) {
  __shared__ double red[4];
  double t = 0.0;
  for (int a = threadIdx.x; a < n; a += 256) t += M[(int64_t)a * n + a].x;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = t;
  __syncthreads();
  if (threadIdx.x == 0) *out = factor * (red[0] + red[1] + red[2] + red[3]);
}

hipError_t launch_trace_re(const void* M, int n, double factor, double* out,
                           hipStream_t st) {
  LACE_LAUNCH(k_trace_re, dim3(1), dim3(256), 0, st,
                     static_cast<const double2*>(M), n, factor, out);
  return hipGetLastError();
}

// Element-wise steps of the polar (Procrustes) iteration on n x n
// complex128 row-major matrices: 0 out = conj(in); 1 out = *s * in;
// 2 out = (3 I - in) / 2; 3 out = in^T.
__global__ void k_polar_elem(int mode, const double2* in, int n,
                             const double* s, double2* out) {
  const int64_t nn = (int64_t)n * n;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const double f = (mode == 1) ? *s : 0.0;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < nn;
       e += stride) {
    const int a = (int)(e / n), b = (int)(e % n);
    const double2 x = in[e];
    double2 y;
    if (mode == 0) y = make_double2(x.x, -x.y);
    else if (mode == 1) y = make_double2(f * x.x, f * x.y);
    else if (mode == 2) y = make_double2(((a == b) ? 1.5 : 0.0) - 0.5 * x.x,
                                         -0.5 * x.y);
    else y = in[(int64_t)b * n + a];
    out[e] = y;
  }
}

// One workgroup on an n x n complex128 row-major B: mode 0 writes
// 1 / sqrt(max_a sum_b |B_ab|) (a bound on the largest eigenvalue of a
// Hermitian positive semidefinite B, by Gershgorin; 0 when B = 0), mode 1
// writes ||B - I||_F / sqrt(n).
__global__ void k_polar_norm(int mode, const double2* B, int n, double* out) {
  __shared__ double red[4];
  double t = 0.0;
  for (int a = threadIdx.x; a < n; a += 256) {
    double r = 0.0;
    for (int b = 0; b < n; ++b) {
      const double2 x = B[(int64_t)a * n + b];
      if (mode == 0) {
        r += sqrt(x.x * x.x + x.y * x.y);
      } else {
        const double re = x.x - (a == b ? 1.0 : 0.0);
        r += re * re + x.y * x.y;
      }
    }
    t = (mode == 0) ? fmax(t, r) : t + r;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double u = __shfl_xor(t, o, 64);
    t = (mode == 0) ? fmax(t, u) : t + u;
  }
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double v = red[0];
    for (int w = 1; w < 4; ++w) v = (mode == 0) ? fmax(v, red[w]) : v + red[w];
    *out = (mode == 0) ? (v > 0.0 ? 1.0 / sqrt(v) : 0.0) : sqrt(v / n);
  }
}

hipError_t launch_polar_elem(int mode, const void* in, int n, const double* s,
                             void* out, hipStream_t st) {
  int64_t blocks = ((int64_t)n * n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  LACE_LAUNCH(k_polar_elem, dim3((unsigned)blocks), dim3(256), 0, st,
                     mode, static_cast<const double2*>(in), n, s,
                     static_cast<double2*>(out));
  return hipGetLastError();
}

hipError_t launch_polar_norm(int mode, const void* B, int n, double* out,
                             hipStream_t st) {
  LACE_LAUNCH(k_polar_norm, dim3(1), dim3(256), 0, st, mode,
                     static_cast<const double2*>(B), n, out);
  return hipGetLastError();
}

}  // namespace lace
