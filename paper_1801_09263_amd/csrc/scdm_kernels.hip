// Selected columns of the density matrix (SCDM) on the grid orbitals.
//
// The localization step of Sec. 2 picks N grid points r_k greedily: each
// pick is the point where the column a_r = conj(psi(r)) of Psi^H (one
// entry per orbital) has the largest part outside the span of the columns
// already picked, i.e. column-pivoted QR of Psi^H.  The residual norms
// d(r) = |a_r|^2 - sum_k |q_k^H a_r|^2 are kept on the device and
// downdated after every pick with the new orthonormal direction q_k, so a
// step reads the orbital grids once (a matrix-vector product over N_g
// points) plus an argmax; no step returns to the host.
//
// Grids are the workspace's orbital grids in the plan precision: complex
// (orbital-major, n^3 points each) or real (Gamma plans).  Sums and the
// directions q_k are FP64.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"

namespace lace {

template <typename T> struct GridVal;
template <> struct GridVal<float2> {
  __device__ static double2 get(const float2* g, int64_t i) {
    const float2 v = g[i];
    return make_double2(v.x, v.y);
  }
};
template <> struct GridVal<double2> {
  __device__ static double2 get(const double2* g, int64_t i) { return g[i]; }
};
template <> struct GridVal<float> {
  __device__ static double2 get(const float* g, int64_t i) {
    return make_double2(g[i], 0.0);
  }
};
template <> struct GridVal<double> {
  __device__ static double2 get(const double* g, int64_t i) {
    return make_double2(g[i], 0.0);
  }
};

// d(r) = sum_n |psi_n(r)|^2 (the diagonal of the density matrix)
template <typename G>
__global__ void k_scdm_density(const G* psi, int n_orb, int64_t ng, double* d) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t r = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; r < ng;
       r += stride) {
    double s = 0.0;
    for (int n = 0; n < n_orb; ++n) {
      const double2 v = GridVal<G>::get(psi, n * ng + r);
      s += v.x * v.x + v.y * v.y;
    }
    d[r] = s;
  }
}

// Block-wise argmax of d over [0, ng): the largest value, the smallest
// index among equals.  Picked points hold -1 and are never chosen again.
struct ArgMax {
  double v;
  int64_t i;
};
__device__ inline ArgMax better(ArgMax a, ArgMax b) {
  if (b.v > a.v || (b.v == a.v && b.i < a.i)) return b;
  return a;
}

template <int NT>
__device__ inline ArgMax block_argmax(ArgMax m) {
  __shared__ double sv[NT / 64];
  __shared__ int64_t si[NT / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    ArgMax t;
    t.v = __shfl_xor(m.v, o, 64);
    t.i = __shfl_xor(m.i, o, 64);
    m = better(m, t);
  }
  if (threadIdx.x % 64 == 0) {
    sv[threadIdx.x / 64] = m.v;
    si[threadIdx.x / 64] = m.i;
  }
  __syncthreads();
  m.v = sv[0];
  m.i = si[0];
  for (int w = 1; w < NT / 64; ++w) m = better(m, ArgMax{sv[w], si[w]});
  return m;
}

constexpr int AM_NT = 256;
constexpr int AM_BLOCKS = 4096;

__global__ void k_argmax_partial(const double* d, int64_t ng, double* pv,
                                 int64_t* pi) {
  ArgMax m{-2.0, 0};
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t r = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; r < ng;
       r += stride)
    m = better(m, ArgMax{d[r], r});
  m = block_argmax<AM_NT>(m);
  if (threadIdx.x == 0) {
    pv[blockIdx.x] = m.v;
    pi[blockIdx.x] = m.i;
  }
}

// Final argmax; records the point as pick k, marks it taken.
__global__ void k_argmax_final(const double* pv, const int64_t* pi, int nparts,
                               double* d, int32_t* points, int k) {
  ArgMax m{-2.0, 0};
  for (int b = threadIdx.x; b < nparts; b += AM_NT) m = better(m, ArgMax{pv[b], pi[b]});
  m = block_argmax<AM_NT>(m);
  if (threadIdx.x == 0) {
    points[k] = (int32_t)m.i;
    d[m.i] = -1.0;
  }
}

// q_k: the picked column a = conj(psi(r_k)) made orthogonal to q_0..q_{k-1}
// (classical Gram-Schmidt, twice) and normalized; Q row-major, q_m = Q[m][.].
// One workgroup.  The column u lives in LDS; h_m = q_m^H u is one wave per
// m (lanes along n, coalesced rows of Q, shuffle sum) into the scratch h;
// u -= sum_m q_m h_m splits the m sum over ngrp thread groups when n_orb
// is small, their partial sums added in LDS.  Dynamic LDS: n_orb double2
// for u plus, when ngrp > 1, ngrp * n_orb for the partials.
__device__ inline double2 wave_sum2(double2 v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o, 64);
    v.y += __shfl_xor(v.y, o, 64);
  }
  return v;
}

template <typename G, int NT>
__global__ __launch_bounds__(NT) void k_scdm_direction(
    const G* psi, int n_orb, int64_t ng, const int32_t* points, int k,
    double2* Q, double2* h, int ngrp) {
  extern __shared__ double2 lds[];
  double2* us = lds;
  double2* part = lds + n_orb;
  __shared__ double red[NT / 64];
  const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  const int64_t r = points[k];
  for (int n = tid; n < n_orb; n += NT) {
    const double2 v = GridVal<G>::get(psi, n * ng + r);
    us[n] = make_double2(v.x, -v.y);
  }
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
    for (int m = wv; m < k; m += NT / 64) {   // h_m = q_m^H u
      const double2* q = Q + (int64_t)m * n_orb;
      double2 sm = make_double2(0.0, 0.0);
#pragma unroll 4
      for (int n = lane; n < n_orb; n += 64) {
        const double2 a = q[n], b = us[n];
        sm.x += a.x * b.x + a.y * b.y;
        sm.y += a.x * b.y - a.y * b.x;
      }
      sm = wave_sum2(sm);
      if (lane == 0) h[m] = sm;
    }
    __syncthreads();
    if (ngrp > 1) {   // thread (g, n): partial over m = g, g + ngrp, ...
      if (tid < ngrp * n_orb) {
        const int n = tid % n_orb, g = tid / n_orb;
        double2 sm = make_double2(0.0, 0.0);
#pragma unroll 8
        for (int m = g; m < k; m += ngrp) {
          const double2 a = Q[(int64_t)m * n_orb + n], hm = h[m];
          sm.x += a.x * hm.x - a.y * hm.y;
          sm.y += a.x * hm.y + a.y * hm.x;
        }
        part[g * n_orb + n] = sm;
      }
      __syncthreads();
      for (int n = tid; n < n_orb; n += NT) {
        double2 sm = us[n];
        for (int g = 0; g < ngrp; ++g) {
          sm.x -= part[g * n_orb + n].x;
          sm.y -= part[g * n_orb + n].y;
        }
        us[n] = sm;
      }
    } else {
      for (int n = tid; n < n_orb; n += NT) {   // u -= sum_m q_m h_m
        double2 sm = us[n];
#pragma unroll 8
        for (int m = 0; m < k; ++m) {
          const double2 a = Q[(int64_t)m * n_orb + n], hm = h[m];
          sm.x -= a.x * hm.x - a.y * hm.y;
          sm.y -= a.x * hm.y + a.y * hm.x;
        }
        us[n] = sm;
      }
    }
    __syncthreads();
  }
  double t = 0.0;
  for (int n = tid; n < n_orb; n += NT) t += us[n].x * us[n].x + us[n].y * us[n].y;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
  if (lane == 0) red[wv] = t;
  __syncthreads();
  double nrm = 0.0;
  for (int w = 0; w < NT / 64; ++w) nrm += red[w];
  const double inv = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
  for (int n = tid; n < n_orb; n += NT)
    Q[(int64_t)k * n_orb + n] = make_double2(us[n].x * inv, us[n].y * inv);
}

// d(r) -= |q_k^H a_r|^2 = |sum_n q_kn psi_n(r)|^2 for points not yet taken,
// fused with the next pick's block-wise argmax (written to pv, pi as
// k_argmax_partial does).  A thread takes VW consecutive points, one
// 16-byte load per orbital (VW = 1 when n_g is not a multiple of the
// vector width); the sum over orbitals runs in orbital order for every
// point, as in a scalar loop.
template <typename G, int VW> struct GridVec {
  G v[VW];
};
template <typename G, int VW>
__device__ inline GridVec<G, VW> ldgrid(const G* p) {
  GridVec<G, VW> r;
  if constexpr (VW * sizeof(G) == 16) {
    const float4 t = *reinterpret_cast<const float4*>(p);
    __builtin_memcpy(&r, &t, 16);
  } else {
#pragma unroll
    for (int e = 0; e < VW; ++e) r.v[e] = p[e];
  }
  return r;
}
template <typename G> struct Cpx;
template <> struct Cpx<float> {
  __device__ static double2 of(float v) { return make_double2(v, 0.0); }
};
template <> struct Cpx<double> {
  __device__ static double2 of(double v) { return make_double2(v, 0.0); }
};
template <> struct Cpx<float2> {
  __device__ static double2 of(float2 v) { return make_double2(v.x, v.y); }
};
template <> struct Cpx<double2> {
  __device__ static double2 of(double2 v) { return v; }
};

template <typename G, int VW>
__global__ __launch_bounds__(AM_NT) void k_scdm_downdate(
    const G* psi, int n_orb, int64_t ng, const double2* Q, int k, double* d,
    double* pv, int64_t* pi) {
  extern __shared__ double2 qs[];
  for (int n = threadIdx.x; n < n_orb; n += AM_NT) qs[n] = Q[(int64_t)k * n_orb + n];
  __syncthreads();
  ArgMax m{-2.0, 0};
  const int64_t stride = int64_t(gridDim.x) * AM_NT * VW;
  for (int64_t r0 = (blockIdx.x * int64_t(AM_NT) + threadIdx.x) * VW; r0 < ng;
       r0 += stride) {
    double sx[VW], sy[VW];
#pragma unroll
    for (int e = 0; e < VW; ++e) sx[e] = sy[e] = 0.0;
    for (int n = 0; n < n_orb; ++n) {
      const GridVec<G, VW> g = ldgrid<G, VW>(psi + n * ng + r0);
      const double2 q = qs[n];
#pragma unroll
      for (int e = 0; e < VW; ++e) {
        const double2 v = Cpx<G>::of(g.v[e]);
        sx[e] += q.x * v.x - q.y * v.y;
        sy[e] += q.x * v.y + q.y * v.x;
      }
    }
#pragma unroll
    for (int e = 0; e < VW; ++e) {
      const double old = d[r0 + e];
      double nv = old;
      if (old >= 0.0) {
        nv = fmax(old - (sx[e] * sx[e] + sy[e] * sy[e]), 0.0);
        d[r0 + e] = nv;
      }
      m = better(m, ArgMax{nv, r0 + e});
    }
  }
  m = block_argmax<AM_NT>(m);
  if (threadIdx.x == 0) {
    pv[blockIdx.x] = m.v;
    pi[blockIdx.x] = m.i;
  }
}

// Y[k][n] = conj(psi_n(r_k)): the picked columns of Psi^H, transposed.
template <typename G>
__global__ void k_scdm_gather(const G* psi, int n_orb, int64_t ng,
                              const int32_t* points, double2* Y) {
  const int64_t total = (int64_t)n_orb * n_orb;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < total;
       e += stride) {
    const int k = (int)(e / n_orb), n = (int)(e % n_orb);
    const double2 v = GridVal<G>::get(psi, n * ng + points[k]);
    Y[e] = make_double2(v.x, -v.y);
  }
}

template <typename G>
static hipError_t scdm_t(const G* psi, int n_orb, int64_t ng, double* d,
                         double* pv, int64_t* pi, double2* Q, double2* h,
                         int32_t* points, double2* Y, hipStream_t st) {
  constexpr int NT = 256;
  constexpr int DIR_NT = 1024;
  const int ngrp = n_orb <= DIR_NT / 2 ? DIR_NT / n_orb : 1;
  const size_t dir_lds = sizeof(double2) * (size_t)n_orb * (ngrp > 1 ? 1 + ngrp : 1);
  int64_t blocks = (ng + NT - 1) / NT;
  if (blocks > 4096) blocks = 4096;
  LACE_LAUNCH(k_scdm_density<G>, dim3((unsigned)blocks), dim3(NT), 0,
                     st, psi, n_orb, ng, d);
  hipError_t e = hipGetLastError();
  constexpr int VW = 16 / (int)sizeof(G);
  const bool vec = ng % VW == 0;
  // one vector of points per downdate thread where the partials allow
  const int64_t per_block = (int64_t)AM_NT * (vec ? VW : 1);
  const int parts = (int)std::min<int64_t>(AM_BLOCKS, (ng + per_block - 1) / per_block);
  const size_t qlds = sizeof(double2) * (size_t)n_orb;
  LACE_LAUNCH(k_argmax_partial, dim3(parts), dim3(AM_NT), 0, st, d, ng,
                     pv, pi);
  for (int k = 0; k < n_orb && e == hipSuccess; ++k) {
    LACE_LAUNCH(k_argmax_final, dim3(1), dim3(AM_NT), 0, st, pv, pi,
                       parts, d, points, k);
    LACE_LAUNCH((k_scdm_direction<G, DIR_NT>), dim3(1), dim3(DIR_NT),
                       dir_lds, st, psi, n_orb, ng, points, k, Q, h, ngrp);
    if (k + 1 < n_orb) {   // downdate, and the next pick's partial argmax
      if (vec)
        LACE_LAUNCH((k_scdm_downdate<G, VW>), dim3(parts), dim3(AM_NT),
                           qlds, st, psi, n_orb, ng, Q, k, d, pv, pi);
      else
        LACE_LAUNCH((k_scdm_downdate<G, 1>), dim3(parts), dim3(AM_NT),
                           qlds, st, psi, n_orb, ng, Q, k, d, pv, pi);
    }
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    int64_t b2 = ((int64_t)n_orb * n_orb + NT - 1) / NT;
    if (b2 > 2048) b2 = 2048;
    LACE_LAUNCH(k_scdm_gather<G>, dim3((unsigned)b2), dim3(NT), 0, st,
                       psi, n_orb, ng, points, Y);
    e = hipGetLastError();
  }
  return e;
}

int64_t scdm_scratch_bytes(int n_orb) {
  return (int64_t)AM_BLOCKS * (sizeof(double) + sizeof(int64_t)) +
         (int64_t)sizeof(double2) * ((int64_t)n_orb + (int64_t)n_orb * n_orb);
}

hipError_t launch_scdm(bool fp64, bool real, const void* psi, int n_orb,
                       int64_t ng, double* d, void* scratch, int32_t* points,
                       void* Y, hipStream_t st) {
  if (n_orb > 48 * 1024 / (int)sizeof(double2)) return hipErrorInvalidValue;
  char* p = static_cast<char*>(scratch);
  double* pv = reinterpret_cast<double*>(p);
  p += AM_BLOCKS * sizeof(double);
  int64_t* pi = reinterpret_cast<int64_t*>(p);
  p += AM_BLOCKS * sizeof(int64_t);
  double2* h = reinterpret_cast<double2*>(p);
  p += sizeof(double2) * n_orb;
  double2* Q = reinterpret_cast<double2*>(p);
  double2* y = static_cast<double2*>(Y);
  if (real)
    return fp64 ? scdm_t(static_cast<const double*>(psi), n_orb, ng, d, pv, pi,
                         Q, h, points, y, st)
                : scdm_t(static_cast<const float*>(psi), n_orb, ng, d, pv, pi,
                         Q, h, points, y, st);
  return fp64 ? scdm_t(static_cast<const double2*>(psi), n_orb, ng, d, pv, pi,
                       Q, h, points, y, st)
              : scdm_t(static_cast<const float2*>(psi), n_orb, ng, d, pv, pi,
                       Q, h, points, y, st);
}

}  // namespace lace
