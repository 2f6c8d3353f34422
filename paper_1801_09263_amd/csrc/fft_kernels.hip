// fft_kernels.hip - 3D FFT passes and the fused pair-exchange pipeline.
//
// Grid layout: an n^3 complex grid is stored x fastest, then y, then z
// (index x + n (y + n z)); batches of grids are back to back.
//
// Pair pipeline (Eq. (2) of the paper, one batch of disjoint pairs):
//   pass A  rho = conj(psi_i) psi_j fused with the forward transform along
//           x and y (whole xy plane in LDS), or along x then y (pencils);
//   pass B  forward z transform, multiply by v(G)/N_g, accumulate the
//           exchange-integral partial sum_G v |rho(G)|^2 in FP64, backward
//           z transform, all in one kernel;
//   pass C  backward y and x transforms fused with
//           W_j -= psi_i V_ij and, for i != j, W_i -= psi_j conj(V_ij)
//           (V_ji = conj(V_ij) because v is real and even in G).
// Pairs inside a batch share no orbital, so pass C needs no atomics and the
// accumulation order is fixed by the schedule.  Batches are read from a
// table in device memory; the launches are sized for a batch's capacity and
// every kernel reads the batch's own slot count.
#include "fft_core.hpp"
#include "internal.hpp"

namespace lace {

// ------------------------------------------------------------- functors
// Prologues produce the values of grid points g .. g+V-1 of slot `slot`;
// epilogues consume them.  V consecutive points are moved with one 16-byte
// access per array.  Epilogues that read memory split into prev() (issue
// the loads) and putv() (combine and store), so a thread can have a whole
// chunk of loads in flight before it stores anything.  Loads never sit
// behind a branch: unused ones read a valid address and are discarded.

template <typename E, int V> struct Vec { E e[V]; };

template <typename E, int V>
__device__ inline Vec<E, V> ldv(const E* p) {
  Vec<E, V> r;
  if constexpr (sizeof(E) * V == 16) {
    const float4 t = *reinterpret_cast<const float4*>(p);
    __builtin_memcpy(&r, &t, 16);
  } else if constexpr (sizeof(E) * V == 8) {
    const float2 t = *reinterpret_cast<const float2*>(p);
    __builtin_memcpy(&r, &t, 8);
  } else {
#pragma unroll
    for (int v = 0; v < V; ++v) r.e[v] = p[v];
  }
  return r;
}
template <typename E, int V>
__device__ inline void stv(E* p, const Vec<E, V>& r) {
  if constexpr (sizeof(E) * V == 16) {
    float4 t;
    __builtin_memcpy(&t, &r, 16);
    *reinterpret_cast<float4*>(p) = t;
  } else if constexpr (sizeof(E) * V == 8) {
    float2 t;
    __builtin_memcpy(&t, &r, 8);
    *reinterpret_cast<float2*>(p) = t;
  } else {
#pragma unroll
    for (int v = 0; v < V; ++v) p[v] = r.e[v];
  }
}

// Nontemporal 16-byte accesses, for the pair buffer of the pipeline: each
// batch's buffer is written once by pass A, read and rewritten once by the
// z pass and read once by pass C, and nothing else reads it, so its lines
// are marked as streaming and leave the caches to the orbitals, the W grids
// and the kernel table, which later batches read again.
typedef float f4_nt __attribute__((ext_vector_type(4)));
template <typename E, int V>
__device__ inline Vec<E, V> ldv_nt(const E* p) {
  static_assert(sizeof(E) * V == 16, "16-byte vectors");
  Vec<E, V> r;
  const f4_nt t = __builtin_nontemporal_load(reinterpret_cast<const f4_nt*>(p));
  __builtin_memcpy(&r, &t, 16);
  return r;
}
template <typename E, int V>
__device__ inline void stv_nt(E* p, const Vec<E, V>& r) {
  static_assert(sizeof(E) * V == 16, "16-byte vectors");
  f4_nt t;
  __builtin_memcpy(&t, &r, 16);
  __builtin_nontemporal_store(t, reinterpret_cast<f4_nt*>(p));
}

struct NoPre {};

// Functor traits.  TABLE: the functor reads a batch of the pair pipeline
// from device memory (bt) and knows its slot count; DYN: the batch says
// whether every slot is a star slot, and the kernel takes the star or the
// general form of the functor for the whole workgroup (as_star).
#define LACE_PLAIN_FUNCTOR              \
  static constexpr bool TABLE = false; \
  static constexpr bool DYN = false;

template <typename T> struct ProGrid {
  LACE_PLAIN_FUNCTOR
  static constexpr int V = 16 / sizeof(C<T>);
  const C<T>* __restrict__ buf;
  int64_t gs;
  __device__ void getv(int g, int slot, C<T>* out) const {
    const Vec<C<T>, V> x = ldv<C<T>, V>(buf + slot * gs + g);
#pragma unroll
    for (int v = 0; v < V; ++v) out[v] = x.e[v];
  }
};
// rho = conj(psi_i) psi_j
template <typename T> struct ProPair {
  static constexpr int V = 16 / sizeof(C<T>);
  static constexpr bool TABLE = true;
  static constexpr bool DYN = false;
  const C<T>* __restrict__ psi;
  int64_t gs;
  const BatchDev* __restrict__ bt;
  __device__ void getv(int g, int slot, C<T>* out) const {
    const Vec<C<T>, V> a = ldv<C<T>, V>(psi + bt->i[slot] * gs + g);
    const Vec<C<T>, V> b = ldv<C<T>, V>(psi + bt->j[slot] * gs + g);
#pragma unroll
    for (int v = 0; v < V; ++v) out[v] = cmul<T>(a.e[v], b.e[v]);
  }
};
template <typename T> struct EpiGrid {
  LACE_PLAIN_FUNCTOR
  static constexpr int V = 16 / sizeof(C<T>);
  static constexpr int CH = 4;   // vectors per chunk of in-flight loads
  using Pre = NoPre;
  C<T>* __restrict__ buf;
  int64_t gs;
  T scale;
  __device__ void prev(int, int, Pre&) const {}
  __device__ void putv(int g, int slot, const C<T>* x, const Pre&) const {
    Vec<C<T>, V> y;
#pragma unroll
    for (int v = 0; v < V; ++v) y.e[v] = scl<T>(x[v], scale);
    stv<C<T>, V>(buf + slot * gs + g, y);
  }
};
// The pair buffer between the passes of the pipeline, accessed nontemporally.
template <typename T> struct EpiSlotBuf : EpiGrid<T> {
  static constexpr int V = EpiGrid<T>::V;
  __device__ void putv(int g, int slot, const C<T>* x, const NoPre&) const {
    Vec<C<T>, V> y;
#pragma unroll
    for (int v = 0; v < V; ++v) y.e[v] = scl<T>(x[v], this->scale);
    stv_nt<C<T>, V>(this->buf + slot * this->gs + g, y);
  }
};
template <typename T> struct ProSlotBuf : ProGrid<T> {
  static constexpr int V = ProGrid<T>::V;
  __device__ void getv(int g, int slot, C<T>* out) const {
    const Vec<C<T>, V> x = ldv_nt<C<T>, V>(this->buf + slot * this->gs + g);
#pragma unroll
    for (int v = 0; v < V; ++v) out[v] = x.e[v];
  }
};
// Two real grids packed as one complex grid: value W_{2p} + i W_{2p+1}
// (zero imaginary part for a last odd grid).  Reads 16 bytes per grid.
template <typename T> struct ProPackReal {
  LACE_PLAIN_FUNCTOR
  static constexpr int V = 16 / sizeof(T);
  const T* __restrict__ w;
  int64_t gs;
  int n_real;
  __device__ void getv(int g, int slot, C<T>* out) const {
    const int a = 2 * slot;
    const bool two = a + 1 < n_real;   // uniform over the workgroup
    const Vec<T, V> x = ldv<T, V>(w + a * gs + g);
    Vec<T, V> y;
    if (two) {
      y = ldv<T, V>(w + (a + 1) * gs + g);
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) y.e[v] = T(0);
    }
#pragma unroll
    for (int v = 0; v < V; ++v) out[v] = mk<T>(x.e[v], y.e[v]);
  }
};
// The inverse: scale * (Re, Im) into the real grids 2p and 2p + 1.
template <typename T> struct EpiSplitReal {
  LACE_PLAIN_FUNCTOR
  static constexpr int V = 16 / sizeof(T);
  static constexpr int CH = 4;
  using Pre = NoPre;
  T* __restrict__ psi;
  int64_t gs;
  int n_real;
  T scale;
  __device__ void prev(int, int, Pre&) const {}
  __device__ void putv(int g, int slot, const C<T>* x, const Pre&) const {
    const int a = 2 * slot;
    Vec<T, V> re, im;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      re.e[v] = x[v].x * scale;
      im.e[v] = x[v].y * scale;
    }
    stv<T, V>(psi + a * gs + g, re);
    if (a + 1 < n_real) stv<T, V>(psi + (a + 1) * gs + g, im);
  }
};

template <typename T> struct AccPre {
  Vec<C<T>, 16 / sizeof(C<T>)> pi, pj, wi, wj;
};
// W_j -= psi_i V and, for i != j, W_i -= psi_j conj(V)
template <typename T> struct EpiAcc {
  static constexpr int V = 16 / sizeof(C<T>);
  static constexpr int CH = 4;
  static constexpr bool TABLE = true;
  static constexpr bool DYN = false;
  using Pre = AccPre<T>;
  const C<T>* __restrict__ psi;
  C<T>* __restrict__ w;
  int64_t gs;
  const BatchDev* __restrict__ bt;
  __device__ void prev(int g, int slot, Pre& r) const {
    // a diagonal pair reads its orbital twice (from cache), and so does a
    // one-sided pair its psi_i and W_j; the stores decide
    const int i = bt->i[slot], j = bt->j[slot];
    const bool os = (bt->one_sided >> slot) & 1ull;
    const int jj = os ? i : j, ii = os ? j : i;
    r.pi = ldv<C<T>, V>(psi + i * gs + g);
    r.wj = ldv<C<T>, V>(w + j * gs + g);
    r.pj = ldv<C<T>, V>(psi + jj * gs + g);
    r.wi = ldv<C<T>, V>(w + ii * gs + g);
  }
  __device__ void putv(int g, int slot, const C<T>* x, const Pre& r) const {
    const int i = bt->i[slot], j = bt->j[slot];
    const bool os = (bt->one_sided >> slot) & 1ull;
    Vec<C<T>, V> yj, yi;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      yj.e[v] = sub<T>(r.wj.e[v], mul<T>(r.pi.e[v], x[v]));
      yi.e[v] = sub<T>(r.wi.e[v], mulc<T>(r.pj.e[v], x[v]));
    }
    stv<C<T>, V>(w + j * gs + g, yj);
    if (i != j && !os) stv<C<T>, V>(w + i * gs + g, yi);
  }
};

// Real orbitals, packed slot: value rho_ij + i rho_kl.  STAR: every slot
// of the launch is a star slot (k = i), whose three orbitals are read once.
template <typename T, bool STAR = false> struct ProQuad {
  static constexpr int V = 16 / sizeof(T);
  static constexpr bool TABLE = true;
  static constexpr bool DYN = false;
  const T* __restrict__ psi;
  int64_t gs;
  const BatchDev* __restrict__ bt;
  __device__ void getv(int g, int slot, C<T>* out) const {
    const int i = bt->i[slot], j = bt->j[slot], k = bt->k[slot], l = bt->l[slot];
    if constexpr (STAR) {
      const Vec<T, V> a = ldv<T, V>(psi + i * gs + g);
      const Vec<T, V> b = ldv<T, V>(psi + j * gs + g);
      const Vec<T, V> d = ldv<T, V>(psi + l * gs + g);
#pragma unroll
      for (int v = 0; v < V; ++v)
        out[v] = mk<T>(a.e[v] * b.e[v], a.e[v] * d.e[v]);
    } else {
      // a slot without a second pair reads orbital i twice and discards it
      const bool two = k >= 0;
      const int kk = two ? k : i, ll = two ? l : i;
      const Vec<T, V> a = ldv<T, V>(psi + i * gs + g);
      const Vec<T, V> b = ldv<T, V>(psi + j * gs + g);
      const Vec<T, V> c = ldv<T, V>(psi + kk * gs + g);
      const Vec<T, V> d = ldv<T, V>(psi + ll * gs + g);
#pragma unroll
      for (int v = 0; v < V; ++v)
        out[v] = mk<T>(a.e[v] * b.e[v], two ? c.e[v] * d.e[v] : T(0));
    }
  }
};
template <typename T> struct QuadPre {
  Vec<T, 16 / sizeof(T)> pi, pj, pk, pl, wi, wj, wk, wl;
};
// V = V_ij + i V_kl (both real):  W_j -= psi_i V_ij, W_i -= psi_j V_ij,
// W_l -= psi_k V_kl, W_k -= psi_l V_kl (one update for a diagonal pair).
// A star slot (k = i) folds both updates of the shared orbital into one;
// when every slot of the launch is a star (STAR), psi_i and W_i are read
// once.  A skipped W is neither updated nor read, nor is the orbital paired
// with it: those loads repeat another orbital of the slot (served by the
// cache).  The two W of the shared orbital of a star are skipped together.
template <typename T, bool STAR = false> struct EpiAccQuad {
  static constexpr int V = 16 / sizeof(T);
  static constexpr int CH = 2;
  static constexpr bool TABLE = true;
  static constexpr bool DYN = false;
  using Pre = QuadPre<T>;
  const T* __restrict__ psi;
  T* __restrict__ w;
  int64_t gs;
  const BatchDev* __restrict__ bt;
  __device__ void flags(int slot, bool s[4]) const {
#pragma unroll
    for (int t = 0; t < 4; ++t) s[t] = (bt->skip[t] >> slot) & 1ull;
  }
  __device__ void prev(int g, int slot, Pre& r) const {
    const int i = bt->i[slot], j = bt->j[slot], k = bt->k[slot], l = bt->l[slot];
    bool sk[4];
    flags(slot, sk);
    if constexpr (STAR) {
      r.pi = ldv<T, V>(psi + (sk[1] && sk[3] ? j : i) * gs + g);
      r.wj = ldv<T, V>(w + (sk[1] ? i : j) * gs + g);
      r.pj = ldv<T, V>(psi + (sk[0] ? i : j) * gs + g);
      r.wi = ldv<T, V>(w + (sk[0] ? j : i) * gs + g);
      r.pl = ldv<T, V>(psi + (sk[2] ? i : l) * gs + g);
      r.wl = ldv<T, V>(w + (sk[3] ? i : l) * gs + g);
    } else {
      const int kk = k >= 0 ? k : i, ll = k >= 0 ? l : i;
      r.pi = ldv<T, V>(psi + (sk[1] ? j : i) * gs + g);
      r.wj = ldv<T, V>(w + (sk[1] ? i : j) * gs + g);
      r.pj = ldv<T, V>(psi + (sk[0] ? i : j) * gs + g);
      r.wi = ldv<T, V>(w + (sk[0] ? j : i) * gs + g);
      r.pk = ldv<T, V>(psi + (sk[3] ? ll : kk) * gs + g);
      r.wl = ldv<T, V>(w + (sk[3] ? kk : ll) * gs + g);
      r.pl = ldv<T, V>(psi + (sk[2] ? kk : ll) * gs + g);
      r.wk = ldv<T, V>(w + (sk[2] ? ll : kk) * gs + g);
    }
  }
  __device__ void putv(int g, int slot, const C<T>* x, const Pre& r) const {
    const int i = bt->i[slot], j = bt->j[slot], k = bt->k[slot], l = bt->l[slot];
    bool sk[4];
    flags(slot, sk);
    if constexpr (STAR) {
      Vec<T, V> yj, yi, yl;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        yj.e[v] = r.wj.e[v] - r.pi.e[v] * x[v].x;
        yi.e[v] = r.wi.e[v] - (sk[0] ? T(0) : r.pj.e[v] * x[v].x);
        yl.e[v] = r.wl.e[v] - r.pi.e[v] * x[v].y;
        if (!sk[2]) yi.e[v] -= r.pl.e[v] * x[v].y;
      }
      if (!sk[1]) stv<T, V>(w + j * gs + g, yj);
      if (!sk[0] || !sk[2]) stv<T, V>(w + i * gs + g, yi);
      if (!sk[3]) stv<T, V>(w + l * gs + g, yl);
    } else {
      const bool star = k == i;
      const bool up_i = !sk[0] || (star && !sk[2]);
      Vec<T, V> yj, yi, yl, yk;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        yj.e[v] = r.wj.e[v] - r.pi.e[v] * x[v].x;
        yi.e[v] = r.wi.e[v] - (sk[0] ? T(0) : r.pj.e[v] * x[v].x);
        yl.e[v] = r.wl.e[v] - r.pk.e[v] * x[v].y;
        yk.e[v] = r.wk.e[v] - r.pl.e[v] * x[v].y;
        if (star && !sk[2]) yi.e[v] -= r.pl.e[v] * x[v].y;
      }
      if (!sk[1]) stv<T, V>(w + j * gs + g, yj);
      if (i != j && up_i) stv<T, V>(w + i * gs + g, yi);
      if (k >= 0) {
        if (!sk[3]) stv<T, V>(w + l * gs + g, yl);
        if (k != l && !star && !sk[2]) stv<T, V>(w + k * gs + g, yk);
      }
    }
  }
};

// The batch decides between the star and the general form (DYN): the
// kernel branches once, at its top, into the whole body of either form, so
// each form keeps its own load schedule (a branch inside the load functions
// serialized a thread's loads).
template <typename T> struct ProQuadD {
  static constexpr int V = 16 / sizeof(T);
  static constexpr bool TABLE = true;
  static constexpr bool DYN = true;
  const T* __restrict__ psi;
  int64_t gs;
  const BatchDev* __restrict__ bt;
  template <bool S> __device__ ProQuad<T, S> form() const { return {psi, gs, bt}; }
};
template <typename T> struct EpiAccQuadD {
  static constexpr int V = 16 / sizeof(T);
  static constexpr int CH = 2;
  static constexpr bool TABLE = true;
  static constexpr bool DYN = true;
  using Pre = QuadPre<T>;
  const T* __restrict__ psi;
  T* __restrict__ w;
  int64_t gs;
  const BatchDev* __restrict__ bt;
  template <bool S> __device__ EpiAccQuad<T, S> form() const { return {psi, w, gs, bt}; }
};

template <bool S, class F> __device__ inline auto as_star(const F& f) {
  if constexpr (F::DYN) return f.template form<S>();
  else return f;
}

// Slots of the launch: the batch's own count for table functors, else the
// host's count.
template <class Pro, class Epi>
__device__ inline int active_slots(const Pro& pro, const Epi& epi, int host) {
  if constexpr (Pro::TABLE) {
    const int n = pro.bt->n;
    return n < host ? n : host;
  } else if constexpr (Epi::TABLE) {
    const int n = epi.bt->n;
    return n < host ? n : host;
  } else {
    return host;
  }
}

// Run body(pro', epi') with the star or the general form of dynamic functors.
template <class Pro, class Epi, class Body>
__device__ __forceinline__ void with_form(const Pro& pro, const Epi& epi,
                                          Body&& body) {
  if constexpr (Pro::DYN || Epi::DYN) {
    int star;
    if constexpr (Pro::DYN) star = pro.bt->star;
    else star = epi.bt->star;
    if (star) body(as_star<true>(pro), as_star<true>(epi));
    else body(as_star<false>(pro), as_star<false>(epi));
  } else {
    body(pro, epi);
  }
}

template <typename T, int N, int NT>
__device__ inline void load_tw(C<T>* tw, const C<T>* tw_g) {
  for (int m = threadIdx.x; m < N; m += NT) tw[m] = tw_g[m];
}

// Fill s[lds(m)], m < NE, from the prologue: thread t takes the vectors
// t, t + NT, ... of V consecutive points (idx(m) .. idx(m) + V - 1 are
// consecutive in memory), all loads first, then the LDS stores.
template <typename T, int NE, int NT, class Pro, class Idx, class Lds>
__device__ inline void stage_in(C<T>* s, const Pro& pro, int slot, Idx idx,
                                Lds lds) {
  constexpr int V = Pro::V;
  static_assert(NE % V == 0, "tile not a multiple of the vector width");
  constexpr int NV = NE / V;
  constexpr int PER = (NV + NT - 1) / NT;
  C<T> x[PER][V];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int mv = threadIdx.x + q * NT;
    if (q < NV / NT || mv < NV) pro.getv(idx(mv * V), slot, x[q]);
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int mv = threadIdx.x + q * NT;
    if (q < NV / NT || mv < NV) {
#pragma unroll
      for (int v = 0; v < V; ++v) s[lds(mv * V + v)] = x[q][v];
    }
  }
}

// Drain s through the epilogue in chunks of CH vectors per thread: the
// chunk's loads are issued before any of its stores.
template <typename T, int NE, int NT, class Epi, class Idx, class Lds>
__device__ inline void stage_out(const C<T>* s, const Epi& epi, int slot,
                                 Idx idx, Lds lds) {
  constexpr int V = Epi::V;
  static_assert(NE % V == 0, "tile not a multiple of the vector width");
  constexpr int NV = NE / V;
  constexpr int PER = (NV + NT - 1) / NT;
  constexpr int CH = PER < Epi::CH ? PER : Epi::CH;   // register budget
#pragma unroll
  for (int q0 = 0; q0 < PER; q0 += CH) {
    typename Epi::Pre pre[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int q = q0 + c, mv = threadIdx.x + q * NT;
      if (q < PER && (q < NV / NT || mv < NV)) epi.prev(idx(mv * V), slot, pre[c]);
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int q = q0 + c, mv = threadIdx.x + q * NT;
      if (q < PER && (q < NV / NT || mv < NV)) {
        C<T> x[V];
#pragma unroll
        for (int v = 0; v < V; ++v) x[v] = s[lds(mv * V + v)];
        epi.putv(idx(mv * V), slot, x, pre[c]);
      }
    }
  }
}

// Workgroups are dealt to the 8 XCDs round robin by id.  Remap the flat
// id so that each XCD receives a contiguous range of logical tiles, which
// then share its L2 (tiles that split a cache line, or read the same
// kernel-table tile).
__device__ inline int xcd_logical(int bid, int total) {
  constexpr int NX = 8;
  const int per = total / NX;
  if (bid >= per * NX) return bid;  // ragged tail keeps identity
  return (bid % NX) * per + bid / NX;
}

// LDS layout.  Every kernel keeps each transform line contiguous in LDS
// with the line stride padded to N + 1 (odd), and lets consecutive lanes
// walk consecutive lines.  A lane stride of N + 1 complex words touches
// distinct banks for 8- and 16-byte elements, for the strided writes of
// the first radix stage as well as for the reads.
template <int N> struct Pad { static constexpr int LS = N + 1; };

// ------------------------------------------- xy-plane pass (whole plane)
template <typename T, int N, int NT, int SIGN, class Pro, class Epi, int RO = 0>
__global__ __launch_bounds__(NT) void k_plane(Pro pro, Epi epi,
                                              const C<T>* tw_g, int nslots) {
  constexpr int LS = Pad<N>::LS;
  __shared__ C<T> s[N * LS];
  __shared__ C<T> tw[N];
  const int z = blockIdx.x, slot = blockIdx.y;
  if (slot >= active_slots(pro, epi, nslots)) return;
  load_tw<T, N, NT>(tw, tw_g);
  const int base = z * N * N;
  auto idx = [base](int m) { return base + m; };
  auto lds = [](int m) { return (m / N) * LS + m % N; };  // row y, col x
  with_form(pro, epi, [&](const auto& pf, const auto& ef) {
    stage_in<T, N * N, NT>(s, pf, slot, idx, lds);
    __syncthreads();
    lds_fft<T, N, N, NT, SIGN, true, 1, RO>(s, LS, 1, tw);  // along x: lines = rows
    lds_fft<T, N, N, NT, SIGN, true, 1, RO>(s, 1, LS, tw);  // along y: lines = columns
    stage_out<T, N * N, NT>(s, ef, slot, idx, lds);
  });
}

// ------------------------------ xy plane in two halves (half the LDS)
// Decimation in frequency along y, H = N/2: rows y and y + H of the input
// plane f give a = f_y + f_{y+H} and b = (f_y - f_{y+H}) w^y (w the N-th
// root of unity of the transform's sign).  The length-N (x) by length-H (y)
// transforms of a and b are the even and the odd rows of the plane's
// transform.  One workgroup forms and transforms one of the two halves in
// an LDS buffer of H rows, so two workgroups share a CU and one's memory
// phases overlap the other's FFT.  Both halves of a plane read the same
// input; the remap puts them on one XCD, back to back, so the second read
// is served by that XCD's L2.  The epilogue is pointwise: the interleaved
// row order of the result costs nothing.
// SPLIT 1: decimation in time instead.  Half h reads only the rows
// y = 2m + h and writes its length-N by length-H transform (E for h = 0, O
// for h = 1) to rows hH .. hH + H - 1; the plane's transform is
// E_k +- w^k O_k, left to the next pass (the z pass), which reads both
// anyway.  Each workgroup then loads half the rows it loads in the
// frequency split.
// SPLIT 2: the frequency split with a and b already formed by the previous
// pass (the z pass) and stored as rows 0 .. H - 1 (a) and H .. N - 1 (b):
// half h reads only its own contiguous half plane.
template <typename T, int N, int NT, int MINW, int SIGN, class Pro, class Epi,
          int SPLIT = 0, int RO = 0>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(MINW)))
void k_half(Pro pro, Epi epi, const C<T>* tw_g, int nslots) {
  constexpr int H = N / 2;
  constexpr int LS = Pad<N>::LS;
  constexpr int V = Pro::V;
  constexpr int NVH = H * N / V;
  constexpr int PER = (NVH + NT - 1) / NT;
  static_assert((H * N) % V == 0 && N % V == 0, "vector width");
  __shared__ C<T> s[H * LS];
  __shared__ C<T> tw[N];
  const int ns = active_slots(pro, epi, nslots);
  if ((int)blockIdx.x >= 2 * N * ns) return;
  const int lg = xcd_logical(blockIdx.x, 2 * N * ns);
  const int half = lg & 1, zs = lg >> 1;
  const int z = zs % N, slot = zs / N;
  load_tw<T, N, NT>(tw, tw_g);
  const int base = z * N * N;
  with_form(pro, epi, [&](const auto& pf, const auto& ef) {
  C<T> f1[PER][V], f2[PER][V];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int mv = threadIdx.x + q * NT;
    if (q < NVH / NT || mv < NVH) {
      const int m0 = mv * V;
      if constexpr (SPLIT == 1) {
        pf.getv(base + (2 * (m0 / N) + half) * N + m0 % N, slot, f1[q]);
      } else if constexpr (SPLIT == 2) {
        pf.getv(base + half * H * N + m0, slot, f1[q]);
      } else {
        pf.getv(base + m0, slot, f1[q]);
        pf.getv(base + H * N + m0, slot, f2[q]);
      }
    }
  }
  __syncthreads();   // twiddles in LDS
  auto lds = [](int m) { return (m / N) * LS + m % N; };
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int mv = threadIdx.x + q * NT;
    if (q < NVH / NT || mv < NVH) {
      const int m0 = mv * V;
      C<T> w = tw[m0 / N];
      if (SIGN > 0) w.y = -w.y;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        C<T> r;
        if (SPLIT != 0) r = f1[q][v];
        else if (half == 0) r = add<T>(f1[q][v], f2[q][v]);
        else r = mul<T>(sub<T>(f1[q][v], f2[q][v]), w);
        s[lds(m0 + v)] = r;
      }
    }
  }
  __syncthreads();
  lds_fft<T, N, H, NT, SIGN, true, 1, RO>(s, LS, 1, tw);   // x: H rows
  lds_fft<T, H, N, NT, SIGN, true, 2, RO>(s, 1, LS, tw);   // y: N columns
  auto out = [base, half](int m) {
    if constexpr (SPLIT == 1) return base + half * H * N + m;
    else return base + (2 * (m / N) + half) * N + m % N;
  };
  stage_out<T, H * N, NT>(s, ef, slot, out, lds);
  });
}

// ---------------------------------------------- x pencils: TY whole rows
template <typename T, int N, int TY, int NT, int SIGN, class Pro, class Epi,
          int RO = 0>
__global__ __launch_bounds__(NT) void k_xlines(Pro pro, Epi epi,
                                               const C<T>* tw_g, int nslots) {
  constexpr int LS = Pad<N>::LS;
  __shared__ C<T> s[TY * LS];
  __shared__ C<T> tw[N];
  const int slot = blockIdx.y;
  if (slot >= active_slots(pro, epi, nslots)) return;
  load_tw<T, N, NT>(tw, tw_g);
  const int base = blockIdx.x * TY * N;
  auto idx = [base](int m) { return base + m; };
  auto lds = [](int m) { return (m / N) * LS + m % N; };
  with_form(pro, epi, [&](const auto& pf, const auto& ef) {
    stage_in<T, TY * N, NT>(s, pf, slot, idx, lds);
    __syncthreads();
    lds_fft<T, N, TY, NT, SIGN, true, 1, RO>(s, LS, 1, tw);
    stage_out<T, TY * N, NT>(s, ef, slot, idx, lds);
  });
}

// ---------------------- y or z pencils: TX adjacent x columns, whole axis
// Element m of a tile: column xx = m % TX (fast in global memory), position
// e = m / TX along the transform axis.  LDS holds column xx as line xx.
template <int N, int AXIS, int TX>
__device__ inline int col_index(int tile, int m) {
  const int xt = tile % (N / TX), f = tile / (N / TX);
  const int xx = m % TX, e = m / TX;
  const int x = xt * TX + xx;
  return AXIS == 1 ? x + N * (e + N * f) : x + N * (f + N * e);
}
// z pencils: a tile is TX consecutive points of the flattened xy plane
// (x + N y), so each z row of a tile is TX contiguous points even where TX
// does not divide N.
template <int N, int TX>
__device__ inline int zcol_index(int tile, int m) {
  return tile * TX + m % TX + N * N * (m / TX);
}
// Paired z tile of the decimation-in-time plane layout: its first TX/2
// columns are points of the first half plane (rows < N/2), the last TX/2
// the same points shifted by half a plane, so that a tile holds E_k and
// O_k of the same (x, k) together.
template <int N, int TX>
__device__ inline int zcol_dit(int tile, int m) {
  constexpr int HC = TX / 2;
  const int c = m % TX;
  return tile * HC + (c < HC ? c : c - HC + N * N / 2) + N * N * (m / TX);
}
template <int N, int TX>
__device__ inline int col_lds(int m) {
  return (m % TX) * Pad<N>::LS + m / TX;
}

// Grid: one flat dimension of ntiles * nslots workgroups, remapped so that
// an XCD takes consecutive tiles and all slots of a tile together.
template <typename T, int N, int AXIS, int TX, int NT, int SIGN, class Pro,
          class Epi, int RO = 0>
__global__ __launch_bounds__(NT) void k_cols(Pro pro, Epi epi,
                                             const C<T>* tw_g, int nslots) {
  constexpr int LS = Pad<N>::LS;
  __shared__ C<T> s[TX * LS];
  __shared__ C<T> tw[N];
  // y pencils: TX adjacent x of one row; z pencils: flattened xy tiles
  constexpr int NTILES = AXIS == 2 ? N * N / TX : N * (N / TX);
  static_assert(AXIS == 2 ? (N * N) % TX == 0 : N % TX == 0, "tile width");
  static_assert(TX % Pro::V == 0 && TX % Epi::V == 0,
                "vectors must not cross a tile row");
  const int ns = active_slots(pro, epi, nslots);
  if ((int)blockIdx.x >= NTILES * ns) return;
  const int lg = xcd_logical(blockIdx.x, NTILES * ns);
  const int tile = lg / ns, slot = lg % ns;
  load_tw<T, N, NT>(tw, tw_g);
  auto idx = [tile](int m) {
    if constexpr (AXIS == 2) return zcol_index<N, TX>(tile, m);
    else return col_index<N, AXIS, TX>(tile, m);
  };
  auto lds = [](int m) { return col_lds<N, TX>(m); };
  with_form(pro, epi, [&](const auto& pf, const auto& ef) {
    stage_in<T, TX * N, NT>(s, pf, slot, idx, lds);
    __syncthreads();
    lds_fft<T, N, TX, NT, SIGN, true, 1, RO>(s, LS, 1, tw);
    stage_out<T, TX * N, NT>(s, ef, slot, idx, lds);
  });
}

template <int NT>
__device__ inline double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    for (int k = 0; k < NT / 64; ++k) t += red[k];
  }
  return t;  // valid in thread 0
}

// ---- pass B: z forward, x v(G)/N_g with energy partial, z backward ----
// Workgroup (tile, group): TX z columns of SL consecutive pair slots, one
// LDS line per column and slot; the kernel-table tile is shared by the SL
// slots.  A tile is TX consecutive points of the flattened xy plane (x + N
// y), so that each z row of a tile is one contiguous piece (256 bytes for
// the tile widths in use) even when TX does not divide N.  Slots past the
// end of the batch load slot 0 (discarded) and are neither stored nor
// summed.
//
// DIT: the xy pass left the decimation-in-time halves E (rows < N/2) and
// O (rows >= N/2) of each plane; tiles pair them (zcol_dit: two pieces of
// TX/2 points per z row), and the loads form the plane's transform
// X_k = E_k + w^k O_k, X_{k+N/2} = E_k - w^k O_k before the z transform,
// in the places the natural layout gives them (so the kernel table is read
// as in that layout).  The stores form the inverse xy pass's frequency
// split in the same places: a_k = Y_k + Y_{k+N/2} in row k and
// b_k = (Y_k - Y_{k+N/2}) w^-k in row k + N/2, Y the result of the inverse
// z transform, so that each half of the inverse xy pass reads only its own
// half plane (its SPLIT 2 form).
template <typename T, int N, int TX, int SL, int NT, int MINW, int ORDER = 0,
          bool DIT = false, int RO = 0>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(MINW)))
void k_zconv(C<T>* __restrict__ tmp, int64_t gs, const T* __restrict__ vtab,
             const BatchDev* __restrict__ bt, double* epart, int ntiles,
             const C<T>* tw_g) {
  constexpr int LS = Pad<N>::LS;
  constexpr int NE1 = TX * N;          // points of one slot's tile
  constexpr int NE = SL * NE1;
  constexpr int V = ProGrid<T>::V;
  constexpr int NV = NE / V;
  constexpr int PER = (NV + NT - 1) / NT;
  __shared__ C<T> s[SL * TX * LS];
  __shared__ C<T> tw[N];
  __shared__ double red[NT / 64];
  const int nslots = bt->n;
  const int ngroups = (nslots + SL - 1) / SL;
  if ((int)blockIdx.x >= ntiles * ngroups) return;
  const int lg = xcd_logical(blockIdx.x, ntiles * ngroups);
  // ORDER 0: all slot groups of a tile together; 1: slot-group-major, the
  // last group first, so that the z pass ends on the slot that pass C
  // reads first (pass C after it measured 480 us against 486 us for order
  // 0 at 120^3 FP32)
  const int tile = ORDER == 0 ? lg / ngroups : lg % ntiles;
  const int slot0 = (ORDER == 0 ? lg % ngroups : ngroups - 1 - lg / ntiles) * SL;
  const int nsl = min(SL, nslots - slot0);
  load_tw<T, N, NT>(tw, tw_g);
  C<T>* g = tmp + slot0 * gs;
  // element m of the group: slot m / NE1, tile point m % NE1
  auto zcol = [](int t, int m) {
    if constexpr (DIT) return zcol_dit<N, TX>(t, m);
    else return zcol_index<N, TX>(t, m);
  };
  auto gidx = [tile, nsl, gs, zcol](int m) {
    const int sl = m / NE1;
    return (sl < nsl ? sl : 0) * (int)gs + zcol(tile, m % NE1);
  };
  auto lds = [](int m) {
    const int sl = m / NE1, r = m % NE1;
    return (sl * TX + r % TX) * LS + r / TX;
  };
  // The forward transform's last stage (radix RL), the kernel multiply
  // with the energy sum, and the inverse transform's first stage run in
  // registers: the inverse takes the plan in reverse order, whose first
  // stage (radix RL, no twiddles) reads exactly the RL outputs that a
  // thread holds after the forward's last stage.
  constexpr int NLN = SL * TX;                 // LDS lines
  constexpr int NST = Plan<N, RO>::nst;
  constexpr int RL = Plan<N, RO>::r[NST - 1];
  constexpr int PL = N / RL;                   // butterflies per line
  constexpr int BF = NLN * PL;
  constexpr int NBF = (BF + NT - 1) / NT;
  static_assert(NT % NLN == 0, "a thread keeps one line (one slot)");
  const int line = threadIdx.x % NLN, col = line % TX, my_sl = line / TX;
  // The kernel table holds one octant, 0 <= kx, ky, kz <= N/2 (v depends on
  // |G| only and the cell is cubic): 1/8 of the grid, small enough to stay
  // in L2 while every slot of the launch reads it.  Octant row of this
  // line's xy point:
  constexpr int VH = N / 2 + 1;
  const int vxy = [&] {
    const int p = zcol(tile, col), lx = p % N, ly = p / N;
    return (ly <= N - ly ? ly : N - ly) * VH + (lx <= N - lx ? lx : N - lx);
  }();
  ProSlotBuf<T> pro{{g, 0}};
  // DIT element pairs (column c < TX/2, column c + TX/2) of each z row
  constexpr int HC = TX / 2;
  constexpr int NVP = NE / 2 / V;
  constexpr int PP = (NVP + NT - 1) / NT;
  static_assert(!DIT || (TX % 2 == 0 && HC % V == 0), "paired tile width");
  auto lo = [](int mp) {   // pair element -> element of the low column
    const int sl = mp / (NE1 / 2), r = mp % (NE1 / 2);
    return sl * NE1 + (r / HC) * TX + r % HC;
  };
  if constexpr (DIT) {
    C<T> fe[PP][V], fo[PP][V];
#pragma unroll
    for (int q = 0; q < PP; ++q) {
      const int mv = threadIdx.x + q * NT;
      if (q < NVP / NT || mv < NVP) {
        const int m = lo(mv * V);
        pro.getv(gidx(m), 0, fe[q]);
        pro.getv(gidx(m + HC), 0, fo[q]);
      }
    }
    __syncthreads();   // twiddles in LDS
#pragma unroll
    for (int q = 0; q < PP; ++q) {
      const int mv = threadIdx.x + q * NT;
      if (q < NVP / NT || mv < NVP) {
        const int m = lo(mv * V);
#pragma unroll
        for (int v = 0; v < V; ++v) {
          // row k of the low point: tile * HC + column, over N
          const int k = (tile * HC + (m + v) % TX) / N;
          const C<T> b = mul<T>(fo[q][v], tw[k]);
          s[lds(m + v)] = add<T>(fe[q][v], b);
          s[lds(m + v + HC)] = sub<T>(fe[q][v], b);
        }
      }
    }
  } else {
    stage_in<T, NE, NT>(s, pro, 0, gidx, lds);
  }
  __syncthreads();
  StagesRange<T, N, 0, NST - 1, NLN, NT, -1, true, 1, RO>::run(s, LS, 1, tw);
  C<T> x[NBF][RL];
#pragma unroll
  for (int b = 0; b < NBF; ++b) {
    const int idx = threadIdx.x + b * NT;
    if (BF % NT == 0 || idx < BF) {
      const int i = idx / NLN;
#pragma unroll
      for (int t = 0; t < RL; ++t) x[b][t] = s[line * LS + i + t * PL];
    }
  }
  __syncthreads();
  double e = 0.0;
#pragma unroll
  for (int b = 0; b < NBF; ++b) {
    const int idx = threadIdx.x + b * NT;
    if (BF % NT == 0 || idx < BF) {
      const int i = idx / NLN;
      if (PL > 1) {   // twiddles of the forward's last stage (k = i < PL)
#pragma unroll
        for (int t = 1; t < RL; ++t) x[b][t] = mul<T>(x[b][t], tw[t * i]);
      }
      T vt[RL];   // kernel values at frequencies i + t PL of the z line
#pragma unroll
      for (int t = 0; t < RL; ++t) {
        const int kz = i + t * PL;
        vt[t] = vtab[(kz <= N - kz ? kz : N - kz) * (VH * VH) + vxy];
      }
      Dft<RL, -1, T>::run(x[b]);
      T eb = T(0);   // the butterfly's RL terms in the transform precision
#pragma unroll
      for (int t = 0; t < RL; ++t) {
        const C<T> r = x[b][t];
        const T v = vt[t];
        eb += v * (r.x * r.x + r.y * r.y);
        x[b][t] = scl<T>(r, v);
      }
      e += double(eb);   // partial sums accumulated in FP64
      Dft<RL, +1, T>::run(x[b]);
#pragma unroll
      for (int t = 0; t < RL; ++t) s[line * LS + i * RL + t] = x[b][t];
    }
  }
  __syncthreads();
  StagesReversed<T, N, NST - 2, NLN, NT, +1, true, 1, RO>::run(s, LS, 1, tw);
  if constexpr (DIT) {
#pragma unroll
    for (int q = 0; q < PP; ++q) {
      const int mv = threadIdx.x + q * NT;
      if ((q < NVP / NT || mv < NVP) && (mv * V) / (NE1 / 2) < nsl) {
        const int m = lo(mv * V);
        Vec<C<T>, V> ya, yb;
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const C<T> a = s[lds(m + v)], b = s[lds(m + v + HC)];
          C<T> w = tw[(tile * HC + (m + v) % TX) / N];
          w.y = -w.y;
          ya.e[v] = add<T>(a, b);
          yb.e[v] = mul<T>(sub<T>(a, b), w);
        }
        stv_nt<C<T>, V>(g + gidx(m), ya);
        stv_nt<C<T>, V>(g + gidx(m + HC), yb);
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int mv = threadIdx.x + q * NT;
      if ((q < NV / NT || mv < NV) && (mv * V) / NE1 < nsl) {
        Vec<C<T>, V> y;
#pragma unroll
        for (int v = 0; v < V; ++v) y.e[v] = s[lds(mv * V + v)];
        stv_nt<C<T>, V>(g + gidx(mv * V), y);
      }
    }
  }
#pragma unroll
  for (int sl = 0; sl < SL; ++sl) {
    const double tot = block_sum<NT>(my_sl == sl ? e : 0.0, red);
    if (threadIdx.x == 0 && sl < nsl) {
      const int slot = slot0 + sl;
      const double wgt = ((bt->one_sided >> slot) & 1ull) ? 0.0
                         : (bt->i[slot] == bt->j[slot]) ? 1.0 : 2.0;
      epart[slot * ntiles + tile] += wgt * tot;
    }
    __syncthreads();   // red is reused by the next slot
  }
}

// ------------------------------------------------------------- helpers
__global__ void k_zero(uint4* p, int64_t n16) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < n16;
       k += stride)
    p[k] = make_uint4(0u, 0u, 0u, 0u);
}
__global__ void k_zero_tail(unsigned char* p, int64_t n) {
  for (int64_t k = threadIdx.x; k < n; k += blockDim.x) p[k] = 0;
}

template <typename T>
__global__ void k_scatter(const double2* coeffs, int64_t n_pw,
                          const int32_t* gidx, C<T>* psi, int64_t gs,
                          int n_orb) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int64_t total = n_pw * n_orb;
  for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < total;
       k += stride) {
    const int64_t j = k / n_pw, m = k % n_pw;
    const double2 c = coeffs[k];
    psi[j * gs + gidx[m]] = mk<T>(T(c.x), T(c.y));
  }
}

template <typename T>
__global__ void k_gather(const C<T>* w, int64_t gs, const int32_t* gidx,
                         int64_t n_pw, int n_orb, double scale,
                         double2* out) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int64_t total = n_pw * n_orb;
  for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < total;
       k += stride) {
    const int64_t j = k / n_pw, m = k % n_pw;
    const C<T> v = w[j * gs + gidx[m]];
    out[k] = make_double2(scale * double(v.x), scale * double(v.y));
  }
}

// Thread t adds part[t], part[t + 256], ... in that order (16 loads in
// flight per step, the additions still in order), then the workgroup sum.
__global__ void k_reduce_sum(const double* part, int64_t count, double factor,
                             double* out) {
  __shared__ double red[256 / 64];
  constexpr int U = 16;
  double t = 0.0;
  int64_t k = threadIdx.x;
  for (; k + (U - 1) * 256 < count; k += U * 256) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = part[k + u * 256];
#pragma unroll
    for (int u = 0; u < U; ++u) t += v[u];
  }
  for (; k < count; k += 256) t += part[k];
  const double tot = block_sum<256>(t, red);
  if (threadIdx.x == 0) *out = factor * tot;
}

// ----------------------------------------------------- tile parameters
template <typename T, int N> struct Cfg {
  // plane pass: whole N x N plane in LDS
  static constexpr bool plane = (int64_t)N * N * sizeof(C<T>) <= 150 * 1024;
  static constexpr int NT_PLANE = sizeof(T) == 4 ? 1024 : 512;
  // y/z pencils: TX columns (>= 128 bytes of x per row when N allows)
  static constexpr int TX0 = sizeof(T) == 4 ? 16 : 8;
  static constexpr int TX = (N % TX0 == 0) ? TX0 : ((N % 8 == 0) ? 8 : 4);
  static constexpr int NT_COLS = 256;
  // z pass: tiles of 256 bytes of the flattened xy plane per z row, one
  // pair slot per workgroup of 256 threads.  Measured at 120^3 FP32 (32
  // slots): 188 us, against 204 us for 128-byte tiles with two slots per
  // 512 threads, 198 us for 256-byte tiles with two slots, 200 us with 512
  // threads.
  static constexpr int SL = 1;
  static constexpr int TXZ0 = 256 / (int)sizeof(C<T>);
  static constexpr int TXZ = (N * N) % TXZ0 == 0 ? TXZ0
                             : (N * N) % (TXZ0 / 2) == 0 ? TXZ0 / 2 : TX;
  static constexpr int NT_Z = 256;
  // waves per SIMD to budget registers for (the fused middle stage in
  // registers needs up to 120 VGPRs at 120^3 FP32, more in FP64, without
  // spilling)
  static constexpr int W_Z = sizeof(T) == 4 ? 4 : 3;
  // z pencils of the 3D transforms: 256 bytes of complex points per z row
  // (128 bytes of each real grid when the last pass splits into real grids)
  static constexpr int TXC20 = 256 / (int)sizeof(C<T>);
  static constexpr int TXC2 = (N * N) % TXC20 == 0 ? TXC20 : TXZ;
  // x pencils: TY rows
  static constexpr int TY = (N % 8 == 0) ? 8 : 4;
  static constexpr int NT_X = 256;
};

// RO: radix order of every transform the engine launches (Plan<N, RO>).
template <typename T, int N, int RO = 0> struct Engine {
  using Cf = Cfg<T, N>;
  static constexpr int64_t NG = (int64_t)N * N * N;

  template <int SIGN, class Pro, class Epi>
  static hipError_t plane(Pro p, Epi e, int count, const C<T>* tw,
                          hipStream_t st) {
    if constexpr (Cf::plane) {
      LACE_LAUNCH((k_plane<T, N, Cf::NT_PLANE, SIGN, Pro, Epi, RO>),
                         dim3(N, count), dim3(Cf::NT_PLANE), 0, st, p, e, tw,
                         count);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  static constexpr int NT_HALF = 512;
  // waves per SIMD to budget registers for: two workgroups of 8 waves when
  // two half planes fit the 160 KiB of LDS of a CU
  static constexpr int W_HALF =
      (N / 2 * (N + 1) + N) * (int)sizeof(C<T>) * 2 <= 160 * 1024 ? 4 : 2;
  template <int SIGN, int SPLIT = 0, class Pro, class Epi>
  static hipError_t half(Pro p, Epi e, int count, const C<T>* tw,
                         hipStream_t st) {
    LACE_LAUNCH((k_half<T, N, NT_HALF, W_HALF, SIGN, Pro, Epi, SPLIT, RO>),
                       dim3(2 * N * count), dim3(NT_HALF), 0, st, p, e, tw,
                       count);
    return hipGetLastError();
  }
  // The pair passes' forward xy pass over half planes splits in time and
  // leaves the combination to the z pass (measured at 120^3 FP32, 32 star
  // slots: 206 us against 219-224 us for the split in frequency); the z
  // pass also forms the inverse pass's frequency split, so that each of
  // its halves reads only its half plane.
  static constexpr bool XY_DIT = N % 2 == 0 && Cf::TXZ % 2 == 0 &&
                              (Cf::TXZ / 2) % ProGrid<T>::V == 0;
  // z tiles: TXZ points of the flattened xy plane per z row by default;
  // half and twice that are the alternatives the autotuner tries.  Index
  // z of zt(z): 0 the default, 1 half, 2 twice (0 when not a divisor of
  // the plane).
  static constexpr bool zt_ok(int tx) {
    return tx >= 2 && (N * N) % tx == 0 && Cf::NT_Z % tx == 0 &&
           (tx / 2) % ProGrid<T>::V == 0;
  }
  static constexpr int zt(int z) {
    const int tx = z == 1 ? Cf::TXZ / 2 : z == 2 ? Cf::TXZ * 2 : Cf::TXZ;
    return zt_ok(tx) ? tx : Cf::TXZ;
  }
  template <bool D, int TX>
  static hipError_t zpass_tx(C<T>* tmp, const T* vtab, const BatchDev* bt,
                             double* epart, int cnt, const C<T>* tw,
                             hipStream_t st) {
    const int ntiles = N * N / TX;
    // the wider tile's LDS allows two workgroups per CU: budget registers
    // for that
    constexpr int MINW = TX > Cf::TXZ ? 2 : Cf::W_Z;
    LACE_LAUNCH((k_zconv<T, N, TX, Cf::SL, Cf::NT_Z, MINW, 1, D, RO>),
                       dim3(ntiles * ((cnt + Cf::SL - 1) / Cf::SL)),
                       dim3(Cf::NT_Z), 0, st, tmp, NG, vtab, bt, epart,
                       ntiles, tw);
    return hipGetLastError();
  }
  template <bool D>
  static hipError_t zpass(C<T>* tmp, const T* vtab, const BatchDev* bt,
                          double* epart, int cnt, const C<T>* tw, int ztile,
                          hipStream_t st) {
    switch (ztile) {
      case 1: return zpass_tx<D, zt(1)>(tmp, vtab, bt, epart, cnt, tw, st);
      case 2: return zpass_tx<D, zt(2)>(tmp, vtab, bt, epart, cnt, tw, st);
      default: return zpass_tx<D, zt(0)>(tmp, vtab, bt, epart, cnt, tw, st);
    }
  }
  template <int SIGN, class Pro, class Epi>
  static hipError_t xlines(Pro p, Epi e, int count, const C<T>* tw,
                           hipStream_t st) {
    LACE_LAUNCH((k_xlines<T, N, Cf::TY, Cf::NT_X, SIGN, Pro, Epi, RO>),
                       dim3(N * N / Cf::TY, count), dim3(Cf::NT_X), 0, st, p,
                       e, tw, count);
    return hipGetLastError();
  }
  template <int AXIS, int SIGN, class Pro, class Epi>
  static hipError_t cols(Pro p, Epi e, int count, const C<T>* tw,
                         hipStream_t st) {
    constexpr int TXC = AXIS == 2 ? Cf::TXC2 : Cf::TX;
    constexpr int ntiles = AXIS == 2 ? N * N / TXC : N * (N / TXC);
    LACE_LAUNCH((k_cols<T, N, AXIS, TXC, Cf::NT_COLS, SIGN, Pro, Epi, RO>),
                       dim3(ntiles * count), dim3(Cf::NT_COLS), 0, st, p, e,
                       tw, count);
    return hipGetLastError();
  }

  // Transform of `count` grids held in g between the passes: the first
  // pass reads through `first`, the last one (z) writes through `last`.
  // oop: `first` reads memory other than g, so the first pass may take the
  // half-plane form (in place, its two workgroups of a plane would
  // overwrite rows that the other one still reads).
  template <int SIGN, class ProF, class EpiL>
  static hipError_t fft3d_io(ProF first, EpiL last, C<T>* g, int count,
                             const C<T>* tw, int mode, hipStream_t st,
                             bool oop = false) {
    ProGrid<T> p{g, NG};
    EpiGrid<T> e1{g, NG, T(1)};
    hipError_t err;
    if (oop && mode == 2) {
      err = half<SIGN>(first, e1, count, tw, st);
    } else if (Cf::plane && mode != 0) {
      err = plane<SIGN>(first, e1, count, tw, st);
    } else {
      err = xlines<SIGN>(first, e1, count, tw, st);
      if (err == hipSuccess) err = cols<1, SIGN>(p, e1, count, tw, st);
    }
    if (err == hipSuccess) err = cols<2, SIGN>(p, last, count, tw, st);
    return err;
  }
  // in-place transform of `count` grids, optional scale on the last pass
  template <int SIGN>
  static hipError_t fft3d(C<T>* g, int count, T scale, const C<T>* tw,
                          int mode, hipStream_t st) {
    return fft3d_io<SIGN>(ProGrid<T>{g, NG}, EpiGrid<T>{g, NG, scale}, g,
                          count, tw, mode, st);
  }
  // packed pairs in src to real grids: inverse transform through g (a
  // buffer apart from src), split into 2 real grids per pair in psi
  static hipError_t to_real(const C<T>* src, C<T>* g, int count, T scale,
                            T* psi, int n_real, const C<T>* tw, int mode,
                            hipStream_t st) {
    return fft3d_io<+1>(ProGrid<T>{src, NG},
                        EpiSplitReal<T>{psi, NG, n_real, scale}, g, count, tw,
                        mode, st, true);
  }
  // packed pairs of real grids: forward transform into g
  static hipError_t from_real(const T* w, int n_real, C<T>* g, int count,
                              const C<T>* tw, int mode, hipStream_t st) {
    return fft3d_io<-1>(ProPackReal<T>{w, NG, n_real},
                        EpiGrid<T>{g, NG, T(1)}, g, count, tw, mode, st, true);
  }

  // One batch of the pair pipeline, read from bt; the grids are sized for
  // cap slots.  Complex orbitals: ProPair / EpiAcc; real orbitals: packed
  // slots (ProQuadD / EpiAccQuadD, star or general form per batch).
  template <class ProA, class EpiC>
  static hipError_t run_batch(const CellDev& c, ProA pa_, EpiC ec,
                              const BatchDev* bt, int cap, C<T>* tmp,
                              double* epart, hipStream_t st, hipEvent_t* ev,
                              const BatchSync* sy) {
    const C<T>* tw = static_cast<const C<T>*>(c.tw);
    ProGrid<T> pt{tmp, NG};
    ProSlotBuf<T> pb{{tmp, NG}};       // the pair buffer, nontemporal
    EpiSlotBuf<T> eb{{tmp, NG, T(1)}};
    const int mode = (c.use_plane == 1 && !Cf::plane) ? 0 : c.use_plane;
    hipError_t err;
    if (ev && (err = hipEventRecord(ev[0], st)) != hipSuccess) return err;
    // pass A
    if (mode == 2) {
      err = half<-1, XY_DIT ? 1 : 0>(pa_, eb, cap, tw, st);
    } else if (mode == 1) {
      err = plane<-1>(pa_, eb, cap, tw, st);
    } else {
      err = xlines<-1>(pa_, EpiGrid<T>{tmp, NG, T(1)}, cap, tw, st);
      if (err == hipSuccess) err = cols<1, -1>(pt, EpiGridT{tmp, NG, T(1), bt}, cap, tw, st);
    }
    if (err != hipSuccess) return err;
    if (ev && (err = hipEventRecord(ev[1], st)) != hipSuccess) return err;
    // pass B
    const T* vtab = static_cast<const T*>(c.vtab);
    err = mode == 2 ? zpass<XY_DIT>(tmp, vtab, bt, epart, cap, tw, c.ztile, st)
                    : zpass<false>(tmp, vtab, bt, epart, cap, tw, c.ztile, st);
    if (err != hipSuccess) return err;
    if (ev && (err = hipEventRecord(ev[2], st)) != hipSuccess) return err;
    if (sy && sy->wait_c && (err = hipStreamWaitEvent(st, sy->wait_c, 0)) != hipSuccess)
      return err;
    // pass C
    if (mode == 2) {
      err = half<+1, XY_DIT ? 2 : 0>(pb, ec, cap, tw, st);
    } else if (mode == 1) {
      err = plane<+1>(pb, ec, cap, tw, st);
    } else {
      err = cols<1, +1>(pt, EpiGridT{tmp, NG, T(1), bt}, cap, tw, st);
      if (err == hipSuccess) err = xlines<+1>(pt, ec, cap, tw, st);
    }
    if (err == hipSuccess && ev) err = hipEventRecord(ev[3], st);
    if (err == hipSuccess && sy && sy->done_c) err = hipEventRecord(sy->done_c, st);
    return err;
  }
  // Grid-to-grid step of the pencil schedule between the pair passes: the
  // pair buffer in and out, limited to the batch's slots.
  struct EpiGridT : EpiGrid<T> {
    static constexpr bool TABLE = true;
    const BatchDev* __restrict__ bt;
    EpiGridT(C<T>* b, int64_t g, T s, const BatchDev* t) : EpiGrid<T>{b, g, s}, bt(t) {}
  };

  static hipError_t pair_batch(const CellDev& c, const BatchDev* bt, int cap,
                               const C<T>* psi, C<T>* w, C<T>* tmp,
                               double* epart, hipStream_t st, hipEvent_t* ev,
                               const BatchSync* sy) {
    return run_batch(c, ProPair<T>{psi, NG, bt}, EpiAcc<T>{psi, w, NG, bt}, bt,
                     cap, tmp, epart, st, ev, sy);
  }
  static hipError_t quad_batch(const CellDev& c, const BatchDev* bt, int cap,
                               const T* psi, T* w, C<T>* tmp, double* epart,
                               hipStream_t st, hipEvent_t* ev,
                               const BatchSync* sy) {
    return run_batch(c, ProQuadD<T>{psi, NG, bt}, EpiAccQuadD<T>{psi, w, NG, bt},
                     bt, cap, tmp, epart, st, ev, sy);
  }

  // energy partials per slot: enough for the smallest z tile
  static int64_t tiles() {
    const int a = zt(0), b = zt(1), c2 = zt(2);
    const int m = a < b ? (a < c2 ? a : c2) : (b < c2 ? b : c2);
    return (int64_t)N * N / m;
  }
};

// ------------------------------------------------------ runtime dispatch
#define LACE_SIZES(X) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(80) X(96) X(120)

bool grid_supported(int n) {
  switch (n) {
#define X(NN) case NN: return true;
    LACE_SIZES(X)
#undef X
    default: return false;
  }
}

bool plane_fits(int n, bool fp64) {
  switch (n) {
#define X(NN) \
  case NN: return fp64 ? Cfg<double, NN>::plane : Cfg<float, NN>::plane;
    LACE_SIZES(X)
#undef X
    default: return false;
  }
}

int ztile_points(int n, bool fp64, int z) {
  switch (n) {
#define X(NN)                                                         \
  case NN:                                                            \
    return fp64 ? (z == 1 ? Engine<double, NN>::zt(1)                 \
                   : z == 2 ? Engine<double, NN>::zt(2)               \
                            : Engine<double, NN>::zt(0))              \
                : (z == 1 ? Engine<float, NN>::zt(1)                  \
                   : z == 2 ? Engine<float, NN>::zt(2)                \
                            : Engine<float, NN>::zt(0));
    LACE_SIZES(X)
#undef X
    default: return 0;
  }
}

// The radix plan of length n read backwards differs from the plan itself.
template <int N> static constexpr bool plan_asym() {
  constexpr int ns = Plan<N, 0>::nst;
  for (int k = 0; k < ns; ++k)
    if (Plan<N, 0>::r[k] != Plan<N, 0>::r[ns - 1 - k]) return true;
  return false;
}
bool radix_orders_differ(int n) {
  switch (n) {
#define X(NN) case NN: return plan_asym<NN>() || plan_asym<NN / 2>();
    LACE_SIZES(X)
#undef X
    default: return false;
  }
}

int64_t energy_tiles(int n, bool fp64) {
  switch (n) {
#define X(NN) \
  case NN: return fp64 ? Engine<double, NN>::tiles() : Engine<float, NN>::tiles();
    LACE_SIZES(X)
#undef X
    default: return 0;
  }
}

template <typename T>
static hipError_t fft3d_t(const CellDev& c, int sign, void* grids, int count,
                          T scale, hipStream_t st) {
  C<T>* g = static_cast<C<T>*>(grids);
  const C<T>* tw = static_cast<const C<T>*>(c.tw);
  switch (c.n) {
#define X(NN)                                                            \
  case NN:                                                               \
    return sign < 0 ? Engine<T, NN>::template fft3d<-1>(g, count, scale, tw, \
                                                         c.use_plane, st)   \
                    : Engine<T, NN>::template fft3d<+1>(g, count, scale, tw, \
                                                         c.use_plane, st);
    LACE_SIZES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fft3d(const CellDev& c, bool fp64, int sign, void* grids,
                        int count, hipStream_t st) {
  return fp64 ? fft3d_t<double>(c, sign, grids, count, 1.0, st)
              : fft3d_t<float>(c, sign, grids, count, 1.0f, st);
}

hipError_t launch_zero(void* p, int64_t bytes, hipStream_t st) {
  if (bytes <= 0) return hipSuccess;
  const int64_t n16 = bytes / 16;
  if (n16 > 0) {
    int64_t blocks = (n16 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    LACE_LAUNCH(k_zero, dim3((unsigned)blocks), dim3(256), 0, st,
                       static_cast<uint4*>(p), n16);
  }
  const int64_t rem = bytes - n16 * 16;
  if (rem > 0)
    LACE_LAUNCH(k_zero_tail, dim3(1), dim3(64), 0, st,
                       static_cast<unsigned char*>(p) + n16 * 16, rem);
  return hipGetLastError();
}

template <typename T>
static hipError_t orb_to_grid_t(const CellDev& c, const void* coeffs,
                                int n_orb, void* psi, hipStream_t st) {
  const int64_t bytes = (int64_t)n_orb * c.ng * sizeof(C<T>);
  hipError_t err = launch_zero(psi, bytes, st);
  if (err != hipSuccess) return err;
  const int64_t total = c.n_pw * n_orb;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  LACE_LAUNCH((k_scatter<T>), dim3((unsigned)blocks), dim3(256), 0, st,
                     static_cast<const double2*>(coeffs), c.n_pw, c.gidx,
                     static_cast<C<T>*>(psi), c.ng, n_orb);
  err = hipGetLastError();
  if (err != hipSuccess) return err;
  return fft3d_t<T>(c, +1, psi, n_orb, T(1.0 / std::sqrt(c.omega)), st);
}

hipError_t launch_orbitals_to_grid(const CellDev& c, bool fp64,
                                   const void* coeffs, int n_orb, void* psi,
                                   hipStream_t st) {
  return fp64 ? orb_to_grid_t<double>(c, coeffs, n_orb, psi, st)
              : orb_to_grid_t<float>(c, coeffs, n_orb, psi, st);
}

template <typename T>
static hipError_t grid_to_pw_t(const CellDev& c, void* w, int n_orb,
                               void* w_pw, hipStream_t st) {
  hipError_t err = fft3d_t<T>(c, -1, w, n_orb, T(1), st);
  if (err != hipSuccess) return err;
  const int64_t total = c.n_pw * n_orb;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  LACE_LAUNCH((k_gather<T>), dim3((unsigned)blocks), dim3(256), 0, st,
                     static_cast<const C<T>*>(w), c.ng, c.gidx, c.n_pw, n_orb,
                     std::sqrt(c.omega) / double(c.ng),
                     static_cast<double2*>(w_pw));
  return hipGetLastError();
}

hipError_t launch_grid_to_pw(const CellDev& c, bool fp64, void* w, int n_orb,
                             void* w_pw, hipStream_t st) {
  return fp64 ? grid_to_pw_t<double>(c, w, n_orb, w_pw, st)
              : grid_to_pw_t<float>(c, w, n_orb, w_pw, st);
}

template <typename T>
static hipError_t pair_batch_t(const CellDev& c, const BatchDev* bt, int cap,
                               const void* psi, void* w, void* tmp,
                               double* epart, hipStream_t st,
                               hipEvent_t* ev, const BatchSync* sy) {
  switch (c.n) {
#define X(NN)                                                               \
  case NN:                                                                  \
    return c.radix ? Engine<T, NN, 1>::pair_batch(                          \
                         c, bt, cap, static_cast<const C<T>*>(psi),         \
                         static_cast<C<T>*>(w), static_cast<C<T>*>(tmp),    \
                         epart, st, ev, sy)                                 \
                   : Engine<T, NN, 0>::pair_batch(                          \
                         c, bt, cap, static_cast<const C<T>*>(psi),         \
                         static_cast<C<T>*>(w), static_cast<C<T>*>(tmp),    \
                         epart, st, ev, sy);
    LACE_SIZES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pair_batch(const CellDev& c, bool fp64, const BatchDev* bt,
                             int cap, const void* psi, void* w, void* tmp,
                             double* epart, hipStream_t st, hipEvent_t* ev,
                             const BatchSync* sy) {
  if (cap <= 0 || cap > SMAX) return hipErrorInvalidValue;
  return fp64 ? pair_batch_t<double>(c, bt, cap, psi, w, tmp, epart, st, ev, sy)
              : pair_batch_t<float>(c, bt, cap, psi, w, tmp, epart, st, ev, sy);
}

hipError_t launch_reduce_sum(const double* part, int64_t count, double factor,
                             double* out, hipStream_t st) {
  LACE_LAUNCH(k_reduce_sum, dim3(1), dim3(256), 0, st, part, count,
                     factor, out);
  return hipGetLastError();
}

// ------------------------------------------ real (Gamma-point) orbitals
// grid p <- C_{2p} + i C_{2p+1} on the sphere (zero elsewhere)
template <typename T>
__global__ void k_scatter_pairs(const double2* coeffs, int64_t n_pw,
                                const int32_t* gidx, C<T>* z, int64_t gs,
                                int n_orb) {
  const int npair = (n_orb + 1) / 2;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int64_t total = n_pw * npair;
  for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < total;
       k += stride) {
    const int64_t p = k / n_pw, m = k % n_pw;
    const double2 a = coeffs[(2 * p) * n_pw + m];
    double2 b = make_double2(0.0, 0.0);
    if (2 * p + 1 < n_orb) b = coeffs[(2 * p + 1) * n_pw + m];
    z[p * gs + gidx[m]] = mk<T>(T(a.x - b.y), T(a.y + b.x));
  }
}

// Unpack two real transforms: with Z = F[W_a + i W_b],
// F[W_a](G) = (Z(G) + conj Z(-G)) / 2, F[W_b](G) = (Z(G) - conj Z(-G)) / 2i.
template <typename T>
__global__ void k_gather_pairs(const C<T>* z, int64_t gs, const int32_t* gidx,
                               const int32_t* negidx, int64_t n_pw, int n_orb,
                               double scale, double2* out) {
  const int npair = (n_orb + 1) / 2;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int64_t total = n_pw * npair;
  for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < total;
       k += stride) {
    const int64_t p = k / n_pw, m = k % n_pw;
    const C<T> a = z[p * gs + gidx[m]];
    const C<T> b = z[p * gs + gidx[negidx[m]]];
    const double ax = a.x, ay = a.y, bx = b.x, by = b.y;
    out[(2 * p) * n_pw + m] =
        make_double2(0.5 * scale * (ax + bx), 0.5 * scale * (ay - by));
    if (2 * p + 1 < n_orb)
      out[(2 * p + 1) * n_pw + m] =
          make_double2(0.5 * scale * (ay + by), -0.5 * scale * (ax - bx));
  }
}

static unsigned grid_for(int64_t total) {
  int64_t blocks = (total + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (blocks < 1) blocks = 1;
  return (unsigned)blocks;
}

template <typename T>
static hipError_t orb_to_grid_real_t(const CellDev& c, const void* coeffs,
                                     int n_orb, void* psi, void* scratch,
                                     hipStream_t st) {
  // the packed coefficients go to the psi buffer (npair complex grids, the
  // bytes of n_orb real ones), are transformed through scratch, and come
  // back to psi as real grids
  const int npair = (n_orb + 1) / 2;
  C<T>* zin = static_cast<C<T>*>(psi);
  hipError_t err = launch_zero(zin, (int64_t)npair * c.ng * sizeof(C<T>), st);
  if (err != hipSuccess) return err;
  LACE_LAUNCH((k_scatter_pairs<T>), dim3(grid_for(c.n_pw * npair)),
                     dim3(256), 0, st, static_cast<const double2*>(coeffs),
                     c.n_pw, c.gidx, zin, c.ng, n_orb);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  const T scale = T(1.0 / std::sqrt(c.omega));
  C<T>* z = static_cast<C<T>*>(scratch);
  T* out = static_cast<T*>(psi);
  const C<T>* tw = static_cast<const C<T>*>(c.tw);
  switch (c.n) {
#define X(NN)                                                               \
  case NN:                                                                  \
    return Engine<T, NN>::to_real(zin, z, npair, scale, out, n_orb, tw,     \
                                  c.use_plane, st);
    LACE_SIZES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_orbitals_to_grid_real(const CellDev& c, bool fp64,
                                        const void* coeffs, int n_orb,
                                        void* psi, void* scratch,
                                        hipStream_t st) {
  return fp64 ? orb_to_grid_real_t<double>(c, coeffs, n_orb, psi, scratch, st)
              : orb_to_grid_real_t<float>(c, coeffs, n_orb, psi, scratch, st);
}

template <typename T>
static hipError_t grid_to_pw_real_t(const CellDev& c, const void* w, int n_orb,
                                    void* scratch, void* w_pw, hipStream_t st) {
  const int npair = (n_orb + 1) / 2;
  C<T>* z = static_cast<C<T>*>(scratch);
  const C<T>* tw = static_cast<const C<T>*>(c.tw);
  hipError_t err = hipErrorInvalidValue;
  switch (c.n) {
#define X(NN)                                                               \
  case NN:                                                                  \
    err = Engine<T, NN>::from_real(static_cast<const T*>(w), n_orb, z,      \
                                   npair, tw, c.use_plane, st);             \
    break;
    LACE_SIZES(X)
#undef X
    default: break;
  }
  if (err != hipSuccess) return err;
  LACE_LAUNCH((k_gather_pairs<T>), dim3(grid_for(c.n_pw * npair)),
                     dim3(256), 0, st, static_cast<const C<T>*>(scratch), c.ng,
                     c.gidx, c.negidx, c.n_pw, n_orb,
                     std::sqrt(c.omega) / double(c.ng),
                     static_cast<double2*>(w_pw));
  return hipGetLastError();
}

hipError_t launch_grid_to_pw_real(const CellDev& c, bool fp64,
                                  const void* w_real, int n_orb, void* scratch,
                                  void* w_pw, hipStream_t st) {
  return fp64 ? grid_to_pw_real_t<double>(c, w_real, n_orb, scratch, w_pw, st)
              : grid_to_pw_real_t<float>(c, w_real, n_orb, scratch, w_pw, st);
}

template <typename T>
static hipError_t quad_batch_t(const CellDev& c, const BatchDev* bt, int cap,
                               const void* psi, void* w, void* tmp,
                               double* epart, hipStream_t st, hipEvent_t* ev,
                               const BatchSync* sy) {
  switch (c.n) {
#define X(NN)                                                                \
  case NN:                                                                   \
    return c.radix ? Engine<T, NN, 1>::quad_batch(                           \
                         c, bt, cap, static_cast<const T*>(psi),             \
                         static_cast<T*>(w), static_cast<C<T>*>(tmp), epart, \
                         st, ev, sy)                                         \
                   : Engine<T, NN, 0>::quad_batch(                           \
                         c, bt, cap, static_cast<const T*>(psi),             \
                         static_cast<T*>(w), static_cast<C<T>*>(tmp), epart, \
                         st, ev, sy);
    LACE_SIZES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_quad_batch(const CellDev& c, bool fp64, const BatchDev* bt,
                             int cap, const void* psi, void* w, void* tmp,
                             double* epart, hipStream_t st, hipEvent_t* ev,
                             const BatchSync* sy) {
  if (cap <= 0 || cap > SMAX) return hipErrorInvalidValue;
  return fp64 ? quad_batch_t<double>(c, bt, cap, psi, w, tmp, epart, st, ev, sy)
              : quad_batch_t<float>(c, bt, cap, psi, w, tmp, epart, st, ev, sy);
}

// per block: sum |C_m - conj C_{-m}|^2 and sum |C_m|^2 over its share
__global__ void k_real_check(const double2* coeffs, int64_t n_pw, int n_orb,
                             const int32_t* negidx, double* part) {
  __shared__ double red[2][4];
  double d = 0.0, t = 0.0;
  const int64_t total = n_pw * n_orb;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < total;
       k += stride) {
    const int64_t j = k / n_pw, m = k % n_pw;
    const double2 a = coeffs[k];
    const double2 b = coeffs[j * n_pw + negidx[m]];
    const double dx = a.x - b.x, dy = a.y + b.y;
    d += dx * dx + dy * dy;
    t += a.x * a.x + a.y * a.y;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    d += __shfl_xor(d, o, 64);
    t += __shfl_xor(t, o, 64);
  }
  if (threadIdx.x % 64 == 0) {
    red[0][threadIdx.x / 64] = d;
    red[1][threadIdx.x / 64] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    part[2 * blockIdx.x + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
}

hipError_t launch_real_check(const CellDev& c, const void* coeffs, int n_orb,
                             double* part, int* nblocks, hipStream_t st) {
  unsigned nb = grid_for(c.n_pw * n_orb);
  if (nb > 1024) nb = 1024;
  *nblocks = (int)nb;
  LACE_LAUNCH(k_real_check, dim3(nb), dim3(256), 0, st,
                     static_cast<const double2*>(coeffs), c.n_pw, n_orb,
                     c.negidx, part);
  return hipGetLastError();
}

}  // namespace lace
