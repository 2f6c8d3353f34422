// screen_kernels.hip - the screening decision of Eq. (6) on the device:
// which unordered pairs (i, j), i <= j, are kept (S_ij >= S_thr), listed
// column by column (j ascending, i ascending within a column).
#include <algorithm>

#include "internal.hpp"

namespace lace {

namespace {

constexpr int KC_NT = 256;   // threads per column workgroup

// Exclusive prefix sum over the KC_NT flags of a workgroup; returns the
// total.  `red` holds KC_NT / 64 ints.
__device__ inline int block_exclusive(int flag, int* excl, int* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long m = __ballot(flag);
  const int below = __popcll(m & ((1ull << lane) - 1ull));
  if (lane == 0) red[wave] = __popcll(m);
  __syncthreads();
  int base = 0, total = 0;
  for (int w = 0; w < KC_NT / 64; ++w) {
    if (w < wave) base += red[w];
    total += red[w];
  }
  *excl = base + below;
  __syncthreads();
  return total;
}

// cnt[j] = #{i <= j : S[i][j] >= thr}; one workgroup per column.
__global__ __launch_bounds__(KC_NT) void k_kept_count(const double* __restrict__ s,
                                                      int n, double thr,
                                                      int32_t* __restrict__ cnt) {
  __shared__ int red[KC_NT / 64];
  const int j = blockIdx.x;
  int c = 0;
  for (int i0 = 0; i0 <= j; i0 += KC_NT) {
    const int i = i0 + (int)threadIdx.x;
    int ex;
    c += block_exclusive(i <= j && s[(int64_t)i * n + j] >= thr, &ex, red);
  }
  if (threadIdx.x == 0) cnt[j] = c;
}

// off[j] = sum of cnt[0 .. j-1], off[n] = total; *total_out = total.
__global__ __launch_bounds__(KC_NT) void k_kept_scan(const int32_t* __restrict__ cnt,
                                                     int n, int64_t* __restrict__ off,
                                                     int64_t* __restrict__ total_out) {
  __shared__ int64_t part[KC_NT];
  // each thread sums a contiguous run of columns, then the runs are scanned
  const int per = (n + KC_NT - 1) / KC_NT;
  const int a = (int)threadIdx.x * per;
  const int b = a + per < n ? a + per : n;
  int64_t t = 0;
  for (int j = a; j < b; ++j) t += cnt[j];
  part[threadIdx.x] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int k = 0; k < KC_NT; ++k) {
      const int64_t v = part[k];
      part[k] = run;
      run += v;
    }
    off[n] = run;
    if (total_out) *total_out = run;
  }
  __syncthreads();
  int64_t run = part[threadIdx.x];
  for (int j = a; j < b; ++j) {
    off[j] = run;
    run += cnt[j];
  }
}

// pairs[2k], pairs[2k + 1] = (i, j) of the k-th kept pair.
__global__ __launch_bounds__(KC_NT) void k_kept_write(const double* __restrict__ s,
                                                      int n, double thr,
                                                      const int64_t* __restrict__ off,
                                                      int32_t* __restrict__ pairs) {
  __shared__ int red[KC_NT / 64];
  const int j = blockIdx.x;
  int64_t base = off[j];
  for (int i0 = 0; i0 <= j; i0 += KC_NT) {
    const int i = i0 + (int)threadIdx.x;
    const int keep = i <= j && s[(int64_t)i * n + j] >= thr;
    int ex;
    const int tot = block_exclusive(keep, &ex, red);
    if (keep) {
      pairs[2 * (base + ex)] = i;
      pairs[2 * (base + ex) + 1] = j;
    }
    base += tot;
  }
}

// Every pair (s == nullptr): the list of all i <= j in the same order.
__global__ void k_all_pairs(int n, int32_t* __restrict__ pairs,
                            int64_t* __restrict__ total_out) {
  const int64_t total = (int64_t)n * (n + 1) / 2;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < total;
       k += (int64_t)gridDim.x * blockDim.x) {
    // column j holds j + 1 pairs starting at j (j + 1) / 2
    int j = (int)((sqrt(8.0 * (double)k + 1.0) - 1.0) * 0.5);
    while ((int64_t)j * (j + 1) / 2 > k) --j;
    while ((int64_t)(j + 1) * (j + 2) / 2 <= k) ++j;
    pairs[2 * k] = (int)(k - (int64_t)j * (j + 1) / 2);
    pairs[2 * k + 1] = j;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && total_out) *total_out = total;
}

}  // namespace

hipError_t launch_kept_pairs(const double* s, int n, double thr, int32_t* cnt,
                             int64_t* off, int32_t* pairs, int64_t* total,
                             hipStream_t st) {
  if (!s) {
    const int64_t tot = (int64_t)n * (n + 1) / 2;
    int64_t blocks = (tot + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    LACE_LAUNCH(k_all_pairs, dim3((unsigned)blocks), dim3(256), 0, st, n, pairs,
                total);
    return hipGetLastError();
  }
  LACE_LAUNCH(k_kept_count, dim3(n), dim3(KC_NT), 0, st, s, n, thr, cnt);
  LACE_LAUNCH(k_kept_scan, dim3(1), dim3(KC_NT), 0, st, cnt, n, off, total);
  LACE_LAUNCH(k_kept_write, dim3(n), dim3(KC_NT), 0, st, s, n, thr, off, pairs);
  return hipGetLastError();
}

// ===================================================================
// Batch schedule of the pair pipeline, built on the device.
//
// Rounds of the circle-method round robin over nv = n_orb rounded up to
// even vertices (vertex nv - 1 fixed): round r pairs nv - 1 with r and
// (r + k, r - k) mod (nv - 1); each round is a set of disjoint pairs, and
// the diagonal pairs form one more round.
//
// Complex orbitals: the kept pairs, round by round, are placed first-fit
// into a window of open batches (no orbital twice in a batch).
//
// Real orbitals: two pair densities share one transform (a slot); two pairs
// that share an orbital make a star slot (three orbital grids instead of
// four).  The union of rounds 2g and 2g + 1 is one cycle through all nv
// vertices, vertex sequence nv - 1, r, r + 2, r - 2, r + 4, r - 4, ...,
// r + 1 (mod nv - 1), edges alternating between the two rounds.  The kept
// edges of the cycle form runs; consecutive edges of a run become star
// slots, and a run of odd length leaves its last edge over.  Left-over
// edges are paired at their smaller orbital, then at their larger one
// (stars again), and what is left is paired as it comes.  One-sided pairs
// (occupied x virtual) form stars around their virtual orbital; diagonal
// pairs go two by two.  The slots are then placed first-fit like the pairs.
//
// The host launches max_batches batches, the count of the round-robin
// schedule (every round, and the diagonal round, in batches of their own),
// which bounds any set of pairs; if first-fit would need more, the table is
// rebuilt as that round-robin schedule.  Entries past the last batch have
// n = 0.

namespace {

struct SlotRec {
  int32_t i, j, k, l;
  int32_t np;      // pairs in the slot (1 or 2)
  uint32_t flags;  // bit 0: one-sided; bits 1..4: W_i, W_j, W_k, W_l skipped
};

__device__ inline bool kbit(const uint64_t* kb, int words, int a, int b) {
  return (kb[(int64_t)a * words + (b >> 6)] >> (b & 63)) & 1ull;
}

// kb[a][b] = 1 for a != b with S[a][b] >= thr (S symmetric, ns x ns:
// orbitals from ns on have no two-sided pairs); db bit a for S[a][a] >= thr.
// s == nullptr: every pair of the first ns orbitals.  One thread per word.
__global__ void k_sched_bits_s(const double* __restrict__ s, int n, int ns,
                               int words, double thr, uint64_t* __restrict__ kb,
                               uint64_t* __restrict__ db) {
  const int64_t total = (int64_t)n * words;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(t / words), w = (int)(t % words);
    uint64_t m = 0;
    for (int c = 0; c < 64; ++c) {
      const int b = w * 64 + c;
      if (b >= ns || a >= ns) break;
      const bool keep = s ? s[(int64_t)a * ns + b] >= thr : true;
      if (b != a && keep) m |= 1ull << c;
    }
    kb[t] = m;
    // the diagonal word w is gathered over its 64 rows by one thread
    if (a == 0) {
      uint64_t d = 0;
      for (int c = 0; c < 64; ++c) {
        const int r = w * 64 + c;
        if (r >= ns) break;
        if (s ? s[(int64_t)r * ns + r] >= thr : true) d |= 1ull << c;
      }
      db[w] = d;
    }
  }
}

// Bits of an explicit pair list (kb and db cleared before).  A bad pair
// (i > j, out of range) or a repeat sets bit 0 of *bad.
__global__ void k_sched_bits_list(const int32_t* __restrict__ pi,
                                  const int32_t* __restrict__ pj, int64_t np,
                                  int n, int words, uint64_t* __restrict__ kb,
                                  uint64_t* __restrict__ db,
                                  int32_t* __restrict__ bad) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < np;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int i = pi[t], j = pj[t];
    if (i < 0 || j < i || j >= n) { atomicOr(bad, 1); continue; }
    const uint64_t bi = 1ull << (i & 63);
    if (i == j) {
      if (atomicOr(reinterpret_cast<unsigned long long*>(db + (i >> 6)), bi) & bi)
        atomicOr(bad, 1);
      continue;
    }
    if (atomicOr(reinterpret_cast<unsigned long long*>(kb + (int64_t)j * words + (i >> 6)), bi) & bi)
      atomicOr(bad, 1);
    atomicOr(reinterpret_cast<unsigned long long*>(kb + (int64_t)i * words + (j >> 6)),
             1ull << (j & 63));
  }
}

// Vertex t of the cycle of rounds r, r + 1 (r even, nv even, m = nv - 1).
__device__ inline int cyc(int t, int r, int nv) {
  const int m = nv - 1;
  if (t == 0) return nv - 1;
  return (t & 1) ? ((r - t + 1) % m + m) % m : (r + t) % m;
}

// Stars and left-over edges of each pair of rounds (one wave per group;
// group nv/2 - 1 is the single last round).  Output regions per group:
// stars at g * (nv / 2), left-overs (a < b) at g * nv.  The lanes test the
// edges of the cycle; the walk along it is uniform over the wave and reads
// the kept bits and the vertex sequence from LDS.
__global__ __launch_bounds__(64) void k_sched_groups(const uint64_t* __restrict__ kb,
                                                     int n_orb, int words,
                                                     SlotRec* __restrict__ gstar,
                                                     int2* __restrict__ gleft,
                                                     int32_t* __restrict__ gcnt) {
  __shared__ int16_t cv[4096];
  __shared__ uint64_t ek[64];
  const int nv = n_orb + (n_orb & 1), m = nv - 1, ng = nv / 2;
  const int g = blockIdx.x, lane = threadIdx.x;
  SlotRec* st = gstar + (int64_t)g * (nv / 2);
  int2* lf = gleft + (int64_t)g * nv;
  auto kept = [&](int a, int b) {
    return a < n_orb && b < n_orb && kbit(kb, words, a, b);
  };
  const uint64_t below = (1ull << lane) - 1ull;
  if (g == ng - 1) {   // round nv - 2 alone: a set of disjoint pairs
    const int r = nv - 2, last = (m - 1) / 2;
    int nl = 0;
    for (int t0 = 0; t0 <= last; t0 += 64) {
      const int t = t0 + lane;
      int x = 0, y = 0;
      bool keep = false;
      if (t <= last) {
        if (t == 0) { x = r; y = nv - 1; }
        else { x = (r + t) % m; y = ((r - t) % m + m) % m; }
        keep = kept(x, y);
      }
      const uint64_t bal = __ballot(keep);
      if (keep) lf[nl + __popcll(bal & below)] = make_int2(min(x, y), max(x, y));
      nl += __popcll(bal);
    }
    if (lane == 0) { gcnt[2 * g] = 0; gcnt[2 * g + 1] = nl; }
    return;
  }
  const int r = 2 * g, nw = (nv + 63) / 64;
  for (int t = lane; t < nv; t += 64) cv[t] = (int16_t)cyc(t, r, nv);
  __syncthreads();
  for (int t0 = 0; t0 < nv; t0 += 64) {
    const int t = t0 + lane;
    const bool e = t < nv && kept(cv[t], cv[t + 1 < nv ? t + 1 : 0]);
    const uint64_t bal = __ballot(e);
    if (lane == 0) ek[t0 >> 6] = bal;
  }
  __syncthreads();
  int ns = 0, nl = 0;
  auto star = [&](int ta) {   // edges ta, ta + 1
    const int t1 = ta + 1 < nv ? ta + 1 : ta + 1 - nv;
    const int t2 = t1 + 1 < nv ? t1 + 1 : t1 + 1 - nv;
    const int x = cv[ta], c = cv[t1], y = cv[t2];
    if (lane == 0) st[ns] = SlotRec{c, x, c, y, 2, 0u};
    ++ns;
  };
  // first edge not kept
  int t0 = -1;
  for (int w = 0; w < nw && t0 < 0; ++w) {
    uint64_t inv = ~ek[w];
    if (w == nw - 1 && (nv & 63)) inv &= (1ull << (nv & 63)) - 1ull;
    if (inv) t0 = 64 * w + __builtin_ctzll(inv);
  }
  if (t0 < 0) {        // the whole cycle is kept
    for (int t = 0; t < nv; t += 2) star(t);
  } else {
    int pend = -1;
    uint64_t word = 0;
    for (int step = 1; step <= nv; ++step) {
      const int t = t0 + step < nv ? t0 + step : t0 + step - nv;
      if (step == 1 || (t & 63) == 0) word = ek[t >> 6];
      if ((word >> (t & 63)) & 1ull) {
        if (pend < 0) pend = t;
        else { star(pend); pend = -1; }
      } else if (pend >= 0) {
        const int x = cv[pend], y = cv[pend + 1 < nv ? pend + 1 : 0];
        if (lane == 0) lf[nl] = make_int2(min(x, y), max(x, y));
        ++nl;
        pend = -1;
      }
    }
  }
  if (lane == 0) { gcnt[2 * g] = ns; gcnt[2 * g + 1] = nl; }
}

// Complex orbitals: the kept pairs of each round (one wave per round,
// round nv - 1 the diagonal one), one-sided pairs included for virtual
// orbitals.  Output region per round at r * nv.
__global__ __launch_bounds__(64) void k_sched_rounds(const uint64_t* __restrict__ kb,
                                                     const uint64_t* __restrict__ db,
                                                     int n_orb, int n_occ, int words,
                                                     SlotRec* __restrict__ rp,
                                                     int32_t* __restrict__ rcnt) {
  const int nv = n_orb + (n_orb & 1), m = nv - 1;
  const int r = blockIdx.x, lane = threadIdx.x;
  SlotRec* out = rp + (int64_t)r * nv;
  const uint64_t below = (1ull << lane) - 1ull;
  int c = 0;
  if (r == nv - 1) {
    for (int a0 = 0; a0 < n_orb; a0 += 64) {
      const int x = a0 + lane;
      const bool keep = x < n_orb && ((db[x >> 6] >> (x & 63)) & 1ull);
      const uint64_t bal = __ballot(keep);
      if (keep) out[c + __popcll(bal & below)] = SlotRec{x, x, -1, -1, 1, 0u};
      c += __popcll(bal);
    }
  } else {
    const int last = (m - 1) / 2;   // pair t = 0: (r, nv - 1); t = k: (r + k, r - k)
    for (int t0 = 0; t0 <= last; t0 += 64) {
      const int t = t0 + lane;
      int x = 0, y = 0;
      bool keep = false, os = false;
      if (t <= last) {
        if (t == 0) { x = r; y = nv - 1; }
        else { x = (r + t) % m; y = ((r - t) % m + m) % m; }
        if (x > y) { const int z = x; x = y; y = z; }
        if (y < n_orb) {
          // a one-sided pair's occupied orbital (i) keeps its W
          os = x < n_occ && y >= n_occ;
          keep = os || (y < n_occ && kbit(kb, words, x, y));
        }
      }
      const uint64_t bal = __ballot(keep);
      if (keep) out[c + __popcll(bal & below)] = SlotRec{x, y, -1, -1, 1, os ? 3u : 0u};
      c += __popcll(bal);
    }
  }
  if (lane == 0) rcnt[r] = c;
}

constexpr int PK_NT = 256;      // packing workgroup
constexpr int PK_WIN = 8;       // open batches considered
constexpr int PK_LCH = 1024;    // left-over edges staged in LDS at a time

// Exclusive prefix of one value per thread over the packing workgroup;
// *total gets the sum.  `wtot` holds PK_NT / 64 values.
__device__ inline int64_t block_scan(int64_t v, int64_t* wtot, int64_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int64_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wtot[wave] = x;
  __syncthreads();
  int64_t base = 0, t = 0;
  for (int w = 0; w < PK_NT / 64; ++w) {
    if (w < wave) base += wtot[w];
    t += wtot[w];
  }
  *total = t;
  __syncthreads();
  return base + x - v;
}

// Exclusive prefix over cnt[0 .. count) (stride apart) into off (global);
// *total gets the sum.  Each thread takes a contiguous run.
__device__ void block_prefix(const int32_t* cnt, int count, int stride,
                             int64_t* off, int64_t* total, int64_t* wtot) {
  const int per = (count + PK_NT - 1) / PK_NT;
  const int a = threadIdx.x * per, b = min(a + per, count);
  int64_t t = 0;
  for (int k = a; k < b; ++k) t += cnt[(int64_t)k * stride];
  int64_t run = block_scan(t, wtot, total);
  for (int k = a; k < b; ++k) {
    off[k] = run;
    run += cnt[(int64_t)k * stride];
  }
  __syncthreads();
}

struct PackArgs {
  int n_orb, n_occ, words, ppb, cap, gamma, force_fallback;
  int64_t max_batches;
};

struct PackScratch {
  const SlotRec* gstar;   // real: per-group stars; complex: per-round pairs
  const int2* gleft;
  const int32_t* gcnt;
  const uint64_t* kb;
  const uint64_t* db;
  SlotRec* slots;         // the ordered slot list
  int64_t* off;           // per-group offsets (stars, left-overs)
  int2* left;             // left-over edges in group order
};

__device__ inline void put_slot(BatchDev* b, int q, const SlotRec& s) {
  b->i[q] = s.i; b->j[q] = s.j; b->k[q] = s.k; b->l[q] = s.l;
  if (s.flags & 1u) b->one_sided |= 1ull << q;
#pragma unroll
  for (int t = 0; t < 4; ++t)
    if ((s.flags >> (1 + t)) & 1u) b->skip[t] |= 1ull << q;
  if (s.k != s.i) b->star = 0;
  b->n = q + 1;
  b->npairs += s.np;
}

__device__ inline void clear_batch(BatchDev* b) {
  b->n = 0; b->star = 1; b->npairs = 0; b->one_sided = 0;
  b->skip[0] = b->skip[1] = b->skip[2] = b->skip[3] = 0;
}

// Round-robin schedule (the bound the host launches for): every round in
// batches of its own.  One thread.
__device__ void fallback_schedule(const PackArgs& a, const uint64_t* kb,
                                  const uint64_t* db, BatchDev* tab,
                                  int32_t* n_batches) {
  const int nv = a.n_orb + (a.n_orb & 1), m = nv - 1;
  const bool virt = a.n_occ < a.n_orb;
  int64_t nb = 0;
  BatchDev* cur = nullptr;
  int cur_slots = 0, cur_pairs = 0;
  const int sp = a.gamma ? (a.ppb >= 2 ? a.ppb / 2 : 1) : a.ppb;
  auto emit = [&](const SlotRec& s) {
    if (!cur || cur_slots == sp || cur_pairs + s.np > a.ppb) {
      cur = tab + nb++;
      clear_batch(cur);
      cur_slots = cur_pairs = 0;
    }
    put_slot(cur, cur_slots++, s);
    cur_pairs += s.np;
  };
  auto close = [&]() { cur = nullptr; };
  for (int r = 0; r < nv; ++r) {
    SlotRec held[2] = {};
    int nh[2] = {0, 0};     // pending single pair per kind (two-sided, one-sided)
    auto take = [&](int x, int y, bool os) {
      SlotRec s{x, y, -1, -1, 1, 0u};
      if (os) s.flags = 1u | (x < a.n_occ ? 2u : 0u);
      if (!a.gamma) { emit(s); return; }
      if (a.ppb == 1) { emit(s); return; }
      const int kd = os ? 1 : 0;
      if (nh[kd]) {
        SlotRec t = held[kd];
        t.k = x; t.l = y; t.np = 2;
        if (os && x < a.n_occ) t.flags |= 8u;
        emit(t);
        nh[kd] = 0;
      } else {
        held[kd] = s;
        nh[kd] = 1;
      }
    };
    if (r == nv - 1) {
      for (int d = 0; d < a.n_orb; ++d)
        if ((db[d >> 6] >> (d & 63)) & 1ull) take(d, d, false);
    } else {
      auto pr = [&](int x, int y) {
        if (x > y) { const int t = x; x = y; y = t; }
        if (y >= a.n_orb) return;
        const bool os = virt && x < a.n_occ && y >= a.n_occ;
        if (os) take(x, y, true);
        else if (y < a.n_occ && kbit(kb, a.words, x, y)) take(x, y, false);
      };
      pr(r, nv - 1);
      for (int k = 1; k <= (m - 1) / 2; ++k) pr((r + k) % m, ((r - k) % m + m) % m);
    }
    for (int kd = 0; kd < 2; ++kd)
      if (nh[kd]) emit(held[kd]);
    close();
  }
  for (int64_t b = nb; b < a.max_batches; ++b) clear_batch(tab + b), tab[b].n = 0;
  *n_batches = (int32_t)nb;
}

// Slot list, then first-fit packing into the batch table.  One workgroup.
__global__ __launch_bounds__(PK_NT) void k_sched_pack(PackArgs a, PackScratch sc,
                                                      BatchDev* __restrict__ tab,
                                                      int32_t* __restrict__ n_batches,
                                                      int64_t* __restrict__ n_pairs) {
  __shared__ int64_t wtot[PK_NT / 64];
  __shared__ int64_t tot[4];
  __shared__ int red[PK_NT / 64];
  __shared__ int32_t st_nb, st_over;
  // the slot-list phase and the first-fit phase share this space
  __shared__ __attribute__((aligned(16))) char pool[8192 * 6];
  int16_t* vcnt = reinterpret_cast<int16_t*>(pool);           // stars of each vertex
  int32_t* voff = reinterpret_cast<int32_t*>(pool + 8192);    // their staging offsets
  int16_t* p1 = reinterpret_cast<int16_t*>(pool + 8192 * 3);  // unpaired edge at v
  int16_t* p2 = reinterpret_cast<int16_t*>(pool + 8192 * 4);  // edge held at v
  int2* lbuf = reinterpret_cast<int2*>(pool + 8192 * 5);      // PK_LCH edges
  uint32_t* inwin = reinterpret_cast<uint32_t*>(pool);        // 4098 words
  int32_t* bst = reinterpret_cast<int32_t*>(pool + 16448);    // PK_WIN x 4 x 64 orbitals
  int32_t* bid = reinterpret_cast<int32_t*>(pool + 24640);    // PK_WIN batch ids
  uint64_t* bbits = reinterpret_cast<uint64_t*>(pool + 24704);  // PK_WIN x 5 header words
  const int n = a.n_orb, nv = n + (n & 1), tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  int64_t nslots = 0;
  // ---------------------------------------------------------- slot list
  if (a.gamma) {
    const int ng = nv / 2;
    block_prefix(sc.gcnt, ng, 2, sc.off, &tot[0], wtot);            // stars
    block_prefix(sc.gcnt + 1, ng, 2, sc.off + ng, &tot[1], wtot);   // left
    const int64_t nstar = tot[0], nleft = tot[1];
    for (int g = wave; g < ng; g += PK_NT / 64) {
      const int64_t o = sc.off[g], ol = sc.off[ng + g];
      const int c = sc.gcnt[2 * g], cl = sc.gcnt[2 * g + 1];
      for (int t = lane; t < c; t += 64)
        sc.slots[o + t] = sc.gstar[(int64_t)g * (nv / 2) + t];
      for (int t = lane; t < cl; t += 64)
        sc.left[ol + t] = sc.gleft[(int64_t)g * nv + t];
    }
    for (int v = tid; v < n; v += PK_NT) { vcnt[v] = 0; p1[v] = -1; p2[v] = -1; }
    __syncthreads();
    nslots = nstar;
    // left-overs, round 1: pairs at the smaller orbital, in edge order.
    // Vertex v belongs to thread v mod PK_NT, which alone reads and writes
    // its entries.  Pass 0 counts each vertex's stars; pass 1 writes them to
    // a staging area (the group-star region, no longer needed) at prefix
    // offsets.  After either pass p1[v] is the edge left unpaired at v.
    SlotRec* stage = const_cast<SlotRec*>(sc.gstar);
    for (int pass = 0; pass < 2; ++pass) {
      for (int64_t c0 = 0; c0 < nleft; c0 += PK_LCH) {
        const int cn = (int)min<int64_t>(PK_LCH, nleft - c0);
        __syncthreads();
        const int cn8 = (cn + 7) & ~7;   // padded with x = -1
        for (int t = tid; t < cn8; t += PK_NT)
          lbuf[t] = t < cn ? sc.left[c0 + t] : make_int2(-1, -1);
        __syncthreads();
        for (int t0 = 0; t0 < cn8; t0 += 8) {
          int2 e8[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) e8[u] = lbuf[t0 + u];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int2 ed = e8[u];
            if (ed.x < 0 || (ed.x & (PK_NT - 1)) != tid) continue;
            const int v = ed.x, h = p1[v];
            if (h < 0) { p1[v] = (int16_t)ed.y; continue; }
            if (pass) stage[voff[v] + vcnt[v]] = SlotRec{v, h, v, ed.y, 2, 0u};
            vcnt[v] = (int16_t)(vcnt[v] + 1);
            p1[v] = -1;
          }
        }
      }
      __syncthreads();
      if (!pass) {
        // offsets of the vertices' stars: contiguous runs per thread
        const int per = (n + PK_NT - 1) / PK_NT;
        const int lo = tid * per, hi = min(lo + per, n);
        int64_t t = 0;
        for (int v = lo; v < hi; ++v) t += vcnt[v];
        int64_t unused;
        int64_t run = block_scan(t, wtot, &unused);
        for (int v = lo; v < hi; ++v) {
          voff[v] = (int32_t)run;
          run += vcnt[v];
          vcnt[v] = 0;
          p1[v] = -1;
        }
        __syncthreads();
      }
    }
    // the stars leave the staging area interleaved: every vertex's first
    // star, then every vertex's second one, ...  (consecutive slots then
    // rarely share their centre, which keeps first-fit from opening a new
    // batch for each of them)
    {
      int64_t base = 0;
      for (int rho = 0;; ++rho) {
        int64_t got = 0;
        for (int v0 = 0; v0 < n; v0 += PK_NT) {
          const int v = v0 + tid;
          const int flag = v < n && vcnt[v] > rho;
          int ex;
          const int t = block_exclusive(flag, &ex, red);
          if (flag) sc.slots[nslots + base + got + ex] = stage[voff[v] + rho];
          got += t;
        }
        if (got == 0) break;
        base += got;
      }
      nslots += base;
    }
    __syncthreads();
    // round 2: the unpaired edges at their larger orbital; then the rest
    // as it comes
    if (tid == 0) {
      int64_t w = nslots;
      for (int v = 0; v < n; ++v) {
        const int y = p1[v];
        if (y < 0) continue;
        const int h = p2[y];
        if (h < 0) { p2[y] = (int16_t)v; continue; }
        sc.slots[w++] = SlotRec{y, h, y, v, 2, 0u};
        p2[y] = -1;
      }
      int hx = -1, hy = -1;
      for (int v = 0; v < n; ++v) {
        const int x = p2[v];
        if (x < 0) continue;
        if (hx < 0) { hx = x; hy = v; continue; }
        // edges (hx, hy) and (x, v)
        if (hx == x || hx == v || hy == x || hy == v) {
          const int c = (hx == x || hx == v) ? hx : hy;
          const int pj = hx == c ? hy : hx, ql = x == c ? v : x;
          sc.slots[w++] = SlotRec{c, pj, c, ql, 2, 0u};
        } else {
          sc.slots[w++] = SlotRec{hx, hy, x, v, 2, 0u};
        }
        hx = -1;
      }
      if (hx >= 0) sc.slots[w++] = SlotRec{hx, hy, -1, -1, 1, 0u};
      tot[3] = w;
    }
    __syncthreads();
    int64_t w = tot[3];
    // one-sided pairs: stars around each virtual orbital u with the
    // occupied pair (2t, 2t + 1), t = (k + u) mod P in round k, so that
    // the stars of one round share no orbital
    if (a.n_occ < n) {
      const int P = a.n_occ / 2, nvirt = n - a.n_occ;
      const int64_t cnt = (int64_t)P * nvirt;
      for (int64_t q = tid; q < cnt; q += PK_NT) {
        const int k = (int)(q / nvirt), u = (int)(q % nvirt);
        const int v = a.n_occ + u, t = 2 * ((k + u) % P);
        sc.slots[w + q] = SlotRec{v, t, v, t + 1, 2, 1u | 4u | 16u};
      }
      w += cnt;
      if (a.n_occ & 1) {
        for (int u = tid; u < nvirt; u += PK_NT)
          sc.slots[w + u] = SlotRec{a.n_occ - 1, a.n_occ + u, -1, -1, 1, 1u | 2u};
        w += nvirt;
      }
    }
    // diagonal pairs, two by two
    if (tid == 0) {
      int hd = -1;
      for (int wd = 0; wd < a.words; ++wd) {
        uint64_t bits = sc.db[wd];
        while (bits) {
          const int d = 64 * wd + __builtin_ctzll(bits);
          bits &= bits - 1ull;
          if (hd < 0) { hd = d; continue; }
          sc.slots[w++] = SlotRec{hd, hd, d, d, 2, 0u};
          hd = -1;
        }
      }
      if (hd >= 0) sc.slots[w++] = SlotRec{hd, hd, -1, -1, 1, 0u};
      tot[2] = w;
    }
    __syncthreads();
    nslots = tot[2];
  } else {
    block_prefix(sc.gcnt, nv, 1, sc.off, &tot[0], wtot);
    for (int r = wave; r < nv; r += PK_NT / 64) {
      const int64_t o = sc.off[r];
      const int c = sc.gcnt[r];
      for (int t = lane; t < c; t += 64)
        sc.slots[o + t] = sc.gstar[(int64_t)r * nv + t];
    }
    nslots = tot[0];
  }
  // clear the table and the window masks
  for (int64_t b = tid; b < a.max_batches; b += PK_NT) clear_batch(tab + b);
  __syncthreads();
  for (int o = tid; o < 4098; o += PK_NT) inwin[o] = 0u;
  __syncthreads();
  // ------------------------------------------------------ first-fit
  // One wave; its state is uniform.  The open batches sit at window
  // positions 0 .. nopen - 1, oldest first, so the first fit is the lowest
  // candidate bit.  inwin[o] has bit x set when orbital o is in the batch at
  // position x (entry 4096 stands for "no orbital" and stays 0; 4097 takes
  // the writes for it).  The slot and pair counts of the positions are the
  // bytes of two 64-bit words; fit1 / fit2 are the positions that can take
  // a one- / two-pair slot.  Each open batch builds its slot lists, id and
  // header bits in one of PK_WIN staging buffers in LDS (phys, 4 bits per
  // position); a batch that leaves the window (full, or the oldest when a
  // new one is needed) is written to the table whole, and the positions
  // above it move down one.  The masks of the next slot are read before
  // the current one is placed, then corrected for it.
  if (wave == 0) {
    constexpr uint32_t NONE_R = 4096u, NONE_W = 4097u;
    uint64_t cnt_s = 0, cnt_p = 0;
    uint32_t fit1 = 0, fit2 = 0, nstar = 0, phys = 0, freep = (1u << PK_WIN) - 1u;
    int nopen = 0, nb = 0, over = a.force_fallback;
    // 64 slot records a lane, packed: orbitals as 16 bits (-1 as NONE_R),
    // then pairs | flags << 8 | (not a star) << 16 | (shares an orbital
    // with the next slot) << 17
    auto load = [&](int64_t base, uint32_t& ij, uint32_t& kl, uint32_t& ex) {
      ij = NONE_R | (NONE_R << 16);
      kl = ij;
      ex = 0;
      if (base + lane < nslots) {
        const SlotRec r = sc.slots[base + lane];
        ij = (uint32_t)r.i | ((uint32_t)r.j << 16);
        kl = (r.k < 0 ? NONE_R : (uint32_t)r.k) | ((r.l < 0 ? NONE_R : (uint32_t)r.l) << 16);
        ex = (uint32_t)r.np | (r.flags << 8) | (r.k != r.i ? 1u << 16 : 0u);
      }
    };
    auto share = [&](uint32_t& ex, uint32_t ij, uint32_t kl, uint32_t nij, uint32_t nkl) {
      const uint32_t o[4] = {ij & 0xFFFFu, ij >> 16, kl & 0xFFFFu, kl >> 16};
      const uint32_t m[4] = {nij & 0xFFFFu, nij >> 16, nkl & 0xFFFFu, nkl >> 16};
      bool hit = false;
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) hit |= o[u] != NONE_R && o[u] == m[v];
      if (hit) ex |= 1u << 17;
    };
    auto masks = [&](uint32_t ij, uint32_t kl) -> uint32_t {
      return inwin[ij & 0xFFFFu] | inwin[ij >> 16] | inwin[kl & 0xFFFFu] | inwin[kl >> 16];
    };
    uint32_t aij, akl, aex, bij, bkl, bex;   // slots c0 .. c0 + 63, and the next 64
    auto mark = [&]() {   // the share bits of chunk a
      uint32_t nij = __shfl_down(aij, 1, 64), nkl = __shfl_down(akl, 1, 64);
      const uint32_t fij = __builtin_amdgcn_readlane(bij, 0);
      const uint32_t fkl = __builtin_amdgcn_readlane(bkl, 0);
      if (lane == 63) { nij = fij; nkl = fkl; }
      share(aex, aij, akl, nij, nkl);
    };
    auto drop = [&](int x, uint32_t& pre) {   // position x leaves the window
      const int ph = (int)((phys >> (4 * x)) & 15u);
      const int ns = (int)((cnt_s >> (8 * x)) & 0xFFu);
      BatchDev* b = tab + bid[ph];
      if (lane < ns) {
        b->i[lane] = bst[(ph * 4 + 0) * 64 + lane];
        b->j[lane] = bst[(ph * 4 + 1) * 64 + lane];
        b->k[lane] = bst[(ph * 4 + 2) * 64 + lane];
        b->l[lane] = bst[(ph * 4 + 3) * 64 + lane];
      }
      if (lane == 0) {
        b->n = ns;
        b->star = (nstar >> x) & 1u ? 0 : 1;
        b->npairs = (int32_t)((cnt_p >> (8 * x)) & 0xFFu);
        b->one_sided = bbits[ph * 5];
        b->skip[0] = bbits[ph * 5 + 1]; b->skip[1] = bbits[ph * 5 + 2];
        b->skip[2] = bbits[ph * 5 + 3]; b->skip[3] = bbits[ph * 5 + 4];
      }
      const uint64_t lowb = (1ull << (8 * x)) - 1ull;
      cnt_s = (cnt_s & lowb) | ((cnt_s >> 8) & ~lowb);
      cnt_p = (cnt_p & lowb) | ((cnt_p >> 8) & ~lowb);
      const uint32_t lown = (1u << (4 * x)) - 1u;
      phys = (phys & lown) | ((phys >> 4) & ~lown);
      freep |= 1u << ph;
      const uint32_t low = (1u << x) - 1u;
      fit1 = (fit1 & low) | ((fit1 >> 1) & ~low);
      fit2 = (fit2 & low) | ((fit2 >> 1) & ~low);
      nstar = (nstar & low) | ((nstar >> 1) & ~low);
      pre = (pre & low) | ((pre >> 1) & ~low);
      for (int o = lane; o < n; o += 64) {
        const uint32_t v = inwin[o];
        inwin[o] = (v & low) | ((v >> 1) & ~low);
      }
      --nopen;
    };
    load(0, aij, akl, aex);
    load(64, bij, bkl, bex);
    mark();
    int64_t c0 = 0;
    uint32_t sij = __builtin_amdgcn_readlane(aij, 0);
    uint32_t skl = __builtin_amdgcn_readlane(akl, 0);
    uint32_t sex = __builtin_amdgcn_readlane(aex, 0);
    uint32_t conf = nslots > 0 ? masks(sij, skl) : 0u;
    for (int64_t q = 0; q < nslots && !over; ++q) {
      // the next slot and its masks, read before this one is placed
      uint32_t nij = 0, nkl = 0, nex = 0, pre = 0;
      if (q + 1 < nslots) {
        const int r = (int)(q + 1 - c0);
        if (r < 64) {
          nij = __builtin_amdgcn_readlane(aij, r);
          nkl = __builtin_amdgcn_readlane(akl, r);
          nex = __builtin_amdgcn_readlane(aex, r);
        } else {
          nij = __builtin_amdgcn_readlane(bij, 0);
          nkl = __builtin_amdgcn_readlane(bkl, 0);
          nex = __builtin_amdgcn_readlane(bex, 0);
        }
        pre = masks(nij, nkl);
      }
      const int np = (int)(sex & 0xFFu);
      const uint32_t cand = (np == 1 ? fit1 : fit2) & ~conf;
      int x;
      if (cand) {
        x = __builtin_ctz(cand);
      } else {
        if (nb >= a.max_batches) { over = 1; break; }
        if (nopen == PK_WIN) drop(0, pre);   // the oldest leaves
        x = nopen++;
        const int ph = __builtin_ctz(freep);
        freep &= ~(1u << ph);
        phys |= (uint32_t)ph << (4 * x);
        if (lane == 0) bid[ph] = nb;
        if (lane < 5) bbits[ph * 5 + lane] = 0ull;
        ++nb;
        fit1 |= 1u << x;
        if (a.ppb >= 2) fit2 |= 1u << x;
      }
      const uint32_t bit = 1u << x;
      const int qs = (int)((cnt_s >> (8 * x)) & 0xFFu);
      const int ph = (int)((phys >> (4 * x)) & 15u);
      const uint32_t oi = sij & 0xFFFFu, oj = sij >> 16, ok = skl & 0xFFFFu, ol = skl >> 16;
      if (lane == 0) {
        int32_t* st = bst + ph * 256 + qs;
        st[0] = (int32_t)oi;
        st[64] = (int32_t)oj;
        st[128] = ok == NONE_R ? -1 : (int32_t)ok;
        st[192] = ol == NONE_R ? -1 : (int32_t)ol;
        atomicOr(&inwin[oi], bit);
        atomicOr(&inwin[oj], bit);
        atomicOr(&inwin[ok == NONE_R ? NONE_W : ok], bit);
        atomicOr(&inwin[ol == NONE_R ? NONE_W : ol], bit);
      }
      cnt_s += 1ull << (8 * x);
      cnt_p += (uint64_t)np << (8 * x);
      const int fs = qs + 1, fp = (int)((cnt_p >> (8 * x)) & 0xFFu);
      if (fs >= a.cap || fp + 1 > a.ppb) fit1 &= ~bit;
      if (fs >= a.cap || fp + 2 > a.ppb) fit2 &= ~bit;
      if ((sex >> 16) & 1u) nstar |= bit;
      const uint32_t fl = (sex >> 8) & 0xFFu;
      if (fl) {   // one-sided or skipped-W bits (virtual orbitals)
        if (lane < 5 && ((fl >> lane) & 1u))
          atomicOr(reinterpret_cast<unsigned long long*>(&bbits[ph * 5 + lane]),
                   1ull << qs);
      }
      // the next slot shares an orbital with this one: not at position x
      if ((sex >> 17) & 1u) pre |= bit;
      if (fp >= a.ppb || fs >= a.cap) drop(x, pre);   // full
      sij = nij; skl = nkl; sex = nex; conf = pre;
      if (q + 1 - c0 == 64) {
        c0 += 64;
        aij = bij; akl = bkl; aex = bex;
        load(c0 + 64, bij, bkl, bex);
        mark();
        sex = __builtin_amdgcn_readlane(aex, 0);   // now with its share bit
      }
    }
    if (!over) {
      uint32_t unused = 0;
      while (nopen) drop(nopen - 1, unused);
    }
    if (lane == 0) { st_nb = nb; st_over = over; }
  }
  __syncthreads();
  {
    int64_t np = 0;
    for (int64_t q = tid; q < nslots; q += PK_NT) np += sc.slots[q].np;
    int64_t total = 0;
    block_scan(np, wtot, &total);
    if (tid == 0) {
      if (n_pairs) *n_pairs = total;
      if (st_over) fallback_schedule(a, sc.kb, sc.db, tab, n_batches);
      else *n_batches = st_nb;
    }
  }
}

}  // namespace

int64_t sched_scratch_bytes(int n_orb) {
  const int64_t nv = n_orb + (n_orb & 1), ng = nv / 2;
  const int64_t words = (n_orb + 63) / 64;
  auto up = [](int64_t x) { return (x + 255) & ~int64_t(255); };
  int64_t b = 0;
  b += up(8 * (int64_t)n_orb * words);                              // kb
  b += up(8 * words);                                               // db
  b += up((int64_t)sizeof(SlotRec) * std::max(ng * (nv / 2), nv * nv));  // gstar
  b += up(8 * ng * nv);                                             // gleft
  b += up(4 * std::max(2 * ng, nv));                                // gcnt
  b += up(8 * (2 * nv + 2));                                        // off
  b += up(8 * ng * nv);                                             // left
  const int64_t nslot = (int64_t)n_orb * (n_orb + 1) / 2 +
                        (int64_t)n_orb * n_orb / 4 + n_orb + 8;
  b += up((int64_t)sizeof(SlotRec) * nslot);                        // slots
  b += up(64);                                                      // flags
  return b;
}

hipError_t launch_schedule(const SchedDesc& d, hipStream_t st) {
  const int n = d.n_orb, nv = n + (n & 1), ng = nv / 2;
  const int words = (n + 63) / 64;
  if (n < 1 || words > 64 || d.ppb < 1 || d.ppb > PMAX) return hipErrorInvalidValue;
  char* p = static_cast<char*>(d.scratch);
  auto up = [](int64_t x) { return (x + 255) & ~int64_t(255); };
  auto take = [&](int64_t bytes) { char* q = p; p += up(bytes); return q; };
  uint64_t* kb = reinterpret_cast<uint64_t*>(take(8 * (int64_t)n * words));
  uint64_t* db = reinterpret_cast<uint64_t*>(take(8 * words));
  SlotRec* gstar = reinterpret_cast<SlotRec*>(
      take((int64_t)sizeof(SlotRec) * std::max((int64_t)ng * (nv / 2), (int64_t)nv * nv)));
  int2* gleft = reinterpret_cast<int2*>(take(8 * (int64_t)ng * nv));
  int32_t* gcnt = reinterpret_cast<int32_t*>(take(4 * std::max(2 * ng, nv)));
  int64_t* off = reinterpret_cast<int64_t*>(take(8 * (2 * (int64_t)nv + 2)));
  int2* left = reinterpret_cast<int2*>(take(8 * (int64_t)ng * nv));
  const int64_t nslot = (int64_t)n * (n + 1) / 2 + (int64_t)n * n / 4 + n + 8;
  SlotRec* slots = reinterpret_cast<SlotRec*>(take((int64_t)sizeof(SlotRec) * nslot));
  int32_t* flags = reinterpret_cast<int32_t*>(take(64));
  hipError_t e = launch_zero(db, 8 * words, st);
  if (e != hipSuccess) return e;
  if (d.pair_i) {
    e = launch_zero(kb, 8 * (int64_t)n * words, st);
    if (e == hipSuccess) e = launch_zero(d.bad ? (void*)d.bad : (void*)flags, 4, st);
    if (e != hipSuccess) return e;
    int64_t blocks = (d.n_pairs + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 1024) blocks = 1024;
    LACE_LAUNCH(k_sched_bits_list, dim3((unsigned)blocks), dim3(256), 0, st,
                d.pair_i, d.pair_j, d.n_pairs, n, words, kb, db,
                d.bad ? d.bad : flags);
  } else {
    int64_t blocks = ((int64_t)n * words + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    LACE_LAUNCH(k_sched_bits_s, dim3((unsigned)blocks), dim3(256), 0, st, d.s,
                n, d.s_n > 0 ? d.s_n : n, words, d.s_thr, kb, db);
  }
  // real orbitals pack two pairs per slot when a batch takes two pairs
  const bool pack = d.gamma && d.ppb >= 2;
  if (pack) {
    LACE_LAUNCH(k_sched_groups, dim3(ng), dim3(64), 0, st, kb, n,
                words, gstar, gleft, gcnt);
  } else {
    LACE_LAUNCH(k_sched_rounds, dim3(nv), dim3(64), 0, st, kb, db,
                n, d.n_occ, words, gstar, gcnt);
  }
  PackArgs a;
  a.n_orb = n; a.n_occ = d.n_occ; a.words = words; a.ppb = d.ppb;
  a.cap = d.gamma ? (d.ppb + 1) / 2 : d.ppb;
  a.gamma = pack ? 1 : 0;
  a.force_fallback = d.force_fallback ? 1 : 0;
  a.max_batches = d.max_batches;
  PackScratch sc{gstar, gleft, gcnt, kb, db, slots, off, left};
  LACE_LAUNCH(k_sched_pack, dim3(1), dim3(PK_NT), 0, st, a, sc, d.table,
              d.n_batches, d.n_kept);
  return hipGetLastError();
}

}  // namespace lace
