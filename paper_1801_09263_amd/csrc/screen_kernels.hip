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
// Complex orbitals: the kept pairs, round by round, form the slot list.
//
// Real orbitals: two pair densities share one transform (a slot); two pairs
// that share an orbital make a star slot (three orbital grids instead of
// four).  The union of rounds 2g and 2g + 1 is one cycle through all nv
// vertices, vertex sequence nv - 1, r, r + 2, r - 2, r + 4, r - 4, ...,
// r + 1 (mod nv - 1), edges alternating between the two rounds.  The kept
// edges of the cycle form runs; consecutive edges of a run become star
// slots, and a run of odd length leaves its last edge over.  Left-over
// edges are paired at their smaller orbital (in group order), then the
// unpaired ones at their larger orbital (stars again), both interleaved by
// rank, and what is left is paired as it comes.  One-sided pairs (occupied
// x virtual) form stars around their virtual orbital; diagonal pairs go
// two by two.
//
// Packing: the slot list is cut into sections (boundaries moved to whole
// groups or rounds), each section is placed first-fit into a window of
// open batches on its own wave (no orbital twice in a batch), and the
// slots of the batches that did not fill are placed first-fit once more
// after the full ones.
//
// The host launches max_batches batches, the count of the round-robin
// schedule (every round, and the diagonal round, in batches of their own),
// which bounds any set of pairs; if the packing would need more, the table
// is rebuilt as that round-robin schedule.  Entries past the last batch
// have n = 0.

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

constexpr int PK_NT = 256;      // list and merge workgroups
constexpr int PK_WIN = 8;       // open batches considered by first-fit

// Exclusive prefix of one value per thread over a PK_NT workgroup;
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
  int n_orb, n_occ, words, ppb, cap, gamma, force_fallback, sections;
  int64_t max_batches;
  int64_t per_bound;      // slots a section's index regions hold
};

struct PackScratch {
  const SlotRec* gstar;   // real: per-group stars; complex: per-round pairs
  const int2* gleft;      // real: per-group left-over edges
  const int32_t* gcnt;
  const uint64_t* kb;
  const uint64_t* db;
  SlotRec* slots;         // the ordered slot list
  int64_t* off;           // per-group offsets
  uint64_t* lb;           // n x ceil(groups / 64): left-over edges by group
  int16_t* ytab;          // n x groups: their larger orbital
  uint64_t* rb;           // n x words: unpaired edges at their larger orbital
  int64_t* count;         // [0] slots, [1] pairs, [2] slots in group (or
                          // round) order, [3] groups (rounds)
  int32_t* idx;           // 2 x sections x per_bound slot indices: the full
                          // batches of each section, then the refill batches
  int32_t* fcnt;          // sections x per_bound: slots of each full batch
  int32_t* pidx;          // sections x per_bound: slots of the other batches
  int32_t* scnt;          // sections x 4: full batches, their slots, others
  int32_t* rlist;         // sections x per_bound: the refill order
  int32_t* dir;           // per batch: first index in idx, slot count
  int32_t* flags;         // [0]: fallback used, [1]: batches
};

// Lowest set bit at or above position p of a bit row that has one.
__device__ inline int next_bit(const uint64_t* row, int p) {
  int w = p >> 6;
  uint64_t m = row[w] & (~0ull << (p & 63));
  while (!m) m = row[++w];
  return 64 * w + __builtin_ctzll(m);
}

// Stars of bit rows: row v lists v's edges, bit b standing for the edge to
// orbital other(v, b); each vertex pairs its edges in ascending bit order,
// and the stars leave interleaved, every vertex's first star, then every
// vertex's second one, ... (consecutive slots then rarely share their
// centre).  pend[v] gets the other orbital of v's unpaired edge (the last
// bit), or -1.  Returns the number of stars written to out.  Called by the
// whole PK_NT workgroup.
template <class Other>
__device__ int64_t emit_stars(const uint64_t* rows, int n, int words, Other other,
                              SlotRec* out, int16_t* vcnt, int16_t* cur,
                              int16_t* pend, int* red) {
  const int tid = threadIdx.x;
  for (int v = tid; v < n; v += PK_NT) {
    int c = 0, last = -1;
    for (int w = 0; w < words; ++w) {
      const uint64_t m = rows[(int64_t)v * words + w];
      c += __popcll(m);
      if (m) last = 64 * w + 63 - __clzll(m);
    }
    vcnt[v] = (int16_t)(c >> 1);
    pend[v] = (int16_t)((c & 1) ? other(v, last) : -1);
    cur[v] = 0;
  }
  __syncthreads();
  int64_t base = 0;
  for (int rho = 0;; ++rho) {
    int64_t got = 0;
    for (int v0 = 0; v0 < n; v0 += PK_NT) {
      const int v = v0 + tid;
      const int flag = v < n && vcnt[v] > rho;
      int ex;
      const int t = block_exclusive(flag, &ex, red);
      if (flag) {
        const uint64_t* row = rows + (int64_t)v * words;
        const int b1 = next_bit(row, cur[v]);
        const int b2 = next_bit(row, b1 + 1);
        cur[v] = (int16_t)(b2 + 1);
        out[base + got + ex] = SlotRec{v, other(v, b1), v, other(v, b2), 2, 0u};
      }
      got += t;
    }
    if (got == 0) break;
    base += got;
  }
  __syncthreads();
  return base;
}

// The ordered slot list, its length and pair count.  One workgroup.
__global__ __launch_bounds__(PK_NT) void k_sched_list(PackArgs a, PackScratch sc) {
  __shared__ int64_t wtot[PK_NT / 64];
  __shared__ int64_t tot[4];
  __shared__ int red[PK_NT / 64];
  __shared__ int16_t vcnt[4096], cur[4096], pend[4096];
  const int n = a.n_orb, nv = n + (n & 1), tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  int64_t nslots = 0;
  if (a.gamma) {
    const int ng = nv / 2;
    block_prefix(sc.gcnt, ng, 2, sc.off, &tot[0], wtot);   // stars per group
    // left-over edges by group: a vertex has at most one per group (two
    // in one group would be adjacent kept edges of one run), so row x of lb
    // has bit g for the left-over (x, y), x < y, of group g, and
    // ytab[x][g] = y; rb rows are orbital bits
    const int gw = (ng + 63) / 64;
    for (int64_t t = tid; t < (int64_t)n * gw; t += PK_NT) sc.lb[t] = 0ull;
    for (int64_t t = tid; t < (int64_t)n * a.words; t += PK_NT) sc.rb[t] = 0ull;
    __syncthreads();
    for (int g = wave; g < ng; g += PK_NT / 64) {
      const int64_t o = sc.off[g];
      const int c = sc.gcnt[2 * g], cl = sc.gcnt[2 * g + 1];
      for (int t = lane; t < c; t += 64)
        sc.slots[o + t] = sc.gstar[(int64_t)g * (nv / 2) + t];
      for (int t = lane; t < cl; t += 64) {
        const int2 e = sc.gleft[(int64_t)g * nv + t];
        sc.ytab[(int64_t)e.x * ng + g] = (int16_t)e.y;
        atomicOr(reinterpret_cast<unsigned long long*>(&sc.lb[(int64_t)e.x * gw + (g >> 6)]),
                 1ull << (g & 63));
      }
    }
    __syncthreads();
    nslots = tot[0];
    // left-overs, first pass: stars at the smaller orbital, in group order
    const int16_t* ytab = sc.ytab;
    nslots += emit_stars(sc.lb, n, gw,
                         [ytab, ng](int v, int g) { return (int)ytab[(int64_t)v * ng + g]; },
                         sc.slots + nslots, vcnt, cur, pend, red);
    // second pass: the unpaired edges, stars at their larger orbital
    for (int v = tid; v < n; v += PK_NT) {
      const int y = pend[v];
      if (y >= 0)
        atomicOr(reinterpret_cast<unsigned long long*>(
                     &sc.rb[(int64_t)y * a.words + (v >> 6)]),
                 1ull << (v & 63));
    }
    __syncthreads();
    nslots += emit_stars(sc.rb, n, a.words, [](int, int x) { return x; },
                         sc.slots + nslots, vcnt, cur, pend, red);
    // what is left (edge (pend[b], b) at each b) is paired as it comes
    if (tid == 0) {
      int64_t w = nslots;
      int hx = -1, hy = -1;
      for (int v = 0; v < n; ++v) {
        const int x = pend[v];
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
    __syncthreads();
  }
  int64_t np = 0;
  for (int64_t q = tid; q < nslots; q += PK_NT) np += sc.slots[q].np;
  int64_t total = 0;
  block_scan(np, wtot, &total);
  if (tid == 0) {
    sc.count[0] = nslots;
    sc.count[1] = total;
    sc.count[2] = tot[0];
    sc.count[3] = a.gamma ? nv / 2 : nv;
  }
}

// First-fit of count slots (slot t of the order: slots[ord(t)]) into a
// window of PK_WIN open batches, no orbital twice in a batch, by one wave.
// The wave's state is uniform.  The open batches sit at window positions
// 0 .. nopen - 1, oldest first, so the first fit is the lowest candidate
// bit.  inwin[o] has bit x set when orbital o is in the batch at position x
// (entry 4096 stands for "no orbital" and stays 0; 4097 takes the writes
// for it).  The slot and pair counts of the positions are the bytes of two
// 64-bit words; fit1 / fit2 are the positions that can take a one- / two-
// pair slot.  Each open batch lists its slots' indices in one of PK_WIN
// LDS rows (phys: the row of each position, 4 bits each).  A batch leaves
// the window when it is full, when it is the oldest and a new one is
// needed, or at the end, oldest first; it is then handed to
// emit(row, slots, full), and the positions above it move down one.  The
// masks of the next slot are read before the current one is placed, then
// corrected for it.  Returns 1 when more than max_open batches would be
// opened (the rest is then not placed).
template <class Ord, class Emit>
__device__ int window_ff(const PackArgs& a, int64_t count, Ord ord,
                         const SlotRec* __restrict__ slots, int64_t max_open,
                         Emit emit, uint32_t* inwin, int32_t* bidx) {
  constexpr uint32_t NONE_R = 4096u, NONE_W = 4097u;
  const int lane = threadIdx.x & 63, n = a.n_orb;
  for (int o = lane; o < 4098; o += 64) inwin[o] = 0u;
  uint64_t cnt_s = 0, cnt_p = 0;
  uint32_t fit1 = 0, fit2 = 0, phys = 0, freep = (1u << PK_WIN) - 1u;
  int nopen = 0, over = 0;
  int64_t nb = 0;
  // 64 slots a lane, packed: orbitals as 16 bits (-1 as NONE_R), then
  // pairs | (shares an orbital with the next slot) << 17, and the index
  auto load = [&](int64_t base, uint32_t& ij, uint32_t& kl, uint32_t& ex, int32_t& ix) {
    ij = NONE_R | (NONE_R << 16);
    kl = ij;
    ex = 0;
    ix = -1;
    if (base + lane < count) {
      ix = ord(base + lane);
      const SlotRec r = slots[ix];
      ij = (uint32_t)r.i | ((uint32_t)r.j << 16);
      kl = (r.k < 0 ? NONE_R : (uint32_t)r.k) | ((r.l < 0 ? NONE_R : (uint32_t)r.l) << 16);
      ex = (uint32_t)r.np;
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
  int32_t aix, bix;
  auto mark = [&]() {   // the share bits of chunk a
    uint32_t nij = __shfl_down(aij, 1, 64), nkl = __shfl_down(akl, 1, 64);
    const uint32_t fij = __builtin_amdgcn_readlane(bij, 0);
    const uint32_t fkl = __builtin_amdgcn_readlane(bkl, 0);
    if (lane == 63) { nij = fij; nkl = fkl; }
    share(aex, aij, akl, nij, nkl);
  };
  auto drop = [&](int x, uint32_t& pre, bool full) {   // position x leaves
    const int ph = (int)((phys >> (4 * x)) & 15u);
    emit(bidx + ph * 64, (int)((cnt_s >> (8 * x)) & 0xFFu), full);
    const uint64_t lowb = (1ull << (8 * x)) - 1ull;
    cnt_s = (cnt_s & lowb) | ((cnt_s >> 8) & ~lowb);
    cnt_p = (cnt_p & lowb) | ((cnt_p >> 8) & ~lowb);
    const uint32_t lown = (1u << (4 * x)) - 1u;
    phys = (phys & lown) | ((phys >> 4) & ~lown);
    freep |= 1u << ph;
    const uint32_t low = (1u << x) - 1u;
    fit1 = (fit1 & low) | ((fit1 >> 1) & ~low);
    fit2 = (fit2 & low) | ((fit2 >> 1) & ~low);
    pre = (pre & low) | ((pre >> 1) & ~low);
    for (int o = lane; o < n; o += 64) {
      const uint32_t v = inwin[o];
      inwin[o] = (v & low) | ((v >> 1) & ~low);
    }
    --nopen;
  };
  load(0, aij, akl, aex, aix);
  load(64, bij, bkl, bex, bix);
  mark();
  int64_t c0 = 0;
  uint32_t sij = __builtin_amdgcn_readlane(aij, 0);
  uint32_t skl = __builtin_amdgcn_readlane(akl, 0);
  uint32_t sex = __builtin_amdgcn_readlane(aex, 0);
  int32_t six = __builtin_amdgcn_readlane(aix, 0);
  uint32_t conf = count > 0 ? masks(sij, skl) : 0u;
  for (int64_t q = 0; q < count; ++q) {
    // the next slot and its masks, read before this one is placed
    uint32_t nij = 0, nkl = 0, nex = 0, pre = 0;
    int32_t nix = -1;
    if (q + 1 < count) {
      const int r = (int)(q + 1 - c0);
      if (r < 64) {
        nij = __builtin_amdgcn_readlane(aij, r);
        nkl = __builtin_amdgcn_readlane(akl, r);
        nex = __builtin_amdgcn_readlane(aex, r);
        nix = __builtin_amdgcn_readlane(aix, r);
      } else {
        nij = __builtin_amdgcn_readlane(bij, 0);
        nkl = __builtin_amdgcn_readlane(bkl, 0);
        nex = __builtin_amdgcn_readlane(bex, 0);
        nix = __builtin_amdgcn_readlane(bix, 0);
      }
      pre = masks(nij, nkl);
    }
    const int np = (int)(sex & 0xFFu);
    const uint32_t cand = (np == 1 ? fit1 : fit2) & ~conf;
    int x;
    if (cand) {
      x = __builtin_ctz(cand);
    } else {
      if (nb >= max_open) { over = 1; break; }
      if (nopen == PK_WIN) drop(0, pre, false);   // the oldest leaves
      x = nopen++;
      const int ph = __builtin_ctz(freep);
      freep &= ~(1u << ph);
      phys |= (uint32_t)ph << (4 * x);
      ++nb;
      fit1 |= 1u << x;
      if (a.ppb >= 2) fit2 |= 1u << x;
    }
    const uint32_t bit = 1u << x;
    const int qs = (int)((cnt_s >> (8 * x)) & 0xFFu);
    const int ph = (int)((phys >> (4 * x)) & 15u);
    const uint32_t oi = sij & 0xFFFFu, oj = sij >> 16, ok = skl & 0xFFFFu, ol = skl >> 16;
    if (lane == 0) {
      bidx[ph * 64 + qs] = six;
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
    // the next slot shares an orbital with this one: not at position x
    if ((sex >> 17) & 1u) pre |= bit;
    if (fp >= a.ppb || fs >= a.cap) drop(x, pre, true);   // full
    sij = nij; skl = nkl; sex = nex; six = nix; conf = pre;
    if (q + 1 - c0 == 64) {
      c0 += 64;
      aij = bij; akl = bkl; aex = bex; aix = bix;
      load(c0 + 64, bij, bkl, bex, bix);
      mark();
      sex = __builtin_amdgcn_readlane(aex, 0);   // now with its share bit
    }
  }
  if (!over) {
    uint32_t unused = 0;
    while (nopen) drop(0, unused, false);
  }
  return over;
}

// Start of section k of the slot list: k * per moved up to the next group
// (round) boundary while it falls among the group-ordered slots, so that a
// section takes whole cycles; section `sections` ends the list.
__device__ inline int64_t section_start(const PackScratch& sc, int sections,
                                        int64_t per, int k) {
  const int64_t ns = sc.count[0], G = sc.count[2];
  const int ng = (int)sc.count[3];
  if (k >= sections) return ns;
  const int64_t t = min(ns, (int64_t)k * per);
  if (t >= G) return t;
  int lo = 0, hi = ng;   // first group g with off[g] >= t (off[ng] = G)
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (sc.off[mid] >= t) hi = mid; else lo = mid + 1;
  }
  return lo < ng ? sc.off[lo] : G;
}

// First-fit of each section of the slot list on its own (one wave per
// section): the full batches' slot indices go to idx (section region) and
// their slot counts to fcnt, the other batches' indices to pidx.
__global__ __launch_bounds__(64) void k_sched_sections(PackArgs a, PackScratch sc) {
  __shared__ uint32_t inwin[4098];
  __shared__ int32_t bidx[PK_WIN * 64];
  const int k = blockIdx.x, lane = threadIdx.x;
  if (k >= a.sections || a.force_fallback) return;
  const int64_t ns = sc.count[0];
  const int64_t per = (ns + a.sections - 1) / a.sections;
  const int64_t lo = section_start(sc, a.sections, per, k);
  const int64_t hi = section_start(sc, a.sections, per, k + 1);
  int32_t* fidx = sc.idx + (int64_t)k * a.per_bound;
  int32_t* fcnt = sc.fcnt + (int64_t)k * a.per_bound;
  int32_t* pidx = sc.pidx + (int64_t)k * a.per_bound;
  int nfb = 0;
  int64_t nfi = 0, npi = 0;
  auto emit = [&](const int32_t* row, int cnt, bool full) {
    int32_t* dst = full ? fidx + nfi : pidx + npi;
    for (int q = lane; q < cnt; q += 64) dst[q] = row[q];
    if (full) {
      if (lane == 0) fcnt[nfb] = cnt;
      ++nfb;
      nfi += cnt;
    } else {
      npi += cnt;
    }
  };
  window_ff(a, hi - lo, [&](int64_t t) { return (int32_t)(lo + t); }, sc.slots,
            INT64_MAX, emit, inwin, bidx);
  if (lane == 0) {
    sc.scnt[4 * k] = nfb;
    sc.scnt[4 * k + 1] = (int32_t)nfi;
    sc.scnt[4 * k + 2] = (int32_t)npi;
  }
}

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

// The sections' full batches in section order, then first-fit of all
// their other slots (section order) on one wave; the batch directory; the
// round-robin fallback when the batches would not fit the table.  One
// workgroup.
__global__ __launch_bounds__(PK_NT) void k_sched_merge(PackArgs a, PackScratch sc,
                                                       BatchDev* __restrict__ tab,
                                                       int32_t* __restrict__ n_batches,
                                                       int64_t* __restrict__ n_pairs) {
  __shared__ uint32_t inwin[4098];
  __shared__ int32_t bidx[PK_WIN * 64];
  __shared__ int32_t sfb[32], sfi[32], spi[32];
  __shared__ int32_t st_nb, st_over;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int S = a.sections;
  if (tid == 0) {
    int32_t fb = 0, fi = 0, pi = 0;
    for (int k = 0; k < S; ++k) {
      sfb[k] = fb; sfi[k] = fi; spi[k] = pi;
      if (!a.force_fallback) {
        fb += sc.scnt[4 * k]; fi += sc.scnt[4 * k + 1]; pi += sc.scnt[4 * k + 2];
      }
    }
    sfb[S] = fb; sfi[S] = fi; spi[S] = pi;
  }
  __syncthreads();
  const int32_t F = sfb[S];
  const int64_t pb = a.per_bound;
  // directory of the full batches: wave w takes sections w, w + 4, ...
  for (int k = wave; k < S; k += PK_NT / 64) {
    const int nfb = sfb[k + 1] - sfb[k];
    int32_t run = 0;
    for (int c0 = 0; c0 < nfb; c0 += 64) {
      const int t = c0 + lane;
      const int32_t v = t < nfb ? sc.fcnt[k * pb + t] : 0;
      int32_t x = v;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
      }
      if (t < nfb) {
        sc.dir[2 * (sfb[k] + t)] = (int32_t)(k * pb) + run + x - v;
        sc.dir[2 * (sfb[k] + t) + 1] = v;
      }
      run += __shfl(x, 63, 64);
    }
  }
  // the refill order
  for (int k = 0; k < S; ++k) {
    const int np = spi[k + 1] - spi[k];
    for (int t = tid; t < np; t += PK_NT) sc.rlist[spi[k] + t] = sc.pidx[k * pb + t];
  }
  __syncthreads();
  if (wave == 0) {
    int32_t* ridx = sc.idx + (int64_t)S * pb;
    int64_t rpos = 0;
    int32_t rb = 0;
    auto emit = [&](const int32_t* row, int cnt, bool) {
      for (int q = lane; q < cnt; q += 64) ridx[rpos + q] = row[q];
      if (lane == 0) {
        sc.dir[2 * (F + rb)] = (int32_t)(S * pb + rpos);
        sc.dir[2 * (F + rb) + 1] = cnt;
      }
      ++rb;
      rpos += cnt;
    };
    int over = a.force_fallback || F > a.max_batches;
    if (!over)
      over = window_ff(a, spi[S], [&](int64_t t) { return sc.rlist[t]; }, sc.slots,
                       a.max_batches - F, emit, inwin, bidx);
    if (lane == 0) { st_nb = F + rb; st_over = over; }
  }
  __syncthreads();
  if (tid == 0) {
    if (n_pairs) *n_pairs = sc.count[1];
    sc.flags[0] = st_over;
    sc.flags[1] = st_nb;
    if (st_over) fallback_schedule(a, sc.kb, sc.db, tab, n_batches);
    else *n_batches = st_nb;
  }
}

// The batch table from the directory: one wave per batch; entries past
// the last batch are cleared.  Skipped when the fallback wrote the table.
__global__ __launch_bounds__(64) void k_sched_fill(PackArgs a, PackScratch sc,
                                                   BatchDev* __restrict__ tab) {
  if (sc.flags[0]) return;
  const int lane = threadIdx.x;
  const int64_t nb = sc.flags[1];
  for (int64_t g = blockIdx.x; g < a.max_batches; g += gridDim.x) {
    BatchDev* b = tab + g;
    if (g >= nb) {
      if (lane == 0) clear_batch(b);
      continue;
    }
    const int32_t start = sc.dir[2 * g], cnt = sc.dir[2 * g + 1];
    const bool on = lane < cnt;
    SlotRec s{-1, -1, -1, -1, 0, 0u};
    if (on) {
      s = sc.slots[sc.idx[start + lane]];
      b->i[lane] = s.i; b->j[lane] = s.j; b->k[lane] = s.k; b->l[lane] = s.l;
    }
    const uint64_t os = __ballot(on && (s.flags & 1u));
    const uint64_t s0 = __ballot(on && ((s.flags >> 1) & 1u));
    const uint64_t s1 = __ballot(on && ((s.flags >> 2) & 1u));
    const uint64_t s2 = __ballot(on && ((s.flags >> 3) & 1u));
    const uint64_t s3 = __ballot(on && ((s.flags >> 4) & 1u));
    const uint64_t ns = __ballot(on && s.k != s.i);
    int np = on ? s.np : 0;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) np += __shfl_xor(np, d, 64);
    if (lane == 0) {
      b->n = cnt;
      b->star = ns ? 0 : 1;
      b->npairs = np;
      b->one_sided = os;
      b->skip[0] = s0; b->skip[1] = s1; b->skip[2] = s2; b->skip[3] = s3;
    }
  }
}

}  // namespace

int sched_sections(int n_orb) {
  const int64_t s = (int64_t)n_orb * n_orb / 4096;
  return s < 1 ? 1 : s > 16 ? 16 : (int)s;
}

int64_t sched_slot_bound(int n_orb) {
  return (int64_t)n_orb * (n_orb + 1) / 2 + (int64_t)n_orb * n_orb / 4 + n_orb + 8;
}

namespace {

struct SchedLayout {
  uint64_t *kb, *db;
  SlotRec* gstar;
  int2* gleft;
  int32_t* gcnt;
  int64_t* off;
  uint64_t* lb;
  int16_t* ytab;
  uint64_t* rb;
  SlotRec* slots;
  int64_t* count;
  int32_t *idx, *fcnt, *pidx, *scnt, *rlist, *dir, *flags;
  int64_t per_bound;
  int64_t bytes;
};

// The scheduler's scratch regions (base == nullptr: sizes only).
SchedLayout sched_layout(int n, void* base) {
  const int64_t nv = n + (n & 1), ng = nv / 2;
  const int64_t words = (n + 63) / 64;
  const int64_t nslot = sched_slot_bound(n);
  const int S = sched_sections(n);
  // a section is its share of the slots, moved to group boundaries: it
  // may take up to one group (round) more
  const int64_t pb = (nslot + S - 1) / S + nv;
  char* p = static_cast<char*>(base);
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    char* q = p ? p + off : nullptr;
    off += (bytes + 255) & ~int64_t(255);
    return q;
  };
  SchedLayout L;
  L.kb = reinterpret_cast<uint64_t*>(take(8 * n * words));
  L.db = reinterpret_cast<uint64_t*>(take(8 * words));
  L.gstar = reinterpret_cast<SlotRec*>(
      take((int64_t)sizeof(SlotRec) * std::max(ng * (nv / 2), nv * nv)));
  L.gleft = reinterpret_cast<int2*>(take(8 * ng * nv));
  L.gcnt = reinterpret_cast<int32_t*>(take(4 * std::max(2 * ng, nv)));
  L.off = reinterpret_cast<int64_t*>(take(8 * (2 * nv + 2)));
  L.lb = reinterpret_cast<uint64_t*>(take(8 * n * ((ng + 63) / 64)));
  L.ytab = reinterpret_cast<int16_t*>(take(2 * n * ng));
  L.rb = reinterpret_cast<uint64_t*>(take(8 * n * words));
  L.slots = reinterpret_cast<SlotRec*>(take((int64_t)sizeof(SlotRec) * nslot));
  L.count = reinterpret_cast<int64_t*>(take(32));
  L.idx = reinterpret_cast<int32_t*>(take(4 * 2 * S * pb));
  L.fcnt = reinterpret_cast<int32_t*>(take(4 * S * pb));
  L.pidx = reinterpret_cast<int32_t*>(take(4 * S * pb));
  L.scnt = reinterpret_cast<int32_t*>(take(4 * 4 * S));
  L.rlist = reinterpret_cast<int32_t*>(take(4 * S * pb));
  L.dir = reinterpret_cast<int32_t*>(take(4 * 2 * nslot));
  L.flags = reinterpret_cast<int32_t*>(take(64));
  L.per_bound = pb;
  L.bytes = off;
  return L;
}

}  // namespace

int64_t sched_scratch_bytes(int n_orb) { return sched_layout(n_orb, nullptr).bytes; }

hipError_t launch_schedule(const SchedDesc& d, hipStream_t st) {
  const int n = d.n_orb, nv = n + (n & 1), ng = nv / 2;
  const int words = (n + 63) / 64;
  if (n < 1 || words > 64 || d.ppb < 1 || d.ppb > PMAX) return hipErrorInvalidValue;
  const SchedLayout L = sched_layout(n, d.scratch);
  hipError_t e = launch_zero(L.db, 8 * words, st);
  if (e != hipSuccess) return e;
  if (d.pair_i) {
    e = launch_zero(L.kb, 8 * (int64_t)n * words, st);
    if (e == hipSuccess) e = launch_zero(d.bad ? (void*)d.bad : (void*)L.flags, 4, st);
    if (e != hipSuccess) return e;
    int64_t blocks = (d.n_pairs + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 1024) blocks = 1024;
    LACE_LAUNCH(k_sched_bits_list, dim3((unsigned)blocks), dim3(256), 0, st,
                d.pair_i, d.pair_j, d.n_pairs, n, words, L.kb, L.db,
                d.bad ? d.bad : L.flags);
  } else {
    int64_t blocks = ((int64_t)n * words + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    LACE_LAUNCH(k_sched_bits_s, dim3((unsigned)blocks), dim3(256), 0, st, d.s,
                n, d.s_n > 0 ? d.s_n : n, words, d.s_thr, L.kb, L.db);
  }
  // real orbitals pack two pairs per slot when a batch takes two pairs
  const bool pack = d.gamma && d.ppb >= 2;
  if (pack) {
    LACE_LAUNCH(k_sched_groups, dim3(ng), dim3(64), 0, st, L.kb, n,
                words, L.gstar, L.gleft, L.gcnt);
  } else {
    LACE_LAUNCH(k_sched_rounds, dim3(nv), dim3(64), 0, st, L.kb, L.db,
                n, d.n_occ, words, L.gstar, L.gcnt);
  }
  PackArgs a;
  a.n_orb = n; a.n_occ = d.n_occ; a.words = words; a.ppb = d.ppb;
  a.cap = d.gamma ? (d.ppb + 1) / 2 : d.ppb;
  a.gamma = pack ? 1 : 0;
  a.force_fallback = d.force_fallback ? 1 : 0;
  a.sections = sched_sections(n);
  a.max_batches = d.max_batches;
  a.per_bound = L.per_bound;
  PackScratch sc{L.gstar, L.gleft, L.gcnt, L.kb, L.db, L.slots, L.off,
                 L.lb, L.ytab, L.rb, L.count, L.idx, L.fcnt, L.pidx, L.scnt,
                 L.rlist, L.dir, L.flags};
  LACE_LAUNCH(k_sched_list, dim3(1), dim3(PK_NT), 0, st, a, sc);
  LACE_LAUNCH(k_sched_sections, dim3(a.sections), dim3(64), 0, st, a, sc);
  LACE_LAUNCH(k_sched_merge, dim3(1), dim3(PK_NT), 0, st, a, sc, d.table,
              d.n_batches, d.n_kept);
  int64_t fb = d.max_batches < 1024 ? d.max_batches : 1024;
  if (fb < 1) fb = 1;
  LACE_LAUNCH(k_sched_fill, dim3((unsigned)fb), dim3(64), 0, st, a, sc, d.table);
  return hipGetLastError();
}

}  // namespace lace
