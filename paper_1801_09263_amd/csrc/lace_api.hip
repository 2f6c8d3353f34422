// lace_api.hip - host side of the C ABI declared in include/lace.h:
// argument validation, plan tables, workspace layout, the pair schedule,
// and the order of launches for the three operations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "internal.hpp"
#include "lace.h"

using namespace lace;

// First-launch guard of every kernel (internal.hpp): the lookup runs under
// this one mutex, once per kernel and device.
hipError_t lace::resolve_kernel(const void* kernel, std::atomic<uint64_t>& done) {
  int d = 0;
  hipError_t e = hipGetDevice(&d);
  if (e != hipSuccess) return e;
  const uint64_t bit = d < 64 ? (1ull << d) : 0ull;
  if (bit && (done.load(std::memory_order_acquire) & bit)) return hipSuccess;
  static std::mutex m;
  std::lock_guard<std::mutex> lock(m);
  if (bit && (done.load(std::memory_order_acquire) & bit)) return hipSuccess;
  hipFuncAttributes attr;
  e = hipFuncGetAttributes(&attr, kernel);
  if (e == hipSuccess && bit) done.fetch_or(bit, std::memory_order_release);
  return e;
}

namespace {

struct CellPlan {
  CellDev dev;
  int32_t* d_gidx = nullptr;
  int32_t* d_negidx = nullptr;
  void* d_vtab = nullptr;
  void* d_tw = nullptr;
};

int default_pairs_per_batch(int n) {
  const char* e = std::getenv("LACE_PAIRS_PER_BATCH");
  if (e) {
    int v = std::atoi(e);
    if (v >= 1 && v <= PMAX) return v;
  }
  // enough xy planes in flight to cover the chip several times
  int p = (4096 + n - 1) / n;
  if (p > 32) p = 32;
  if (p < 8) p = 8;
  return p;
}

}  // namespace

struct Profile {
  bool on = false;
  std::vector<hipEvent_t> pool;     // created events, reused across calls
  size_t used = 0;                  // events handed out since the last read
  struct Rec {
    size_t ev;                      // index of the first of 4 events
    int64_t pairs;
    double bytes[3];                // algorithmic bytes per pass
  };
  std::vector<Rec> recs;
  double ms[3] = {0, 0, 0};
  int64_t launches[3] = {0, 0, 0};
  int64_t pairs[3] = {0, 0, 0};
  double bytes[3] = {0, 0, 0};
};

// Cached HIP graph of the device work of one batched call.
struct GraphCache {
  std::vector<uint64_t> key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct lace_plan {
  lace_precision prec;
  bool fp64 = false;   // grid precision
  bool gamma = false;  // real orbitals, packed transforms
  int device = 0;
  std::vector<CellPlan> cells;
  Profile prof;
  // internal streams (default priority) for concurrent jobs, created lazily
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;   // fork/join events, no timing
  hipStream_t origin = nullptr;     // capture stream of the batched call
  hipEvent_t s_ready = nullptr;     // screened exchange: S copied to the host
  GraphCache graph;
};

// ---------------------------------------------------------------- helpers
static int hip_status(hipError_t e) { return e == hipSuccess ? LACE_OK : LACE_EHIP; }

static size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  size_t info, psi, w, tmp, epart, s, part, mw, a, z, t, u, dens, scdm, pts,
      total;
  int pairs_per_batch;
};

// bytes of one complex grid point in the plan precision
static size_t grid_bytes(const lace_plan* p) { return p->fp64 ? 16 : 8; }
// bytes of one orbital grid point (real for Gamma plans)
static size_t orb_bytes(const lace_plan* p) {
  return p->gamma ? grid_bytes(p) / 2 : grid_bytes(p);
}

static Layout layout_for(const lace_plan* p, int cell, int n_orb, int n_vec) {
  const CellDev& c = p->cells[cell].dev;
  const bool fp64 = p->fp64;
  Layout L{};
  L.pairs_per_batch = c.ppb;
  const size_t gb = (size_t)c.ng * grid_bytes(p);
  size_t off = 0;
  // the Cholesky info word of builds that pass no info pointer: first, so
  // that lace_get_info finds it without the layout
  L.info = off; off += 256;
  // pair buffer and energy partials sized for the largest batch, so that
  // one workspace serves every tuning of the cell
  // orbital and W grids; for real orbitals these hold n_orb real grids and
  // double as the scratch of ceil(n_orb / 2) packed complex transforms
  const size_t ob = p->gamma ? gb * ((n_orb + 1) / 2) : gb * n_orb;
  L.psi = off; off += align_up(ob);
  L.w = off; off += align_up(ob);
  // two pair buffers and two sets of energy partials: consecutive batches
  // alternate between them, so that one batch's passes A and B can run
  // while the previous batch's pass C still reads its buffer
  L.tmp = off; off += align_up(gb * PMAX * 2);
  L.epart = off;
  off += align_up(sizeof(double) * PMAX * 2 * energy_tiles(c.n, fp64));
  L.s = off; off += align_up(sizeof(double) * n_orb * n_orb);
  int64_t part = gemm_ip_part_bytes(n_orb, n_orb, c.n_pw, true);
  part = std::max(part, gemm_ip_part_bytes(n_orb, n_orb, c.ng, false));
  part = std::max(part, gemm_ip_part_bytes(n_orb, std::max(n_vec, 1), c.n_pw, true));
  L.part = off; off += align_up((size_t)part);
  L.mw = off; off += align_up(16 * (size_t)n_orb * n_orb);
  L.a = off; off += align_up(16 * (size_t)n_orb * n_orb);
  L.z = off; off += align_up(16 * (size_t)n_orb * std::max(n_orb, n_vec));
  L.t = off; off += align_up(16 * (size_t)n_orb * std::max(n_vec, 1));
  L.u = off; off += align_up(16 * (size_t)n_orb * n_orb);
  L.dens = off; off += align_up(sizeof(double) * (size_t)c.ng);
  L.scdm = off; off += align_up((size_t)scdm_scratch_bytes(n_orb));
  L.pts = off; off += align_up(sizeof(int32_t) * (size_t)n_orb);
  L.total = off;
  return L;
}

static char* at(void* ws, size_t off) { return static_cast<char*>(ws) + off; }

static hipError_t enqueue_orbitals(const lace_plan* p, const CellDev& c,
                                   const void* psi_g, int n_orb,
                                   const Layout& L, void* ws, hipStream_t st);
static hipError_t enqueue_screen(const lace_plan* p, const CellDev& c, int n_orb,
                                 const Layout& L, void* ws, double* s_out,
                                 hipStream_t st);

static bool device_ok(const lace_plan* p) {
  int d = -1;
  if (hipGetDevice(&d) != hipSuccess) return false;
  return d == p->device;
}

static void free_cell(CellPlan& c) {
  if (c.d_gidx) (void)hipFree(c.d_gidx);
  if (c.d_negidx) (void)hipFree(c.d_negidx);
  c.d_negidx = nullptr;
  if (c.d_vtab) (void)hipFree(c.d_vtab);
  if (c.d_tw) (void)hipFree(c.d_tw);
  c.d_gidx = nullptr; c.d_vtab = nullptr; c.d_tw = nullptr;
}

// Next free profiling event (created on first use).
static hipEvent_t prof_event(Profile& pr) {
  if (pr.used == pr.pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    pr.pool.push_back(e);
  }
  return pr.pool[pr.used++];
}

// Fold the recorded intervals into the totals (events must be complete).
static hipError_t prof_collect(Profile& pr) {
  for (const auto& r : pr.recs) {
    for (int k = 0; k < 3; ++k) {
      float t = 0.f;
      hipError_t e = hipEventElapsedTime(&t, pr.pool[r.ev + k], pr.pool[r.ev + k + 1]);
      if (e != hipSuccess) return e;
      pr.ms[k] += t;
      pr.launches[k] += 1;
      pr.pairs[k] += r.pairs;
      pr.bytes[k] += r.bytes[k];
    }
  }
  pr.recs.clear();
  pr.used = 0;
  return hipSuccess;
}

// Signed frequency of FFT index k on an n-point axis.
static int signed_freq(int k, int n) { return k < (n + 1) / 2 ? k : k - n; }

// Round of an unordered pair in the circle-method round robin over n'
// vertices (n' = n_orb rounded up to even): vertex n'-1 stays fixed and
// round r pairs it with r and pairs (r + k, r - k) mod (n'-1); so pair
// (i, j) with i < j < n'-1 sits in round (i + j) / 2 mod (n'-1), and every
// round is a set of disjoint pairs.  Diagonal pairs form one extra round.
static int pair_round(int i, int j, int nv) {
  if (i == j) return nv - 1;
  if (j == nv - 1) return i;
  const int64_t m = nv - 1;                  // odd
  return (int)(((int64_t)(i + j) * (nv / 2)) % m);  // (nv/2) = 1/2 mod m
}

// One batch of the pair pipeline: its pairs and, for plans of real
// orbitals, the packed slots (the pairs then listed slot by slot).
struct Batch {
  PairArgs p;
  QuadArgs q;
};

// Group pairs into batches of at most per_batch pairs in which no orbital
// appears twice, so the accumulation into W has no write conflicts.  Pairs
// are taken round by round (stable within a round) and placed first-fit
// into a small window of open batches; a round is itself conflict-free, so
// batches fill to per_batch except at round boundaries.
static void build_schedule(const std::vector<std::pair<int, int>>& pairs,
                           int n_orb, int per_batch,
                           std::vector<Batch>& outb,
                           std::vector<int32_t>* batch_of = nullptr,
                           const std::vector<char>* one_sided = nullptr) {
  std::vector<PairArgs> out;
  const int nv = n_orb + (n_orb & 1);
  std::vector<int> order(pairs.size());
  std::vector<int> round(pairs.size());
  for (size_t k = 0; k < pairs.size(); ++k) {
    order[k] = (int)k;
    round[k] = pair_round(pairs[k].first, pairs[k].second, nv);
  }
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return round[a] < round[b]; });
  if (batch_of) batch_of->assign(pairs.size(), -1);
  const int words = (n_orb + 63) / 64;
  struct Open {
    size_t idx;
    std::vector<uint64_t> used;
  };
  std::vector<Open> open;
  const size_t window = 8;
  for (int k : order) {
    const int i = pairs[k].first, j = pairs[k].second;
    bool placed = false;
    for (size_t o = 0; o < open.size(); ++o) {
      Open& ob = open[o];
      const bool ui = (ob.used[i / 64] >> (i % 64)) & 1ull;
      const bool uj = (ob.used[j / 64] >> (j % 64)) & 1ull;
      if (ui || uj) continue;
      PairArgs& b = out[ob.idx];
      if (one_sided && (*one_sided)[k]) b.one_sided |= 1ull << b.n;
      b.i[b.n] = i; b.j[b.n] = j; ++b.n;
      if (batch_of) (*batch_of)[k] = (int32_t)ob.idx;
      ob.used[i / 64] |= 1ull << (i % 64);
      ob.used[j / 64] |= 1ull << (j % 64);
      if (b.n == per_batch) open.erase(open.begin() + o);
      placed = true;
      break;
    }
    if (placed) continue;
    PairArgs b;
    std::memset(&b, 0, sizeof(b));
    b.n = 1; b.i[0] = i; b.j[0] = j;
    if (one_sided && (*one_sided)[k]) b.one_sided = 1ull;
    out.push_back(b);
    if (batch_of) (*batch_of)[k] = (int32_t)(out.size() - 1);
    if (per_batch > 1) {
      Open ob;
      ob.idx = out.size() - 1;
      ob.used.assign(words, 0ull);
      ob.used[i / 64] |= 1ull << (i % 64);
      ob.used[j / 64] |= 1ull << (j % 64);
      open.push_back(ob);
      if (open.size() > window) open.erase(open.begin());
    }
  }
  outb.resize(out.size());
  for (size_t b = 0; b < out.size(); ++b) {
    outb[b].p = out[b];
    outb[b].q.n = 0;
  }
}

// Plans of real orbitals pack two pair densities into one complex
// transform (a slot); slots of one batch use disjoint orbitals.  A slot
// whose two pairs share an orbital (a star slot) reads and updates three
// orbital grids instead of four.  Stars come from trails: a walk along
// pairs not yet used, cut into runs of two consecutive pairs, which share
// the orbital between them.  Off-diagonal pairs are first walked two
// round-robin rounds at a time (each round a set of disjoint pairs, so the
// stars of one group overlap little and pack densely into batches); what
// is left (one pair per trail of odd length) is walked once more as a
// whole, and the rest is packed two by two, then the diagonal pairs; a
// last odd pair of either kind gets a slot of its own.
struct Slot {
  int i, j, k, l;   // k = l = -1: a single pair; k = i: a star slot
  int pk[2];        // the slot's pairs (indices into the pair list, or -1)
  bool os;          // one-sided pairs (occupied x virtual)
};

static int slot_orbitals(const Slot& s, int o[4]) {
  int n = 0;
  for (int v : {s.i, s.j, s.k, s.l}) {
    if (v < 0) continue;
    bool seen = false;
    for (int t = 0; t < n; ++t) seen = seen || o[t] == v;
    if (!seen) o[n++] = v;
  }
  return n;
}

static Slot make_slot(const std::vector<std::pair<int, int>>& pairs, int a,
                      int b) {
  Slot s;
  s.pk[0] = a;
  s.pk[1] = b;
  s.os = false;
  int i = pairs[a].first, j = pairs[a].second;
  if (b < 0) {
    s.i = i; s.j = j; s.k = s.l = -1;
    return s;
  }
  int k = pairs[b].first, l = pairs[b].second;
  if (i != j) {   // a shared orbital goes first in both pairs
    if (j == k || j == l) std::swap(i, j);
    if (k != i && l == i) std::swap(k, l);
  }
  s.i = i; s.j = j; s.k = k; s.l = l;
  return s;
}

// Trail decomposition of the off-diagonal pairs `edges`: consecutive pairs
// of each walk become star slots, the last pair of an odd walk goes to
// `left`.  Walks start at orbitals with an odd number of unused pairs.
// Adjacency buffers of trail_slots, reused across its calls.
struct TrailWork {
  std::vector<int> off, rem, cur, adj;
};

static void trail_slots(const std::vector<std::pair<int, int>>& pairs,
                        const std::vector<int>& edges, int n_orb,
                        std::vector<char>& done, std::vector<Slot>& slots,
                        std::vector<int>& left, TrailWork& tw) {
  std::vector<int>& off = tw.off;
  std::vector<int>& rem = tw.rem;
  std::vector<int>& cur = tw.cur;
  std::vector<int>& adj = tw.adj;
  off.assign(n_orb + 1, 0);
  rem.resize(n_orb);
  for (int e : edges) {
    ++off[pairs[e].first + 1];
    ++off[pairs[e].second + 1];
  }
  for (int v = 0; v < n_orb; ++v) off[v + 1] += off[v];
  adj.resize(off[n_orb]);
  cur.assign(off.begin(), off.end() - 1);
  for (int e : edges)
    for (int v : {pairs[e].first, pairs[e].second}) adj[cur[v]++] = e;
  for (int v = 0; v < n_orb; ++v) {
    cur[v] = off[v];
    rem[v] = off[v + 1] - off[v];
  }
  auto walk = [&](int v) {
    int pend = -1;
    for (;;) {
      while (cur[v] < off[v + 1] && done[adj[cur[v]]]) ++cur[v];
      if (cur[v] == off[v + 1]) break;
      const int e = adj[cur[v]++];
      done[e] = 1;
      --rem[pairs[e].first];
      --rem[pairs[e].second];
      if (pend < 0) {
        pend = e;
      } else {
        slots.push_back(make_slot(pairs, pend, e));
        pend = -1;
      }
      v = pairs[e].first == v ? pairs[e].second : pairs[e].first;
    }
    if (pend >= 0) left.push_back(pend);
  };
  for (int e : edges)
    for (int v : {pairs[e].first, pairs[e].second})
      if (rem[v] & 1) walk(v);
  for (int e : edges)
    if (!done[e]) walk(pairs[e].first);
}

// Off-diagonal pairs of one kind (two-sided, or one-sided) into slots.
static void star_slots(const std::vector<std::pair<int, int>>& pairs,
                       std::vector<int> off, int n_orb, std::vector<char>& done,
                       std::vector<Slot>& slots) {
  const int nv = n_orb + (n_orb & 1);
  std::vector<int> round(pairs.size(), 0), left, rest, group;
  // stable counting sort of the pairs by round (rounds are < nv)
  std::vector<int> start(nv + 1, 0), sorted(off.size());
  for (int k : off) {
    round[k] = pair_round(pairs[k].first, pairs[k].second, nv);
    ++start[round[k] + 1];
  }
  for (int r = 0; r < nv; ++r) start[r + 1] += start[r];
  for (int k : off) sorted[start[round[k]]++] = k;
  off.swap(sorted);
  TrailWork tw;
  for (size_t a = 0; a < off.size();) {
    const int g = round[off[a]] / 2;
    group.clear();
    while (a < off.size() && round[off[a]] / 2 == g) group.push_back(off[a++]);
    trail_slots(pairs, group, n_orb, done, slots, left, tw);
  }
  for (int e : left) done[e] = 0;
  trail_slots(pairs, left, n_orb, done, slots, rest, tw);
  for (size_t t = 0; t < rest.size(); t += 2)
    slots.push_back(make_slot(pairs, rest[t],
                              t + 1 < rest.size() ? rest[t + 1] : -1));
}

static void make_slots(const std::vector<std::pair<int, int>>& pairs,
                       int n_orb, bool pack, std::vector<Slot>& slots,
                       const std::vector<char>* one_sided) {
  slots.clear();
  auto is_os = [&](int k) { return one_sided && (*one_sided)[k]; };
  if (!pack) {
    for (size_t k = 0; k < pairs.size(); ++k) {
      slots.push_back(make_slot(pairs, (int)k, -1));
      slots.back().os = is_os((int)k);
    }
    return;
  }
  std::vector<int> off, offo, diag;
  for (size_t k = 0; k < pairs.size(); ++k) {
    if (is_os((int)k)) offo.push_back((int)k);
    else if (pairs[k].first == pairs[k].second) diag.push_back((int)k);
    else off.push_back((int)k);
  }
  std::vector<char> done(pairs.size(), 0);
  star_slots(pairs, off, n_orb, done, slots);
  const size_t first_os = slots.size();
  star_slots(pairs, offo, n_orb, done, slots);
  for (size_t t = first_os; t < slots.size(); ++t) slots[t].os = true;
  for (size_t t = 0; t < diag.size(); t += 2)
    slots.push_back(make_slot(pairs, diag[t],
                              t + 1 < diag.size() ? diag[t + 1] : -1));
}

// Slots into batches of at most per_batch pairs and (per_batch + 1) / 2
// slots, first-fit over a window of open batches, no orbital twice in a
// batch.
static void build_slot_schedule(const std::vector<std::pair<int, int>>& pairs,
                                int n_orb, int per_batch,
                                std::vector<Batch>& out,
                                std::vector<int32_t>* batch_of = nullptr,
                                std::vector<int32_t>* slot_of = nullptr,
                                const std::vector<char>* one_sided = nullptr,
                                int n_occ = -1) {
  out.clear();
  std::vector<Slot> slots;
  make_slots(pairs, n_orb, per_batch >= 2, slots, one_sided);
  if (batch_of) batch_of->assign(pairs.size(), -1);
  if (slot_of) slot_of->assign(pairs.size(), -1);
  const int cap_slots = (per_batch + 1) / 2;
  const int words = (n_orb + 63) / 64;
  struct Open {
    size_t idx;
    std::vector<uint64_t> used;
  };
  std::vector<Open> open;
  const size_t window = 8;
  auto put = [&](size_t idx, const Slot& sl) {
    Batch& b = out[idx];
    const int q = b.q.n++;
    b.q.i[q] = sl.i; b.q.j[q] = sl.j; b.q.k[q] = sl.k; b.q.l[q] = sl.l;
    if (sl.os) {   // the occupied orbital of a one-sided pair keeps its W
      b.q.one_sided |= 1ull << q;
      const int pos[4] = {sl.i, sl.j, sl.k, sl.l};
      for (int t = 0; t < 4; ++t)
        if (pos[t] >= 0 && pos[t] < n_occ) b.q.skip[t] |= 1ull << q;
    }
    for (int t = 0; t < 2; ++t) {
      const int k = sl.pk[t];
      if (k < 0) continue;
      b.p.i[b.p.n] = pairs[k].first;
      b.p.j[b.p.n] = pairs[k].second;
      if (sl.os) b.p.one_sided |= 1ull << b.p.n;
      ++b.p.n;
      if (batch_of) (*batch_of)[k] = (int32_t)idx;
      if (slot_of) (*slot_of)[k] = q;
    }
  };
  for (const Slot& sl : slots) {
    int o[4];
    const int no = slot_orbitals(sl, o);
    const int np = sl.pk[1] >= 0 ? 2 : 1;
    bool placed = false;
    for (size_t w = 0; w < open.size() && !placed; ++w) {
      Open& ob = open[w];
      const Batch& b = out[ob.idx];
      if (b.p.n + np > per_batch) continue;
      bool clash = false;
      for (int t = 0; t < no; ++t)
        clash = clash || ((ob.used[o[t] / 64] >> (o[t] % 64)) & 1ull);
      if (clash) continue;
      put(ob.idx, sl);
      for (int t = 0; t < no; ++t) ob.used[o[t] / 64] |= 1ull << (o[t] % 64);
      if (out[ob.idx].p.n == per_batch || out[ob.idx].q.n == cap_slots)
        open.erase(open.begin() + w);
      placed = true;
    }
    if (placed) continue;
    Batch nb;
    std::memset(&nb, 0, sizeof(nb));
    out.push_back(nb);
    put(out.size() - 1, sl);
    if (out.back().p.n < per_batch && out.back().q.n < cap_slots) {
      Open ob;
      ob.idx = out.size() - 1;
      ob.used.assign(words, 0ull);
      for (int t = 0; t < no; ++t) ob.used[o[t] / 64] |= 1ull << (o[t] % 64);
      open.push_back(ob);
      if (open.size() > window) open.erase(open.begin());
    }
  }
}

// one_sided (optional): per pair, occupied x virtual; n_occ: orbitals
// below it are occupied.
static void schedule_for(const lace_plan* p,
                         const std::vector<std::pair<int, int>>& pairs,
                         int n_orb, int per_batch, std::vector<Batch>& out,
                         const std::vector<char>* one_sided = nullptr,
                         int n_occ = -1) {
  if (p->gamma)
    build_slot_schedule(pairs, n_orb, per_batch, out, nullptr, nullptr,
                        one_sided, n_occ);
  else
    build_schedule(pairs, n_orb, per_batch, out, nullptr, one_sided);
}

// ------------------------------------------------------------------ API
// The entry points keep the C linkage of their declarations in lace.h.

const char* lace_status_string(int s) {
  switch (s) {
    case LACE_OK: return "ok";
    case LACE_EINVAL: return "invalid argument";
    case LACE_ENOMEM: return "workspace too small or allocation failed";
    case LACE_ENOTPD: return "-M_s is not positive definite";
    case LACE_EUNSUPPORTED: return "unsupported grid size or sphere outside the grid";
    case LACE_EHIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

int lace_plan_create(const lace_cell_desc* cells, int n_cells,
                     lace_precision prec, lace_plan** out) {
  if (!cells || !out || n_cells < 1) return LACE_EINVAL;
  if (prec != LACE_FP64 && prec != LACE_FP32 && prec != LACE_FP64_GAMMA &&
      prec != LACE_FP32_GAMMA)
    return LACE_EINVAL;
  const bool gamma = prec == LACE_FP64_GAMMA || prec == LACE_FP32_GAMMA;
  // validate everything before touching the device
  for (int ci = 0; ci < n_cells; ++ci) {
    const lace_cell_desc& d = cells[ci];
    if (!(d.L > 0.0) || d.n_pw < 1 || !d.miller || !std::isfinite(d.L) ||
        !(d.omega >= 0.0) || !std::isfinite(d.omega))
      return LACE_EINVAL;
    if (!grid_supported(d.n)) return LACE_EUNSUPPORTED;
    const int n = d.n;
    std::vector<uint8_t> seen((size_t)n * n * n, 0);
    for (int64_t m = 0; m < d.n_pw; ++m) {
      for (int a = 0; a < 3; ++a) {
        const int v = d.miller[3 * m + a];
        if (2 * std::abs(v) >= n) return LACE_EUNSUPPORTED;
      }
      const int x = (d.miller[3 * m] % n + n) % n;
      const int y = (d.miller[3 * m + 1] % n + n) % n;
      const int z = (d.miller[3 * m + 2] % n + n) % n;
      const size_t g = (size_t)x + (size_t)n * (y + (size_t)n * z);
      if (seen[g]) return LACE_EINVAL;
      seen[g] = 1;
    }
    if (gamma) {
      for (int64_t m = 0; m < d.n_pw; ++m) {
        const int x = ((-d.miller[3 * m]) % n + n) % n;
        const int y = ((-d.miller[3 * m + 1]) % n + n) % n;
        const int z = ((-d.miller[3 * m + 2]) % n + n) % n;
        if (!seen[(size_t)x + (size_t)n * (y + (size_t)n * z)]) return LACE_EINVAL;
      }
    }
  }
  lace_plan* p = new (std::nothrow) lace_plan;
  if (!p) return LACE_ENOMEM;
  p->prec = prec;
  p->fp64 = prec == LACE_FP64 || prec == LACE_FP64_GAMMA;
  p->gamma = gamma;
  if (hipGetDevice(&p->device) != hipSuccess) { delete p; return LACE_EHIP; }
  p->cells.resize(n_cells);
  const bool fp64 = p->fp64;
  for (int ci = 0; ci < n_cells; ++ci) {
    const lace_cell_desc& d = cells[ci];
    CellPlan& cp = p->cells[ci];
    const int n = d.n;
    const int64_t ng = (int64_t)n * n * n;
    const double rc = d.rc > 0.0 ? d.rc : 0.5 * d.L;
    cp.dev.n = n; cp.dev.ng = ng; cp.dev.n_pw = d.n_pw;
    cp.dev.L = d.L; cp.dev.rc = rc; cp.dev.omega = d.L * d.L * d.L;
    cp.dev.ppb = default_pairs_per_batch(n);
    cp.dev.use_plane = plane_fits(n, fp64) ? 1 : 2;
    // sphere -> grid map
    std::vector<int32_t> gidx(d.n_pw);
    for (int64_t m = 0; m < d.n_pw; ++m) {
      const int x = (d.miller[3 * m] % n + n) % n;
      const int y = (d.miller[3 * m + 1] % n + n) % n;
      const int z = (d.miller[3 * m + 2] % n + n) % n;
      gidx[m] = x + n * (y + n * z);
    }
    std::vector<int32_t> negidx;
    if (gamma) {
      std::vector<int32_t> at_grid((size_t)ng, -1);
      for (int64_t m = 0; m < d.n_pw; ++m) at_grid[gidx[m]] = (int32_t)m;
      negidx.resize(d.n_pw);
      for (int64_t m = 0; m < d.n_pw; ++m) {
        const int x = ((-d.miller[3 * m]) % n + n) % n;
        const int y = ((-d.miller[3 * m + 1]) % n + n) % n;
        const int z = ((-d.miller[3 * m + 2]) % n + n) % n;
        negidx[m] = at_grid[x + (int64_t)n * (y + (int64_t)n * z)];
      }
    }
    // kernel table v(G)/N_g: truncated Coulomb 8 pi sin^2(|G| rc / 2) / |G|^2,
    // v(0) = 2 pi rc^2; or, for omega > 0, the short-range erfc(omega r) / r:
    // -4 pi expm1(-|G|^2 / (4 omega^2)) / |G|^2, v(0) = pi / omega^2
    const double om = d.omega;
    std::vector<double> v(ng);
    const double g1 = 2.0 * M_PI / d.L;
    for (int z = 0; z < n; ++z)
      for (int y = 0; y < n; ++y)
        for (int x = 0; x < n; ++x) {
          const double gx = g1 * signed_freq(x, n), gy = g1 * signed_freq(y, n),
                       gz = g1 * signed_freq(z, n);
          const double gg2 = gx * gx + gy * gy + gz * gz;
          double val;
          if (om > 0.0) {
            val = gg2 == 0.0 ? M_PI / (om * om)
                             : -4.0 * M_PI * std::expm1(-gg2 / (4.0 * om * om)) / gg2;
          } else if (gg2 == 0.0) {
            val = 2.0 * M_PI * rc * rc;
          } else {
            const double s = std::sin(0.5 * std::sqrt(gg2) * rc);
            val = 8.0 * M_PI * s * s / gg2;
          }
          v[x + (int64_t)n * (y + (int64_t)n * z)] = val / double(ng);
        }
    // twiddles exp(-2 pi i m / n)
    std::vector<double> tw(2 * n);
    for (int m = 0; m < n; ++m) {
      const double ang = 2.0 * M_PI * double(m) / double(n);
      tw[2 * m] = std::cos(ang);
      tw[2 * m + 1] = -std::sin(ang);
    }
    hipError_t e = hipSuccess;
    e = hipMalloc(&cp.d_gidx, sizeof(int32_t) * d.n_pw);
    // the device keeps one octant of the table (0 <= kx, ky, kz <= n/2):
    // v depends on the squares of the signed frequencies only, so the
    // entry at k and at n - k is the same value
    const int vh = n / 2 + 1;
    const int64_t nv = (int64_t)vh * vh * vh;
    std::vector<double> voct((size_t)nv);
    for (int z = 0; z < vh; ++z)
      for (int y = 0; y < vh; ++y)
        for (int x = 0; x < vh; ++x)
          voct[(size_t)((z * vh + y) * vh + x)] = v[x + (int64_t)n * (y + (int64_t)n * z)];
    if (e == hipSuccess) e = hipMalloc(&cp.d_vtab, (fp64 ? 8 : 4) * (size_t)nv);
    if (e == hipSuccess) e = hipMalloc(&cp.d_tw, (fp64 ? 16 : 8) * (size_t)n);
    if (e == hipSuccess && gamma) {
      e = hipMalloc(&cp.d_negidx, sizeof(int32_t) * d.n_pw);
      if (e == hipSuccess)
        e = hipMemcpy(cp.d_negidx, negidx.data(), sizeof(int32_t) * d.n_pw,
                      hipMemcpyHostToDevice);
    }
    if (e == hipSuccess)
      e = hipMemcpy(cp.d_gidx, gidx.data(), sizeof(int32_t) * d.n_pw,
                    hipMemcpyHostToDevice);
    if (e == hipSuccess) {
      if (fp64) {
        e = hipMemcpy(cp.d_vtab, voct.data(), 8 * (size_t)nv, hipMemcpyHostToDevice);
        if (e == hipSuccess)
          e = hipMemcpy(cp.d_tw, tw.data(), 16 * (size_t)n, hipMemcpyHostToDevice);
      } else {
        std::vector<float> vf((size_t)nv), twf(2 * n);
        for (int64_t k = 0; k < nv; ++k) vf[k] = static_cast<float>(voct[k]);
        for (int k = 0; k < 2 * n; ++k) twf[k] = static_cast<float>(tw[k]);
        e = hipMemcpy(cp.d_vtab, vf.data(), 4 * (size_t)nv, hipMemcpyHostToDevice);
        if (e == hipSuccess)
          e = hipMemcpy(cp.d_tw, twf.data(), 8 * (size_t)n, hipMemcpyHostToDevice);
      }
    }
    if (e != hipSuccess) {
      for (auto& c2 : p->cells) free_cell(c2);
      delete p;
      return e == hipErrorOutOfMemory ? LACE_ENOMEM : LACE_EHIP;
    }
    cp.dev.gidx = cp.d_gidx;
    cp.dev.negidx = cp.d_negidx;
    cp.dev.vtab = cp.d_vtab;
    cp.dev.tw = cp.d_tw;
  }
  *out = p;
  return LACE_OK;
}

int lace_plan_destroy(lace_plan* p) {
  if (!p) return LACE_OK;
  (void)hipDeviceSynchronize();
  for (auto& c : p->cells) free_cell(c);
  for (auto ev : p->prof.pool) (void)hipEventDestroy(ev);
  if (p->graph.exec) (void)hipGraphExecDestroy(p->graph.exec);
  if (p->graph.graph) (void)hipGraphDestroy(p->graph.graph);
  for (auto ev : p->events) (void)hipEventDestroy(ev);
  if (p->s_ready) (void)hipEventDestroy(p->s_ready);
  for (auto st : p->streams) (void)hipStreamDestroy(st);
  if (p->origin) (void)hipStreamDestroy(p->origin);
  delete p;
  return LACE_OK;
}

int lace_workspace_size(const lace_plan* p, int cell, int n_orb, int n_vec,
                        size_t* bytes) {
  if (!p || !bytes || cell < 0 || cell >= (int)p->cells.size() || n_orb < 1 ||
      n_vec < 0)
    return LACE_EINVAL;
  *bytes = layout_for(p, cell, n_orb, n_vec).total;
  return LACE_OK;
}

static int check_common(const lace_plan* p, int cell, int n_orb) {
  if (!p || cell < 0 || cell >= (int)p->cells.size() || n_orb < 1)
    return LACE_EINVAL;
  if (!device_ok(p)) return LACE_EINVAL;
  return LACE_OK;
}

int lace_screen(lace_plan* p, int cell, const void* psi_g, int n_orb,
                double* s_out, void* ws, size_t ws_bytes, lace_stream_t stream) {
  int rc = check_common(p, cell, n_orb);
  if (rc) return rc;
  if (!psi_g || !s_out || !ws) return LACE_EINVAL;
  const Layout L = layout_for(p, cell, n_orb, 0);
  if (ws_bytes < L.total) return LACE_ENOMEM;
  const CellDev& c = p->cells[cell].dev;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = enqueue_orbitals(p, c, psi_g, n_orb, L, ws, st);
  if (e == hipSuccess) e = enqueue_screen(p, c, n_orb, L, ws, s_out, st);
  return hip_status(e);
}

// Host copy of an explicit pair list after validation; false on a bad list.
static bool copy_pairs(const int32_t* pair_i, const int32_t* pair_j,
                       int64_t n_pairs, int n_orb,
                       std::vector<std::pair<int, int>>& pairs) {
  std::vector<uint8_t> seen((size_t)n_orb * n_orb, 0);
  pairs.clear();
  pairs.reserve(n_pairs);
  for (int64_t k = 0; k < n_pairs; ++k) {
    const int i = pair_i[k], j = pair_j[k];
    if (i < 0 || j < 0 || i > j || j >= n_orb) return false;
    if (seen[(size_t)i * n_orb + j]) return false;
    seen[(size_t)i * n_orb + j] = 1;
    pairs.emplace_back(i, j);
  }
  return true;
}

static void all_pairs(int n_orb, std::vector<std::pair<int, int>>& pairs) {
  pairs.clear();
  pairs.reserve((size_t)n_orb * (n_orb + 1) / 2);
  for (int j = 0; j < n_orb; ++j)
    for (int i = 0; i <= j; ++i) pairs.emplace_back(i, j);
}

// Kept pairs from a host copy of S: S_ij >= s_thr (upper triangle, Eq. (6)).
static void kept_from_s(const std::vector<double>& hs, int n_orb, double s_thr,
                        std::vector<std::pair<int, int>>& pairs) {
  pairs.clear();
  for (int j = 0; j < n_orb; ++j)
    for (int i = 0; i <= j; ++i)
      if (hs[(size_t)i * n_orb + j] >= s_thr) pairs.emplace_back(i, j);
}

// Grid orbitals into the workspace (real grids for Gamma plans, packed two
// per complex transform in the W region).
static hipError_t enqueue_orbitals(const lace_plan* p, const CellDev& c,
                                   const void* psi_g, int n_orb,
                                   const Layout& L, void* ws, hipStream_t st) {
  if (p->gamma)
    return launch_orbitals_to_grid_real(c, p->fp64, psi_g, n_orb,
                                        at(ws, L.psi), at(ws, L.w), st);
  return launch_orbitals_to_grid(c, p->fp64, psi_g, n_orb, at(ws, L.psi), st);
}

// S into the workspace from the grid orbitals already in it.
static hipError_t enqueue_screen(const lace_plan* p, const CellDev& c, int n_orb,
                                 const Layout& L, void* ws, double* s_out,
                                 hipStream_t st) {
  const double dv = c.omega / double(c.ng);
  const int64_t pb = (int64_t)(L.mw - L.part);
  if (p->gamma)
    return launch_gemm_ip_abs_real(p->fp64, at(ws, L.psi), c.ng, n_orb, c.ng,
                                   dv, s_out, at(ws, L.part), pb, st);
  return launch_gemm_ip_abs(p->fp64, at(ws, L.psi), c.ng, n_orb, c.ng, dv,
                            s_out, at(ws, L.part), pb, st);
}

// Algorithmic bytes of one batch per pass (see lace_profile_read).
static void batch_bytes(const lace_plan* p, const CellDev& c, const Batch& bt,
                        double out[3]) {
  const double U = double(c.ng) * grid_bytes(p);
  const double G = double(c.ng) * orb_bytes(p);
  // orbs: orbital grids read by pass A; orbs_c: orbital grids read by pass
  // C plus twice the W grids it updates
  double orbs = 0.0, orbs_c = 0.0, slots = 0.0;
  if (p->gamma) {
    for (int q = 0; q < bt.q.n; ++q) {
      const int pos[4] = {bt.q.i[q], bt.q.j[q], bt.q.k[q], bt.q.l[q]};
      const int mate[4] = {1, 0, 3, 2};
      int all[4], upd[4], rd[4], na = 0, nu = 0, nr = 0;
      auto add = [](int* set, int& n, int v) {
        for (int t = 0; t < n; ++t) if (set[t] == v) return;
        set[n++] = v;
      };
      for (int t = 0; t < 4; ++t) {
        if (pos[t] < 0) continue;
        add(all, na, pos[t]);
        if (!((bt.q.skip[t] >> q) & 1ull)) {
          add(upd, nu, pos[t]);
          add(rd, nr, pos[mate[t]]);
        }
      }
      orbs += na;
      orbs_c += nr + 2 * nu;
    }
    slots = bt.q.n;
  } else {
    for (int k = 0; k < bt.p.n; ++k) {
      const bool diag = bt.p.i[k] == bt.p.j[k];
      const bool os = (bt.p.one_sided >> k) & 1ull;
      orbs += diag ? 1.0 : 2.0;
      orbs_c += (diag || os) ? 3.0 : 6.0;
    }
    slots = bt.p.n;
  }
  out[0] = orbs * G + slots * U;
  out[1] = 2.0 * slots * U;
  out[2] = slots * U + orbs_c * G;
}

// One batch of the pair pipeline (pairs, or packed slots for Gamma plans).
// `lane` picks the pair buffer and the energy partials (0 or 1).
static hipError_t enqueue_batch(const lace_plan* p, const CellDev& c,
                                const Batch& bt, const Layout& L, void* ws,
                                int lane, hipStream_t st, hipEvent_t* ev,
                                const BatchSync* sy = nullptr) {
  void* tmp = at(ws, L.tmp + (size_t)lane * PMAX * c.ng * grid_bytes(p));
  double* epart = reinterpret_cast<double*>(at(ws, L.epart)) +
                  (size_t)lane * PMAX * energy_tiles(c.n, p->fp64);
  if (p->gamma)
    return launch_quad_batch(c, p->fp64, bt.q, at(ws, L.psi), at(ws, L.w),
                             tmp, epart, st, ev, sy);
  const PairArgs& b = bt.p;
  if (ev)
    return launch_pair_batch_timed(c, p->fp64, b, at(ws, L.psi), at(ws, L.w),
                                   tmp, epart, st, ev);
  return launch_pair_batch(c, p->fp64, b, at(ws, L.psi), at(ws, L.w), tmp,
                           epart, st, sy);
}

static hipError_t ensure_streams(lace_plan* p, int k);
static hipError_t link(lace_plan* p, hipStream_t from, hipStream_t to, int k);

// Pair pipeline over a schedule, energy reduction, W back to plane waves.
// Requires the grid orbitals in the workspace.
// overlap: run consecutive batches on two internal streams (batch b on
// lane b % 2): a batch's passes A and B overlap the previous batch's passes,
// and its pass C waits for the previous pass C (they may share W grids), so
// W is summed in batch order either way.  Profiled calls run on one stream.
// W and the energy partials start at zero.
static hipError_t enqueue_exchange_zero(const lace_plan* p, const CellDev& c,
                                        int n_orb, const Layout& L, void* ws,
                                        hipStream_t st) {
  const int64_t ntiles = energy_tiles(c.n, p->fp64);
  hipError_t e = launch_zero(at(ws, L.w), (int64_t)c.ng * n_orb * orb_bytes(p), st);
  if (e == hipSuccess)
    e = launch_zero(at(ws, L.epart), (int64_t)sizeof(double) * PMAX * 2 * ntiles, st);
  return e;
}

// zeroed: the caller has already enqueued enqueue_exchange_zero on st.
static hipError_t enqueue_exchange(lace_plan* p, const CellDev& c, int n_orb,
                                   const std::vector<Batch>& sched,
                                   const Layout& L, void* ws, void* w_g,
                                   double* e_x, hipStream_t st, bool profile,
                                   bool overlap = false, bool zeroed = false) {
  const bool fp64 = p->fp64;
  void* w = at(ws, L.w);
  const int64_t ntiles = energy_tiles(c.n, fp64);
  double* epart = reinterpret_cast<double*>(at(ws, L.epart));
  hipError_t e = zeroed ? hipSuccess : enqueue_exchange_zero(p, c, n_orb, L, ws, st);
  Profile& pr = p->prof;
  const bool timed = profile && pr.on;
  const bool two = overlap && !timed && sched.size() > 1;
  hipStream_t lane[2] = {st, st};
  hipEvent_t cdone[2] = {nullptr, nullptr};
  if (e == hipSuccess && two) {
    e = ensure_streams(p, 2);
    if (e == hipSuccess) {
      lane[0] = p->streams[0];
      lane[1] = p->streams[1];
      cdone[0] = p->events[2];
      cdone[1] = p->events[3];
      e = link(p, st, lane[0], 0);
      if (e == hipSuccess) e = link(p, st, lane[1], 1);
    }
  }
  if (e == hipSuccess && timed && pr.used + 4 * sched.size() > 65536) {
    // bound the number of outstanding events: fold what is recorded
    e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = prof_collect(pr);
  }
  for (size_t b = 0; e == hipSuccess && b < sched.size(); ++b) {
    if (timed) {
      const size_t first = pr.used;
      hipEvent_t ev[4];
      for (int k = 0; k < 4; ++k) ev[k] = prof_event(pr);
      if (!ev[0] || !ev[1] || !ev[2] || !ev[3]) return hipErrorOutOfMemory;
      Profile::Rec r;
      r.ev = first;
      r.pairs = sched[b].p.n;
      batch_bytes(p, c, sched[b], r.bytes);
      pr.recs.push_back(r);
      e = enqueue_batch(p, c, sched[b], L, ws, (int)(b % 2), st, ev);
    } else if (two) {
      BatchSync sy{b > 0 ? cdone[(b - 1) % 2] : nullptr, cdone[b % 2]};
      e = enqueue_batch(p, c, sched[b], L, ws, (int)(b % 2), lane[b % 2],
                        nullptr, &sy);
    } else {
      e = enqueue_batch(p, c, sched[b], L, ws, (int)(b % 2), st, nullptr);
    }
  }
  if (e == hipSuccess && two) {
    e = link(p, lane[0], st, 0);
    if (e == hipSuccess) e = link(p, lane[1], st, 1);
  }
  if (e == hipSuccess && e_x)
    e = launch_reduce_sum(epart, (int64_t)PMAX * 2 * ntiles,
                          -0.5 * c.omega / double(c.ng), e_x, st);
  if (e == hipSuccess) {
    if (p->gamma)  // the orbital grids are no longer needed: scratch
      e = launch_grid_to_pw_real(c, fp64, w, n_orb, at(ws, L.psi), w_g, st);
    else
      e = launch_grid_to_pw(c, fp64, w, n_orb, w_g, st);
  }
  return e;
}

// M, E_x trace, -M_s, Cholesky, Z = L^{-H}, xi = W Z.
// info: the call's Cholesky info word (device), or NULL for the workspace's.
static hipError_t enqueue_build_ace(const CellPlan& cp, int n_orb, int sym,
                                    const Layout& L, void* ws,
                                    const void* psi_g, const void* w_g,
                                    void* xi_g, void* m_out, double* ex_tr,
                                    int32_t* info, hipStream_t st) {
  const CellDev& c = cp.dev;
  void* m = m_out ? m_out : at(ws, L.mw);
  hipError_t e = launch_gemm_ip_c128(psi_g, c.n_pw, n_orb, w_g, c.n_pw, n_orb,
                                     c.n_pw, 1.0, m, at(ws, L.part),
                                     (int64_t)(L.mw - L.part), st);
  if (e == hipSuccess && ex_tr) e = launch_trace_re(m, n_orb, 0.5, ex_tr, st);
  if (e == hipSuccess) e = launch_neg_sym(m, n_orb, sym, at(ws, L.a), st);
  if (e == hipSuccess)
    e = launch_cholesky(at(ws, L.a), n_orb,
                        info ? info : reinterpret_cast<int32_t*>(at(ws, L.info)),
                        at(ws, L.u),
                        at(ws, L.part), (int64_t)(L.mw - L.part), st);
  if (e == hipSuccess) e = launch_trinv_adj(at(ws, L.a), n_orb, at(ws, L.z), st);
  if (e == hipSuccess)
    e = launch_gemm_tall(w_g, c.n_pw, c.n_pw, n_orb, at(ws, L.z), n_orb, xi_g,
                         c.n_pw, st);
  return e;
}

int lace_apply_exchange(lace_plan* p, int cell, const void* psi_g, int n_orb,
                        double s_thr, const int32_t* pair_i,
                        const int32_t* pair_j, int64_t n_pairs, void* w_g,
                        double* e_x, int64_t* n_kept, void* ws, size_t ws_bytes,
                        lace_stream_t stream) {
  int rc = check_common(p, cell, n_orb);
  if (rc) return rc;
  if (!psi_g || !w_g || !ws) return LACE_EINVAL;
  if (!(s_thr >= 0.0 && s_thr < 1.0)) return LACE_EINVAL;
  if ((pair_i == nullptr) != (pair_j == nullptr)) return LACE_EINVAL;
  if (pair_i && n_pairs < 0) return LACE_EINVAL;
  const Layout L = layout_for(p, cell, n_orb, 0);
  if (ws_bytes < L.total) return LACE_ENOMEM;
  std::vector<std::pair<int, int>> pairs;
  if (pair_i && !copy_pairs(pair_i, pair_j, n_pairs, n_orb, pairs))
    return LACE_EINVAL;
  const CellDev& c = p->cells[cell].dev;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = enqueue_orbitals(p, c, psi_g, n_orb, L, ws, st);
  if (e != hipSuccess) return LACE_EHIP;
  bool zeroed = false;
  if (!pair_i) {
    if (s_thr > 0.0) {
      double* s = reinterpret_cast<double*>(at(ws, L.s));
      e = enqueue_screen(p, c, n_orb, L, ws, s, st);
      if (e != hipSuccess) return LACE_EHIP;
      std::vector<double> hs((size_t)n_orb * n_orb);
      e = hipMemcpyAsync(hs.data(), s, sizeof(double) * hs.size(),
                         hipMemcpyDeviceToHost, st);
      if (e == hipSuccess && !p->s_ready)
        e = hipEventCreateWithFlags(&p->s_ready, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventRecord(p->s_ready, st);
      // the device clears W while the host builds the pair list and the
      // schedule
      if (e == hipSuccess) e = enqueue_exchange_zero(p, c, n_orb, L, ws, st);
      if (e == hipSuccess) e = hipEventSynchronize(p->s_ready);
      if (e != hipSuccess) return LACE_EHIP;
      zeroed = true;
      kept_from_s(hs, n_orb, s_thr, pairs);
    } else {
      all_pairs(n_orb, pairs);
    }
  }
  std::vector<Batch> sched;
  schedule_for(p, pairs, n_orb, c.ppb, sched);
  e = enqueue_exchange(p, c, n_orb, sched, L, ws, w_g, e_x, st, true, true,
                       zeroed);
  if (e != hipSuccess) return LACE_EHIP;
  if (n_kept) *n_kept = (int64_t)pairs.size();
  return LACE_OK;
}

// Newton-Schulz steps of the polar factor; quadratic near convergence and
// growing the smallest singular value by 3/2 per step before that, so 30
// steps resolve singular values down to ~1e-4 of the largest.
static constexpr int kAlignSteps = 30;

// Polar factor U of an n x n complex matrix A, given Y_0 = A^T (row-major)
// in the workspace's `a` block: X_0 = A s with s from a Gershgorin bound,
// then X <- X (3 I - X^H X) / 2, kept transposed (Y = X^T).  Leaves U
// (row-major) in the `mw` block; resid (device, may be NULL) gets
// ||U^H U - I||_F / sqrt(n).
static hipError_t enqueue_polar(const Layout& L, void* ws, int n, double* resid,
                                hipStream_t st) {
  void* part = at(ws, L.part);
  const int64_t pb = (int64_t)(L.mw - L.part);
  void* g = at(ws, L.mw);     // C, finally U
  void* y0 = at(ws, L.a);     // Y, ping
  void* y1 = at(ws, L.u);     // pong
  void* b = at(ws, L.z);      // X^H X
  double* sc = reinterpret_cast<double*>(at(ws, L.s));
  hipError_t e = launch_gemm_ip_c128(y0, n, n, y0, n, n, n, 1.0, b, part, pb, st);
  if (e == hipSuccess) e = launch_polar_norm(0, b, n, sc, st);
  if (e == hipSuccess) e = launch_polar_elem(1, y0, n, sc, y1, st);
  void* cur = y1;
  void* nxt = y0;
  for (int it = 0; it < kAlignSteps && e == hipSuccess; ++it) {
    // X <- X C, C = (3 I - X^H X) / 2: Y'[b][a] = sum_k Y[k][a] C[k][b]
    e = launch_gemm_ip_c128(cur, n, n, cur, n, n, n, 1.0, b, part, pb, st);
    if (e == hipSuccess) e = launch_polar_elem(2, b, n, nullptr, g, st);
    if (e == hipSuccess) e = launch_gemm_tall(cur, n, n, n, g, n, nxt, n, st);
    std::swap(cur, nxt);
  }
  if (e == hipSuccess && resid) {
    e = launch_gemm_ip_c128(cur, n, n, cur, n, n, n, 1.0, b, part, pb, st);
    if (e == hipSuccess) e = launch_polar_norm(1, b, n, resid, st);
  }
  if (e == hipSuccess) e = launch_polar_elem(3, cur, n, nullptr, g, st);  // U = Y^T
  return e;
}

int lace_align(lace_plan* p, int cell, const void* psi_new, const void* psi_old,
               int n_orb, void* psi_out, double* resid, void* ws,
               size_t ws_bytes, lace_stream_t stream) {
  int rc = check_common(p, cell, n_orb);
  if (rc) return rc;
  if (!psi_new || !psi_old || !psi_out || !ws) return LACE_EINVAL;
  if (psi_out == psi_new || psi_out == psi_old) return LACE_EINVAL;
  const Layout L = layout_for(p, cell, n_orb, 0);
  if (ws_bytes < L.total) return LACE_ENOMEM;
  const CellDev& c = p->cells[cell].dev;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int n = n_orb;
  // G[x][y] = <psi_old_x | psi_new_y> = conj(A[y][x]), A = psi_new^H psi_old,
  // so Y_0 = A^T = conj(G)
  hipError_t e = launch_gemm_ip_c128(psi_old, c.n_pw, n, psi_new, c.n_pw, n,
                                     c.n_pw, 1.0, at(ws, L.mw), at(ws, L.part),
                                     (int64_t)(L.mw - L.part), st);
  if (e == hipSuccess) e = launch_polar_elem(0, at(ws, L.mw), n, nullptr, at(ws, L.a), st);
  if (e == hipSuccess) e = enqueue_polar(L, ws, n, resid, st);
  // psi_out_b = sum_a psi_new_a U[a][b]
  if (e == hipSuccess)
    e = launch_gemm_tall(psi_new, c.n_pw, c.n_pw, n, at(ws, L.mw), n, psi_out,
                         c.n_pw, st);
  return hip_status(e);
}

int lace_scdm(lace_plan* p, int cell, const void* psi_g, int n_orb,
              void* phi_g, int32_t* points, double* resid, void* ws,
              size_t ws_bytes, lace_stream_t stream) {
  int rc = check_common(p, cell, n_orb);
  if (rc) return rc;
  if (!psi_g || !phi_g || !ws || phi_g == psi_g) return LACE_EINVAL;
  const CellDev& c = p->cells[cell].dev;
  if ((int64_t)n_orb > c.ng || n_orb > 3072) return LACE_EINVAL;
  const Layout L = layout_for(p, cell, n_orb, 0);
  if (ws_bytes < L.total) return LACE_ENOMEM;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int32_t* pts = points ? points : reinterpret_cast<int32_t*>(at(ws, L.pts));
  hipError_t e = enqueue_orbitals(p, c, psi_g, n_orb, L, ws, st);
  if (e == hipSuccess)
    e = launch_scdm(p->fp64, p->gamma, at(ws, L.psi), n_orb, c.ng,
                    reinterpret_cast<double*>(at(ws, L.dens)), at(ws, L.scdm),
                    pts, at(ws, L.a), st);
  if (e == hipSuccess) e = enqueue_polar(L, ws, n_orb, resid, st);
  // phi_k = sum_n psi_n U[n][k]
  if (e == hipSuccess)
    e = launch_gemm_tall(psi_g, c.n_pw, c.n_pw, n_orb, at(ws, L.mw), n_orb,
                         phi_g, c.n_pw, st);
  return hip_status(e);
}

int lace_apply_exchange_virtual(lace_plan* p, int cell, const void* psi_g,
                                int n_occ, int n_virt, double s_thr, void* w_g,
                                double* e_x, int64_t* n_kept, void* ws,
                                size_t ws_bytes, lace_stream_t stream) {
  if (n_occ < 1 || n_virt < 0) return LACE_EINVAL;
  const int n_orb = n_occ + n_virt;
  int rc = check_common(p, cell, n_orb);
  if (rc) return rc;
  if (!psi_g || !w_g || !ws) return LACE_EINVAL;
  if (!(s_thr >= 0.0 && s_thr < 1.0)) return LACE_EINVAL;
  const Layout L = layout_for(p, cell, n_orb, 0);
  if (ws_bytes < L.total) return LACE_ENOMEM;
  const CellDev& c = p->cells[cell].dev;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = enqueue_orbitals(p, c, psi_g, n_orb, L, ws, st);
  if (e != hipSuccess) return LACE_EHIP;
  // occupied pairs, screened among the occupied orbitals
  std::vector<std::pair<int, int>> pairs;
  if (s_thr > 0.0) {
    double* s = reinterpret_cast<double*>(at(ws, L.s));
    e = enqueue_screen(p, c, n_occ, L, ws, s, st);
    if (e != hipSuccess) return LACE_EHIP;
    std::vector<double> hs((size_t)n_occ * n_occ);
    e = hipMemcpyAsync(hs.data(), s, sizeof(double) * hs.size(),
                       hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return LACE_EHIP;
    kept_from_s(hs, n_occ, s_thr, pairs);
  } else {
    all_pairs(n_occ, pairs);
  }
  // every occupied x virtual pair, one-sided
  std::vector<char> os(pairs.size(), 0);
  for (int v = n_occ; v < n_orb; ++v)
    for (int i = 0; i < n_occ; ++i) {
      pairs.emplace_back(i, v);
      os.push_back(1);
    }
  std::vector<Batch> sched;
  schedule_for(p, pairs, n_orb, c.ppb, sched, &os, n_occ);
  e = enqueue_exchange(p, c, n_orb, sched, L, ws, w_g, e_x, st, true, true);
  if (e != hipSuccess) return LACE_EHIP;
  if (n_kept) *n_kept = (int64_t)pairs.size();
  return LACE_OK;
}

int lace_build_ace(lace_plan* p, int cell, const void* psi_g, const void* w_g,
                   int n_orb, lace_sym sym, void* xi_g, void* m_out,
                   double* ex_tr, int32_t* info, void* ws, size_t ws_bytes,
                   lace_stream_t stream) {
  int rc = check_common(p, cell, n_orb);
  if (rc) return rc;
  if (!psi_g || !w_g || !xi_g || !ws) return LACE_EINVAL;
  if (sym != LACE_SYM_AVG && sym != LACE_SYM_UPPER && sym != LACE_SYM_LOWER)
    return LACE_EINVAL;
  const Layout L = layout_for(p, cell, n_orb, 0);
  if (ws_bytes < L.total) return LACE_ENOMEM;
  return hip_status(enqueue_build_ace(p->cells[cell], n_orb, (int)sym, L, ws,
                                      psi_g, w_g, xi_g, m_out, ex_tr, info,
                                      static_cast<hipStream_t>(stream)));
}

int lace_apply_ace(lace_plan* p, int cell, const void* xi_g, int n_orb,
                   const void* x_g, int n_vec, void* y_g, void* ws,
                   size_t ws_bytes, lace_stream_t stream) {
  int rc = check_common(p, cell, n_orb);
  if (rc) return rc;
  if (!xi_g || !x_g || !y_g || !ws || n_vec < 1) return LACE_EINVAL;
  if (x_g == y_g) return LACE_EINVAL;
  const Layout L = layout_for(p, cell, n_orb, n_vec);
  if (ws_bytes < L.total) return LACE_ENOMEM;
  const CellDev& c = p->cells[cell].dev;
  hipStream_t st = static_cast<hipStream_t>(stream);
  // T = -(xi^H x), then y = xi T
  hipError_t e = launch_gemm_ip_c128(xi_g, c.n_pw, n_orb, x_g, c.n_pw, n_vec,
                                     c.n_pw, -1.0, at(ws, L.t), at(ws, L.part),
                                     (int64_t)(L.mw - L.part), st);
  if (e == hipSuccess)
    e = launch_gemm_tall(xi_g, c.n_pw, c.n_pw, n_orb, at(ws, L.t), n_vec, y_g,
                         c.n_pw, st);
  return hip_status(e);
}

int lace_fft3d(lace_plan* p, int cell, int direction, void* grids, int count,
               lace_stream_t stream) {
  if (!p || cell < 0 || cell >= (int)p->cells.size() || !grids || count < 1)
    return LACE_EINVAL;
  if (direction != -1 && direction != 1) return LACE_EINVAL;
  if (!device_ok(p)) return LACE_EINVAL;
  return hip_status(launch_fft3d(p->cells[cell].dev, p->fp64,
                                 direction, grids, count,
                                 static_cast<hipStream_t>(stream)));
}

int lace_schedule_pairs(const int32_t* pair_i, const int32_t* pair_j,
                        int64_t n_pairs, int n_orb, int per_batch,
                        int32_t* batch_of, int64_t* n_batches) {
  if (!pair_i || !pair_j || !batch_of || !n_batches || n_pairs < 0 ||
      n_orb < 1 || per_batch < 1 || per_batch > PMAX)
    return LACE_EINVAL;
  std::vector<std::pair<int, int>> pairs;
  pairs.reserve(n_pairs);
  for (int64_t k = 0; k < n_pairs; ++k) {
    const int i = pair_i[k], j = pair_j[k];
    if (i < 0 || j < i || j >= n_orb) return LACE_EINVAL;
    pairs.emplace_back(i, j);
  }
  std::vector<Batch> sched;
  std::vector<int32_t> bo;
  build_schedule(pairs, n_orb, per_batch, sched, &bo);
  for (int64_t k = 0; k < n_pairs; ++k) batch_of[k] = bo[k];
  *n_batches = (int64_t)sched.size();
  return LACE_OK;
}

int lace_schedule_slots(const int32_t* pair_i, const int32_t* pair_j,
                        int64_t n_pairs, int n_orb, int per_batch,
                        int32_t* batch_of, int32_t* slot_of,
                        int64_t* n_batches) {
  if (!pair_i || !pair_j || !batch_of || !slot_of || !n_batches ||
      n_pairs < 0 || n_orb < 1 || per_batch < 1 || per_batch > PMAX)
    return LACE_EINVAL;
  std::vector<std::pair<int, int>> pairs;
  pairs.reserve(n_pairs);
  for (int64_t k = 0; k < n_pairs; ++k) {
    const int i = pair_i[k], j = pair_j[k];
    if (i < 0 || j < i || j >= n_orb) return LACE_EINVAL;
    pairs.emplace_back(i, j);
  }
  std::vector<Batch> sched;
  std::vector<int32_t> bo, so;
  build_slot_schedule(pairs, n_orb, per_batch, sched, &bo, &so);
  for (int64_t k = 0; k < n_pairs; ++k) {
    batch_of[k] = bo[k];
    slot_of[k] = so[k];
  }
  *n_batches = (int64_t)sched.size();
  return LACE_OK;
}

int lace_set_tuning(lace_plan* p, int cell, int ppb, int use_plane) {
  if (!p || cell < 0 || cell >= (int)p->cells.size()) return LACE_EINVAL;
  if (ppb < 1 || ppb > PMAX || use_plane < 0 || use_plane > 2)
    return LACE_EINVAL;
  CellDev& c = p->cells[cell].dev;
  if (use_plane == 1 && !plane_fits(c.n, p->fp64)) return LACE_EUNSUPPORTED;
  c.ppb = ppb;
  c.use_plane = use_plane;
  return LACE_OK;
}

int lace_get_tuning(const lace_plan* p, int cell, int* ppb, int* use_plane) {
  if (!p || cell < 0 || cell >= (int)p->cells.size()) return LACE_EINVAL;
  if (ppb) *ppb = p->cells[cell].dev.ppb;
  if (use_plane) *use_plane = p->cells[cell].dev.use_plane;
  return LACE_OK;
}

int lace_autotune(lace_plan* p, int cell, const void* psi_g, int n_orb,
                  void* ws, size_t ws_bytes, lace_stream_t stream,
                  int* cand_ppb, int* cand_plane, double* cand_us, int* n_cand) {
  int rc = check_common(p, cell, n_orb);
  if (rc) return rc;
  if (!psi_g || !ws) return LACE_EINVAL;
  const Layout L = layout_for(p, cell, n_orb, 0);
  if (ws_bytes < L.total) return LACE_ENOMEM;
  CellDev& c = p->cells[cell].dev;
  const bool fp64 = p->fp64;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = enqueue_orbitals(p, c, psi_g, n_orb, L, ws, st);
  if (e != hipSuccess) return LACE_EHIP;
  // every candidate schedules all pairs its own way and is timed on its
  // first batches holding at least 4 * PMAX pairs: steady-state batches of
  // that candidate's own schedule
  std::vector<std::pair<int, int>> pairs;
  all_pairs(n_orb, pairs);
  struct Cand { int ppb, plane; double us; };
  std::vector<Cand> cands;
  const int ppbs[4] = {8, 16, 32, 64};
  for (int plane = 2; plane >= 0; --plane) {
    if (plane == 1 && !plane_fits(c.n, fp64)) continue;
    for (int k = 0; k < 4; ++k) cands.push_back({ppbs[k], plane, 0.0});
  }
  const int save_ppb = c.ppb, save_plane = c.use_plane;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess)
    return LACE_EHIP;
  for (auto& cd : cands) {
    c.ppb = cd.ppb;
    c.use_plane = cd.plane;
    std::vector<Batch> sched;
    schedule_for(p, pairs, n_orb, cd.ppb, sched);
    int64_t timed_pairs = 0;
    size_t nb = 0;
    while (nb < sched.size() && timed_pairs < 4 * PMAX)
      timed_pairs += sched[nb++].p.n;
    sched.resize(nb);
    double best = 1e30;
    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
      e = hipEventRecord(t0, st);
      for (size_t b = 0; e == hipSuccess && b < sched.size(); ++b)
        e = enqueue_batch(p, c, sched[b], L, ws, (int)(b % 2), st, nullptr);
      if (e == hipSuccess) e = hipEventRecord(t1, st);
      if (e == hipSuccess) e = hipEventSynchronize(t1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
      if (rep > 0 && ms < best) best = ms;   // first repetition warms up
    }
    cd.us = 1e3 * best / double(timed_pairs);
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (e != hipSuccess) {
    c.ppb = save_ppb;
    c.use_plane = save_plane;
    return LACE_EHIP;
  }
  size_t bi = 0;
  for (size_t k = 1; k < cands.size(); ++k)
    if (cands[k].us < cands[bi].us) bi = k;
  c.ppb = cands[bi].ppb;
  c.use_plane = cands[bi].plane;
  if (n_cand) {
    const int cap = *n_cand;
    for (int k = 0; k < (int)cands.size() && k < cap; ++k) {
      if (cand_ppb) cand_ppb[k] = cands[k].ppb;
      if (cand_plane) cand_plane[k] = cands[k].plane;
      if (cand_us) cand_us[k] = cands[k].us;
    }
    *n_cand = (int)cands.size();
  }
  return LACE_OK;
}

// ------------------------------------------------------------ batching
static hipError_t ensure_streams(lace_plan* p, int k) {
  while ((int)p->streams.size() < k) {
    hipStream_t s;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    p->streams.push_back(s);
  }
  while ((int)p->events.size() < k + 2) {
    hipEvent_t ev;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return e;
    p->events.push_back(ev);
  }
  if (!p->origin) {
    hipError_t e = hipStreamCreateWithFlags(&p->origin, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// `to` waits for everything enqueued so far on `from` (event k).
static hipError_t link(lace_plan* p, hipStream_t from, hipStream_t to, int k) {
  hipError_t e = hipEventRecord(p->events[k], from);
  if (e == hipSuccess) e = hipStreamWaitEvent(to, p->events[k], 0);
  return e;
}

static void hash_mix(std::vector<uint64_t>& key, uint64_t v) { key.push_back(v); }

int lace_apply_exchange_batched(lace_plan* p, lace_job* jobs, int n_jobs,
                                int flags, lace_stream_t stream) {
  if (!p || !jobs || n_jobs < 1) return LACE_EINVAL;
  if (!device_ok(p)) return LACE_EINVAL;
  if (flags & ~LACE_BATCH_GRAPH) return LACE_EINVAL;
  std::vector<Layout> lay(n_jobs);
  for (int k = 0; k < n_jobs; ++k) {
    const lace_job& j = jobs[k];
    int rc = check_common(p, j.cell, j.n_orb);
    if (rc) return rc;
    if (!j.psi_g || !j.w_g || !j.ws) return LACE_EINVAL;
    if (!(j.s_thr >= 0.0 && j.s_thr < 1.0)) return LACE_EINVAL;
    if (j.xi_g && j.sym != LACE_SYM_AVG && j.sym != LACE_SYM_UPPER &&
        j.sym != LACE_SYM_LOWER)
      return LACE_EINVAL;
    lay[k] = layout_for(p, j.cell, j.n_orb, 0);
    if (j.ws_bytes < lay[k].total) return LACE_ENOMEM;
    for (int q = 0; q < k; ++q)
      if (jobs[q].ws == j.ws || jobs[q].w_g == j.w_g ||
          (j.info && jobs[q].info == j.info))
        return LACE_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int ns = n_jobs < 8 ? n_jobs : 8;
  hipError_t e = ensure_streams(p, ns);
  if (e != hipSuccess) return LACE_EHIP;
  // jobs to streams, largest first onto the least loaded stream
  std::vector<int> order(n_jobs), on(n_jobs);
  for (int k = 0; k < n_jobs; ++k) order[k] = k;
  auto cost = [&](int k) {
    const CellDev& c = p->cells[jobs[k].cell].dev;
    return double(c.ng) * jobs[k].n_orb * jobs[k].n_orb;
  };
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return cost(a) > cost(b); });
  std::vector<double> load(ns, 0.0);
  for (int k : order) {
    int best = 0;
    for (int q = 1; q < ns; ++q) if (load[q] < load[best]) best = q;
    on[k] = best;
    load[best] += cost(k);
  }
  // phase 1: grid orbitals and screening, eagerly
  for (int q = 0; q < ns && e == hipSuccess; ++q) e = link(p, st, p->streams[q], q);
  bool any_screen = false;
  for (int k = 0; k < n_jobs && e == hipSuccess; ++k) {
    const lace_job& j = jobs[k];
    const CellDev& c = p->cells[j.cell].dev;
    hipStream_t js = p->streams[on[k]];
    e = enqueue_orbitals(p, c, j.psi_g, j.n_orb, lay[k], j.ws, js);
    if (e == hipSuccess && j.s_thr > 0.0) {
      any_screen = true;
      e = enqueue_screen(p, c, j.n_orb, lay[k], j.ws,
                         reinterpret_cast<double*>(at(j.ws, lay[k].s)), js);
    }
  }
  if (e != hipSuccess) return LACE_EHIP;
  std::vector<std::vector<Batch>> scheds(n_jobs);
  {
    std::vector<std::vector<double>> hs(n_jobs);
    for (int k = 0; k < n_jobs && e == hipSuccess; ++k) {
      if (jobs[k].s_thr > 0.0) {
        hs[k].resize((size_t)jobs[k].n_orb * jobs[k].n_orb);
        e = hipMemcpyAsync(hs[k].data(), at(jobs[k].ws, lay[k].s),
                           sizeof(double) * hs[k].size(), hipMemcpyDeviceToHost,
                           p->streams[on[k]]);
      }
    }
    if (any_screen)
      for (int q = 0; q < ns && e == hipSuccess; ++q)
        e = hipStreamSynchronize(p->streams[q]);
    if (e != hipSuccess) return LACE_EHIP;
    for (int k = 0; k < n_jobs; ++k) {
      std::vector<std::pair<int, int>> pairs;
      if (jobs[k].s_thr > 0.0) kept_from_s(hs[k], jobs[k].n_orb, jobs[k].s_thr, pairs);
      else all_pairs(jobs[k].n_orb, pairs);
      jobs[k].n_kept = (int64_t)pairs.size();
      schedule_for(p, pairs, jobs[k].n_orb, p->cells[jobs[k].cell].dev.ppb,
                   scheds[k]);
    }
  }
  // phase 2: pair pipelines, back-transforms, ACE builds
  auto enqueue_phase2 = [&]() -> hipError_t {
    hipError_t r = hipSuccess;
    for (int k = 0; k < n_jobs && r == hipSuccess; ++k) {
      const lace_job& j = jobs[k];
      const CellPlan& cp = p->cells[j.cell];
      hipStream_t js = p->streams[on[k]];
      r = enqueue_exchange(p, cp.dev, j.n_orb, scheds[k], lay[k], j.ws, j.w_g,
                           j.e_x, js, false);
      if (r == hipSuccess && j.xi_g)
        r = enqueue_build_ace(cp, j.n_orb, j.sym, lay[k], j.ws, j.psi_g, j.w_g,
                              j.xi_g, j.m_out, j.ex_tr, j.info, js);
    }
    return r;
  };
  if (!(flags & LACE_BATCH_GRAPH)) {
    e = enqueue_phase2();
    for (int q = 0; q < ns && e == hipSuccess; ++q)
      e = link(p, p->streams[q], st, q);
    return hip_status(e);
  }
  // graph: key on everything the captured work depends on
  std::vector<uint64_t> key;
  hash_mix(key, (uint64_t)n_jobs);
  for (int k = 0; k < n_jobs; ++k) {
    const lace_job& j = jobs[k];
    const CellDev& c = p->cells[j.cell].dev;
    for (uint64_t v : {(uint64_t)j.cell, (uint64_t)(uintptr_t)j.psi_g,
                       (uint64_t)j.n_orb, (uint64_t)(uintptr_t)j.w_g,
                       (uint64_t)(uintptr_t)j.e_x, (uint64_t)j.sym,
                       (uint64_t)(uintptr_t)j.xi_g, (uint64_t)(uintptr_t)j.m_out,
                       (uint64_t)(uintptr_t)j.ex_tr, (uint64_t)(uintptr_t)j.info,
                       (uint64_t)(uintptr_t)j.ws,
                       (uint64_t)on[k], (uint64_t)c.ppb, (uint64_t)c.use_plane,
                       (uint64_t)scheds[k].size()})
      hash_mix(key, v);
    uint64_t h = 1469598103934665603ull;
    for (const auto& bt : scheds[k]) {
      for (int q = 0; q < bt.p.n; ++q)
        h = (h ^ (uint64_t)(bt.p.i[q] * 65536 + bt.p.j[q] + 1)) *
            1099511628211ull;
      for (int q = 0; q < bt.q.n; ++q)
        for (int v : {bt.q.i[q], bt.q.j[q], bt.q.k[q], bt.q.l[q]})
          h = (h ^ (uint64_t)(v + 2)) * 1099511628211ull;
      h = (h ^ 0x9e3779b97f4a7c15ull) * 1099511628211ull;   // batch boundary
    }
    hash_mix(key, h);
  }
  // the origin stream waits for phase 1 on every internal stream
  for (int q = 0; q < ns && e == hipSuccess; ++q) e = link(p, p->streams[q], p->origin, q);
  if (e != hipSuccess) return LACE_EHIP;
  if (!p->graph.exec || p->graph.key != key) {
    if (p->graph.exec) { (void)hipGraphExecDestroy(p->graph.exec); p->graph.exec = nullptr; }
    if (p->graph.graph) { (void)hipGraphDestroy(p->graph.graph); p->graph.graph = nullptr; }
    e = hipStreamBeginCapture(p->origin, hipStreamCaptureModeThreadLocal);
    for (int q = 0; q < ns && e == hipSuccess; ++q)
      e = link(p, p->origin, p->streams[q], ns);
    hipError_t r = (e == hipSuccess) ? enqueue_phase2() : e;
    for (int q = 0; q < ns && r == hipSuccess; ++q)
      r = link(p, p->streams[q], p->origin, q);
    hipGraph_t g = nullptr;
    hipError_t ec = hipStreamEndCapture(p->origin, &g);
    if (r != hipSuccess || ec != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      return LACE_EHIP;
    }
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) { (void)hipGraphDestroy(g); return LACE_EHIP; }
    p->graph.graph = g;
    p->graph.exec = ex;
    p->graph.key = key;
  }
  e = hipGraphLaunch(p->graph.exec, p->origin);
  if (e == hipSuccess) e = link(p, p->origin, st, ns + 1);
  return hip_status(e);
}

int lace_profile_enable(lace_plan* p, int enable) {
  if (!p) return LACE_EINVAL;
  Profile& pr = p->prof;
  if (enable) {
    if (!pr.recs.empty() && hipDeviceSynchronize() != hipSuccess) return LACE_EHIP;
    pr.recs.clear();
    pr.used = 0;
    for (int k = 0; k < 3; ++k) {
      pr.ms[k] = 0; pr.launches[k] = 0; pr.pairs[k] = 0; pr.bytes[k] = 0;
    }
  }
  pr.on = enable != 0;
  return LACE_OK;
}

int lace_profile_read(lace_plan* p, double* ms, int64_t* launches,
                      int64_t* pairs, double* alg_bytes) {
  if (!p) return LACE_EINVAL;
  Profile& pr = p->prof;
  if (hipDeviceSynchronize() != hipSuccess) return LACE_EHIP;
  if (prof_collect(pr) != hipSuccess) return LACE_EHIP;
  for (int k = 0; k < 3; ++k) {
    if (ms) ms[k] = pr.ms[k];
    if (launches) launches[k] = pr.launches[k];
    if (pairs) pairs[k] = pr.pairs[k];
    if (alg_bytes) alg_bytes[k] = pr.bytes[k];
  }
  return LACE_OK;
}

int lace_check_real(lace_plan* p, int cell, const void* psi_g, int n_orb,
                    void* ws, size_t ws_bytes, lace_stream_t stream,
                    double* rel_dev) {
  int rc = check_common(p, cell, n_orb);
  if (rc) return rc;
  if (!p->gamma || !psi_g || !ws || !rel_dev) return LACE_EINVAL;
  const Layout L = layout_for(p, cell, n_orb, 0);
  if (ws_bytes < L.total) return LACE_ENOMEM;
  hipStream_t st = static_cast<hipStream_t>(stream);
  double* part = reinterpret_cast<double*>(at(ws, L.part));
  int nb = 0;
  hipError_t e = launch_real_check(p->cells[cell].dev, psi_g, n_orb, part, &nb, st);
  std::vector<double> h(2 * (size_t)nb);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h.data(), part, sizeof(double) * h.size(),
                       hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return LACE_EHIP;
  double d = 0.0, t = 0.0;
  for (int k = 0; k < nb; ++k) { d += h[2 * k]; t += h[2 * k + 1]; }
  *rel_dev = t > 0.0 ? std::sqrt(d / t) : 0.0;
  return LACE_OK;
}

int lace_get_info(const void* ws, lace_stream_t stream, int32_t* info_host) {
  if (!ws || !info_host) return LACE_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int32_t v = 0;
  // the word sits at offset 0 of every workspace layout
  hipError_t e = hipMemcpyAsync(&v, ws, sizeof(v), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return LACE_EHIP;
  *info_host = v;
  return v == 0 ? LACE_OK : LACE_ENOTPD;
}

