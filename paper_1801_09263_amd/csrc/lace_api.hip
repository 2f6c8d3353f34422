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

// Scratch of lace_apply_ace_noalloc: one fixed array per GPU, for callers
// that cannot allocate.  In host code the array's name is not a device
// address; its address on each device is looked up once, with that device
// current, when the first plan is created there, and kept here.
static constexpr size_t kNoAllocScratchBytes = size_t(96) << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};
}  // namespace

// Looks up the scratch array's address on device d (the current device).
static void noalloc_scratch_init(int d) {
  if (d < 0 || d >= kMaxDevices) return;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch_done[d]) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  g_scratch_ptr[d] = e == hipSuccess ? ptr : nullptr;
  g_scratch_err[d] = e;
  g_scratch_done[d] = true;
}

// The device address of device d's scratch array, or nullptr when the
// lookup failed or has not run.
static void* noalloc_scratch(int d) {
  if (d < 0 || d >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  return g_scratch_done[d] && g_scratch_err[d] == hipSuccess ? g_scratch_ptr[d] : nullptr;
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
  GraphCache graph;
  // LACE_SCHEDULE_FALLBACK=1: schedules take the round-robin form (tests)
  bool force_fallback = false;
};

// ---------------------------------------------------------------- helpers
static int hip_status(hipError_t e) { return e == hipSuccess ? LACE_OK : LACE_EHIP; }

static size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  size_t info, psi, w, tmp, epart, s, part, mw, a, z, t, u, dens, scdm, pts,
      tab, sched, kcnt, koff, total;
  int64_t max_batches;
  int pairs_per_batch;
};

// The status block at the start of every workspace: the Cholesky info word
// of builds that pass none (offset 0, where lace_get_info reads it), the
// batch count of the last schedule, the count of pairs it holds.
struct Status {
  int32_t info;
  int32_t n_batches;
  int64_t n_kept;
};

// bytes of one complex grid point in the plan precision
static size_t grid_bytes(const lace_plan* p) { return p->fp64 ? 16 : 8; }
// bytes of one orbital grid point (real for Gamma plans)
static size_t orb_bytes(const lace_plan* p) {
  return p->gamma ? grid_bytes(p) / 2 : grid_bytes(p);
}

// The most batches a schedule of any set of pairs of n_orb orbitals takes
// with at most ppb pairs per batch: the count of the round-robin schedule,
// which runs each round (a set of disjoint pairs, at most nv/2 of them)
// and the diagonal round in batches of their own.  Real orbitals pack two
// pairs of one kind per slot (one-sided pairs with the virtual orbitals are
// a second kind) and a batch holds at most ppb / 2 two-pair slots.
static int64_t batch_bound(int n_orb, int ppb, bool gamma, bool virt) {
  const int64_t nv = n_orb + (n_orb & 1), pr = nv / 2;
  auto cdiv = [](int64_t a, int64_t b) { return (a + b - 1) / b; };
  if (!gamma) return (nv - 1) * cdiv(pr, ppb) + cdiv(n_orb, ppb);
  if (ppb == 1) return (nv - 1) * pr + n_orb;
  const int64_t sp = ppb / 2;
  const int64_t slots_r = virt ? pr / 2 + 1 : cdiv(pr, 2);
  return (nv - 1) * cdiv(slots_r, sp) + cdiv(cdiv(n_orb, 2), sp);
}

// Batches the host launches, and the most a schedule may use before the
// round-robin fallback replaces it.  Slot schedules of real orbitals get a
// margin above the round-robin bound: their star slots read three orbital
// grids where the fallback's slots read four, which outweighs a few more
// batches (a nearly complete pair set of 64 orbitals packs into 66 batches
// of stars against the fallback's 64 without).  Complex plans gain nothing
// from more batches than the round robin.
static int64_t bound_margin(int64_t b) { return std::max<int64_t>(4, b / 64); }
static int64_t launch_bound(int n_orb, int ppb, bool gamma, bool virt) {
  const int64_t b = batch_bound(n_orb, ppb, gamma, virt);
  return gamma && ppb >= 2 ? b + bound_margin(b) : b;
}

static Layout layout_for(const lace_plan* p, int cell, int n_orb, int n_vec) {
  const CellDev& c = p->cells[cell].dev;
  const bool fp64 = p->fp64;
  Layout L{};
  L.pairs_per_batch = c.ppb;
  const size_t gb = (size_t)c.ng * grid_bytes(p);
  size_t off = 0;
  // the status block: first, so that lace_get_info finds the info word
  // without the layout
  L.info = off; off += 256;
  // orbital and W grids; for real orbitals these hold n_orb real grids and
  // double as the scratch of ceil(n_orb / 2) packed complex transforms
  const size_t ob = p->gamma ? gb * ((n_orb + 1) / 2) : gb * n_orb;
  L.psi = off; off += align_up(ob);
  L.w = off; off += align_up(ob);
  // two pair buffers and two sets of energy partials, each sized for the
  // largest batch (so that one workspace serves every tuning of the cell):
  // consecutive batches alternate between them, so that one batch's passes
  // A and B can run while the previous batch's pass C still reads its buffer
  L.tmp = off; off += align_up(gb * SMAX * 2);
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
  // batch table: the launch bound of one pair per batch, one-sided pairs
  // included, which every tuning's launch bound stays below (batch_bound
  // falls as ppb grows)
  L.max_batches = batch_bound(n_orb, 1, p->gamma, true);
  L.max_batches += bound_margin(L.max_batches);
  L.tab = off; off += align_up(sizeof(BatchDev) * (size_t)L.max_batches);
  L.sched = off; off += align_up((size_t)sched_scratch_bytes(n_orb));
  L.kcnt = off; off += align_up(sizeof(int32_t) * (size_t)n_orb);
  L.koff = off; off += align_up(sizeof(int64_t) * ((size_t)n_orb + 1));
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
  {
    const char* fb = std::getenv("LACE_SCHEDULE_FALLBACK");
    p->force_fallback = fb && fb[0] == '1';
  }
  p->fp64 = prec == LACE_FP64 || prec == LACE_FP64_GAMMA;
  p->gamma = gamma;
  if (hipGetDevice(&p->device) != hipSuccess) { delete p; return LACE_EHIP; }
  noalloc_scratch_init(p->device);
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
    cp.dev.ppb = std::min(default_pairs_per_batch(n), gamma ? PMAX : SMAX);
    cp.dev.ztile = 0;
    cp.dev.radix = 0;
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

// The device schedule keeps one bit per orbital pair in 64-bit words of at
// most 4096 orbitals.
static constexpr int kMaxExchangeOrbitals = 4096;

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
static void batch_bytes(const lace_plan* p, const CellDev& c, const BatchDev& bt,
                        double out[3]) {
  const double U = double(c.ng) * grid_bytes(p);
  const double G = double(c.ng) * orb_bytes(p);
  // orbs: orbital grids read by pass A; orbs_c: orbital grids read by pass
  // C plus twice the W grids it updates
  double orbs = 0.0, orbs_c = 0.0;
  for (int q = 0; q < bt.n; ++q) {
    if (p->gamma) {
      const int pos[4] = {bt.i[q], bt.j[q], bt.k[q], bt.l[q]};
      const int mate[4] = {1, 0, 3, 2};
      int all[4], upd[4], rd[4], na = 0, nu = 0, nr = 0;
      auto add = [](int* set, int& n, int v) {
        for (int t = 0; t < n; ++t) if (set[t] == v) return;
        set[n++] = v;
      };
      for (int t = 0; t < 4; ++t) {
        if (pos[t] < 0) continue;
        add(all, na, pos[t]);
        if (!((bt.skip[t] >> q) & 1ull)) {
          add(upd, nu, pos[t]);
          add(rd, nr, pos[mate[t]]);
        }
      }
      orbs += na;
      orbs_c += nr + 2 * nu;
    } else {
      const bool diag = bt.i[q] == bt.j[q];
      const bool os = (bt.one_sided >> q) & 1ull;
      orbs += diag ? 1.0 : 2.0;
      orbs_c += (diag || os) ? 3.0 : 6.0;
    }
  }
  out[0] = orbs * G + bt.n * U;
  out[1] = 2.0 * bt.n * U;
  out[2] = bt.n * U + orbs_c * G;
}

// One batch of the pair pipeline (pairs, or packed slots for Gamma plans).
// `lane` picks the pair buffer and the energy partials (0 or 1).
// Slot capacity of a batch with at most ppb pairs.
static int slot_cap(const lace_plan* p, int ppb) {
  return p->gamma ? (ppb + 1) / 2 : ppb;
}

// Batch b of the workspace's batch table through the pair pipeline.
// `lane` picks the pair buffer and the energy partials (0 or 1).
static hipError_t enqueue_batch(const lace_plan* p, const CellDev& c,
                                int64_t b, int ppb, const Layout& L, void* ws,
                                int lane, hipStream_t st, hipEvent_t* ev,
                                const BatchSync* sy = nullptr) {
  void* tmp = at(ws, L.tmp + (size_t)lane * SMAX * c.ng * grid_bytes(p));
  double* epart = reinterpret_cast<double*>(at(ws, L.epart)) +
                  (size_t)lane * PMAX * energy_tiles(c.n, p->fp64);
  const BatchDev* bt = reinterpret_cast<const BatchDev*>(at(ws, L.tab)) + b;
  const int cap = slot_cap(p, ppb);
  if (p->gamma)
    return launch_quad_batch(c, p->fp64, bt, cap, at(ws, L.psi), at(ws, L.w),
                             tmp, epart, st, ev, sy);
  return launch_pair_batch(c, p->fp64, bt, cap, at(ws, L.psi), at(ws, L.w),
                           tmp, epart, st, ev, sy);
}

static hipError_t ensure_streams(lace_plan* p, int k);
static hipError_t link(lace_plan* p, hipStream_t from, hipStream_t to, int k);

// Which pairs to run: kept by S >= s_thr (s: device S, or nullptr for every
// pair), or an explicit device list.  n_occ < n_orb: orbitals from n_occ on
// are virtual, with every occupied x virtual pair one-sided.
struct PairSource {
  const double* s = nullptr;
  double s_thr = 0.0;
  int s_n = 0;                 // orbitals S covers (two-sided pairs)
  const int32_t* pair_i = nullptr;
  const int32_t* pair_j = nullptr;
  int64_t n_pairs = 0;
  int n_occ = 0;
};

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

static Status* status_of(void* ws, const Layout& L) {
  return reinterpret_cast<Status*>(at(ws, L.info));
}

// The batch schedule of `src` into the workspace's table, on the device.
static hipError_t enqueue_schedule(const lace_plan* p, const CellDev& c,
                                   int n_orb, int ppb, const PairSource& src,
                                   const Layout& L, void* ws, int64_t* n_kept,
                                   hipStream_t st) {
  Status* stw = status_of(ws, L);
  SchedDesc d{};
  d.n_orb = n_orb;
  d.n_occ = src.n_occ;
  d.ppb = ppb;
  d.gamma = p->gamma;
  d.force_fallback = p->force_fallback;
  d.max_batches = launch_bound(n_orb, ppb, p->gamma, src.n_occ < n_orb);
  d.s = src.s;
  d.s_n = src.s_n;
  d.s_thr = src.s_thr;
  d.pair_i = src.pair_i;
  d.pair_j = src.pair_j;
  d.n_pairs = src.n_pairs;
  d.table = reinterpret_cast<BatchDev*>(at(ws, L.tab));
  d.n_batches = &stw->n_batches;
  d.n_kept = n_kept ? n_kept : &stw->n_kept;
  d.scratch = at(ws, L.sched);
  (void)c;
  return launch_schedule(d, st);
}

// Schedule, pair pipeline, energy reduction, W back to plane waves.
// Requires the grid orbitals in the workspace.  Without profiling the host
// launches the bound of the schedule's batch count (launch_bound) and the
// kernels of batches past the schedule's end return at once, so nothing
// waits on the host.  Consecutive batches alternate between two internal
// streams when `overlap` (batch b on lane b % 2): a batch's passes A and B
// overlap the previous batch's passes, and its pass C waits for the
// previous pass C (they may share W grids), so W is summed in batch order
// either way.  Profiled calls read the schedule back (they synchronize the
// stream) and run the batches it holds one launch at a time on `st`.
// Batches 0 .. nb - 1 of the workspace's table through the pair pipeline.
// two: on two internal streams (batch b on lane b % 2), a batch's passes A
// and B overlapping the previous batch's pass C, the C passes in batch
// order; the caller's stream waits for both lanes at the end.  Else all on
// the caller's stream.
static hipError_t enqueue_batches(lace_plan* p, const CellDev& c, int64_t nb,
                                  int ppb, const Layout& L, void* ws,
                                  hipStream_t st, bool two) {
  two = two && nb > 1;
  hipStream_t lane[2] = {st, st};
  hipEvent_t cdone[2] = {nullptr, nullptr};
  hipError_t e = hipSuccess;
  if (two) {
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
  for (int64_t b = 0; e == hipSuccess && b < nb; ++b) {
    if (two) {
      BatchSync sy{b > 0 ? cdone[(b - 1) % 2] : nullptr, cdone[b % 2]};
      e = enqueue_batch(p, c, b, ppb, L, ws, (int)(b % 2), lane[b % 2], nullptr,
                        &sy);
    } else {
      e = enqueue_batch(p, c, b, ppb, L, ws, (int)(b % 2), st, nullptr);
    }
  }
  if (e == hipSuccess && two) {
    e = link(p, lane[0], st, 0);
    if (e == hipSuccess) e = link(p, lane[1], st, 1);
  }
  return e;
}

static hipError_t enqueue_exchange(lace_plan* p, const CellDev& c, int n_orb,
                                   const PairSource& src, const Layout& L,
                                   void* ws, void* w_g, double* e_x,
                                   int64_t* n_kept, hipStream_t st,
                                   bool profile, bool overlap = false) {
  const bool fp64 = p->fp64;
  void* w = at(ws, L.w);
  const int64_t ntiles = energy_tiles(c.n, fp64);
  double* epart = reinterpret_cast<double*>(at(ws, L.epart));
  const int ppb = c.ppb;
  hipError_t e = enqueue_exchange_zero(p, c, n_orb, L, ws, st);
  if (e == hipSuccess) e = enqueue_schedule(p, c, n_orb, ppb, src, L, ws, n_kept, st);
  Profile& pr = p->prof;
  const bool timed = profile && pr.on;
  int64_t nb = launch_bound(n_orb, ppb, p->gamma, src.n_occ < n_orb);
  std::vector<BatchDev> host_tab;
  if (e == hipSuccess && timed) {
    // read the schedule back: the profile records each batch's bytes and
    // launches only the batches the schedule holds
    Status h{};
    e = hipMemcpyAsync(&h, status_of(ws, L), sizeof(h), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) {
      nb = h.n_batches;
      host_tab.resize((size_t)nb);
      if (nb > 0)
        e = hipMemcpyAsync(host_tab.data(), at(ws, L.tab), sizeof(BatchDev) * nb,
                           hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    if (e == hipSuccess && pr.used + 4 * (size_t)nb > 65536) e = prof_collect(pr);
  }
  // Under stream capture the batches stay on the caller's stream: a capture
  // of the two-lane form (events recorded and waited for by turns on two
  // internal streams) ended in a host fault in the runtime's capture end,
  // whose cause is not known; the library's own graph (the batched call)
  // runs every job on one stream as well.
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (e == hipSuccess && overlap && hipStreamIsCapturing(st, &cap) != hipSuccess)
    cap = hipStreamCaptureStatusNone;
  const bool two = overlap && !timed && cap == hipStreamCaptureStatusNone;
  if (e == hipSuccess && timed) {
    for (int64_t b = 0; e == hipSuccess && b < nb; ++b) {
      const size_t first = pr.used;
      hipEvent_t ev[4];
      for (int k = 0; k < 4; ++k) ev[k] = prof_event(pr);
      if (!ev[0] || !ev[1] || !ev[2] || !ev[3]) return hipErrorOutOfMemory;
      Profile::Rec r;
      r.ev = first;
      r.pairs = host_tab[(size_t)b].npairs;
      batch_bytes(p, c, host_tab[(size_t)b], r.bytes);
      pr.recs.push_back(r);
      e = enqueue_batch(p, c, b, ppb, L, ws, (int)(b % 2), st, ev);
    }
  } else if (e == hipSuccess) {
    e = enqueue_batches(p, c, nb, ppb, L, ws, st, two);
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
                        double* e_x, int64_t* n_kept, int32_t* kept, void* ws,
                        size_t ws_bytes, lace_stream_t stream) {
  int rc = check_common(p, cell, n_orb);
  if (rc) return rc;
  if (n_orb > kMaxExchangeOrbitals) return LACE_EINVAL;
  if (!psi_g || !w_g || !ws) return LACE_EINVAL;
  if (!(s_thr >= 0.0 && s_thr < 1.0)) return LACE_EINVAL;
  if ((pair_i == nullptr) != (pair_j == nullptr)) return LACE_EINVAL;
  if (pair_i && (n_pairs < 0 || n_pairs > (int64_t)n_orb * (n_orb + 1) / 2))
    return LACE_EINVAL;
  const Layout L = layout_for(p, cell, n_orb, 0);
  if (ws_bytes < L.total) return LACE_ENOMEM;
  const CellDev& c = p->cells[cell].dev;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = enqueue_orbitals(p, c, psi_g, n_orb, L, ws, st);
  PairSource src;
  src.n_occ = n_orb;
  src.s_n = n_orb;
  if (pair_i) {
    src.pair_i = pair_i;
    src.pair_j = pair_j;
    src.n_pairs = n_pairs;
  } else if (s_thr > 0.0) {
    double* s = reinterpret_cast<double*>(at(ws, L.s));
    if (e == hipSuccess) e = enqueue_screen(p, c, n_orb, L, ws, s, st);
    src.s = s;
    src.s_thr = s_thr;
  }
  if (e == hipSuccess && kept && !pair_i)
    e = launch_kept_pairs(src.s, n_orb, s_thr,
                          reinterpret_cast<int32_t*>(at(ws, L.kcnt)),
                          reinterpret_cast<int64_t*>(at(ws, L.koff)), kept,
                          nullptr, st);
  if (e == hipSuccess)
    e = enqueue_exchange(p, c, n_orb, src, L, ws, w_g, e_x, n_kept, st, true,
                         true);
  return hip_status(e);
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
  if (n_orb > kMaxExchangeOrbitals) return LACE_EINVAL;
  int rc = check_common(p, cell, n_orb);
  if (rc) return rc;
  if (!psi_g || !w_g || !ws) return LACE_EINVAL;
  if (!(s_thr >= 0.0 && s_thr < 1.0)) return LACE_EINVAL;
  const Layout L = layout_for(p, cell, n_orb, 0);
  if (ws_bytes < L.total) return LACE_ENOMEM;
  const CellDev& c = p->cells[cell].dev;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = enqueue_orbitals(p, c, psi_g, n_orb, L, ws, st);
  // occupied pairs screened among the occupied orbitals; every occupied x
  // virtual pair one-sided
  PairSource src;
  src.n_occ = n_occ;
  src.s_n = n_occ;
  if (s_thr > 0.0) {
    double* s = reinterpret_cast<double*>(at(ws, L.s));
    if (e == hipSuccess) e = enqueue_screen(p, c, n_occ, L, ws, s, st);
    src.s = s;
    src.s_thr = s_thr;
  }
  if (e == hipSuccess)
    e = enqueue_exchange(p, c, n_orb, src, L, ws, w_g, e_x, n_kept, st, true,
                         true);
  return hip_status(e);
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

int lace_apply_ace_noalloc(lace_plan* p, int cell, const void* xi_g, int n_orb,
                           const void* x_g, int n_vec, void* y_g,
                           lace_stream_t stream) {
  int rc = check_common(p, cell, n_orb);
  if (rc) return rc;
  if (!xi_g || !x_g || !y_g || n_vec < 1) return LACE_EINVAL;
  if (x_g == y_g) return LACE_EINVAL;
  const CellDev& c = p->cells[cell].dev;
  // T = -(xi^H x) and the split-K partials of the same product, in the
  // device's scratch array
  const size_t t_bytes = align_up(16 * (size_t)n_orb * (size_t)n_vec);
  const int64_t part_bytes = gemm_ip_part_bytes(n_orb, n_vec, c.n_pw, true);
  if (t_bytes + (size_t)part_bytes > kNoAllocScratchBytes) return LACE_ENOMEM;
  char* base = static_cast<char*>(noalloc_scratch(p->device));
  if (!base) return LACE_EHIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = launch_gemm_ip_c128(xi_g, c.n_pw, n_orb, x_g, c.n_pw, n_vec,
                                     c.n_pw, -1.0, base, base + t_bytes,
                                     part_bytes, st);
  if (e == hipSuccess)
    e = launch_gemm_tall(xi_g, c.n_pw, c.n_pw, n_orb, base, n_vec, y_g, c.n_pw, st);
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

// Host form of the device schedule (screen_kernels.hip), step for step, so
// that the host-only entry points return the schedule the library runs.
namespace {

struct HSlot { int i, j, k, l, np; uint32_t flags; };

struct HostSched {
  int n, n_occ, ppb, cap, words;
  bool gamma, force_fallback;
  int64_t max_batches;
  std::vector<uint64_t> kb, db;
  bool kbit(int a, int b) const {
    return (kb[(size_t)a * words + (b >> 6)] >> (b & 63)) & 1ull;
  }
  bool dbit(int a) const { return (db[a >> 6] >> (a & 63)) & 1ull; }
};

int cyc_host(int t, int r, int nv) {
  const int m = nv - 1;
  if (t == 0) return nv - 1;
  return (t & 1) ? ((r - t + 1) % m + m) % m : (r + t) % m;
}

void put_host(BatchDev& b, int q, const HSlot& s) {
  b.i[q] = s.i; b.j[q] = s.j; b.k[q] = s.k; b.l[q] = s.l;
  if (s.flags & 1u) b.one_sided |= 1ull << q;
  for (int t = 0; t < 4; ++t)
    if ((s.flags >> (1 + t)) & 1u) b.skip[t] |= 1ull << q;
  if (s.k != s.i) b.star = 0;
  b.n = q + 1;
  b.npairs += s.np;
}

void clear_host(BatchDev& b) {
  std::memset(&b, 0, sizeof(b));
  b.star = 1;
}

// The ordered slot list; goff[g] is where group (round) g's slots start
// and G the number of slots in group order.
void slot_list(const HostSched& h, std::vector<HSlot>& slots,
               std::vector<int64_t>& goff, int64_t& G) {
  const int n = h.n, nv = n + (n & 1), m = nv - 1;
  auto kept = [&](int a, int b) { return a < n && b < n && h.kbit(a, b); };
  slots.clear();
  goff.clear();
  if (!h.gamma || h.ppb < 2) {   // single-pair slots
    for (int r = 0; r < nv; ++r) {
      goff.push_back((int64_t)slots.size());
      auto add = [&](int a, int b) {
        if (a > b) std::swap(a, b);
        if (b >= n) return;
        const bool os = a < h.n_occ && b >= h.n_occ;
        if (os || (b < h.n_occ && h.kbit(a, b)))
          slots.push_back({a, b, -1, -1, 1, os ? 3u : 0u});
      };
      if (r == nv - 1) {
        for (int a = 0; a < n; ++a)
          if (h.dbit(a)) slots.push_back({a, a, -1, -1, 1, 0u});
      } else {
        add(r, nv - 1);
        for (int k = 1; k <= (m - 1) / 2; ++k) add((r + k) % m, ((r - k) % m + m) % m);
      }
    }
    G = (int64_t)slots.size();
    return;
  }
  const int ng = nv / 2;
  std::vector<std::pair<int, int>> left;
  for (int g = 0; g < ng; ++g) {
    goff.push_back((int64_t)slots.size());
    if (g == ng - 1) {
      const int r = nv - 2;
      if (kept(r, nv - 1)) left.emplace_back(std::min(r, nv - 1), std::max(r, nv - 1));
      for (int k = 1; k <= (m - 1) / 2; ++k) {
        const int a = (r + k) % m, b = ((r - k) % m + m) % m;
        if (kept(a, b)) left.emplace_back(std::min(a, b), std::max(a, b));
      }
      continue;
    }
    const int r = 2 * g;
    auto ek = [&](int t) { return kept(cyc_host(t, r, nv), cyc_host((t + 1) % nv, r, nv)); };
    auto star = [&](int ta) {
      const int a = cyc_host(ta % nv, r, nv), c = cyc_host((ta + 1) % nv, r, nv),
                b = cyc_host((ta + 2) % nv, r, nv);
      slots.push_back({c, a, c, b, 2, 0u});
    };
    int t0 = -1;
    for (int t = 0; t < nv && t0 < 0; ++t)
      if (!ek(t)) t0 = t;
    if (t0 < 0) {
      for (int t = 0; t < nv; t += 2) star(t);
    } else {
      int pend = -1;
      for (int step = 1; step <= nv; ++step) {
        const int t = (t0 + step) % nv;
        if (ek(t)) {
          if (pend < 0) pend = t;
          else { star(pend); pend = -1; }
        } else if (pend >= 0) {
          const int pa = cyc_host(pend, r, nv), pb = cyc_host((pend + 1) % nv, r, nv);
          left.emplace_back(std::min(pa, pb), std::max(pa, pb));
          pend = -1;
        }
      }
    }
  }
  G = (int64_t)slots.size();
  // stars of edge rows: each vertex pairs its edges in row order; the stars
  // leave interleaved by rank; pend[v] is the other orbital of v's unpaired
  // edge (the last), or -1
  auto emit_stars = [&](const std::vector<std::vector<int>>& rows, std::vector<int>& pend) {
    size_t most = 0;
    for (int v = 0; v < n; ++v) {
      most = std::max(most, rows[v].size() / 2);
      pend[v] = (rows[v].size() & 1) ? rows[v].back() : -1;
    }
    for (size_t rho = 0; rho < most; ++rho)
      for (int v = 0; v < n; ++v)
        if (rho < rows[v].size() / 2)
          slots.push_back({v, rows[v][2 * rho], v, rows[v][2 * rho + 1], 2, 0u});
  };
  // left-overs, first pass: at the smaller orbital, in group order
  std::vector<std::vector<int>> rows(n);
  for (const auto& e : left) rows[e.first].push_back(e.second);
  std::vector<int> pend(n, -1);
  emit_stars(rows, pend);
  // second pass: the unpaired edges at their larger orbital
  std::vector<std::vector<int>> rows2(n);
  for (int v = 0; v < n; ++v)
    if (pend[v] >= 0) rows2[pend[v]].push_back(v);   // v ascending
  emit_stars(rows2, pend);
  // what is left, edge (pend[b], b) at each b, is paired as it comes
  int hx = -1, hy = -1;
  for (int v = 0; v < n; ++v) {
    const int x = pend[v];
    if (x < 0) continue;
    if (hx < 0) { hx = x; hy = v; continue; }
    if (hx == x || hx == v || hy == x || hy == v) {
      const int c = (hx == x || hx == v) ? hx : hy;
      const int pj = hx == c ? hy : hx, ql = x == c ? v : x;
      slots.push_back({c, pj, c, ql, 2, 0u});
    } else {
      slots.push_back({hx, hy, x, v, 2, 0u});
    }
    hx = -1;
  }
  if (hx >= 0) slots.push_back({hx, hy, -1, -1, 1, 0u});
  if (h.n_occ < n) {
    const int P = h.n_occ / 2, nvirt = n - h.n_occ;
    for (int k = 0; k < P; ++k)
      for (int u = 0; u < nvirt; ++u) {
        const int v = h.n_occ + u, t = 2 * ((k + u) % P);
        slots.push_back({v, t, v, t + 1, 2, 1u | 4u | 16u});
      }
    if (h.n_occ & 1)
      for (int u = 0; u < nvirt; ++u)
        slots.push_back({h.n_occ - 1, h.n_occ + u, -1, -1, 1, 1u | 2u});
  }
  int hd = -1;
  for (int d = 0; d < n; ++d) {
    if (!h.dbit(d)) continue;
    if (hd < 0) { hd = d; continue; }
    slots.push_back({hd, hd, d, d, 2, 0u});
    hd = -1;
  }
  if (hd >= 0) slots.push_back({hd, hd, -1, -1, 1, 0u});
}

void fallback_host(const HostSched& h, std::vector<BatchDev>& tab, int64_t& nb) {
  const int n = h.n, nv = n + (n & 1), m = nv - 1;
  const bool virt = h.n_occ < n;
  const int sp = h.gamma ? (h.ppb >= 2 ? h.ppb / 2 : 1) : h.ppb;
  nb = 0;
  int cur = -1, cur_slots = 0, cur_pairs = 0;
  auto emit = [&](const HSlot& s) {
    if (cur < 0 || cur_slots == sp || cur_pairs + s.np > h.ppb) {
      cur = (int)nb++;
      clear_host(tab[cur]);
      cur_slots = cur_pairs = 0;
    }
    put_host(tab[cur], cur_slots++, s);
    cur_pairs += s.np;
  };
  for (int r = 0; r < nv; ++r) {
    HSlot held[2] = {};
    int nh[2] = {0, 0};
    auto take = [&](int x, int y, bool os) {
      HSlot s{x, y, -1, -1, 1, 0u};
      if (os) s.flags = 1u | (x < h.n_occ ? 2u : 0u);
      if (!h.gamma || h.ppb == 1) { emit(s); return; }
      const int kd = os ? 1 : 0;
      if (nh[kd]) {
        HSlot t = held[kd];
        t.k = x; t.l = y; t.np = 2;
        if (os && x < h.n_occ) t.flags |= 8u;
        emit(t);
        nh[kd] = 0;
      } else {
        held[kd] = s;
        nh[kd] = 1;
      }
    };
    if (r == nv - 1) {
      for (int d = 0; d < n; ++d)
        if (h.dbit(d)) take(d, d, false);
    } else {
      auto pr = [&](int x, int y) {
        if (x > y) std::swap(x, y);
        if (y >= n) return;
        const bool os = virt && x < h.n_occ && y >= h.n_occ;
        if (os) take(x, y, true);
        else if (y < h.n_occ && h.kbit(x, y)) take(x, y, false);
      };
      pr(r, nv - 1);
      for (int k = 1; k <= (m - 1) / 2; ++k) pr((r + k) % m, ((r - k) % m + m) % m);
    }
    for (int kd = 0; kd < 2; ++kd)
      if (nh[kd]) emit(held[kd]);
    cur = -1;
  }
  for (int64_t b = nb; b < h.max_batches; ++b) clear_host(tab[(size_t)b]);
}

// First-fit over a window of 8 open batches, as on the device: the slots
// in the order ord; emit(list, full) gets each batch as it leaves the
// window (full; the oldest when a new one is needed; the rest at the end,
// oldest first).  Returns true when more than max_open batches would be
// opened.
template <class Emit>
bool ff_host(const HostSched& h, const std::vector<HSlot>& slots,
             const std::vector<int>& ord, int64_t max_open, Emit emit) {
  struct Win { std::vector<int> list; int pairs; std::vector<uint64_t> mask; };
  std::vector<Win> win;
  int64_t opened = 0;
  for (int q : ord) {
    const HSlot& s = slots[(size_t)q];
    const int orb[4] = {s.i, s.j, s.k, s.l};
    int pick = -1;
    for (size_t x = 0; x < win.size() && pick < 0; ++x) {
      const Win& w = win[x];
      bool ok = w.pairs + s.np <= h.ppb && (int)w.list.size() + 1 <= h.cap;
      for (int t = 0; t < 4 && ok; ++t)
        if (orb[t] >= 0 && ((w.mask[orb[t] >> 6] >> (orb[t] & 63)) & 1ull)) ok = false;
      if (ok) pick = (int)x;
    }
    if (pick < 0) {
      if (opened >= max_open) return true;
      if (win.size() == 8) {
        emit(win[0].list, false);
        win.erase(win.begin());
      }
      win.push_back({{}, 0, std::vector<uint64_t>(h.words, 0ull)});
      ++opened;
      pick = (int)win.size() - 1;
    }
    Win& w = win[(size_t)pick];
    w.list.push_back(q);
    w.pairs += s.np;
    for (int t = 0; t < 4; ++t)
      if (orb[t] >= 0) w.mask[orb[t] >> 6] |= 1ull << (orb[t] & 63);
    if (w.pairs >= h.ppb || (int)w.list.size() >= h.cap) {
      emit(w.list, true);
      win.erase(win.begin() + pick);
    }
  }
  for (const Win& w : win) emit(w.list, false);
  return false;
}

// The slot list cut into sched_sections(n) sections, each packed on its
// own; their full batches in section order, then first-fit of all other
// slots (section order) into further batches; as on the device.
void host_schedule(const HostSched& h, std::vector<BatchDev>& tab, int64_t& nb) {
  std::vector<HSlot> slots;
  std::vector<int64_t> goff;
  int64_t G = 0;
  slot_list(h, slots, goff, G);
  tab.assign((size_t)h.max_batches, BatchDev{});
  for (auto& b : tab) clear_host(b);
  nb = 0;
  bool over = h.force_fallback;
  std::vector<std::vector<int>> batches;
  if (!over) {
    const int S = sched_sections(h.n);
    const int64_t N = (int64_t)slots.size(), per = (N + S - 1) / S;
    // section k starts at k * per, moved up to the next group boundary
    // while among the group-ordered slots
    auto start = [&](int k) -> int64_t {
      if (k >= S) return N;
      const int64_t t = std::min(N, (int64_t)k * per);
      if (t >= G) return t;
      for (int64_t o : goff)
        if (o >= t) return o;
      return G;
    };
    std::vector<int> rest;
    for (int k = 0; k < S; ++k) {
      const int64_t lo = start(k), hi = start(k + 1);
      std::vector<int> ord;
      for (int64_t q = lo; q < hi; ++q) ord.push_back((int)q);
      ff_host(h, slots, ord, INT64_MAX, [&](const std::vector<int>& l, bool full) {
        if (full) batches.push_back(l);
        else rest.insert(rest.end(), l.begin(), l.end());
      });
    }
    const int64_t F = (int64_t)batches.size();
    if (F > h.max_batches) {
      over = true;
    } else {
      over = ff_host(h, slots, rest, h.max_batches - F,
                     [&](const std::vector<int>& l, bool) { batches.push_back(l); });
    }
  }
  if (over) {
    fallback_host(h, tab, nb);
    return;
  }
  nb = (int64_t)batches.size();
  for (int64_t b = 0; b < nb; ++b)
    for (size_t q = 0; q < batches[(size_t)b].size(); ++q)
      put_host(tab[(size_t)b], (int)q, slots[(size_t)batches[(size_t)b][q]]);
}

// Host schedule of an explicit pair list; batch and slot of every pair.
int schedule_list(const int32_t* pair_i, const int32_t* pair_j, int64_t n_pairs,
                  int n_orb, int per_batch, bool gamma, int32_t* batch_of,
                  int32_t* slot_of, int64_t* n_batches) {
  if (!pair_i || !pair_j || !batch_of || !n_batches || n_pairs < 0 ||
      n_orb < 1 || n_orb > 4096 || per_batch < 1 ||
      per_batch > (gamma ? PMAX : SMAX))
    return LACE_EINVAL;
  HostSched h;
  h.n = n_orb; h.n_occ = n_orb; h.ppb = per_batch;
  h.cap = gamma ? (per_batch + 1) / 2 : per_batch;
  h.words = (n_orb + 63) / 64;
  h.gamma = gamma;
  h.force_fallback = false;
  h.max_batches = launch_bound(n_orb, per_batch, gamma, false);
  h.kb.assign((size_t)n_orb * h.words, 0ull);
  h.db.assign((size_t)h.words, 0ull);
  for (int64_t k = 0; k < n_pairs; ++k) {
    const int i = pair_i[k], j = pair_j[k];
    if (i < 0 || j < i || j >= n_orb) return LACE_EINVAL;
    uint64_t* w = i == j ? &h.db[i >> 6] : &h.kb[(size_t)j * h.words + (i >> 6)];
    if ((*w >> (i & 63)) & 1ull) return LACE_EINVAL;   // repeated pair
    *w |= 1ull << (i & 63);
    if (i != j) h.kb[(size_t)i * h.words + (j >> 6)] |= 1ull << (j & 63);
  }
  std::vector<BatchDev> tab;
  int64_t nb = 0;
  host_schedule(h, tab, nb);
  std::vector<int64_t> where((size_t)n_orb * n_orb, -1);
  for (int64_t b = 0; b < nb; ++b)
    for (int q = 0; q < tab[(size_t)b].n; ++q) {
      const BatchDev& d = tab[(size_t)b];
      const int64_t code = b * 64 + q;
      where[(size_t)std::min(d.i[q], d.j[q]) * n_orb + std::max(d.i[q], d.j[q])] = code;
      if (d.k[q] >= 0)
        where[(size_t)std::min(d.k[q], d.l[q]) * n_orb + std::max(d.k[q], d.l[q])] = code;
    }
  for (int64_t k = 0; k < n_pairs; ++k) {
    const int64_t code = where[(size_t)pair_i[k] * n_orb + pair_j[k]];
    if (code < 0) return LACE_EINVAL;
    batch_of[k] = (int32_t)(code / 64);
    if (slot_of) slot_of[k] = (int32_t)(code % 64);
  }
  *n_batches = nb;
  return LACE_OK;
}

}  // namespace

int lace_schedule_pairs(const int32_t* pair_i, const int32_t* pair_j,
                        int64_t n_pairs, int n_orb, int per_batch,
                        int32_t* batch_of, int64_t* n_batches) {
  return schedule_list(pair_i, pair_j, n_pairs, n_orb, per_batch, false,
                       batch_of, nullptr, n_batches);
}

int lace_schedule_slots(const int32_t* pair_i, const int32_t* pair_j,
                        int64_t n_pairs, int n_orb, int per_batch,
                        int32_t* batch_of, int32_t* slot_of,
                        int64_t* n_batches) {
  if (!slot_of) return LACE_EINVAL;
  return schedule_list(pair_i, pair_j, n_pairs, n_orb, per_batch, true,
                       batch_of, slot_of, n_batches);
}

int lace_read_schedule(const lace_plan* p, int cell, int n_orb, const void* ws,
                       lace_stream_t stream, const int32_t* pair_i,
                       const int32_t* pair_j, int64_t n_pairs,
                       int32_t* batch_of, int32_t* slot_of,
                       int64_t* n_batches) {
  if (!p || cell < 0 || cell >= (int)p->cells.size() || n_orb < 1 || !ws ||
      !n_batches || n_pairs < 0 || (n_pairs > 0 && (!pair_i || !pair_j || !batch_of || !slot_of)))
    return LACE_EINVAL;
  const Layout L = layout_for(p, cell, n_orb, 0);
  hipStream_t st = static_cast<hipStream_t>(stream);
  Status h{};
  void* w = const_cast<void*>(ws);
  hipError_t e = hipMemcpyAsync(&h, status_of(w, L), sizeof(h),
                                hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return LACE_EHIP;
  if (h.n_batches < 0 || h.n_batches > L.max_batches) return LACE_EINVAL;
  std::vector<BatchDev> tab((size_t)h.n_batches);
  if (h.n_batches > 0) {
    e = hipMemcpyAsync(tab.data(), at(w, L.tab), sizeof(BatchDev) * tab.size(),
                       hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return LACE_EHIP;
  }
  std::vector<int64_t> where((size_t)n_orb * n_orb, -1);
  for (size_t b = 0; b < tab.size(); ++b)
    for (int q = 0; q < tab[b].n && q < SMAX; ++q) {
      const BatchDev& d = tab[b];
      const int64_t code = (int64_t)b * 64 + q;
      for (int t = 0; t < 2; ++t) {
        const int a = t ? d.k[q] : d.i[q], c = t ? d.l[q] : d.j[q];
        if (a < 0 || c < 0 || a >= n_orb || c >= n_orb) continue;
        where[(size_t)std::min(a, c) * n_orb + std::max(a, c)] = code;
      }
    }
  for (int64_t k = 0; k < n_pairs; ++k) {
    const int i = pair_i[k], j = pair_j[k];
    if (i < 0 || j < i || j >= n_orb) return LACE_EINVAL;
    const int64_t code = where[(size_t)i * n_orb + j];
    batch_of[k] = code < 0 ? -1 : (int32_t)(code / 64);
    slot_of[k] = code < 0 ? -1 : (int32_t)(code % 64);
  }
  *n_batches = h.n_batches;
  return LACE_OK;
}

int lace_set_tuning(lace_plan* p, int cell, int ppb, int use_plane, int z_tile,
                    int radix_order) {
  if (!p || cell < 0 || cell >= (int)p->cells.size()) return LACE_EINVAL;
  if (ppb < 1 || ppb > (p->gamma ? PMAX : SMAX) || use_plane < 0 || use_plane > 2)
    return LACE_EINVAL;
  if (z_tile < 0 || z_tile > 2 || radix_order < 0 || radix_order > 1)
    return LACE_EINVAL;
  CellDev& c = p->cells[cell].dev;
  if (use_plane == 1 && !plane_fits(c.n, p->fp64)) return LACE_EUNSUPPORTED;
  c.ppb = ppb;
  c.use_plane = use_plane;
  c.ztile = z_tile;
  c.radix = radix_order;
  return LACE_OK;
}

int lace_get_tuning(const lace_plan* p, int cell, int* ppb, int* use_plane,
                    int* z_tile, int* radix_order) {
  if (!p || cell < 0 || cell >= (int)p->cells.size()) return LACE_EINVAL;
  const CellDev& c = p->cells[cell].dev;
  if (ppb) *ppb = c.ppb;
  if (use_plane) *use_plane = c.use_plane;
  if (z_tile) *z_tile = c.ztile;
  if (radix_order) *radix_order = c.radix;
  return LACE_OK;
}

int lace_autotune(lace_plan* p, int cell, const void* psi_g, int n_orb,
                  double s_thr, void* ws, size_t ws_bytes, lace_stream_t stream,
                  int* cand_ppb, int* cand_plane, int* cand_ztile,
                  int* cand_radix, double* cand_us, int* n_cand) {
  int rc = check_common(p, cell, n_orb);
  if (rc) return rc;
  if (n_orb > kMaxExchangeOrbitals) return LACE_EINVAL;
  if (!psi_g || !ws || !(s_thr >= 0.0 && s_thr < 1.0)) return LACE_EINVAL;
  const Layout L = layout_for(p, cell, n_orb, 0);
  if (ws_bytes < L.total) return LACE_ENOMEM;
  CellDev& c = p->cells[cell].dev;
  const bool fp64 = p->fp64;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = enqueue_orbitals(p, c, psi_g, n_orb, L, ws, st);
  // the pairs the exchange will run: those S keeps at s_thr (Eq. (6))
  PairSource all;
  all.n_occ = n_orb;
  all.s_n = n_orb;
  if (e == hipSuccess && s_thr > 0.0) {
    double* s = reinterpret_cast<double*>(at(ws, L.s));
    e = enqueue_screen(p, c, n_orb, L, ws, s, st);
    all.s = s;
    all.s_thr = s_thr;
  }
  if (e != hipSuccess) return LACE_EHIP;
  // every candidate schedules the pairs its own way and is timed on two
  // lanes as the exchange runs them
  struct Cand { int ppb, plane, ztile, radix; double us; bool full; };
  std::vector<Cand> cands;
  // stage 1: pairs per batch (up to SMAX slots of one pair, complex, or
  // two, real) and the xy schedule, each timed on its first batches
  const int ppbs[5] = {8, 16, 32, 64, 128};
  const int nppb = p->gamma ? 5 : 4;
  for (int plane = 2; plane >= 0; --plane) {
    if (plane == 1 && !plane_fits(c.n, fp64)) continue;
    for (int k = 0; k < nppb; ++k) cands.push_back({ppbs[k], plane, 0, 0, 0.0, false});
  }
  const CellDev save = c;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess)
    return LACE_EHIP;
  // us per pair of a candidate: its first batches holding at least 16 *
  // PMAX pairs, or (full) its whole schedule, on two lanes as the exchange
  // runs them (the best of the repetitions after the first), plus their
  // share of the schedule's build time
  auto time_cand = [&](Cand& cd, bool full) {
    c.ppb = cd.ppb;
    c.use_plane = cd.plane;
    c.ztile = cd.ztile;
    c.radix = cd.radix;
    // the schedule's own build time, charged to the timed pairs in
    // proportion (batches that never fill leave every slot to the one-wave
    // refill, which makes the build cost depend on the candidate)
    if (e == hipSuccess) e = hipEventRecord(t0, st);
    if (e == hipSuccess) e = enqueue_schedule(p, c, n_orb, cd.ppb, all, L, ws, nullptr, st);
    if (e == hipSuccess) e = hipEventRecord(t1, st);
    if (e == hipSuccess) e = hipEventSynchronize(t1);
    float sched_ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&sched_ms, t0, t1);
    Status h{};
    if (e == hipSuccess)
      e = hipMemcpyAsync(&h, status_of(ws, L), sizeof(h), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    std::vector<BatchDev> tab((size_t)std::max(h.n_batches, 0));
    if (e == hipSuccess && !tab.empty())
      e = hipMemcpyAsync(tab.data(), at(ws, L.tab), sizeof(BatchDev) * tab.size(),
                         hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    int64_t timed_pairs = 0, all_pairs = 0;
    for (const BatchDev& b : tab) all_pairs += b.npairs;
    size_t nb = 0;
    while (nb < tab.size() && (full || timed_pairs < 16 * PMAX))
      timed_pairs += tab[nb++].npairs;
    // the whole schedule as the exchange launches it: up to the bound,
    // the batches past the schedule's end included
    if (full) nb = (size_t)launch_bound(n_orb, cd.ppb, p->gamma, false);
    double best = 1e30;
    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
      e = hipEventRecord(t0, st);
      if (e == hipSuccess) e = enqueue_batches(p, c, (int64_t)nb, cd.ppb, L, ws, st, true);
      if (e == hipSuccess) e = hipEventRecord(t1, st);
      if (e == hipSuccess) e = hipEventSynchronize(t1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
      if (rep > 0 && ms < best) best = ms;   // first repetition warms up
    }
    const double share = all_pairs > 0 ? double(timed_pairs) / double(all_pairs) : 0.0;
    const double us = timed_pairs > 0
                          ? 1e3 * (best + sched_ms * share) / double(timed_pairs)
                          : 1e30;
    // the whole-schedule time is the best over the rounds it is taken in
    cd.us = full && cd.full ? std::min(cd.us, us) : us;
    cd.full = full;
  };
  for (auto& cd : cands) time_cand(cd, false);
  // the three fastest of stage 1 again over their whole schedules (the
  // first batches, stars of whole cycles, pack differently from the rest)
  std::vector<size_t> order(cands.size());
  for (size_t k = 0; k < order.size(); ++k) order[k] = k;
  std::sort(order.begin(), order.end(),
            [&](size_t x, size_t y) { return cands[x].us < cands[y].us; });
  // (in two interleaved rounds, so that a drift of the clock over the
  // tuning does not favour one of them)
  for (int round = 0; round < 2; ++round)
    for (size_t k = 0; k < order.size() && k < 3; ++k) time_cand(cands[order[k]], true);
  auto best_full = [&]() {
    size_t bi = cands.size();
    for (size_t k = 0; k < cands.size(); ++k)
      if (cands[k].full && (bi == cands.size() || cands[k].us < cands[bi].us)) bi = k;
    return bi;
  };
  // stage 2, for the fastest so far: the z tiles half and twice as wide
  // (where the plane allows them) and the reversed radix order, each over
  // the whole schedule
  const size_t stage1 = cands.size();
  if (e == hipSuccess) {
    const Cand b = cands[best_full()];
    const int def = ztile_points(c.n, fp64, 0);
    for (int z = 1; z <= 2; ++z)
      if (ztile_points(c.n, fp64, z) != def)
        cands.push_back({b.ppb, b.plane, z, 0, 0.0, false});
    if (radix_orders_differ(c.n)) cands.push_back({b.ppb, b.plane, 0, 1, 0.0, false});
  }
  for (int round = 0; round < 2; ++round)
    for (size_t k = stage1; k < cands.size(); ++k) time_cand(cands[k], true);
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (e != hipSuccess) {
    c = save;
    return LACE_EHIP;
  }
  const Cand& win = cands[best_full()];
  c.ppb = win.ppb;
  c.use_plane = win.plane;
  c.ztile = win.ztile;
  c.radix = win.radix;
  if (n_cand) {
    const int cap = *n_cand;
    for (int k = 0; k < (int)cands.size() && k < cap; ++k) {
      if (cand_ppb) cand_ppb[k] = cands[k].ppb;
      if (cand_plane) cand_plane[k] = cands[k].plane;
      if (cand_ztile) cand_ztile[k] = cands[k].ztile;
      if (cand_radix) cand_radix[k] = cands[k].radix;
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
    if (j.n_orb > kMaxExchangeOrbitals) return LACE_EINVAL;
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
  // every job's device work on its stream: grid orbitals, screening,
  // schedule, pair pipeline, W to plane waves, ACE build
  auto enqueue_all = [&]() -> hipError_t {
    hipError_t r = hipSuccess;
    for (int k = 0; k < n_jobs && r == hipSuccess; ++k) {
      const lace_job& j = jobs[k];
      const CellPlan& cp = p->cells[j.cell];
      const CellDev& c = cp.dev;
      hipStream_t js = p->streams[on[k]];
      r = enqueue_orbitals(p, c, j.psi_g, j.n_orb, lay[k], j.ws, js);
      PairSource src;
      src.n_occ = j.n_orb;
      src.s_n = j.n_orb;
      if (r == hipSuccess && j.s_thr > 0.0) {
        double* sm = reinterpret_cast<double*>(at(j.ws, lay[k].s));
        r = enqueue_screen(p, c, j.n_orb, lay[k], j.ws, sm, js);
        src.s = sm;
        src.s_thr = j.s_thr;
      }
      if (r == hipSuccess)
        r = enqueue_exchange(p, c, j.n_orb, src, lay[k], j.ws, j.w_g, j.e_x,
                             j.n_kept, js, false);
      if (r == hipSuccess && j.xi_g)
        r = enqueue_build_ace(cp, j.n_orb, j.sym, lay[k], j.ws, j.psi_g, j.w_g,
                              j.xi_g, j.m_out, j.ex_tr, j.info, js);
    }
    return r;
  };
  if (!(flags & LACE_BATCH_GRAPH)) {
    for (int q = 0; q < ns && e == hipSuccess; ++q) e = link(p, st, p->streams[q], q);
    if (e == hipSuccess) e = enqueue_all();
    for (int q = 0; q < ns && e == hipSuccess; ++q)
      e = link(p, p->streams[q], st, q);
    return hip_status(e);
  }
  // graph: key on everything the captured work depends on (the pair lists
  // are built inside it, so a replay follows the current orbitals)
  std::vector<uint64_t> key;
  hash_mix(key, (uint64_t)n_jobs);
  for (int k = 0; k < n_jobs; ++k) {
    const lace_job& j = jobs[k];
    const CellDev& c = p->cells[j.cell].dev;
    uint64_t thr_bits = 0;
    std::memcpy(&thr_bits, &j.s_thr, sizeof(thr_bits));
    for (uint64_t v : {(uint64_t)j.cell, (uint64_t)(uintptr_t)j.psi_g,
                       (uint64_t)j.n_orb, thr_bits, (uint64_t)(uintptr_t)j.w_g,
                       (uint64_t)(uintptr_t)j.e_x, (uint64_t)(uintptr_t)j.n_kept,
                       (uint64_t)j.sym, (uint64_t)(uintptr_t)j.xi_g,
                       (uint64_t)(uintptr_t)j.m_out, (uint64_t)(uintptr_t)j.ex_tr,
                       (uint64_t)(uintptr_t)j.info, (uint64_t)(uintptr_t)j.ws,
                       (uint64_t)on[k], (uint64_t)c.ppb, (uint64_t)c.use_plane})
      hash_mix(key, v);
  }
  // the origin stream waits for the caller's stream
  e = link(p, st, p->origin, ns);
  if (e != hipSuccess) return LACE_EHIP;
  if (!p->graph.exec || p->graph.key != key) {
    if (p->graph.exec) { (void)hipGraphExecDestroy(p->graph.exec); p->graph.exec = nullptr; }
    if (p->graph.graph) { (void)hipGraphDestroy(p->graph.graph); p->graph.graph = nullptr; }
    e = hipStreamBeginCapture(p->origin, hipStreamCaptureModeThreadLocal);
    for (int q = 0; q < ns && e == hipSuccess; ++q)
      e = link(p, p->origin, p->streams[q], q);
    hipError_t r = (e == hipSuccess) ? enqueue_all() : e;
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

