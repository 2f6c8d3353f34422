// Drives the library's host layer from several threads at once, each with
// its own plan, workspace and buffers (the serving loop's use), through
// every entry point.  Built with the stand-in runtime and launchers under
// the thread or the address and undefined-behaviour sanitizers.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

#include "lace.h"

#define CHECK(x)                                                        \
  do {                                                                  \
    int rc_ = (x);                                                      \
    if (rc_ != LACE_OK) {                                               \
      std::fprintf(stderr, "%s:%d %s -> %d\n", __FILE__, __LINE__, #x, rc_); \
      std::exit(3);                                                     \
    }                                                                   \
  } while (0)

static std::vector<int32_t> sphere(int mmax) {
  std::vector<int32_t> m;
  for (int z = -mmax; z <= mmax; ++z)
    for (int y = -mmax; y <= mmax; ++y)
      for (int x = -mmax; x <= mmax; ++x)
        if (x * x + y * y + z * z <= mmax * mmax) {
          m.push_back(x); m.push_back(y); m.push_back(z);
        }
  return m;
}

// lace_apply_ace_noalloc shares one scratch array per GPU: its callers
// order their calls, as its contract asks.
static std::mutex noalloc_order;

static void worker(int t, int reps) {
  const lace_precision precs[4] = {LACE_FP32_GAMMA, LACE_FP32, LACE_FP64,
                                   LACE_FP64_GAMMA};
  const lace_precision prec = precs[t % 4];
  std::vector<int32_t> m0 = sphere(3), m1 = sphere(5);
  lace_cell_desc cells[2] = {};
  cells[0].L = 10.0; cells[0].n = 8; cells[0].n_pw = (int64_t)m0.size() / 3;
  cells[0].miller = m0.data();
  cells[1].L = 16.0; cells[1].n = 12; cells[1].n_pw = (int64_t)m1.size() / 3;
  cells[1].miller = m1.data();
  lace_plan* plan = nullptr;
  CHECK(lace_plan_create(cells, 2, prec, &plan));
  const int n_orb[2] = {37 + t, 70};
  std::vector<void*> own;
  auto dev = [&](size_t bytes) {
    void* p = std::calloc(bytes, 1);
    own.push_back(p);
    return p;
  };
  for (int rep = 0; rep < reps; ++rep) {
    for (int c = 0; c < 2; ++c) {
      const int n = n_orb[c];
      const int64_t npw = cells[c].n_pw;
      size_t wsb = 0;
      CHECK(lace_workspace_size(plan, c, n, n, &wsb));
      void* ws = dev(wsb);
      void* psi = dev(16 * npw * n);
      void* psi2 = dev(16 * npw * n);
      void* w = dev(16 * npw * n);
      void* xi = dev(16 * npw * n);
      void* y = dev(16 * npw * n);
      void* m = dev(16 * (size_t)n * n);
      double* s = static_cast<double*>(dev(8 * (size_t)n * n));
      double* e = static_cast<double*>(dev(64));
      int32_t* info = static_cast<int32_t*>(dev(64));
      int32_t* pts = static_cast<int32_t*>(dev(4 * (size_t)n));
      int64_t* kept = static_cast<int64_t*>(dev(64));
      int32_t* klist = static_cast<int32_t*>(dev(4 * (size_t)n * (n + 1)));
      CHECK(lace_screen(plan, c, psi, n, s, ws, wsb, nullptr));
      for (double thr : {0.0, 0.05, 0.4})
        CHECK(lace_apply_exchange(plan, c, psi, n, thr, nullptr, nullptr, 0, w,
                                  e, kept, thr > 0.1 ? klist : nullptr, ws, wsb,
                                  nullptr));
      std::vector<int32_t> pi, pj;
      for (int j = 0; j < n; ++j)
        for (int i = 0; i <= j; i += 3) { pi.push_back(i); pj.push_back(j); }
      int32_t* dpi = static_cast<int32_t*>(dev(4 * pi.size()));
      int32_t* dpj = static_cast<int32_t*>(dev(4 * pj.size()));
      std::memcpy(dpi, pi.data(), 4 * pi.size());
      std::memcpy(dpj, pj.data(), 4 * pj.size());
      CHECK(lace_apply_exchange(plan, c, psi, n, 0.0, dpi, dpj,
                                (int64_t)pi.size(), w, e, kept, nullptr, ws, wsb,
                                nullptr));
      int32_t bo[8], so[8];
      int64_t nbr = 0;
      CHECK(lace_read_schedule(plan, c, n, ws, nullptr, pi.data(), pj.data(), 8,
                               bo, so, &nbr));
      CHECK(lace_apply_exchange_virtual(plan, c, psi, n - 5, 5, 0.1, w, e,
                                        nullptr, ws, wsb, nullptr));
      for (int sym = 0; sym < 3; ++sym)
        CHECK(lace_build_ace(plan, c, psi, w, n, (lace_sym)sym, xi, m, e + 1,
                             sym == 1 ? info : nullptr, ws, wsb, nullptr));
      int32_t hinfo = -1;
      CHECK(lace_get_info(ws, nullptr, &hinfo));
      CHECK(lace_apply_ace(plan, c, xi, n, psi, n, y, ws, wsb, nullptr));
      {
        std::lock_guard<std::mutex> order(noalloc_order);
        CHECK(lace_apply_ace_noalloc(plan, c, xi, n, psi, n, y, nullptr));
      }
      CHECK(lace_align(plan, c, psi, psi2, n, y, e + 2, ws, wsb, nullptr));
      CHECK(lace_scdm(plan, c, psi, n, y, pts, e + 3, ws, wsb, nullptr));
      double dev_real = 0;
      if (prec == LACE_FP32_GAMMA || prec == LACE_FP64_GAMMA)
        CHECK(lace_check_real(plan, c, psi, n, ws, wsb, nullptr, &dev_real));
      int ppb[16], pl[16], nc = 16;
      double us[16];
      int zt[16], ro[16];
      CHECK(lace_autotune(plan, c, psi, n, 0.1, ws, wsb, nullptr, ppb, pl, zt, ro, us, &nc));
      CHECK(lace_profile_enable(plan, 1));
      CHECK(lace_apply_exchange(plan, c, psi, n, 0.05, nullptr, nullptr, 0, w,
                                e, kept, nullptr, ws, wsb, nullptr));
      double ms[3], bytes[3];
      int64_t la[3], pr[3];
      CHECK(lace_profile_read(plan, ms, la, pr, bytes));
      CHECK(lace_profile_enable(plan, 0));
      CHECK(lace_fft3d(plan, c, -1, w, 1, nullptr));
    }
    // two jobs per cell in one batched call, eager and as a graph
    lace_job jobs[4] = {};
    for (int k = 0; k < 4; ++k) {
      const int c = k % 2, n = n_orb[c];
      const int64_t npw = cells[c].n_pw;
      size_t wsb = 0;
      CHECK(lace_workspace_size(plan, c, n, 0, &wsb));
      jobs[k].cell = c;
      jobs[k].psi_g = dev(16 * npw * n);
      jobs[k].n_orb = n;
      jobs[k].s_thr = k < 2 ? 0.0 : 0.05;
      jobs[k].w_g = dev(16 * npw * n);
      jobs[k].e_x = static_cast<double*>(dev(8));
      jobs[k].n_kept = static_cast<int64_t*>(dev(8));
      jobs[k].sym = k % 3;
      jobs[k].xi_g = dev(16 * npw * n);
      jobs[k].m_out = dev(16 * (size_t)n * n);
      jobs[k].ex_tr = static_cast<double*>(dev(8));
      jobs[k].info = k == 3 ? static_cast<int32_t*>(dev(4)) : nullptr;
      jobs[k].ws = dev(wsb);
      jobs[k].ws_bytes = wsb;
    }
    CHECK(lace_apply_exchange_batched(plan, jobs, 4, 0, nullptr));
    CHECK(lace_apply_exchange_batched(plan, jobs, 4, LACE_BATCH_GRAPH, nullptr));
    CHECK(lace_apply_exchange_batched(plan, jobs, 4, LACE_BATCH_GRAPH, nullptr));
    for (void* p : own) std::free(p);
    own.clear();
  }
  CHECK(lace_plan_destroy(plan));
}

int main(int argc, char** argv) {
  const int threads = argc > 1 ? std::atoi(argv[1]) : 4;
  const int reps = argc > 2 ? std::atoi(argv[2]) : 2;
  std::vector<std::thread> th;
  for (int t = 0; t < threads; ++t) th.emplace_back(worker, t, reps);
  for (auto& x : th) x.join();
  // host-only schedules
  std::vector<int32_t> pi, pj;
  for (int j = 0; j < 50; ++j)
    for (int i = 0; i <= j; ++i) { pi.push_back(i); pj.push_back(j); }
  std::vector<int32_t> bo(pi.size()), so(pi.size());
  int64_t nb = 0;
  CHECK(lace_schedule_pairs(pi.data(), pj.data(), (int64_t)pi.size(), 50, 16,
                            bo.data(), &nb));
  CHECK(lace_schedule_slots(pi.data(), pj.data(), (int64_t)pi.size(), 50, 16,
                            bo.data(), so.data(), &nb));
  std::printf("host layer: %d threads x %d reps ok\n", threads, reps);
  return 0;
}
