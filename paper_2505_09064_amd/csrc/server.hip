// Serving engine: continuous batching of independent V-ASMG-PCG solve requests
// (one mesh + one load case each) on one GPU.
//
// A request's life: submit (inputs deep-copied) -> host setup by one of the
// setup workers (the region-tree hierarchy, the expensive step of the method)
// -> admission, first in first out, as soon as a device slot is free and the
// request's device bytes fit the HBM budget next to the hierarchies already
// resident -> upload, solve and free on the slot's own non-blocking stream
// (stream-ordered allocations, so one request's upload or free never waits for
// another's kernels) -> result waiting for vasmg_server_wait. Requests that
// arrive while others are on the device are set up in parallel with them and
// admitted as slots and memory free up; their kernels overlap on the GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/vasmg.h"

namespace vasmg {
void set_host_threads(int n);   // setup.cpp: OpenMP threads of the calling thread's setups
int host_thread_budget();       // setup.cpp: the default OpenMP team size
}

namespace {

using Clock = std::chrono::steady_clock;

// Packed coarsest levels stay within the size the coarse solve applies as one
// explicit inverse.
constexpr int64_t kPackCoarseMax = 256;

struct Request {
  int64_t id = 0;
  int32_t dim = 0;
  int64_t nv = 0, ne = 0;
  std::vector<double> coords, E, nu, rhs, x;
  std::vector<int32_t> elems;
  std::vector<uint8_t> fixed;
  double rtol = 1e-6;
  vasmg_handle h = nullptr;
  int64_t bytes = 0;
  int64_t dofs = 0, coarse_dofs = 0;   // fine and coarsest-level DOFs of the hierarchy
  bool done = false;
  vasmg_request_result res{};
};

using ReqPtr = std::shared_ptr<Request>;

}  // namespace

struct vasmg_server {
  vasmg_server_config cfg{};
  Clock::time_point t0;
  int device = 0;
  int64_t budget = 0;

  std::mutex mu;
  std::condition_variable cv;
  std::deque<ReqPtr> setup_q, admit_q;
  std::unordered_map<int64_t, ReqPtr> reqs;
  int64_t next_id = 0;
  int64_t in_use = 0, peak = 0;
  int setups_active = 0, running = 0;
  int64_t submitted = 0, completed = 0;
  bool stop = false;
  std::vector<std::thread> workers;

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
  }

  static void note(const ReqPtr& r, const char* what, const char* why) {
    if (r->res.message[0]) return;       // keep the first failure
    std::snprintf(r->res.message, sizeof(r->res.message), "%s: %s", what, why ? why : "");
  }

  // caller holds mu; t_done < 0: now
  void finish(const ReqPtr& r, int status, double t_done = -1.0) {
    r->res.status = status;
    r->res.t_done_ms = t_done < 0.0 ? now_ms() : t_done;
    r->done = true;
    ++completed;
    cv.notify_all();
  }

  // hw_threads: the host's threads; a setup takes its share among the setups
  // running or queued when it starts (a lone large mesh gets them all). The
  // hierarchy does not depend on the thread count.
  void setup_loop(int hw_threads) {
    if (cfg.options.setup_device) (void)hipSetDevice(device);   // device Galerkin products
    for (;;) {
      ReqPtr r;
      {
        std::unique_lock<std::mutex> g(mu);
        cv.wait(g, [&] { return stop || !setup_q.empty(); });
        if (setup_q.empty()) return;       // stopping and nothing left to set up
        r = setup_q.front();
        setup_q.pop_front();
        ++setups_active;
        // setups running or about to start (queued requests go to idle workers)
        const int busy = std::min(cfg.setup_workers,
                                  setups_active + static_cast<int>(setup_q.size()));
        vasmg::set_host_threads(std::max(1, hw_threads / std::max(1, busy)));
      }
      r->res.t_setup_start_ms = now_ms();
      vasmg_mesh m{r->dim, r->nv, r->coords.data(), r->ne, r->elems.data(),
                   r->E.data(), r->nu.data(), r->fixed.data()};
      vasmg_options o = cfg.options;
      o.host_only = 1;
      o.block_rhs = 0;
      const int64_t mesh_dofs = static_cast<int64_t>(r->nv) * r->dim;
      if (mesh_dofs <= (r->dim == 2 ? cfg.host_setup_max_dofs_2d : cfg.host_setup_max_dofs_3d))
        o.setup_device = 0;
      r->res.setup_device = o.setup_device ? 1 : 0;
      vasmg_handle h = nullptr;
      int st = vasmg_setup(&m, &o, &h);
      if (st != VASMG_OK) note(r, "setup", vasmg_last_error());
      int64_t bytes = 0;
      if (st == VASMG_OK) st = vasmg_device_bytes(h, &bytes);
      if (st == VASMG_OK) {
        int32_t nl = 0, dim = 0;
        int64_t nd = 0, nvc = 0, nb = 0, pn = 0;
        int32_t nc = 0;
        st = vasmg_hierarchy_info(h, &nl, &nd, &dim);
        if (st == VASMG_OK) st = vasmg_level_info(h, nl - 1, &nvc, &nb, &nc, &pn);
        r->dofs = nd;
        r->coarse_dofs = nvc * dim;
      }
      r->res.t_setup_end_ms = now_ms();
      // the mesh copies are no longer needed
      std::vector<double>().swap(r->coords);
      std::vector<int32_t>().swap(r->elems);
      std::lock_guard<std::mutex> g(mu);
      --setups_active;
      if (st == VASMG_OK && bytes > budget) {
        st = VASMG_ENOMEM;
        note(r, "admission", "device bytes exceed the whole budget");
      }
      if (st != VASMG_OK) {
        if (h) vasmg_free(h);
        finish(r, st);
        continue;
      }
      r->h = h;
      r->bytes = bytes;
      r->res.device_bytes = bytes;
      admit_q.push_back(r);
      cv.notify_all();
    }
  }

  bool packable(const Request& q) const {
    const vasmg_options& o = cfg.options;
    return cfg.pack_max_dofs > 0 && cfg.pack_max_parts > 1 && q.dofs <= cfg.pack_max_dofs &&
           o.preconditioner == VASMG_PRECOND_VASMG && o.cycle == VASMG_CYCLE_V &&
           o.smoother == VASMG_SMOOTHER_GS && o.color_blocks == 0;
  }

  // One request alone on the slot: upload, solve, result back. Returns its status;
  // r->bytes ends as the device bytes it held.
  int run_single(hipStream_t st, bool have_stream, const ReqPtr& r) {
    int status = have_stream ? vasmg_upload(r->h, st) : VASMG_EDEVICE;
    if (status != VASMG_OK) note(r, "upload", have_stream ? vasmg_last_error() : "no stream");
    double *d_rhs = nullptr, *d_x = nullptr;
    const size_t vbytes = sizeof(double) * static_cast<size_t>(r->nv) * r->dim;
    if (status == VASMG_OK) {
      int64_t actual = 0;
      vasmg_device_bytes(r->h, &actual);
      actual += 2 * static_cast<int64_t>(vbytes);
      std::lock_guard<std::mutex> g(mu);
      in_use += actual - r->bytes;       // the estimate is an upper bound
      r->bytes = actual;
      r->res.device_bytes = actual;
      peak = std::max(peak, in_use);
    }
    if (status == VASMG_OK) {
      hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&d_rhs), vbytes, st);
      if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void**>(&d_x), vbytes, st);
      if (e == hipSuccess) e = hipMemcpyAsync(d_rhs, r->rhs.data(), vbytes, hipMemcpyHostToDevice, st);
      if (e != hipSuccess) {
        status = VASMG_ENOMEM;
        note(r, "vectors", hipGetErrorString(e));
      }
    }
    if (status == VASMG_OK) {
      status = vasmg_solve_device(r->h, d_rhs, nullptr, d_x, 1, r->rtol, st, &r->res.info);
      if (status != VASMG_OK) note(r, "solve", vasmg_last_error());
      r->x.resize(static_cast<size_t>(r->nv) * r->dim);
      hipError_t e = hipMemcpyAsync(r->x.data(), d_x, vbytes, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) {
        status = VASMG_EDEVICE;
        note(r, "result copy", hipGetErrorString(e));
      }
    }
    if (d_rhs) (void)hipFreeAsync(d_rhs, st);
    if (d_x) (void)hipFreeAsync(d_x, st);
    vasmg_free(r->h);                    // stream-ordered frees on st
    r->h = nullptr;
    if (have_stream) (void)hipStreamSynchronize(st);   // memory back before it is counted free
    return status;
  }

  // Small requests packed into one handle (vasmg_pack): one upload, one solve
  // with a PCG recurrence per request, results split back. statuses[i] per request.
  void run_pack(hipStream_t st, bool have_stream, const std::vector<ReqPtr>& batch,
                std::vector<int>& statuses, int64_t& held) {
    const int n = static_cast<int>(batch.size());
    statuses.assign(n, VASMG_OK);
    std::vector<vasmg_handle> hs;
    int64_t nv = 0;
    for (const ReqPtr& r : batch) {
      hs.push_back(r->h);
      nv += r->nv;
    }
    const int dim = batch[0]->dim;
    vasmg_handle ph = nullptr;
    int status = have_stream ? vasmg_pack(hs.data(), n, &ph) : VASMG_EDEVICE;
    const char* what = "pack";
    if (status == VASMG_OK) {
      status = vasmg_upload(ph, st);
      what = "upload";
    }
    std::string why = status == VASMG_OK ? "" : (have_stream ? vasmg_last_error() : "no stream");
    for (const ReqPtr& r : batch) {   // the host hierarchies are in the packed handle now
      vasmg_free(r->h);
      r->h = nullptr;
    }
    double *d_rhs = nullptr, *d_x = nullptr;
    const size_t vbytes = sizeof(double) * static_cast<size_t>(nv) * dim;
    if (status == VASMG_OK) {
      int64_t actual = 0;
      vasmg_device_bytes(ph, &actual);
      actual += 2 * static_cast<int64_t>(vbytes);
      std::lock_guard<std::mutex> g(mu);
      in_use += actual - held;
      held = actual;
      peak = std::max(peak, in_use);
    }
    std::vector<double> stage;
    if (status == VASMG_OK) {
      stage.resize(static_cast<size_t>(nv) * dim);
      size_t o = 0;
      for (const ReqPtr& r : batch) {
        std::copy(r->rhs.begin(), r->rhs.end(), stage.begin() + o);
        o += r->rhs.size();
      }
      hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&d_rhs), vbytes, st);
      if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void**>(&d_x), vbytes, st);
      if (e == hipSuccess) e = hipMemcpyAsync(d_rhs, stage.data(), vbytes, hipMemcpyHostToDevice, st);
      if (e != hipSuccess) {
        status = VASMG_ENOMEM;
        what = "vectors";
        why = hipGetErrorString(e);
      }
    }
    std::vector<vasmg_solve_info> infos(n);
    if (status == VASMG_OK) {
      const int s = vasmg_solve_packed_device(ph, d_rhs, d_x, batch[0]->rtol, st, infos.data());
      hipError_t e = hipMemcpyAsync(stage.data(), d_x, vbytes, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) {
        status = VASMG_EDEVICE;
        what = "result copy";
        why = hipGetErrorString(e);
      } else if (s != VASMG_OK && s != VASMG_ENOTCONV && s != VASMG_EBREAKDOWN) {
        status = s;
        what = "solve";
        why = vasmg_last_error();
      }
    }
    size_t o = 0;
    for (int i = 0; i < n; ++i) {
      const ReqPtr& r = batch[i];
      if (status != VASMG_OK) {
        statuses[i] = status;
        note(r, what, why.c_str());
        continue;
      }
      r->res.info = infos[i];
      r->x.assign(stage.begin() + o, stage.begin() + o + r->rhs.size());
      o += r->rhs.size();
      statuses[i] = infos[i].status;
      if (statuses[i] != VASMG_OK)
        note(r, "solve", statuses[i] == VASMG_ENOTCONV ? "PCG did not reach rtol within max_iters"
                                                      : "PCG breakdown");
      r->res.device_bytes = held;
    }
    if (d_rhs) (void)hipFreeAsync(d_rhs, st);
    if (d_x) (void)hipFreeAsync(d_x, st);
    vasmg_free(ph);
    if (have_stream) (void)hipStreamSynchronize(st);
  }

  void slot_loop(int slot) {
    (void)hipSetDevice(device);
    hipStream_t st = nullptr;
    const bool have_stream = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    for (;;) {
      std::vector<ReqPtr> batch;
      int64_t held = 0;
      {
        std::unique_lock<std::mutex> g(mu);
        cv.wait(g, [&] {
          if (!admit_q.empty() && in_use + admit_q.front()->bytes <= budget) return true;
          return stop && admit_q.empty() && setup_q.empty() && setups_active == 0;
        });
        if (admit_q.empty()) break;        // stopping and nothing left to run
        const ReqPtr r0 = admit_q.front();
        admit_q.pop_front();
        batch.push_back(r0);
        held = r0->bytes;
        if (packable(*r0)) {
          // small requests set up and waiting behind it join it: same dimension
          // and tolerance, their coarsest levels together within kPackCoarseMax
          int64_t coarse = r0->coarse_dofs;
          auto gather = [&] {
            for (auto it = admit_q.begin();
                 it != admit_q.end() && static_cast<int>(batch.size()) < cfg.pack_max_parts;) {
              const ReqPtr& q = *it;
              if (packable(*q) && q->dim == r0->dim && q->rtol == r0->rtol &&
                  coarse + q->coarse_dofs <= kPackCoarseMax && in_use + held + q->bytes <= budget) {
                coarse += q->coarse_dofs;
                held += q->bytes;
                batch.push_back(q);
                it = admit_q.erase(it);
              } else {
                ++it;
              }
            }
          };
          gather();
          // batching window: while setups are still running, wait up to
          // pack_wait_ms for more small requests (each finished setup wakes us)
          const auto deadline = Clock::now() + std::chrono::milliseconds(cfg.pack_wait_ms);
          while (cfg.pack_wait_ms > 0 && static_cast<int>(batch.size()) < cfg.pack_max_parts &&
                 (setups_active > 0 || !setup_q.empty())) {
            const bool timed_out = cv.wait_until(g, deadline) == std::cv_status::timeout;
            gather();
            if (timed_out) break;
          }
        }
        in_use += held;
        peak = std::max(peak, in_use);
        running += static_cast<int>(batch.size());
      }
      const double t_admit = now_ms();
      for (const ReqPtr& r : batch) {
        r->res.t_admit_ms = t_admit;
        r->res.slot = slot;
        r->res.pack_size = static_cast<int32_t>(batch.size());
      }
      std::vector<int> statuses;
      if (batch.size() == 1) {
        statuses.push_back(run_single(st, have_stream, batch[0]));
        held = batch[0]->bytes;
      } else {
        run_pack(st, have_stream, batch, statuses, held);
      }
      std::lock_guard<std::mutex> g(mu);
      in_use -= held;
      running -= static_cast<int>(batch.size());
      const double t_done = now_ms();   // a pack's requests complete together
      for (size_t i = 0; i < batch.size(); ++i) finish(batch[i], statuses[i], t_done);
    }
    if (have_stream) (void)hipStreamDestroy(st);
  }
};

extern "C" {

vasmg_status vasmg_server_default_config(vasmg_server_config* cfg) {
  if (!cfg) return VASMG_EINVAL;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->slots = 4;
  cfg->setup_workers = 4;
  cfg->hbm_budget_bytes = 0;
  cfg->pack_max_dofs = 0;
  cfg->pack_max_parts = 16;
  cfg->pack_wait_ms = 0;
  cfg->host_setup_max_dofs_2d = 131072;
  cfg->host_setup_max_dofs_3d = 16384;
  const vasmg_status st = vasmg_default_options(3, &cfg->options);
  cfg->options.leaf_capacity = 0;          // each request: its dimension's default
  return st;
}

vasmg_status vasmg_server_create(const vasmg_server_config* cfg, vasmg_server_handle* out) {
  if (!cfg || !out) return VASMG_EINVAL;
  *out = nullptr;
  if (cfg->slots < 1 || cfg->slots > 64 || cfg->setup_workers < 1 || cfg->setup_workers > 64 ||
      cfg->hbm_budget_bytes < 0 || cfg->pack_max_dofs < 0 || cfg->pack_max_parts < 0 ||
      cfg->pack_max_parts > 256 || cfg->pack_wait_ms < 0 || cfg->pack_wait_ms > 10000 ||
      cfg->host_setup_max_dofs_2d < 0 || cfg->host_setup_max_dofs_3d < 0)
    return VASMG_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return VASMG_EDEVICE;
  auto s = std::make_unique<vasmg_server>();
  s->cfg = *cfg;
  s->cfg.options.autotune = 0;             // a request's result must not depend on the mix
  s->t0 = Clock::now();
  if (hipGetDevice(&s->device) != hipSuccess) return VASMG_EDEVICE;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return VASMG_EDEVICE;
  s->budget = cfg->hbm_budget_bytes > 0 ? cfg->hbm_budget_bytes
                                        : static_cast<int64_t>(0.8 * static_cast<double>(free_b));
  // the process's share of the host (OMP_NUM_THREADS where set), not every core
  const int hw = std::max(1, std::min(static_cast<int>(std::thread::hardware_concurrency()),
                                      vasmg::host_thread_budget()));
  vasmg_server* sp = s.get();
  for (int i = 0; i < cfg->setup_workers; ++i)
    s->workers.emplace_back([sp, hw] { sp->setup_loop(hw); });
  for (int i = 0; i < cfg->slots; ++i) s->workers.emplace_back([sp, i] { sp->slot_loop(i); });
  *out = s.release();
  return VASMG_OK;
}

vasmg_status vasmg_server_submit(vasmg_server_handle s, const vasmg_mesh* mesh, const double* rhs,
                                 double rtol, int64_t* id) {
  if (!s || !mesh || !rhs || !id || (mesh->dim != 2 && mesh->dim != 3) || mesh->n_vertices < 1 ||
      mesh->n_elements < 1 || !mesh->coords || !mesh->elems || !mesh->E || !mesh->nu ||
      !mesh->fixed || !(rtol > 0.0))
    return VASMG_EINVAL;
  auto r = std::make_shared<Request>();
  const int d = mesh->dim;
  const int64_t nv = mesh->n_vertices, ne = mesh->n_elements;
  r->dim = d;
  r->nv = nv;
  r->ne = ne;
  r->coords.assign(mesh->coords, mesh->coords + nv * d);
  r->elems.assign(mesh->elems, mesh->elems + ne * (d + 1));
  r->E.assign(mesh->E, mesh->E + ne);
  r->nu.assign(mesh->nu, mesh->nu + ne);
  r->fixed.assign(mesh->fixed, mesh->fixed + nv * d);
  r->rhs.assign(rhs, rhs + nv * d);
  r->rtol = rtol;
  r->res.slot = -1;
  std::lock_guard<std::mutex> g(s->mu);
  if (s->stop) return VASMG_EINVAL;
  r->id = s->next_id++;
  r->res.id = r->id;
  r->res.t_submit_ms = s->now_ms();
  s->reqs[r->id] = r;
  s->setup_q.push_back(r);
  ++s->submitted;
  *id = r->id;
  s->cv.notify_all();
  return VASMG_OK;
}

vasmg_status vasmg_server_wait(vasmg_server_handle s, int64_t id, double* x,
                               vasmg_request_result* res) {
  if (!s) return VASMG_EINVAL;
  std::unique_lock<std::mutex> g(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return VASMG_EINVAL;
  ReqPtr r = it->second;
  s->cv.wait(g, [&] { return r->done; });
  s->reqs.erase(it);
  g.unlock();
  if (x && !r->x.empty()) std::memcpy(x, r->x.data(), sizeof(double) * r->x.size());
  if (x && r->x.empty()) std::memset(x, 0, sizeof(double) * static_cast<size_t>(r->nv) * r->dim);
  if (res) *res = r->res;
  return static_cast<vasmg_status>(r->res.status);
}

vasmg_status vasmg_server_stats(vasmg_server_handle s, vasmg_server_counters* out) {
  if (!s || !out) return VASMG_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->waiting_setup = static_cast<int64_t>(s->setup_q.size()) + s->setups_active;
  out->waiting_admission = static_cast<int64_t>(s->admit_q.size());
  out->running = s->running;
  out->bytes_in_use = s->in_use;
  out->peak_bytes = s->peak;
  out->budget_bytes = s->budget;
  out->t_now_ms = s->now_ms();
  return VASMG_OK;
}

void vasmg_server_destroy(vasmg_server_handle s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    s->cv.notify_all();
  }
  for (auto& t : s->workers) t.join();
  for (auto& kv : s->reqs)
    if (kv.second->h) vasmg_free(kv.second->h);
  delete s;
}

}  // extern "C"
