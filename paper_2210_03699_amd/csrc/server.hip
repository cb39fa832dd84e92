// Solve server: continuous batching of independent CTR-IBIM solves on one GPU.
//
// A request moves through: submitted -> host setup on a background thread
// (geometry and correction sets) -> waiting for admission -> device setup on
// one of two admission threads (uploads, correction weights, Krylov basis; a
// stream each) -> active -> done (G_pol and the solution kept on the host;
// its device memory freed on the reaper thread) or failed.  Each round of
// the direct-sum solves does one persistent batched pair-kernel launch over
// the work items of all of them, one batched finishing launch per precision
// and one launch per GMRES stage; the solves that the options send to the
// treecode run their rounds (their own launches, then one launch per GMRES
// stage) on a second stream, each round started when the previous one has
// completed.  Every request gets the blocks and reduction order of
// ibim_solve and ibim_energy, so results do not depend on the mix of requests.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ibim.h"
#include "context.h"
#include "krylov.h"
#include "operator.h"

using namespace ibim;

namespace {

enum class Phase { kIter, kResid };

struct Request {
  int64_t ticket = 0;
  // inputs (released after the host setup)
  std::vector<double> sdf;
  int dims[3] = {0, 0, 0};
  double origin[3] = {0, 0, 0};
  double h = 0, eps = 0, eps_in = 0, eps_out = 0, kappa = 0, tol = 0;
  std::vector<double> zq, q;
  // lifecycle
  int state = IBIM_REQ_WAITING;
  bool prepared = false;  // host setup finished (guarded by the server mutex)
  int error = 0;
  std::string error_msg;
  ibim_ctx* ctx = nullptr;
  size_t estimate = 0;
  size_t held = 0;  // device bytes charged to the budget (the estimate while admitting)
  size_t setup_bytes = 0;  // device bytes once set up
  int admit_error = 0;     // result of the device setup on the admission thread
  std::string admit_msg;
  int slot = -1;
  double* d_b = nullptr;  // right-hand side
  double* d_x = nullptr;  // iterate
  DeviceArena arena;      // the block its device setup allocated from
  // GMRES state (the driver of ibim_solve, one step per round)
  Phase phase = Phase::kIter;
  bool final_check = false;
  int j = 0, total = 0;
  double bnorm = -1.0, resid = 0.0, explicit_rel = -1.0;
  bool converged = false;
  // results
  double g_pol = 0.0;
  std::vector<double> x_host;
  int64_t M = 0;
  std::chrono::steady_clock::time_point t_submit, t_admit;
  double seconds = 0.0;
  int applies = 0;
};

}  // namespace

struct ibim_server {
  ibim_options opt{};
  size_t budget = 0, used = 0, peak = 0;
  int max_slots = 1;
  hipStream_t stream = nullptr;
  // device setup of newly admitted requests (uploads, weights, right-hand
  // side) runs on these streams, one per admission thread, while the rounds
  // execute
  static constexpr int kAdmitters = 2;
  hipStream_t setup[kAdmitters] = {};
  int grid = 0;
  int64_t next_ticket = 1;
  std::map<int64_t, std::unique_ptr<Request>> reqs;
  std::vector<Request*> waiting;  // submission order
  std::vector<Request*> active;       // direct-sum solves: one round per step on `stream`
  std::vector<Request*> tree_active;  // treecode solves: rounds on `tstream`
  std::vector<Request*> tree_round;   // the treecode solves of the round in flight
  bool tree_busy = false;             // a treecode round is in flight (tevent marks its end)
  hipStream_t tstream = nullptr;
  hipEvent_t tevent = nullptr;
  std::vector<int> free_slots;
  ibim_server_stats st{};
  // device buffers of the batched launch and of the per-round status
  PairArgs* d_args = nullptr;
  PairArgs* h_args = nullptr;
  size_t args_cap = 0;
  int32_t* d_items = nullptr;
  int32_t* h_items = nullptr;
  size_t items_cap = 0;
  // problems on the symmetric float64 kernel and their (problem, item) list
  SymArgs* d_sargs = nullptr;
  SymArgs* h_sargs = nullptr;
  size_t sargs_cap = 0;
  int32_t* d_swork = nullptr;
  int32_t* h_swork = nullptr;
  size_t swork_cap = 0;
  KrylovStepArgs* d_steps = nullptr;  // batched GMRES step of the solves in Arnoldi phase
  KrylovStepArgs* h_steps = nullptr;
  size_t steps_cap = 0;
  KrylovStepArgs* d_tsteps = nullptr;  // the same for the treecode rounds
  KrylovStepArgs* h_tsteps = nullptr;
  size_t tsteps_cap = 0;
  SymFinishArgs* d_fin = nullptr;  // batched finishing launches (float64, mixed)
  SymFinishArgs* h_fin = nullptr;
  size_t fin_cap = 0;
  SymMixedFinishArgs* d_finm = nullptr;
  SymMixedFinishArgs* h_finm = nullptr;
  size_t finm_cap = 0;
  int sym_grid = 0;
  int* d_counter = nullptr;  // two counters: one-directional and symmetric launches
  double* d_status = nullptr;   // 8 doubles per slot
  double* h_status = nullptr;   // pinned, copied at the end of each direct round
  double* h_tstatus = nullptr;  // pinned, copied at the end of each treecode round
  // background host setup
  std::mutex mu;
  std::condition_variable cv;        // work for the setup threads
  std::condition_variable ready_cv;  // a host setup finished
  std::deque<Request*> prep_queue;
  std::vector<std::thread> workers;
  bool stopping = false;
  // device memory of finished or failed requests is freed on its own thread
  // (each hipFree waits for the device), so rounds do not stall on it; the
  // bytes still held count against the budget until they are freed.  A
  // request's setup allocates from one block (DeviceArena), so freeing it
  // takes one such wait, not one per array
  struct Reap {
    ibim_ctx* ctx;
    double *b, *x;
    DeviceArena arena;
    size_t bytes;
  };
  std::deque<Reap> reap_queue;
  std::condition_variable reap_cv;
  size_t reaping = 0;  // bytes queued or being freed (under mu)
  bool reap_stop = false;
  std::thread reaper;
  // device setup of admitted requests while rounds run: the main thread
  // reserves a slot and the estimated bytes and queues the request; the
  // admission thread sets it up on the setup stream; the next round picks it up
  std::deque<Request*> admit_queue;
  std::vector<Request*> admitted;     // set up (or failed), not yet picked up
  std::condition_variable admit_cv;   // work for the admission threads
  std::condition_variable admitted_cv;
  int admitting = 0;                  // queued or being set up (main thread)
  bool admit_stop = false;
  std::thread admitter[kAdmitters];
};

namespace {

constexpr int kStatusStride = 8;  // per slot: |g_{j+1}|, H(j+1,j), ||b||^2, ||r||^2

__global__ void zero_ints_kernel(int* p, int n) {
  if (blockIdx.x == 0 && (int)threadIdx.x < n) p[threadIdx.x] = 0;
}

void worker_main(ibim_server* srv, int omp_threads) {
  // the setup threads share the host cores instead of each starting a full team
  set_host_setup_threads(omp_threads);
  for (;;) {
    Request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      srv->cv.wait(lk, [&] { return srv->stopping || !srv->prep_queue.empty(); });
      if (srv->stopping && srv->prep_queue.empty()) return;
      r = srv->prep_queue.front();
      srv->prep_queue.pop_front();
    }
    ibim_options o = srv->opt;
    ibim_ctx* c = nullptr;
    const int code = ctx_create_host(r->sdf.data(), r->dims[0], r->dims[1], r->dims[2],
                                     r->origin, r->h, r->eps, r->eps_in, r->eps_out, r->kappa,
                                     r->zq.data(), r->q.data(), (int)r->q.size(), o, &c);
    std::string msg = code ? std::string(ibim_last_error()) : std::string();
    size_t est = c ? ctx_footprint_estimate(c) + 4 * 2 * (size_t)c->plan.M * 8 : 0;
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      r->ctx = c;
      r->error = code;
      r->error_msg = msg;
      r->estimate = est;
      std::vector<double>().swap(r->sdf);
      r->prepared = true;
    }
    srv->ready_cv.notify_all();
  }
}

void reaper_main(ibim_server* srv) {
  (void)hipSetDevice(srv->opt.device);
  for (;;) {
    ibim_server::Reap job;
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      srv->reap_cv.wait(lk, [&] { return srv->reap_stop || !srv->reap_queue.empty(); });
      if (srv->reap_queue.empty()) return;  // stopping and drained
      job = srv->reap_queue.front();
      srv->reap_queue.pop_front();
    }
    ibim_destroy(job.ctx);
    dfree(job.b);
    dfree(job.x);
    arena_release(&job.arena);
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->reaping -= job.bytes;
  }
}

size_t reaping_bytes(ibim_server* srv) {
  std::lock_guard<std::mutex> lk(srv->mu);
  return srv->reaping;
}

void release_device(ibim_server* srv, Request* r) {
  if (r->ctx || r->d_b || r->d_x || r->arena.base) {
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      srv->reap_queue.push_back(ibim_server::Reap{r->ctx, r->d_b, r->d_x, r->arena, r->held});
      srv->reaping += r->held;
    }
    srv->reap_cv.notify_one();
    r->ctx = nullptr;
    r->d_b = nullptr;
    r->d_x = nullptr;
    r->arena = DeviceArena{};
  }
  srv->used -= r->held;
  r->held = 0;
  if (r->slot >= 0) srv->free_slots.push_back(r->slot);
  r->slot = -1;
}

void mark_failed(ibim_server* srv, Request* r, int code, const std::string& msg) {
  release_device(srv, r);
  r->state = IBIM_REQ_FAILED;
  r->error = code;
  r->error_msg = msg;
  srv->st.failed++;
}

// Device setup and the first GMRES cycle's start (r = b, V0 = b/||b||) on
// the setup stream, for a request holding a reserved slot.  Touches only the
// request and its slot, so it may run on the admission thread.
int admit_device(ibim_server* srv, Request* r, hipStream_t s) {
  ibim_ctx* c = r->ctx;
  c->opt.device = srv->opt.device;
  // the request's device arrays come from one block of its estimated
  // footprint, freed with one hipFree when the request is reaped (without
  // the block they come from hipMalloc one by one)
  {
    DeviceScope ds(srv->opt.device);
    if (!ds.ok) return fail(IBIM_EHIP, "hipSetDevice failed");
    if (arena_create(&r->arena, r->estimate) != hipSuccess) (void)hipGetLastError();
  }
  ArenaScope scope(&r->arena);
  if (int e = ctx_setup_device(c, s)) return e;
  if (int e = ensure_krylov(c)) return e;
  const int64_t N = c->kr.n;
  HIP_TRY(dalloc(&r->d_b, (size_t)N), "right-hand side allocation");
  HIP_TRY(dalloc(&r->d_x, (size_t)N), "iterate allocation");
  r->setup_bytes = c->device_bytes + 2 * (size_t)N * 8;
  if (r->arena.base)  // the whole block is held, plus what did not fit in it
    r->setup_bytes = std::max(r->setup_bytes, r->arena.size + r->arena.outside);
  {
    const size_t top = std::max(c->setup_peak_bytes, r->setup_bytes);
    if (top > r->estimate) {
      std::lock_guard<std::mutex> lk(srv->mu);
      srv->st.estimate_shortfall = std::max(srv->st.estimate_shortfall, top - r->estimate);
    }
  }
  r->M = c->P.M;
  double* st = srv->d_status + (size_t)r->slot * kStatusStride;
  if (int e = rhs_impl(c, r->d_b, s)) return e;
  if (c->opt.precond == IBIM_PRECOND_DIAG)
    HIP_TRY(launch_row_scaling(c, r->d_b, r->d_b, s), "row scaling");  // as ibim_solve
  Krylov& K = c->kr;
  HIP_TRY(K.dots(r->d_b, N, 1, r->d_b, N, st + 2, 0, s), "dots");
  HIP_TRY(launch_fill(r->d_x, N, 0.0, s), "fill");
  HIP_TRY(launch_copy(r->d_b, K.tmp, N, s), "copy");
  HIP_TRY(K.normalize(K.tmp, st + 2, K.V, N, s), "normalize");
  HIP_TRY(K.init_g(st + 2, s), "init_g");
  // the request's device state is complete before the main stream uses it
  HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  r->phase = Phase::kIter;
  r->j = 0;
  r->total = 0;
  r->applies = 0;
  r->bnorm = -1.0;
  r->t_admit = std::chrono::steady_clock::now();
  return IBIM_OK;
}

void admitter_main(ibim_server* srv, int idx) {
  (void)hipSetDevice(srv->opt.device);
  for (;;) {
    Request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      srv->admit_cv.wait(lk, [&] { return srv->admit_stop || !srv->admit_queue.empty(); });
      if (srv->admit_stop) return;  // queued requests are released by the server's destroy
      r = srv->admit_queue.front();
      srv->admit_queue.pop_front();
    }
    const int e = admit_device(srv, r, srv->setup[idx]);
    const std::string msg = e ? std::string(ibim_last_error()) : std::string();
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      r->admit_error = e;
      r->admit_msg = msg;
      srv->admitted.push_back(r);
    }
    srv->admitted_cv.notify_all();
  }
}

// Main thread, after the device setup: the budget charge becomes the actual
// bytes and the request joins *fresh, or it fails alone.
void finish_admission(ibim_server* srv, Request* r, int e, const std::string& msg,
                      std::vector<Request*>* fresh) {
  if (e) {
    mark_failed(srv, r, e, msg);
    return;
  }
  srv->used = srv->used - r->held + r->setup_bytes;
  r->held = r->setup_bytes;
  if (srv->used > srv->peak) srv->peak = srv->used;
  r->state = IBIM_REQ_ACTIVE;
  srv->st.admitted++;
  fresh->push_back(r);
}

// Requests whose device setup finished on the admission thread, in the
// order they finished (wait: block until at least one is there).
void collect_admitted(ibim_server* srv, std::vector<Request*>* fresh, bool wait) {
  std::vector<Request*> done;
  {
    std::unique_lock<std::mutex> lk(srv->mu);
    if (wait) srv->admitted_cv.wait(lk, [&] { return !srv->admitted.empty(); });
    done.swap(srv->admitted);
  }
  for (Request* r : done) {
    --srv->admitting;
    finish_admission(srv, r, r->admit_error, r->admit_msg, fresh);
  }
}

// Finishing a request: G_pol from psi at the charges, solution to the host,
// on the stream its rounds ran on.
int finish_request(ibim_server* srv, Request* r, hipStream_t s) {
  ibim_ctx* c = r->ctx;
  const int nc = (int)c->q.size();
  std::vector<double> psi(nc > 0 ? nc : 1);
  if (int e = energy_launch(c, r->d_x, s)) return e;
  r->x_host.resize((size_t)c->kr.n);
  if (nc > 0)
    HIP_TRY(hipMemcpyAsync(psi.data(), c->d_psi, nc * sizeof(double), hipMemcpyDeviceToHost, s),
            "copy");
  HIP_TRY(hipMemcpyAsync(r->x_host.data(), r->d_x, (size_t)c->kr.n * sizeof(double),
                         hipMemcpyDeviceToHost, s),
          "copy");
  HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  r->g_pol = nc > 0 ? energy_sum(c, psi.data()) : 0.0;
  if (!std::isfinite(r->g_pol)) return fail(IBIM_ENAN, "energy is not finite");
  r->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - r->t_admit).count();
  release_device(srv, r);
  r->state = IBIM_REQ_DONE;
  srv->st.finished++;
  return IBIM_OK;
}

// Grows a device array and its pinned host staging copy to hold n elements.
template <class T>
int ensure_staging(T** d, T** h, size_t* cap, size_t n) {
  if (n <= *cap) return IBIM_OK;
  dfree(*d);
  if (*h) (void)hipHostFree(*h);
  *h = nullptr;
  *cap = 0;
  const size_t c = 2 * n;
  HIP_TRY(dalloc(d, c), "alloc");
  HIP_TRY(hipHostMalloc((void**)h, c * sizeof(T), hipHostMallocDefault), "pinned allocation");
  *cap = c;
  return IBIM_OK;
}

// Admission, first fit in submission order: requests whose host setup is
// done and whose footprint fits the remaining budget get a slot and their
// device setup on the setup stream, here (now: appended to *fresh) or on the
// admission thread (picked up by a later round).
void admit_waiting(ibim_server* srv, std::vector<Request*>* fresh, bool now) {
  std::vector<Request*> still;
  for (Request* r : srv->waiting) {
    bool prepared;
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      prepared = r->prepared;
    }
    if (!prepared) {
      still.push_back(r);
      continue;
    }
    if (r->error) {
      mark_failed(srv, r, r->error, r->error_msg);
      continue;
    }
    const bool slot = !srv->free_slots.empty();
    if (slot && srv->used + reaping_bytes(srv) + r->estimate <= srv->budget) {
      r->slot = srv->free_slots.back();
      srv->free_slots.pop_back();
      r->held = r->estimate;  // reserved until the device setup reports its bytes
      srv->used += r->held;
      if (now) {
        const int e = admit_device(srv, r, srv->setup[0]);
        finish_admission(srv, r, e, e ? std::string(ibim_last_error()) : std::string(), fresh);
      } else {
        {
          std::lock_guard<std::mutex> lk(srv->mu);
          srv->admit_queue.push_back(r);
        }
        ++srv->admitting;
        srv->admit_cv.notify_one();
      }
    } else {
      if (srv->active.empty() && srv->tree_active.empty() && fresh->empty() &&
          srv->admitting == 0 && slot &&
          r->estimate > srv->budget) {
        mark_failed(srv, r, IBIM_ENOMEM, "request footprint exceeds the server's HBM budget");
        continue;
      }
      if (slot) ++srv->st.held_for_budget;
      else ++srv->st.held_for_slot;
      still.push_back(r);
    }
  }
  srv->waiting.swap(still);
}

// Step 3 of a round for `reqs` (all on the treecode, or none) on stream s:
// correction (+ row scaling), then one GMRES or residual step each, and the
// status slots copied to the pinned host buffer hstat.  The finishing
// kernels of the requests on the symmetric kernels run as one launch per
// precision, and the GMRES (Arnoldi + Givens) steps of all solves as one
// launch per stage, from the staging buffers passed in.
int finish_and_step(ibim_server* srv, const std::vector<Request*>& reqs, hipStream_t s,
                    bool tree, KrylovStepArgs** d_steps, KrylovStepArgs** h_steps,
                    size_t* steps_cap, double* hstat) {
  const size_t na = reqs.size();
  if (int e = ensure_staging(d_steps, h_steps, steps_cap, na)) return e;
  if (!tree) {
    if (int e = ensure_staging(&srv->d_fin, &srv->h_fin, &srv->fin_cap, na)) return e;
    if (int e = ensure_staging(&srv->d_finm, &srv->h_finm, &srv->finm_cap, na)) return e;
  }
  const bool unscale = srv->opt.precond == IBIM_PRECOND_DIAG;
  int nsteps = 0, nfin = 0, nfinm = 0;
  for (Request* r : reqs) {
    ibim_ctx* c = r->ctx;
    Krylov& K = c->kr;
    const int64_t N = K.n;
    const double* u = r->phase == Phase::kIter ? K.V + (int64_t)r->j * N : r->d_x;
    double* out = r->phase == Phase::kIter ? K.V + (int64_t)(r->j + 1) * N : K.tmp2;
    r->applies++;
    if (c->opt.summation == IBIM_SUM_DIRECT && c->sym.enabled) {
      if (c->opt.precision == IBIM_MIXED)
        srv->h_finm[nfinm++] =
            make_finish_sym_mixed_args(c->P, c->sym, c->d_careful, u, c->sym_scratch, out);
      else
        srv->h_fin[nfin++] = make_finish_sym_args(c->P, c->sym, u, c->sym_scratch, out);
      continue;
    }
    if (c->opt.summation == IBIM_SUM_TREE) {
      HIP_TRY(launch_tree_sum(c->tree, c->P, u, s), "treecode launch");
      HIP_TRY(launch_tree_finish(c->tree, c->P, u, out, s), "finish");
    } else if (c->opt.precision == IBIM_MIXED) {
      HIP_TRY(launch_finish_mixed(c->P, c->pair, u, c->partial, out, s), "finish");
    } else {
      HIP_TRY(launch_finish(c->P, c->pair, c->opt.precision, u, c->partial, out, s), "finish");
    }
    if (unscale) HIP_TRY(launch_row_scaling(c, out, out, s), "row scaling");
  }
  if (!tree) {
    HIP_TRY(launch_finish_sym_batched(srv->h_fin, nfin, srv->d_fin, unscale, s), "finish");
    HIP_TRY(launch_finish_sym_mixed_batched(srv->h_finm, nfinm, srv->d_finm, unscale, s),
            "finish");
  }
  for (Request* r : reqs) {
    ibim_ctx* c = r->ctx;
    Krylov& K = c->kr;
    const int64_t N = K.n;
    double* st = srv->d_status + (size_t)r->slot * kStatusStride;
    if (r->phase == Phase::kIter) {
      // as ibim_solve's dots/sub/dots/sub/dots/normalize/givens on out = V_{j+1}
      KrylovStepArgs& a = (*h_steps)[nsteps++];
      a.V = K.V;
      a.H = K.H;
      a.cs = K.cs;
      a.sn = K.sn;
      a.g = K.g;
      a.hcol = K.hcol;
      a.hcol2 = K.hcol2;
      a.scal = K.scal;
      a.partial = K.partial;
      a.status = st;  // straight into the request's status slot
      a.n = N;
      a.m = K.m;
      a.j = r->j;
    } else {
      HIP_TRY(K.residual(r->d_b, K.tmp2, K.tmp, N, s), "residual");
      HIP_TRY(K.dots(K.tmp, N, 1, K.tmp, N, st + 3, 0, s), "dots");
    }
  }
  HIP_TRY(krylov_step_batched(*h_steps, nsteps, *d_steps, s), "batched GMRES step");
  HIP_TRY(hipMemcpyAsync(hstat, srv->d_status,
                         (size_t)srv->max_slots * kStatusStride * sizeof(double),
                         hipMemcpyDeviceToHost, s),
          "copy");
  return IBIM_OK;
}

// Step 4 for `reqs` once their round has completed: the GMRES decisions from
// their status slots in hstat, follow-up work on stream s (the stream their
// round ran on).  Requests still solving are appended to *keep.
int decide(ibim_server* srv, const std::vector<Request*>& reqs, hipStream_t s,
           const double* hstat, std::vector<Request*>* keep) {
  for (Request* r : reqs) {
    ibim_ctx* c = r->ctx;
    Krylov& K = c->kr;
    const int64_t N = K.n;
    const double* hs = hstat + (size_t)r->slot * kStatusStride;
    double* st = srv->d_status + (size_t)r->slot * kStatusStride;
    if (r->bnorm < 0.0) r->bnorm = std::sqrt(hs[2]);
    bool done = false;
    int err = 0;
    if (!std::isfinite(r->bnorm)) {
      err = fail(IBIM_ENAN, "right-hand side is not finite");
    } else if (r->bnorm == 0.0) {
      r->converged = true;
      r->explicit_rel = 0.0;
      r->resid = 0.0;
      done = true;
    } else if (r->phase == Phase::kIter) {
      r->total++;
      r->resid = hs[0];
      const int jend = r->j + 1;
      if (!std::isfinite(r->resid)) {
        err = fail(IBIM_ENAN, "NaN in the GMRES recurrence");
      } else {
        const bool conv = r->resid <= r->tol * r->bnorm || hs[1] == 0.0;
        if (conv || jend == K.m || r->total >= c->opt.max_iter) {
          HIP_TRY(K.backsolve(jend, s), "backsolve");
          HIP_TRY(K.add(K.V, N, jend, K.y, r->d_x, N, s), "update");
          r->converged = conv;
          r->final_check = conv || r->total >= c->opt.max_iter;
          if (r->final_check && !c->opt.check_residual) {
            done = true;
          } else {
            r->phase = Phase::kResid;
          }
        } else {
          r->j++;
        }
      }
    } else {
      const double beta = std::sqrt(hs[3]);
      if (!std::isfinite(beta)) {
        err = fail(IBIM_ENAN, "NaN in the residual");
      } else if (r->final_check) {
        r->explicit_rel = beta / r->bnorm;
        done = true;
      } else if (beta <= r->tol * r->bnorm) {
        // converged at a restart: the residual just formed is the explicit one
        r->converged = true;
        r->resid = beta;
        r->explicit_rel = c->opt.check_residual ? beta / r->bnorm : -1.0;
        done = true;
      } else {
        HIP_TRY(K.normalize(K.tmp, st + 3, K.V, N, s), "normalize");
        HIP_TRY(K.init_g(st + 3, s), "init_g");
        r->phase = Phase::kIter;
        r->j = 0;
      }
    }
    if (err) {
      mark_failed(srv, r, err, ibim_last_error());
      continue;
    }
    if (done) {
      if (int e = finish_request(srv, r, s)) mark_failed(srv, r, e, ibim_last_error());
      continue;
    }
    keep->push_back(r);
  }
  return IBIM_OK;
}

bool on_tree(const Request* r) { return r->ctx->opt.summation == IBIM_SUM_TREE; }

int step_impl(ibim_server* srv) {
  hipStream_t s = srv->stream;
  std::vector<Request*> fresh;
  // requests set up on the admission thread join this round
  collect_admitted(srv, &fresh, false);
  const bool none = srv->active.empty() && srv->tree_active.empty();
  if (none && fresh.empty() && srv->admitting > 0) collect_admitted(srv, &fresh, true);
  // with no solve running, wait for a host setup rather than return idle
  if (none && fresh.empty() && !srv->waiting.empty()) {
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->ready_cv.wait(lk, [&] {
      for (Request* r : srv->waiting)
        if (r->prepared) return true;
      return false;
    });
  }
  const bool idle = none && fresh.empty();
  if (idle) {
    // nothing on the device: admit here and run the new requests' first round now
    admit_waiting(srv, &fresh, true);
  }
  for (Request* r : fresh) (on_tree(r) ? srv->tree_active : srv->active).push_back(r);
  fresh.clear();
  const int n_active = (int)(srv->active.size() + srv->tree_active.size());
  if (n_active > srv->st.max_active_seen) srv->st.max_active_seen = n_active;
  if (n_active == 0) return IBIM_OK;

  // the treecode solves run their own rounds on a second stream, the next one
  // launched when the previous has completed, so that the direct solves'
  // rounds do not wait for their long launches
  if (srv->tree_busy) {
    hipError_t q = hipEventQuery(srv->tevent);
    if (q == hipErrorNotReady && srv->active.empty()) q = hipEventSynchronize(srv->tevent);
    if (q == hipSuccess) {
      srv->tree_busy = false;
      std::vector<Request*> next;
      if (int e = decide(srv, srv->tree_round, srv->tstream, srv->h_tstatus, &next)) return e;
      // then the treecode solves admitted while the round ran
      for (Request* r : srv->tree_active)
        if (std::find(srv->tree_round.begin(), srv->tree_round.end(), r) == srv->tree_round.end())
          next.push_back(r);
      srv->tree_active.swap(next);
      srv->tree_round.clear();
    } else if (q != hipErrorNotReady) {
      return hip_fail(q, "treecode round");
    }
  }
  if (!srv->tree_busy && !srv->tree_active.empty()) {
    srv->tree_round = srv->tree_active;
    if (int e = finish_and_step(srv, srv->tree_round, srv->tstream, true, &srv->d_tsteps,
                                &srv->h_tsteps, &srv->tsteps_cap, srv->h_tstatus))
      return e;
    HIP_TRY(hipEventRecord(srv->tevent, srv->tstream), "event");
    srv->tree_busy = true;
  }
  if (srv->active.empty()) {
    if (!idle) admit_waiting(srv, &fresh, false);
    return IBIM_OK;
  }

  // the direct solves' round: batched pair launches over all of them, one for
  // the problems on the one-directional kernels, one for those on the
  // symmetric kernel
  size_t nargs = 0, nitems = 0, nsargs = 0, nswork = 0;
  for (Request* r : srv->active) {
    const ibim_ctx* c = r->ctx;
    if (c->sym.enabled) {
      ++nsargs;
      nswork += (size_t)c->n_sym_items;
    } else {
      ++nargs;
      nitems += (size_t)c->pair.ntile * (size_t)c->pair.nsplit;
    }
  }
  if (int e = ensure_staging(&srv->d_args, &srv->h_args, &srv->args_cap, nargs)) return e;
  if (int e = ensure_staging(&srv->d_items, &srv->h_items, &srv->items_cap, 3 * nitems)) return e;
  if (int e = ensure_staging(&srv->d_sargs, &srv->h_sargs, &srv->sargs_cap, nsargs)) return e;
  if (int e = ensure_staging(&srv->d_swork, &srv->h_swork, &srv->swork_cap, 2 * nswork)) return e;
  size_t ia = 0, it = 0, isa = 0, isw = 0;
  for (Request* r : srv->active) {
    ibim_ctx* c = r->ctx;
    const int64_t N = c->kr.n;
    const double* u = r->phase == Phase::kIter ? c->kr.V + (int64_t)r->j * N : r->d_x;
    if (c->sym.enabled) {
      srv->h_sargs[isa] =
          make_sym_args(c->P, c->sym, c->d_sym_items, c->d_careful, u, c->sym_scratch);
      for (int q = 0; q < c->n_sym_items; ++q) {
        srv->h_swork[2 * isw] = (int32_t)isa;
        srv->h_swork[2 * isw + 1] = q;
        ++isw;
      }
      ++isa;
    } else {
      srv->h_args[ia] = make_pair_args(c->P, c->pair, u, c->partial);
      for (int t = 0; t < c->pair.ntile; ++t)
        for (int sp = 0; sp < c->pair.nsplit; ++sp) {
          srv->h_items[3 * it] = (int32_t)ia;
          srv->h_items[3 * it + 1] = t;
          srv->h_items[3 * it + 2] = sp;
          ++it;
        }
      ++ia;
    }
  }
  hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(64), 0, s, srv->d_counter, 2);
  HIP_TRY(hipGetLastError(), "zero");
  if (nitems > 0) {
    HIP_TRY(hipMemcpyAsync(srv->d_args, srv->h_args, nargs * sizeof(PairArgs),
                           hipMemcpyHostToDevice, s),
            "copy");
    HIP_TRY(hipMemcpyAsync(srv->d_items, srv->h_items, 3 * nitems * sizeof(int32_t),
                           hipMemcpyHostToDevice, s),
            "copy");
    HIP_TRY(launch_pair_batched(srv->opt.precision, srv->d_args, srv->d_items, (int)nitems,
                                srv->d_counter, srv->grid, s),
            "batched pair launch");
  }
  if (nswork > 0) {
    HIP_TRY(hipMemcpyAsync(srv->d_sargs, srv->h_sargs, nsargs * sizeof(SymArgs),
                           hipMemcpyHostToDevice, s),
            "copy");
    HIP_TRY(hipMemcpyAsync(srv->d_swork, srv->h_swork, 2 * nswork * sizeof(int32_t),
                           hipMemcpyHostToDevice, s),
            "copy");
    if (srv->opt.precision == IBIM_MIXED)
      HIP_TRY(launch_pair_sym_mixed_batched(srv->d_sargs, srv->d_swork, (int)nswork,
                                            srv->d_counter + 1, srv->sym_grid, s),
              "batched symmetric pair launch");
    else
      HIP_TRY(launch_pair_sym_batched(srv->d_sargs, srv->d_swork, (int)nswork,
                                      srv->d_counter + 1, srv->sym_grid, s),
              "batched symmetric pair launch");
  }
  srv->st.rounds++;
  srv->st.batched_items += (int64_t)(nitems + nswork);

  if (int e = finish_and_step(srv, srv->active, s, false, &srv->d_steps, &srv->h_steps,
                              &srv->steps_cap, srv->h_status))
    return e;
  // requests that became ready are set up on the admission thread while the
  // round runs; they join a later round
  if (!idle) admit_waiting(srv, &fresh, false);
  HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  std::vector<Request*> keep;
  if (int e = decide(srv, srv->active, s, srv->h_status, &keep)) return e;
  srv->active.swap(keep);
  return IBIM_OK;
}

Request* find(ibim_server* srv, int64_t ticket) {
  auto it = srv->reqs.find(ticket);
  return it == srv->reqs.end() ? nullptr : it->second.get();
}

}  // namespace

extern "C" {

int ibim_server_create(const ibim_options* opt, size_t hbm_budget_bytes, int max_slots,
                       int host_threads, void* stream, ibim_server** out) {
  if (!out) return fail(IBIM_EINVAL, "out is NULL");
  *out = nullptr;
  if (hbm_budget_bytes == 0 || max_slots < 1 || max_slots > 4096 || host_threads < 1 ||
      host_threads > 64)
    return fail(IBIM_EINVAL, "need hbm_budget_bytes > 0, 1 <= max_slots <= 4096, "
                             "1 <= host_threads <= 64");
  ibim_options o;
  ibim_default_options(&o);
  if (opt) o = *opt;
  if (o.device < 0) return fail(IBIM_EINVAL, "the server needs a device (options.device >= 0)");
  if (int r = check_options(o)) return r;
  ibim_server* srv = new (std::nothrow) ibim_server();
  if (!srv) return fail(IBIM_ENOMEM, "host allocation failed");
  srv->opt = o;
  srv->budget = hbm_budget_bytes;
  srv->max_slots = max_slots;
  srv->stream = reinterpret_cast<hipStream_t>(stream);
  for (int sl = max_slots - 1; sl >= 0; --sl) srv->free_slots.push_back(sl);
  {
    DeviceScope ds(o.device);
    srv->grid = pair_batched_grid(o.precision);
    srv->sym_grid =
        o.precision == IBIM_MIXED ? pair_sym_mixed_batched_grid() : pair_sym_batched_grid();
    hipError_t e = hipSuccess;
    for (int t = 0; t < ibim_server::kAdmitters && e == hipSuccess; ++t)
      e = hipStreamCreateWithFlags(&srv->setup[t], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&srv->tstream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&srv->tevent, hipEventDisableTiming);
    if (e == hipSuccess) e = dalloc(&srv->d_counter, 2);
    if (e == hipSuccess) e = dalloc(&srv->d_status, (size_t)max_slots * kStatusStride);
    if (e == hipSuccess)
      e = hipHostMalloc((void**)&srv->h_status, (size_t)max_slots * kStatusStride * sizeof(double),
                        hipHostMallocDefault);
    if (e == hipSuccess)
      e = hipHostMalloc((void**)&srv->h_tstatus,
                        (size_t)max_slots * kStatusStride * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) {
      ibim_server_destroy(srv);
      return hip_fail(e, "server allocation");
    }
  }
  srv->st.budget_bytes = hbm_budget_bytes;
  int cores = (int)std::thread::hardware_concurrency();
  if (const char* env = std::getenv("OMP_NUM_THREADS")) {
    const int v = std::atoi(env);
    if (v > 0) cores = v;
  }
  const int per = std::max(1, cores / host_threads);
  for (int t = 0; t < host_threads; ++t) srv->workers.emplace_back(worker_main, srv, per);
  srv->reaper = std::thread(reaper_main, srv);
  for (int t = 0; t < ibim_server::kAdmitters; ++t)
    srv->admitter[t] = std::thread(admitter_main, srv, t);
  *out = srv;
  return IBIM_OK;
}

int ibim_server_submit(ibim_server* srv, const double* sdf, int nx, int ny, int nz,
                       const double origin[3], double h, double eps_tube, double eps_in,
                       double eps_out, double kappa, const double* charge_xyz,
                       const double* charge_q, int n_charges, double tol, int64_t* ticket) {
  if (!srv || !sdf || !origin || !ticket) return fail(IBIM_EINVAL, "NULL argument");
  if (nx < 1 || ny < 1 || nz < 1 || n_charges < 0 || !(tol > 0) ||
      (n_charges > 0 && (!charge_xyz || !charge_q)))
    return fail(IBIM_EINVAL, "bad request arguments");
  auto r = std::make_unique<Request>();
  r->ticket = srv->next_ticket++;
  r->sdf.assign(sdf, sdf + (size_t)nx * ny * nz);
  r->dims[0] = nx;
  r->dims[1] = ny;
  r->dims[2] = nz;
  for (int a = 0; a < 3; ++a) r->origin[a] = origin[a];
  r->h = h;
  r->eps = eps_tube;
  r->eps_in = eps_in;
  r->eps_out = eps_out;
  r->kappa = kappa;
  r->tol = tol;
  r->zq.assign(charge_xyz, charge_xyz + 3 * (size_t)n_charges);
  r->q.assign(charge_q, charge_q + (size_t)n_charges);
  r->t_submit = std::chrono::steady_clock::now();
  Request* raw = r.get();
  *ticket = raw->ticket;
  srv->reqs.emplace(raw->ticket, std::move(r));
  srv->waiting.push_back(raw);
  srv->st.submitted++;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->prep_queue.push_back(raw);
  }
  srv->cv.notify_one();
  return IBIM_OK;
}

int ibim_server_step(ibim_server* srv, int* active, int* waiting) {
  if (!srv) return fail(IBIM_EINVAL, "NULL server");
  DeviceScope ds(srv->opt.device);
  const int e = step_impl(srv);
  if (active) *active = (int)(srv->active.size() + srv->tree_active.size());
  if (waiting) *waiting = (int)srv->waiting.size() + srv->admitting;
  return e;
}

int ibim_server_poll(ibim_server* srv, int64_t ticket, int* state, double* g_pol,
                     ibim_solve_info* info) {
  if (!srv || !state) return fail(IBIM_EINVAL, "NULL argument");
  Request* r = find(srv, ticket);
  if (!r) return fail(IBIM_EINVAL, "unknown ticket");
  *state = r->state;
  if (r->state == IBIM_REQ_FAILED) return fail(r->error, r->error_msg);
  if (r->state == IBIM_REQ_DONE) {
    if (g_pol) *g_pol = r->g_pol;
    if (info)
      *info = ibim_solve_info{r->total, r->applies, r->converged ? 1 : 0, r->resid / r->bnorm,
                              r->explicit_rel, r->seconds};
  }
  return IBIM_OK;
}

int ibim_server_solution(ibim_server* srv, int64_t ticket, double* x, int64_t* M) {
  if (!srv || !M) return fail(IBIM_EINVAL, "NULL argument");
  Request* r = find(srv, ticket);
  if (!r) return fail(IBIM_EINVAL, "unknown ticket");
  if (r->state != IBIM_REQ_DONE) return fail(IBIM_EINVAL, "request is not finished");
  *M = r->M;
  if (x) std::memcpy(x, r->x_host.data(), r->x_host.size() * sizeof(double));
  return IBIM_OK;
}

int ibim_server_release(ibim_server* srv, int64_t ticket) {
  if (!srv) return fail(IBIM_EINVAL, "NULL server");
  Request* r = find(srv, ticket);
  if (!r) return fail(IBIM_EINVAL, "unknown ticket");
  if (r->state != IBIM_REQ_DONE && r->state != IBIM_REQ_FAILED)
    return fail(IBIM_EINVAL, "request is still in progress");
  srv->reqs.erase(ticket);
  return IBIM_OK;
}

int ibim_server_get_stats(ibim_server* srv, ibim_server_stats* st) {
  if (!srv || !st) return fail(IBIM_EINVAL, "NULL argument");
  srv->st.bytes_in_use = srv->used;
  srv->st.bytes_peak = srv->peak;
  srv->st.active = (int)(srv->active.size() + srv->tree_active.size());
  srv->st.waiting = (int)srv->waiting.size() + srv->admitting;  // as ibim_server_step
  {
    // estimate_shortfall is written by the admission thread
    std::lock_guard<std::mutex> lk(srv->mu);
    *st = srv->st;
  }
  return IBIM_OK;
}

void ibim_server_destroy(ibim_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stopping = true;
  }
  srv->cv.notify_all();
  for (auto& t : srv->workers) t.join();
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->admit_stop = true;
  }
  srv->admit_cv.notify_all();
  for (auto& t : srv->admitter)
    if (t.joinable()) t.join();  // setups in progress complete
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->reap_stop = true;
  }
  srv->reap_cv.notify_all();
  if (srv->reaper.joinable()) srv->reaper.join();  // frees what is still queued first
  DeviceScope ds(srv->opt.device);
  for (hipStream_t st : srv->setup) {
    if (!st) continue;
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  if (srv->tstream) {
    (void)hipStreamSynchronize(srv->tstream);  // a treecode round still in flight
    (void)hipStreamDestroy(srv->tstream);
  }
  if (srv->tevent) (void)hipEventDestroy(srv->tevent);
  for (auto& kv : srv->reqs) {
    Request* r = kv.second.get();
    if (r->ctx) ibim_destroy(r->ctx);
    r->ctx = nullptr;
    dfree(r->d_b);
    dfree(r->d_x);
  }
  dfree(srv->d_args);
  dfree(srv->d_items);
  dfree(srv->d_sargs);
  dfree(srv->d_swork);
  dfree(srv->d_steps);
  dfree(srv->d_tsteps);
  if (srv->h_tsteps) (void)hipHostFree(srv->h_tsteps);
  if (srv->h_tstatus) (void)hipHostFree(srv->h_tstatus);
  dfree(srv->d_fin);
  dfree(srv->d_finm);
  if (srv->h_fin) (void)hipHostFree(srv->h_fin);
  if (srv->h_finm) (void)hipHostFree(srv->h_finm);
  if (srv->h_sargs) (void)hipHostFree(srv->h_sargs);
  if (srv->h_swork) (void)hipHostFree(srv->h_swork);
  if (srv->h_steps) (void)hipHostFree(srv->h_steps);
  dfree(srv->d_counter);
  dfree(srv->d_status);
  if (srv->h_args) (void)hipHostFree(srv->h_args);
  if (srv->h_items) (void)hipHostFree(srv->h_items);
  if (srv->h_status) (void)hipHostFree(srv->h_status);
  delete srv;
}

}  // extern "C"
