// Continuous-batching job loop (see lf.h).
//
// Jobs wait in arrival order and are admitted while their HBM fits the
// budget and a slot is free.  The Euler steps of every job that is stepping
// advance together in "ticks": one tick issues, on the server's stream, up to
// `chunk` step launches, and each launch covers the slices of all the jobs
// still stepping at that point of the tick (one grouped kernel over their
// independent field objects; jobs with per-pair coefficients in a second
// grouped kernel).  Jobs join at the next tick after admission and leave at
// the end of a phase, so the set of jobs in a launch changes from tick to
// tick without moving any job's data.  Everything that is not a step runs on
// a host worker thread per job, on the job's own stream, while ticks go on
// for the others: admission (mesh, operator, vertex order, fields), the
// Lloyd re-seeding and re-initialisation between phases, and labels plus
// dual mesh at the end.  lf_server_poll never waits for the GPU: it books a
// tick whose event has completed, collects finished worker threads, admits,
// and issues the next tick.
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "lf_internal.h"

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

enum JobState { kQueued, kActive, kDone, kFailed, kCancelled };
// what an active job is doing
enum Work { kStepping, kAdmitting, kPhaseEnd, kFinishing };

struct Job {
  int64_t id = 0;
  std::vector<double> V;
  std::vector<int32_t> F, seeds;
  int32_t n_v = 0, n_f = 0, n_s = 0, op = 0, steps = 0, rounds = 0, dual = 0;
  lf_params P;
  double conv_eps = 0;  // > 0: phases end at convergence
  int32_t conv_every = 0;
  int32_t n_types = 0;  // per-pair coefficients
  std::vector<int32_t> layer_types;
  std::vector<double> table;
  bool chunk_quiet = true;  // the current convergence chunk has been quiet so far
  int64_t chunk_pos = 0;     // steps of the current convergence chunk done
  int64_t bytes = 0;         // HBM charged to the budget
  double t_submit = 0, t_admit = 0, t_done = 0;
  JobState state = kQueued;
  Work work = kStepping;
  lf_ctx* ctx = nullptr;
  lf_mesh* mesh = nullptr;
  lf_fields* f = nullptr;
  int32_t round = 0;
  int64_t left = 0, steps_run = 0;
  int64_t tick_steps = 0;  // steps of this job in the tick in flight (0: not in it)
  // host worker (admission, phase ends)
  std::thread worker;
  std::atomic<bool> worker_done{false};
  lf_status worker_st = LF_OK;
  std::string worker_msg;
  std::vector<int32_t> out_seeds, labels, tris;
  lf_status err = LF_OK;
  std::string err_msg;
};

// HBM a job holds while active, estimated before admission.  Per vertex:
// positions 24, the operator twice (caller's and step order: row pointers,
// diagonal, about 7 off-diagonal entries of 8 bytes each) and its slices
// (8 x 8), vertex order 8, two fixed-width field buffers 64, the CSR view 40,
// re-seeding and dual-mesh tables about 60: 380 bytes.  Per face: indices 12
// and the operator assembly's half-edges (transient, 3 x 20): 80 bytes.  Plus
// overflow areas, counters and workspace rows: 4 MiB.  Once admitted, a job
// is charged the larger of this and what its fields and mesh actually hold
// (overflow growth included).
int64_t job_bytes(int64_t n_v, int64_t n_f) {
  return 380 * n_v + 80 * n_f + (4 << 20);
}

void release(Job* j) {
  if (j->worker.joinable()) j->worker.join();
  if (j->f) lf_fields_destroy(j->f);
  if (j->mesh) lf_mesh_destroy(j->mesh);
  if (j->ctx) lf_ctx_destroy(j->ctx);
  j->f = nullptr;
  j->mesh = nullptr;
  j->ctx = nullptr;
}

}  // namespace

struct lf_server {
  int32_t device = 0;
  int64_t budget = 0, in_use = 0, peak = 0;
  int32_t max_active = 1, chunk = 64;
  int64_t next_id = 1;
  std::deque<Job*> queue;
  std::vector<Job*> active;
  std::map<int64_t, Job*> jobs;
  int32_t n_done = 0;
  // ticks
  lf_ctx* ctx = nullptr;  // the server's stream
  hipEvent_t tick_ev = nullptr;
  bool tick_in_flight = false;
  std::vector<Job*> tick_jobs;
  lf::StepArgs* d_args = nullptr;    // grouped launch tables, device
  int32_t* d_first = nullptr;
  lf::StepArgs* h_args = nullptr;    // their pinned host staging
  int32_t* h_first = nullptr;
  int64_t args_cap = 0, first_cap = 0;
  int64_t ticks = 0, launches = 0;
};

namespace {

lf_status sfail(lf_status st, const std::string& m) {
  lf::set_error(m);
  return st;
}

void job_failed(lf_server* s, Job* j, lf_status st, const std::string& msg) {
  j->err = st;
  j->err_msg = msg;
  j->state = kFailed;
  j->t_done = now_ms();
  release(j);
  s->in_use -= j->bytes;
  ++s->n_done;
}

void charge(lf_server* s, Job* j) {
  if (!j->f) return;
  const int64_t b = lf::fields_bytes(j->f) + lf::mesh_bytes(j->mesh);
  if (b > j->bytes) {
    s->in_use += b - j->bytes;
    j->bytes = b;
    if (s->in_use > s->peak) s->peak = s->in_use;
  }
}

// worker bodies: the job's own context and stream; each ends with the stream
// drained, so that the server's stream may use the job's buffers next
void admit_work(Job* j, int32_t device) {
  lf_status st = lf_ctx_create(device, nullptr, &j->ctx);
  if (!st) st = lf_mesh_create(j->ctx, j->V.data(), j->n_v, j->F.data(), j->n_f, j->op, &j->mesh);
  if (!st) st = lf_fields_create(j->mesh, j->seeds.data(), j->n_s, &j->P, &j->f);
  if (!st && j->n_types > 0)
    st = lf_fields_set_coefficients(j->f, j->n_types, j->layer_types.data(), j->table.data());
  if (!st) st = lf_sync(j->f);
  if (st) j->worker_msg = lf_last_error();
  j->worker_st = st;
  j->worker_done.store(true, std::memory_order_release);
}

// end of a phase: re-seed and re-initialise (kPhaseEnd), or the final labels,
// seeds and dual mesh (kFinishing)
void phase_work(Job* j) {
  lf_status st = LF_OK;
  if (j->work == kPhaseEnd) {
    std::vector<int32_t> ns((size_t)j->n_s);
    st = lf_lloyd_reseed(j->f, ns.data(), nullptr);
    if (!st) st = lf_fields_reset(j->f, ns.data());
    if (!st) st = lf_sync(j->f);
  } else {
    j->labels.resize((size_t)j->n_v);
    st = lf_labels(j->f, j->labels.data(), 0);
    j->out_seeds.resize((size_t)j->n_s);
    if (!st) st = lf_fields_seeds(j->f, j->out_seeds.data());
    if (!st && j->dual) {
      int64_t nt = 0, nnz = 0;
      st = lf_dual_mesh(j->f, j->P.tau, &nt, nullptr, &nnz, nullptr, nullptr);
      if (!st) {
        j->tris.resize((size_t)(3 * nt));
        std::vector<int32_t> rp((size_t)j->n_s + 1), col((size_t)std::max<int64_t>(nnz, 1));
        st = lf_dual_mesh(j->f, j->P.tau, &nt, j->tris.data(), &nnz, rp.data(), col.data());
      }
    }
  }
  if (st) j->worker_msg = lf_last_error();
  j->worker_st = st;
  j->worker_done.store(true, std::memory_order_release);
}

void start_worker(Job* j, Work w, int32_t device) {
  if (j->worker.joinable()) j->worker.join();
  j->work = w;
  j->worker_done.store(false, std::memory_order_relaxed);
  if (w == kAdmitting) j->worker = std::thread(admit_work, j, device);
  else j->worker = std::thread(phase_work, j);
}

// a phase has run its steps: the next phase or the end
void end_phase(lf_server* s, Job* j) {
  start_worker(j, j->round < j->rounds ? kPhaseEnd : kFinishing, s->device);
}

template <class T>
lf_status grow_pinned(T** h, T** d, int64_t* cap, int64_t need) {
  if (need <= *cap) return LF_OK;
  const int64_t c = std::max<int64_t>(need, 2 * *cap);
  T *nh = nullptr, *nd = nullptr;
  LF_HIP(hipHostMalloc((void**)&nh, sizeof(T) * c, 0));
  hipError_t e = lf::dalloc(&nd, c);
  if (e != hipSuccess) {
    (void)hipHostFree(nh);
    return lf::hip_fail(e, "grouped launch tables");
  }
  if (*h) (void)hipHostFree(*h);
  if (*d) (void)hipFree(*d);
  *h = nh;
  *d = nd;
  *cap = c;
  return LF_OK;
}

// One tick: every stepping job issues its next steps (a chunk, or the rest of
// its convergence chunk, at most what its phase has left); launch k of the
// tick covers the jobs with more than k steps in it.
lf_status issue_tick(lf_server* s) {
  std::vector<Job*> js;
  for (Job* j : s->active)
    if (j->work == kStepping && j->left > 0) js.push_back(j);
  if (js.empty()) return LF_OK;
  hipStream_t st = s->ctx->stream;
  LF_HIP(hipSetDevice(s->device));
  int64_t M = 0;
  for (Job* j : js) {
    j->tick_steps = std::min<int64_t>(
        j->conv_eps > 0 ? j->conv_every - j->chunk_pos : s->chunk, j->left);
    M = std::max(M, j->tick_steps);
    lf_status e = lf::ensure_step_buffers(j->f, j->tick_steps);
    if (e) return e;
  }
  // launch tables: for each launch k, the scalar jobs then the typed jobs
  // still stepping, their arguments and first slices
  int64_t n_args = 0, n_first = 0;
  for (int64_t k = 0; k < M; ++k)
    for (Job* j : js)
      if (j->tick_steps > k) ++n_args;
  n_first = n_args + 2 * M;
  lf_status e = grow_pinned(&s->h_args, &s->d_args, &s->args_cap, n_args);
  if (!e) e = grow_pinned(&s->h_first, &s->d_first, &s->first_cap, n_first);
  if (e) return e;
  struct Group { int64_t a0, f0; int32_t n, total; bool typed; };
  std::vector<Group> groups;
  int64_t a = 0, fi = 0;
  for (int64_t k = 0; k < M; ++k) {
    for (int typed = 0; typed < 2; ++typed) {
      Group g{a, fi, 0, 0, typed == 1};
      int32_t slices = 0;
      for (Job* j : js) {
        if (j->tick_steps <= k || (j->n_types > 0) != (typed == 1)) continue;
        s->h_args[a] = lf::chunk_step_args(j->f, k, j->tick_steps);
        s->h_args[a++].wide_rows = nullptr;  // a grouped launch steps wide rows in place
        s->h_first[fi++] = slices;
        slices += j->mesh->n_slices;
        ++g.n;
      }
      if (g.n == 0) {
        a = g.a0;
        fi = g.f0;
        continue;
      }
      s->h_first[fi++] = slices;
      g.total = slices;
      groups.push_back(g);
    }
  }
  LF_HIP(hipMemcpyAsync(s->d_args, s->h_args, sizeof(lf::StepArgs) * a, hipMemcpyHostToDevice, st));
  LF_HIP(hipMemcpyAsync(s->d_first, s->h_first, sizeof(int32_t) * fi, hipMemcpyHostToDevice, st));
  for (Job* j : js) LF_HIP(lf::launch_reset_flags(j->f->flags, j->f->parts, j->tick_steps, st));
  for (const Group& g : groups)
    LF_HIP(lf::launch_step_group(s->d_args + g.a0, s->d_first + g.f0, g.n, g.total, g.typed, st));
  for (Job* j : js) {
    e = lf::chunk_tail(j->f, j->tick_steps, st);
    if (e) return e;
  }
  LF_HIP(hipEventRecord(s->tick_ev, st));
  s->tick_jobs = js;
  s->tick_in_flight = true;
  ++s->ticks;
  s->launches += (int64_t)groups.size();
  return LF_OK;
}

// books the completed tick for every job in it
void book_tick(lf_server* s) {
  s->tick_in_flight = false;
  std::vector<Job*> js;
  js.swap(s->tick_jobs);
  for (Job* j : js) {
    if (j->state != kActive) continue;  // cancelled meanwhile
    const int64_t n = j->tick_steps;
    j->tick_steps = 0;
    int64_t rem = 0;
    lf_status st = lf::step_book(j->f, n, &rem);
    // growth or a cleared failure ran on the job's stream: drain it before
    // the server's stream touches the job again
    if (!st) st = lf_sync(j->f);
    if (st) {
      std::string msg = lf_last_error();
      s->active.erase(std::find(s->active.begin(), s->active.end(), j));
      job_failed(s, j, st, msg);
      continue;
    }
    const int64_t ok = n - rem;
    j->left -= ok;
    j->steps_run += ok;
    if (j->conv_eps > 0) {
      j->chunk_quiet = j->chunk_quiet && lf::chunk_quiet(j->f, ok, j->conv_eps);
      j->chunk_pos += ok;
      if (j->chunk_pos == j->conv_every) {
        if (j->chunk_quiet) j->left = 0;
        j->chunk_pos = 0;
        j->chunk_quiet = true;
      }
    }
    charge(s, j);
    if (j->left == 0) end_phase(s, j);
  }
}

}  // namespace

extern "C" {

lf_status lf_server_create(int32_t device, int64_t budget, int32_t max_active, int32_t chunk,
                           lf_server** out) try {
  if (!out || budget <= 0 || max_active < 1 || chunk < 1 || chunk > lf::kMaxChunk)
    return sfail(LF_EINVAL, "invalid argument");
  *out = nullptr;
  lf_server* s = new lf_server();
  s->device = device;
  s->budget = budget;
  s->max_active = max_active;
  s->chunk = chunk;
  *out = s;  // the server's stream and event are made by the first poll
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_server_destroy(lf_server* s) try {
  if (!s) return LF_OK;
  if (s->tick_in_flight) (void)hipEventSynchronize(s->tick_ev);
  if (s->ctx) (void)hipSetDevice(s->device);
  for (auto& kv : s->jobs) {
    release(kv.second);
    delete kv.second;
  }
  if (s->tick_ev) (void)hipEventDestroy(s->tick_ev);
  if (s->h_args) (void)hipHostFree(s->h_args);
  if (s->h_first) (void)hipHostFree(s->h_first);
  if (s->d_args) (void)hipFree(s->d_args);
  if (s->d_first) (void)hipFree(s->d_first);
  if (s->ctx) lf_ctx_destroy(s->ctx);
  delete s;
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_server_submit(lf_server* s, const lf_job* job, int64_t* id) try {
  if (!s || !job || !id || !job->V || !job->F || !job->seeds || job->n_v < 3 || job->n_f < 1 ||
      job->n_s < 1 || job->steps < 0 || job->lloyd_rounds < 0 || job->conv_eps < 0 ||
      (job->conv_eps > 0 && (job->conv_every < 1 || job->conv_every > lf::kMaxChunk)) ||
      job->n_types < 0 || job->n_types > 65536 ||
      (job->n_types > 0 && (!job->layer_types || !job->table)))
    return sfail(LF_EINVAL, "invalid job");
  Job* j = new Job();
  j->bytes = job_bytes(job->n_v, job->n_f);
  if (job->n_types > 0)  // the coefficient table and the layer types on the device
    j->bytes += 16ll * job->n_types * job->n_types + 4ll * (job->n_s + 1);
  if (j->bytes > s->budget) {
    delete j;
    return sfail(LF_ENOMEM, "the job alone exceeds the HBM budget");
  }
  try {
    j->V.assign(job->V, job->V + 3ll * job->n_v);
    j->F.assign(job->F, job->F + 3ll * job->n_f);
    j->seeds.assign(job->seeds, job->seeds + job->n_s);
    if (job->n_types > 0) {  // checked when the job is admitted
      j->layer_types.assign(job->layer_types, job->layer_types + job->n_s + 1);
      j->table.assign(job->table, job->table + 3ll * job->n_types * job->n_types);
    }
  } catch (const std::bad_alloc&) {
    delete j;
    return sfail(LF_ENOMEM, "the job's inputs do not fit in host memory");
  }
  j->id = s->next_id++;
  j->n_v = job->n_v;
  j->n_f = job->n_f;
  j->n_s = job->n_s;
  j->op = job->op;
  j->steps = job->steps;
  j->rounds = job->lloyd_rounds;
  j->dual = job->dual_mesh;
  j->P = job->params;
  j->conv_eps = job->conv_eps;
  j->conv_every = job->conv_every;
  j->n_types = job->n_types;
  j->t_submit = now_ms();
  s->queue.push_back(j);
  s->jobs[j->id] = j;
  *id = j->id;
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_server_poll(lf_server* s, int32_t* n_queued, int32_t* n_active, int32_t* n_done) try {
  if (!s) return sfail(LF_EINVAL, "NULL argument");
  if (!s->ctx) {
    lf_status st = lf_ctx_create(s->device, nullptr, &s->ctx);
    if (st) return st;
    LF_HIP(hipEventCreateWithFlags(&s->tick_ev, hipEventDisableTiming));
  }
  LF_HIP(hipSetDevice(s->device));
  // a completed tick: book it (jobs whose phase ended go to their workers)
  if (s->tick_in_flight && hipEventQuery(s->tick_ev) == hipSuccess) book_tick(s);
  // finished workers
  for (size_t k = 0; k < s->active.size();) {
    Job* j = s->active[k];
    if (j->work == kStepping || !j->worker_done.load(std::memory_order_acquire)) {
      ++k;
      continue;
    }
    j->worker.join();
    if (j->worker_st) {
      s->active.erase(s->active.begin() + (long)k);
      job_failed(s, j, j->worker_st, j->worker_msg);
      continue;
    }
    if (j->work == kFinishing) {
      j->state = kDone;
      j->t_done = now_ms();
      release(j);
      s->in_use -= j->bytes;
      ++s->n_done;
      s->active.erase(s->active.begin() + (long)k);
      continue;
    }
    if (j->work == kAdmitting) {
      j->f->measure_all = j->conv_eps > 0;
      j->t_admit = now_ms();
      j->round = 0;
      j->left = j->steps;
      charge(s, j);
    } else {  // re-seeded and re-initialised: the next phase
      ++j->round;
      j->left = j->steps;
      j->chunk_pos = 0;
      j->chunk_quiet = true;
    }
    j->work = kStepping;
    if (j->left == 0) end_phase(s, j);
    ++k;
  }
  // admission, in arrival order, while memory and slots allow
  while (!s->queue.empty() && (int32_t)s->active.size() < s->max_active &&
         s->in_use + s->queue.front()->bytes <= s->budget) {
    Job* j = s->queue.front();
    s->queue.pop_front();
    s->in_use += j->bytes;
    if (s->in_use > s->peak) s->peak = s->in_use;
    j->state = kActive;
    s->active.push_back(j);
    start_worker(j, kAdmitting, s->device);
  }
  // the next tick
  if (!s->tick_in_flight) {
    lf_status st = issue_tick(s);
    if (st) return st;
  }
  if (n_queued) *n_queued = (int32_t)s->queue.size();
  if (n_active) *n_active = (int32_t)s->active.size();
  if (n_done) *n_done = s->n_done;
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
} catch (const std::system_error&) {
  return sfail(LF_ENOMEM, "could not start a worker thread");
}

lf_status lf_server_cancel(lf_server* s, int64_t id) try {
  if (!s) return sfail(LF_EINVAL, "NULL argument");
  auto it = s->jobs.find(id);
  if (it == s->jobs.end()) return sfail(LF_EINVAL, "unknown job");
  Job* j = it->second;
  if (j->state == kQueued) {
    s->queue.erase(std::find(s->queue.begin(), s->queue.end(), j));
  } else if (j->state == kActive) {
    // a tick in flight finishes first (it may hold this job's steps); a
    // worker finishes its part; then the job's memory is released at once
    if (j->tick_steps > 0 && s->tick_in_flight) LF_HIP(hipEventSynchronize(s->tick_ev));
    j->tick_steps = 0;
    auto t = std::find(s->tick_jobs.begin(), s->tick_jobs.end(), j);
    if (t != s->tick_jobs.end()) s->tick_jobs.erase(t);
    release(j);
    s->in_use -= j->bytes;
    s->active.erase(std::find(s->active.begin(), s->active.end(), j));
  } else {
    return sfail(LF_EINVAL, "job already finished");
  }
  j->state = kCancelled;
  j->t_done = now_ms();
  ++s->n_done;
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_server_result(lf_server* s, int64_t id, int32_t* seeds, int32_t* labels,
                           int64_t* n_tri, int32_t* tris, double* latency_ms, double* queue_ms,
                           int64_t* steps) try {
  if (!s) return sfail(LF_EINVAL, "NULL argument");
  auto it = s->jobs.find(id);
  if (it == s->jobs.end()) return sfail(LF_EINVAL, "unknown job");
  Job* j = it->second;
  if (j->state == kFailed) return sfail(j->err, "job failed: " + j->err_msg);
  if (j->state == kCancelled) return sfail(LF_EINVAL, "job cancelled");
  if (j->state != kDone) return sfail(LF_EBUSY, "job not finished");
  if (seeds) memcpy(seeds, j->out_seeds.data(), sizeof(int32_t) * j->out_seeds.size());
  if (labels) memcpy(labels, j->labels.data(), sizeof(int32_t) * j->labels.size());
  if (n_tri) *n_tri = (int64_t)j->tris.size() / 3;
  if (tris) memcpy(tris, j->tris.data(), sizeof(int32_t) * j->tris.size());
  if (latency_ms) *latency_ms = j->t_done - j->t_submit;
  if (queue_ms) *queue_ms = j->t_admit - j->t_submit;
  if (steps) *steps = j->steps_run;
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_server_times(lf_server* s, int64_t id, double* submit_ms, double* admit_ms,
                          double* done_ms) try {
  if (!s) return sfail(LF_EINVAL, "NULL argument");
  auto it = s->jobs.find(id);
  if (it == s->jobs.end()) return sfail(LF_EINVAL, "unknown job");
  Job* j = it->second;
  if (submit_ms) *submit_ms = j->t_submit;
  if (admit_ms) *admit_ms = j->t_admit;
  if (done_ms) *done_ms = j->t_done;
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_server_release(lf_server* s, int64_t id) try {
  if (!s) return sfail(LF_EINVAL, "NULL argument");
  auto it = s->jobs.find(id);
  if (it == s->jobs.end()) return sfail(LF_EINVAL, "unknown job");
  Job* j = it->second;
  if (j->state != kDone && j->state != kFailed && j->state != kCancelled)
    return sfail(LF_EBUSY, "job not finished");
  delete j;
  s->jobs.erase(it);
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_server_memory(lf_server* s, int64_t* in_use, int64_t* peak) try {
  if (!s) return sfail(LF_EINVAL, "NULL argument");
  if (in_use) *in_use = s->in_use;
  if (peak) *peak = s->peak;
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_server_stats(lf_server* s, int64_t* ticks, int64_t* launches) try {
  if (!s) return sfail(LF_EINVAL, "NULL argument");
  if (ticks) *ticks = s->ticks;
  if (launches) *launches = s->launches;
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

}  // extern "C"
