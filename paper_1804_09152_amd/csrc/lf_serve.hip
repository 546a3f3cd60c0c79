// Continuous-batching job loop (see lf.h): jobs are admitted while their HBM
// estimate fits the budget and a slot is free, each active job runs on its
// own stream, chunks of steps of all active jobs are in flight together, and
// a finished job's memory is released at once.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "lf_internal.h"

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

enum JobState { kQueued, kActive, kDone, kFailed, kCancelled };

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
  bool chunk_quiet = true;  // the current chunk has been quiet so far
  int64_t chunk_pos = 0;     // steps of the current chunk done
  int64_t bytes = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  JobState state = kQueued;
  lf_ctx* ctx = nullptr;
  lf_mesh* mesh = nullptr;
  lf_fields* f = nullptr;
  int32_t round = 0;
  int64_t left = 0, issued = 0, steps_run = 0;
  bool in_flight = false;
  std::vector<int32_t> out_seeds, labels, tris;
  lf_status err = LF_OK;
  std::string err_msg;
};

// HBM a job holds while active (an upper estimate).  Per vertex: positions
// 24, the operator twice (caller's and step order: row pointers, diagonal,
// about 7 off-diagonal entries of 8 bytes each) and its slices (8 x 8),
// vertex order 8, two fixed-width field buffers 64, CSR view and scratch
// about 40: 320 bytes.  Per face: indices 12 and the operator assembly's
// half-edges (transient, 3 x 20): 80 bytes.  Plus overflow areas, counters
// and workspace rows: 4 MiB.
int64_t job_bytes(int64_t n_v, int64_t n_f) {
  return 320 * n_v + 80 * n_f + (4 << 20);
}

void release(Job* j) {
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
};

namespace {

lf_status sfail(lf_status st, const std::string& m) {
  lf::set_error(m);
  return st;
}

void job_failed(lf_server* s, Job* j, lf_status st) {
  j->err = st;
  j->err_msg = lf_last_error();
  j->state = kFailed;
  j->t_done = now_ms();
  release(j);
  s->in_use -= j->bytes;
  ++s->n_done;
}

lf_status admit(lf_server* s, Job* j) {
  lf_status st = lf_ctx_create(s->device, nullptr, &j->ctx);
  if (!st) st = lf_mesh_create(j->ctx, j->V.data(), j->n_v, j->F.data(), j->n_f, j->op, &j->mesh);
  if (!st) st = lf_fields_create(j->mesh, j->seeds.data(), j->n_s, &j->P, &j->f);
  if (!st && j->n_types > 0)
    st = lf_fields_set_coefficients(j->f, j->n_types, j->layer_types.data(), j->table.data());
  if (st) return st;
  j->f->measure_all = j->conv_eps > 0;
  j->state = kActive;
  j->t_admit = now_ms();
  j->round = 0;
  j->left = j->steps;
  j->in_flight = false;
  return LF_OK;
}

// end of a phase: re-seed and re-initialise, or finish the job
lf_status next_phase(lf_server* s, Job* j, bool* finished) {
  *finished = false;
  if (j->round < j->rounds) {
    std::vector<int32_t> ns((size_t)j->n_s);
    lf_status st = lf_lloyd_reseed(j->f, ns.data(), nullptr);
    if (!st) st = lf_fields_reset(j->f, ns.data());
    if (st) return st;
    ++j->round;
    j->left = j->steps;
    j->chunk_pos = 0;
    j->chunk_quiet = true;
    return LF_OK;
  }
  j->labels.resize((size_t)j->n_v);
  lf_status st = lf_labels(j->f, j->labels.data(), 0);
  if (st) return st;
  j->out_seeds.resize((size_t)j->n_s);
  st = lf_fields_seeds(j->f, j->out_seeds.data());
  if (st) return st;
  if (j->dual) {
    int64_t nt = 0, nnz = 0;
    st = lf_dual_mesh(j->f, j->P.tau, &nt, nullptr, &nnz, nullptr, nullptr);
    if (st) return st;
    j->tris.resize((size_t)(3 * nt));
    std::vector<int32_t> rp((size_t)j->n_s + 1), col((size_t)std::max<int64_t>(nnz, 1));
    st = lf_dual_mesh(j->f, j->P.tau, &nt, j->tris.data(), &nnz, rp.data(), col.data());
    if (st) return st;
  }
  j->state = kDone;
  j->t_done = now_ms();
  release(j);
  s->in_use -= j->bytes;
  ++s->n_done;
  *finished = true;
  return LF_OK;
}

}  // namespace

extern "C" {

lf_status lf_server_create(int32_t device, int64_t budget, int32_t max_active, int32_t chunk,
                           lf_server** out) try {
  if (!out || budget <= 0 || max_active < 1 || chunk < 1) return sfail(LF_EINVAL, "invalid argument");
  lf_server* s = new lf_server();
  s->device = device;
  s->budget = budget;
  s->max_active = max_active;
  s->chunk = chunk;
  *out = s;
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_server_destroy(lf_server* s) try {
  if (!s) return LF_OK;
  for (auto& kv : s->jobs) {
    Job* j = kv.second;
    if (j->f && j->in_flight) {
      int64_t rem = 0;
      lf::step_complete(j->f, &rem);
    }
    release(j);
    delete j;
  }
  delete s;
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_server_submit(lf_server* s, const lf_job* job, int64_t* id) try {
  if (!s || !job || !id || !job->V || !job->F || !job->seeds || job->n_v < 3 || job->n_f < 1 ||
      job->n_s < 1 || job->steps < 0 || job->lloyd_rounds < 0 || job->conv_eps < 0 ||
      (job->conv_eps > 0 && job->conv_every < 1) || job->n_types < 0 || job->n_types > 65536 ||
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
  // admission, in arrival order, while memory and slots allow
  while (!s->queue.empty() && (int32_t)s->active.size() < s->max_active &&
         s->in_use + s->queue.front()->bytes <= s->budget) {
    Job* j = s->queue.front();
    s->queue.pop_front();
    s->in_use += j->bytes;
    if (s->in_use > s->peak) s->peak = s->in_use;
    lf_status st = admit(s, j);
    if (st) {
      job_failed(s, j, st);
      continue;
    }
    s->active.push_back(j);
  }
  // book finished chunks, start phases, issue the next chunks
  for (size_t k = 0; k < s->active.size();) {
    Job* j = s->active[k];
    bool gone = false;
    lf_status st = LF_OK;
    if (j->in_flight && lf::step_ready(j->f)) {
      int64_t rem = 0;
      st = lf::step_complete(j->f, &rem);
      j->in_flight = false;
      const int64_t ok = j->issued - rem;
      j->left -= ok;
      j->steps_run += ok;
      // a phase converges at the end of a whole quiet chunk of conv_every steps
      if (!st && j->conv_eps > 0) {
        j->chunk_quiet = j->chunk_quiet && lf::chunk_quiet(j->f, ok, j->conv_eps);
        j->chunk_pos += ok;
        if (j->chunk_pos == j->conv_every) {
          if (j->chunk_quiet) j->left = 0;
          j->chunk_pos = 0;
          j->chunk_quiet = true;
        }
      }
    }
    if (!st && !j->in_flight) {
      if (j->left == 0) st = next_phase(s, j, &gone);
      if (!st && !gone && j->left > 0) {
        j->issued = std::min<int64_t>(
            j->conv_eps > 0 ? j->conv_every - j->chunk_pos : s->chunk, j->left);
        st = lf::step_issue(j->f, j->issued);
        j->in_flight = !st;
      }
    }
    if (st) {
      job_failed(s, j, st);
      gone = true;
    }
    if (gone) s->active.erase(s->active.begin() + (long)k);
    else ++k;
  }
  if (n_queued) *n_queued = (int32_t)s->queue.size();
  if (n_active) *n_active = (int32_t)s->active.size();
  if (n_done) *n_done = s->n_done;
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_server_cancel(lf_server* s, int64_t id) try {
  if (!s) return sfail(LF_EINVAL, "NULL argument");
  auto it = s->jobs.find(id);
  if (it == s->jobs.end()) return sfail(LF_EINVAL, "unknown job");
  Job* j = it->second;
  if (j->state == kQueued) {
    s->queue.erase(std::find(s->queue.begin(), s->queue.end(), j));
  } else if (j->state == kActive) {
    // the chunk in flight finishes first; then the job's memory is released
    if (j->in_flight) {
      int64_t rem = 0;
      lf::step_complete(j->f, &rem);
      j->in_flight = false;
    }
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

}  // extern "C"
