// C ABI of the layered-field library: contexts, meshes, fields, stepping
// with device-side capacity checks, import / export, labels, statistics.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "lf_internal.h"

namespace lf {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

lf_status hip_fail(hipError_t e, const char* what) {
  g_err = std::string("HIP error ") + hipGetErrorString(e) + " in " + what;
  return (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? LF_ENOMEM : LF_EDEVICE;
}

lf_status host_oom() {
  g_err = "out of host memory";
  return LF_ENOMEM;
}

static lf_status fail(lf_status st, const std::string& msg) {
  set_error(msg);
  return st;
}

// device buffer released at scope exit unless released
template <class T>
struct DevBuf {
  T* p = nullptr;
  ~DevBuf() {
    if (p) hipFree(p);
  }
  hipError_t alloc(int64_t n) { return dalloc(&p, n); }
  T* release() {
    T* q = p;
    p = nullptr;
    return q;
  }
};

// a float kept as its bit pattern in an integer counter
static float bits_float(unsigned long long u) {
  const uint32_t w = (uint32_t)u;
  float x;
  memcpy(&x, &w, sizeof x);
  return x;
}

StepArgs step_args(lf_fields* f, int parity) {
  StepArgs a;
  lf_mesh* m = f->mesh;
  a.lell = f->lell;
  a.lptr = f->slptr;
  a.lent = f->slent;
  a.op_w = f->op_w;
  a.pad0_ = 0;
  a.ldiag = f->sldiag;
  a.slice_cls = f->slice_cls;
  a.wide_rows = f->wide_rows;
  a.u_in = f->ell[parity];
  a.u_out = f->ell[1 - parity];
  a.ovf_in = f->ovf[parity];
  a.ovf_out = f->ovf[1 - parity];
  a.ovf_cap = f->ovf_cap;
  a.ovf_ctr = f->counters + (1 - parity);
  a.ovf_ctr_next = f->counters + parity;
  a.n_v = m->n_v;
  a.n_slices = m->n_slices;
  a.c.a = (float)f->P.a;
  a.c.w = (float)f->P.w;
  a.c.e = (float)f->P.e;
  a.c.mu = (float)f->P.mu;
  a.c.dt = (float)f->P.dt;
  a.c.theta = (float)f->P.theta;
  a.c.base_mode = f->P.base_mode;
  a.c.n_s = f->n_s;
  a.c.tau = (float)f->P.tau;
  a.c.n_types = f->n_types;
  a.c.types = f->types;
  a.c.tab = f->coef;
  a.wide = f->wide;
  a.wide_cap = f->wide_cap;
  a.pad_ = 0;
  a.wide_ctr = f->counters + 2 + (1 - parity);
  a.wide_ctr_next = f->counters + 2 + parity;
  a.flags = f->flags;
  a.parts = nullptr;
  a.step_idx = 0;
  a.measure = 0;
  return a;
}

static lf_status clear_step_state(lf_fields* f) {
  hipStream_t s = f->mesh->ctx->stream;
  LF_HIP(launch_fill_i32((int32_t*)f->counters, 4, 0, s));
  LF_HIP(launch_reset_flags(f->flags, nullptr, 0, s));
  return LF_OK;
}

// four times more workspace rows for vertices touching many layers
static lf_status grow_wide(lf_fields* f) {
  const int64_t c = 4ll * f->wide_cap;
  if (c > (1ll << 24)) return fail(LF_ECAPACITY, "wide-row workspace would exceed 2^24 rows");
  WideRow* p = nullptr;
  LF_HIP(dalloc(&p, c));
  LF_HIP(hipStreamSynchronize(f->mesh->ctx->stream));
  (void)hipFree(f->wide);
  f->wide = p;
  f->wide_cap = (int32_t)c;
  f->grow_events++;
  return LF_OK;
}

// grows both overflow areas to at least `need` entries (plus 20%), keeping
// the current one's contents
static lf_status grow(lf_fields* f, int64_t need) {
  const int64_t lim = (1ll << 31) - 1;
  if (need > lim) return fail(LF_ECAPACITY, "overflow area would exceed 2^31 entries");
  int64_t ncap = std::max(need + need / 5, f->ovf_cap + f->ovf_cap / 5) + 1024;
  ncap = std::min(ncap, lim);
  hipStream_t s = f->mesh->ctx->stream;
  DevBuf<Ent> a, b;
  LF_HIP(a.alloc(ncap));
  LF_HIP(b.alloc(ncap));
  LF_HIP(hipMemcpyAsync(a.p, f->ovf[f->cur], sizeof(Ent) * f->ovf_cap, hipMemcpyDeviceToDevice, s));
  LF_HIP(hipStreamSynchronize(s));
  (void)hipFree(f->ovf[0]);
  (void)hipFree(f->ovf[1]);
  f->ovf[f->cur] = a.release();
  f->ovf[1 - f->cur] = b.release();
  f->ovf_cap = ncap;
  f->grow_events++;
  return clear_step_state(f);
}

// CSR buffer for at least n entries (contents not kept)
static lf_status reserve_csr(lf_fields* f, int64_t n) {
  if (n <= f->csr_cap && f->uent) return LF_OK;
  const int64_t c = std::max<int64_t>(n + n / 5, f->mesh->n_v) + 1024;
  Ent* p = nullptr;
  LF_HIP(dalloc(&p, c));
  LF_HIP(hipStreamSynchronize(f->mesh->ctx->stream));
  (void)hipFree(f->uent);
  f->uent = p;
  f->csr_cap = c;
  return LF_OK;
}

lf_status fields_csr(lf_fields* f, const int32_t** uptr, const Ent** uent) {
  if (!f->csr_valid) {
    hipStream_t s = f->mesh->ctx->stream;
    const int32_t n_v = f->mesh->n_v;
    lf_status st = reserve_csr(f, f->nnz);
    if (st) return st;
    LF_HIP(ell_to_csr_ptr(f->ell[f->cur], f->inv, n_v, f->owner, f->uptr, f->scan_tmp, s));
    LF_HIP(ell_to_csr_fill(f->ell[f->cur], f->ovf[f->cur], f->inv, n_v, f->uptr, f->uent, s));
    f->csr_valid = true;
  }
  *uptr = f->uptr;
  *uent = f->uent;
  return LF_OK;
}

}  // namespace lf

using namespace lf;

extern "C" {

const char* lf_last_error(void) { return g_err.c_str(); }

void lf_params_default(lf_params* p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->w = 0.2;
  p->a = 0.04;
  p->e = 1.0;
  p->mu = 0.1;
  p->dt = 5.0;
  p->theta = 1e-3;
  p->tau = 0.25;
  p->base_mode = 0;
  p->capacity_hint = 0;
}

lf_status lf_ctx_create(int32_t device, void* hip_stream, lf_ctx** out) try {
  if (!out) return fail(LF_EINVAL, "out is NULL");
  *out = nullptr;
  int n = 0;
  LF_HIP(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(LF_EINVAL, "no such device");
  LF_HIP(hipSetDevice(device));
  lf_ctx* c = new lf_ctx();
  c->device = device;
  c->own_stream = hip_stream == nullptr;
  if (c->own_stream) {
    hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete c;
      return hip_fail(e, "hipStreamCreate");
    }
  } else {
    c->stream = (hipStream_t)hip_stream;
  }
  *out = c;
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_ctx_destroy(lf_ctx* c) try {
  if (!c) return LF_OK;
  hipSetDevice(c->device);
  if (c->own_stream) hipStreamDestroy(c->stream);
  delete c;
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

}  // extern "C"

namespace lf {

// spreads the low 21 bits of x to every third bit
// bounding box of every part's vertices: box[6 p .. 6 p + 5] = lo xyz, hi xyz
static std::vector<double> part_boxes(const double* V, const int32_t* part_off, int32_t n_parts) {
  std::vector<double> box(6 * (size_t)n_parts);
  for (int32_t p = 0; p < n_parts; ++p) {
    const int32_t a = part_off[p], b = part_off[p + 1];
    double* bx = box.data() + 6 * (size_t)p;
    if (a >= b) continue;  // an empty part keeps a zero box
    for (int d = 0; d < 3; ++d) bx[d] = bx[3 + d] = V[3ll * a + d];
    for (int32_t v = a; v < b; ++v)
      for (int d = 0; d < 3; ++d) {
        bx[d] = std::min(bx[d], V[3ll * v + d]);
        bx[3 + d] = std::max(bx[3 + d], V[3ll * v + d]);
      }
  }
  return box;
}

lf_status mesh_create(lf_ctx* ctx, const double* V, int32_t n_v, const int32_t* F, int32_t n_f,
                      int32_t op, const int32_t* part_off, int32_t n_parts, lf_mesh** out) {
  if (!ctx || !V || !F || !out) return fail(LF_EINVAL, "NULL argument");
  *out = nullptr;
  if (n_v < 3 || n_v >= kMaxVerts || n_f < 1 || (int64_t)n_f > 4ll * n_v)
    return fail(LF_EINVAL, "mesh size out of range (3 <= n_v < 2^25, 1 <= n_f <= 4 n_v)");
  if (op != LF_OP_GRAPH && op != LF_OP_COTAN) return fail(LF_EINVAL, "unknown operator");
  for (int64_t f = 0; f < n_f; ++f) {
    const int32_t a = F[3 * f], b = F[3 * f + 1], c = F[3 * f + 2];
    if (a < 0 || b < 0 || c < 0 || a >= n_v || b >= n_v || c >= n_v)
      return fail(LF_EINVAL, "face " + std::to_string(f) + " has a vertex id out of range");
    if (a == b || b == c || a == c)
      return fail(LF_EINVAL, "face " + std::to_string(f) + " repeats a vertex");
  }
  LF_HIP(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  lf_mesh* m = new lf_mesh();
  m->ctx = ctx;
  m->n_v = n_v;
  m->n_f = n_f;
  m->op = op;
  m->n_slices = (n_v + kSlice - 1) / kSlice;
  auto bail = [&](hipError_t e, const char* what) {
    lf_mesh_destroy(m);
    return hip_fail(e, what);
  };
  hipError_t e = dalloc(&m->V, 3ll * n_v);
  if (e == hipSuccess) e = dalloc(&m->F, 3ll * n_f);
  if (e == hipSuccess)
    e = hipMemcpyAsync(m->V, V, sizeof(double) * 3 * n_v, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(m->F, F, sizeof(int32_t) * 3 * n_f, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return bail(e, "mesh upload");
  int bad = 0;
  e = build_operator(m->V, m->F, n_v, n_f, op, &m->lptr, &m->lent, &m->ldiag, &m->nnz_off, &bad, s);
  if (e != hipSuccess) return bail(e, "operator");
  if (bad) {
    lf_mesh_destroy(m);
    return fail(LF_EINVAL, "zero-area face: cotangent weights undefined");
  }
  // the step's vertex order (a Morton curve per part, sorted on the GPU) and
  // its copy of the operator
  const std::vector<double> box = part_boxes(V, part_off, n_parts);
  e = dalloc(&m->perm, n_v);
  if (e == hipSuccess) e = dalloc(&m->inv, n_v);
  if (e == hipSuccess) e = locality_order(m->V, n_v, part_off, n_parts, box.data(), m->perm, m->inv, s);
  if (e == hipSuccess)
    e = permute_operator(m->lptr, m->lent, m->ldiag, m->perm, m->inv, n_v, m->nnz_off, &m->slptr,
                         &m->slent, &m->sldiag, s);
  if (e == hipSuccess) e = build_slices(m->slptr, m->slent, n_v, &m->lell, &m->op_w, s);
  if (e != hipSuccess) return bail(e, "operator in step order");
  *out = m;
  return LF_OK;
}

}  // namespace lf

extern "C" {

lf_status lf_mesh_create(lf_ctx* ctx, const double* V, int32_t n_v, const int32_t* F, int32_t n_f,
                         int32_t op, lf_mesh** out) try {
  const int32_t part[2] = {0, n_v};
  return mesh_create(ctx, V, n_v, F, n_f, op, part, 1, out);
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_mesh_destroy(lf_mesh* m) try {
  if (!m) return LF_OK;
  hipSetDevice(m->ctx->device);
  (void)hipFree(m->V);
  (void)hipFree(m->F);
  (void)hipFree(m->lptr);
  (void)hipFree(m->lent);
  (void)hipFree(m->ldiag);
  (void)hipFree(m->lell);
  (void)hipFree(m->perm);
  (void)hipFree(m->inv);
  (void)hipFree(m->slptr);
  (void)hipFree(m->slent);
  (void)hipFree(m->sldiag);
  delete m;
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_mesh_operator(lf_mesh* m, int64_t* nnz, int32_t* rowptr, int32_t* col, float* val,
                           int32_t is_dev) try {
  if (!m || !nnz) return fail(LF_EINVAL, "NULL argument");
  const int64_t total = m->nnz_off + m->n_v;
  *nnz = total;
  if (!rowptr && !col && !val) return LF_OK;
  if (!rowptr || !col || !val) return fail(LF_EINVAL, "rowptr, col and val must all be given");
  LF_HIP(hipSetDevice(m->ctx->device));
  hipStream_t s = m->ctx->stream;
  if (is_dev) {
    LF_HIP(launch_operator_export(m->lptr, m->lent, m->ldiag, m->n_v, rowptr, col, val, s));
    LF_HIP(hipStreamSynchronize(s));
    return LF_OK;
  }
  DevBuf<int32_t> dp, dc;
  DevBuf<float> dv;
  LF_HIP(dp.alloc(m->n_v + 1));
  LF_HIP(dc.alloc(total));
  LF_HIP(dv.alloc(total));
  LF_HIP(launch_operator_export(m->lptr, m->lent, m->ldiag, m->n_v, dp.p, dc.p, dv.p, s));
  LF_HIP(hipMemcpyAsync(rowptr, dp.p, sizeof(int32_t) * (m->n_v + 1), hipMemcpyDeviceToHost, s));
  LF_HIP(hipMemcpyAsync(col, dc.p, sizeof(int32_t) * total, hipMemcpyDeviceToHost, s));
  LF_HIP(hipMemcpyAsync(val, dv.p, sizeof(float) * total, hipMemcpyDeviceToHost, s));
  LF_HIP(hipStreamSynchronize(s));
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

static lf_status check_seeds(const int32_t* seeds, int32_t n_s, int32_t n_v) {
  if (n_s < 1 || n_s >= n_v) return fail(LF_EINVAL, "need 1 <= n_s < n_v seeds");
  if (!seeds) return fail(LF_EINVAL, "seeds is NULL");
  std::vector<char> used(n_v, 0);
  for (int32_t k = 0; k < n_s; ++k) {
    const int32_t v = seeds[k];
    if (v < 0 || v >= n_v) return fail(LF_EINVAL, "seed " + std::to_string(k) + " out of range");
    if (used[v]) return fail(LF_EINVAL, "seed vertex " + std::to_string(v) + " repeated");
    used[v] = 1;
  }
  return LF_OK;
}

static lf_status init_fields(lf_fields* f) {
  hipStream_t s = f->mesh->ctx->stream;
  const int32_t n_v = f->mesh->n_v;
  LF_HIP(hipMemcpyAsync(f->d_seeds, f->seeds.data(), sizeof(int32_t) * f->n_s,
                        hipMemcpyHostToDevice, s));
  if (f->region_owner.empty()) {
    LF_HIP(launch_fill_i32(f->owner, n_v, f->n_s, s));
    LF_HIP(launch_scatter_owner(f->d_seeds, f->n_s, f->owner, s));
    if (f->rings > 0) {
      DevBuf<int32_t> tmp;
      LF_HIP(tmp.alloc(n_v));
      int32_t* a = f->owner;
      int32_t* b = tmp.p;
      for (int32_t r = 0; r < f->rings; ++r) {
        LF_HIP(launch_ring_grow(f->mesh->lptr, f->mesh->lent, a, b, n_v, f->n_s, s));
        std::swap(a, b);
      }
      if (a != f->owner)
        LF_HIP(hipMemcpyAsync(f->owner, a, sizeof(int32_t) * n_v, hipMemcpyDeviceToDevice, s));
      LF_HIP(hipStreamSynchronize(s));
    }
  } else {
    LF_HIP(hipMemcpyAsync(f->owner, f->region_owner.data(), sizeof(int32_t) * n_v,
                          hipMemcpyHostToDevice, s));
  }
  f->cur = 0;
  f->next_reorder = f->steps + 128;  // once the fronts have met
  LF_HIP(launch_init_fields(f->owner, f->perm, n_v, f->ell[0], s));
  f->nnz = n_v;
  f->csr_valid = false;
  lf_status st = clear_step_state(f);
  if (st) return st;
  LF_HIP(hipStreamSynchronize(s));
  return LF_OK;
}

lf_status lf_fields_destroy(lf_fields* f) try {
  if (!f) return LF_OK;
  (void)hipSetDevice(f->mesh->ctx->device);
  // steps still in flight (lf_step_async) finish before their buffers go;
  // those not issued yet are dropped
  if (f->pending) (void)hipStreamSynchronize(f->mesh->ctx->stream);
  drop_graphs(f);
  fields_order_reset(f);
  for (int k = 0; k < 2; ++k) {
    (void)hipFree(f->ell[k]);
    (void)hipFree(f->ovf[k]);
  }
  (void)hipFree(f->d_seeds);
  (void)hipFree(f->owner);
  (void)hipFree(f->counters);
  (void)hipFree(f->wide);
  (void)hipFree(f->wide_rows);
  (void)hipFree(f->parts);
  (void)hipFree(f->stats);
  (void)hipFree(f->flags);
  (void)hipFree(f->uptr);
  (void)hipFree(f->uent);
  (void)hipFree(f->scan_tmp);
  (void)hipFree(f->types);
  (void)hipFree(f->coef);
  if (f->flags_host) (void)hipHostFree(f->flags_host);
  if (f->stats_pinned) (void)hipHostFree(f->stats_pinned);
  if (f->done_ev) (void)hipEventDestroy(f->done_ev);
  for (auto e : f->ev0) (void)hipEventDestroy(e);
  for (auto e : f->ev1) (void)hipEventDestroy(e);
  dual_release(f);
  delete f;
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

// owner of every vertex (region id, n_s outside all regions) and the first
// vertex of every region, from a caller's region lists
static lf_status check_regions(const int32_t* ptr, const int32_t* verts, int32_t n_s, int32_t n_v,
                               std::vector<int32_t>& owner, std::vector<int32_t>& first) {
  if (!ptr || !verts) return fail(LF_EINVAL, "NULL argument");
  if (n_s < 1 || n_s >= n_v) return fail(LF_EINVAL, "need 1 <= n_s < n_v regions");
  if (ptr[0] != 0) return fail(LF_EINVAL, "region_ptr[0] must be 0");
  owner.assign((size_t)n_v, n_s);
  first.resize((size_t)n_s);
  for (int32_t k = 0; k < n_s; ++k) {
    if (ptr[k + 1] <= ptr[k]) return fail(LF_EINVAL, "region " + std::to_string(k) + " is empty");
    if (ptr[k + 1] > n_v) return fail(LF_EINVAL, "regions hold more vertices than the mesh");
    first[(size_t)k] = verts[ptr[k]];
    for (int32_t p = ptr[k]; p < ptr[k + 1]; ++p) {
      const int32_t v = verts[p];
      if (v < 0 || v >= n_v)
        return fail(LF_EINVAL, "region " + std::to_string(k) + " has a vertex out of range");
      if (owner[(size_t)v] != n_s)
        return fail(LF_EINVAL, "vertex " + std::to_string(v) + " is in two regions");
      owner[(size_t)v] = k;
    }
  }
  return LF_OK;
}

static lf_status fields_new(lf_mesh* m, const int32_t* seeds, int32_t n_s, const lf_params* P,
                            std::vector<int32_t>&& region_owner, int32_t rings, lf_fields** out);

lf_status lf_fields_create(lf_mesh* m, const int32_t* seeds, int32_t n_s, const lf_params* P,
                           lf_fields** out) try {
  if (!m || !out) return fail(LF_EINVAL, "NULL argument");
  *out = nullptr;
  lf_status st = check_seeds(seeds, n_s, m->n_v);
  if (st) return st;
  return fields_new(m, seeds, n_s, P, std::vector<int32_t>(), 0, out);
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_fields_create_rings(lf_mesh* m, const int32_t* seeds, int32_t n_s, int32_t rings,
                                 const lf_params* P, lf_fields** out) try {
  if (!m || !out) return fail(LF_EINVAL, "NULL argument");
  *out = nullptr;
  if (rings < 0 || rings > 1024) return fail(LF_EINVAL, "rings must be in [0, 1024]");
  lf_status st = check_seeds(seeds, n_s, m->n_v);
  if (st) return st;
  return fields_new(m, seeds, n_s, P, std::vector<int32_t>(), rings, out);
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_fields_create_regions(lf_mesh* m, const int32_t* region_ptr,
                                   const int32_t* region_vertices, int32_t n_s, const lf_params* P,
                                   lf_fields** out) try {
  if (!m || !out) return fail(LF_EINVAL, "NULL argument");
  *out = nullptr;
  std::vector<int32_t> owner, first;
  lf_status st = check_regions(region_ptr, region_vertices, n_s, m->n_v, owner, first);
  if (st) return st;
  return fields_new(m, first.data(), n_s, P, std::move(owner), 0, out);
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_fields_reset_regions(lf_fields* f, const int32_t* region_ptr,
                                  const int32_t* region_vertices) try {
  if (!f) return fail(LF_EINVAL, "NULL argument");
  LF_SETTLE(f);
  std::vector<int32_t> owner, first;
  lf_status st = check_regions(region_ptr, region_vertices, f->n_s, f->mesh->n_v, owner, first);
  if (st) return st;
  LF_HIP(hipSetDevice(f->mesh->ctx->device));
  f->seeds = std::move(first);
  f->region_owner = std::move(owner);
  f->rings = 0;
  return init_fields(f);
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

}  // extern "C"

static lf_status fields_new(lf_mesh* m, const int32_t* seeds, int32_t n_s, const lf_params* P,
                            std::vector<int32_t>&& region_owner, int32_t rings, lf_fields** out) {
  lf_status st = LF_OK;
  lf_params prm;
  if (P) prm = *P;
  else lf_params_default(&prm);
  if (!(prm.dt > 0) || !(prm.mu >= 0) || !(prm.theta >= 0 && prm.theta < 1) ||
      (prm.base_mode != 0 && prm.base_mode != 1))
    return fail(LF_EINVAL, "invalid parameters");
  LF_HIP(hipSetDevice(m->ctx->device));
  lf_fields* f = new lf_fields();
  f->mesh = m;
  f->n_s = n_s;
  f->P = prm;
  f->seeds.assign(seeds, seeds + n_s);
  f->region_owner = std::move(region_owner);
  f->rings = rings;
  fields_order_reset(f);
  const int64_t hint = prm.capacity_hint > 0 ? prm.capacity_hint
                                             : std::max<int64_t>(4096, m->n_v / 16);
  f->ovf_cap = std::min<int64_t>(hint, (1ll << 31) - 1);
  hipError_t e = hipSuccess;
#define ALLOC(x, n)                          \
  if (e == hipSuccess) e = dalloc(&(x), (n));
  ALLOC(f->d_seeds, n_s);
  ALLOC(f->owner, m->n_v);
  for (int k = 0; k < 2; ++k) {
    ALLOC(f->ell[k], m->n_v + 1);
    ALLOC(f->ovf[k], f->ovf_cap);
  }
  ALLOC(f->counters, 4);
  f->wide_cap = 1024;
  ALLOC(f->wide, f->wide_cap);
  ALLOC(f->flags, 1);
  ALLOC(f->uptr, m->n_v + 1);
  ALLOC(f->scan_tmp, scan_tmp_elems(m->n_v));
#undef ALLOC
  if (e == hipSuccess) e = hipHostMalloc((void**)&f->flags_host, sizeof(StepFlags), 0);
  if (e != hipSuccess) {
    lf_fields_destroy(f);
    return hip_fail(e, "allocating field state");
  }
  e = launch_reset_flags(f->flags, nullptr, 0, m->ctx->stream);
  for (int k = 0; k < 2 && e == hipSuccess; ++k) {
    // row n_v: the empty row read in place of a missing neighbour
    static const EllRow empty{{Ent{-1, 0.f}, Ent{-1, 0.f}, Ent{-1, 0.f}}};
    e = hipMemcpy(f->ell[k] + m->n_v, &empty, sizeof(EllRow), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    lf_fields_destroy(f);
    return hip_fail(e, "reset flags");
  }
  st = init_fields(f);
  if (st) {
    lf_fields_destroy(f);
    return st;
  }
  *out = f;
  return LF_OK;
}

extern "C" {

lf_status lf_fields_reset(lf_fields* f, const int32_t* seeds) try {
  if (!f) return fail(LF_EINVAL, "NULL argument");
  LF_SETTLE(f);
  lf_status st = check_seeds(seeds, f->n_s, f->mesh->n_v);
  if (st) return st;
  LF_HIP(hipSetDevice(f->mesh->ctx->device));
  f->seeds.assign(seeds, seeds + f->n_s);
  f->region_owner.clear();
  return init_fields(f);
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_fields_seeds(lf_fields* f, int32_t* seeds) try {
  if (!f || !seeds) return fail(LF_EINVAL, "NULL argument");
  LF_SETTLE(f);
  memcpy(seeds, f->seeds.data(), sizeof(int32_t) * f->n_s);
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

static hipEvent_t pool_event(std::vector<hipEvent_t>& pool, size_t k) {
  while (pool.size() <= k) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    pool.push_back(e);
  }
  return pool[k];
}

}  // extern "C"

namespace lf {

void book_steps(lf_fields* f, const StepStats* st, int64_t ok) {
  for (int64_t k = 0; k < ok; ++k) {
    f->skel_total += st[k].skel;
    f->out_total += st[k].out;
    f->in_total += st[k].in;
    f->events_total += st[k].events;
  }
  f->cur = (int)((f->cur + ok) & 1);
  f->steps += ok;
  if (ok > 0) {
    f->nnz = (int64_t)st[ok - 1].out;
    f->csr_valid = false;
    f->last_changed = st[ok - 1].changed;
    f->last_dmax = bits_float(st[ok - 1].dmax);
  }
}

int64_t mesh_bytes(const lf_mesh* m) {
  const int64_t nv = m->n_v;
  return 24 * nv + 12ll * m->n_f + 2 * (4 * (nv + 1) + 8 * m->nnz_off + 4 * nv) + 8 * nv +
         8ll * m->n_slices * m->op_w * kSlice;
}

int64_t fields_bytes(const lf_fields* f) {
  const int64_t nv = f->mesh->n_v;
  return 2 * (int64_t)sizeof(EllRow) * (nv + 1) + 2 * 8 * f->ovf_cap + 4 * nv + 4ll * f->n_s +
         (int64_t)sizeof(WideRow) * f->wide_cap + (f->wide_rows ? 4 * nv : 0) +
         4 * (nv + 1) + 8 * f->csr_cap +
         8 * scan_tmp_elems(nv) + (int64_t)sizeof(StepStats) * f->stats_cap * (1 + kParts) +
         4ll * (f->n_s + 1) * (f->n_types > 0) + 16ll * f->n_types * f->n_types +
         (f->own_order ? 2 * 4 * nv + 4 * (nv + 1) + 8 * f->mesh->nnz_off + 4 * nv +
                             8ll * f->mesh->n_slices * f->op_w * kSlice + f->mesh->n_slices
                       : 0);
}

// Step counters and host copies for chunks of up to n steps.
lf_status ensure_step_buffers(lf_fields* f, int64_t n) {
  hipStream_t s = f->mesh->ctx->stream;
  if (n > f->stats_cap) {
    const int64_t c = std::max<int64_t>(n, 2 * f->stats_cap);
    StepStats *p = nullptr, *q = nullptr;
    LF_HIP(dalloc(&p, c));
    if (dalloc(&q, c * kParts) != hipSuccess) {
      (void)hipFree(p);
      return fail(LF_ENOMEM, "step counters");
    }
    LF_HIP(hipStreamSynchronize(s));
    (void)hipFree(f->stats);
    (void)hipFree(f->parts);
    f->stats = p;
    f->parts = q;
    f->stats_cap = c;
  }
  if (n > f->stats_pinned_cap) {
    const int64_t c = std::max<int64_t>(n, 2 * f->stats_pinned_cap);
    StepStats* p = nullptr;
    LF_HIP(hipHostMalloc((void**)&p, sizeof(StepStats) * c, 0));
    LF_HIP(hipStreamSynchronize(s));
    if (f->stats_pinned) (void)hipHostFree(f->stats_pinned);
    f->stats_pinned = p;
    f->stats_pinned_cap = c;
  }
  if (!f->done_ev) LF_HIP(hipEventCreateWithFlags(&f->done_ev, hipEventDisableTiming));
  return LF_OK;
}

StepArgs chunk_step_args(lf_fields* f, int64_t k, int64_t n) {
  StepArgs a = step_args(f, (int)((f->cur + k) & 1));
  a.parts = f->parts + k * kParts;
  a.step_idx = (uint32_t)k;
  a.measure = (f->measure_all || k == n - 1) ? 1u : 0u;
  return a;
}

static lf_status chunk_tail_copies(lf_fields* f, int64_t n, hipStream_t s) {
  LF_HIP(hipMemcpyAsync(f->flags_host, f->flags, sizeof(StepFlags), hipMemcpyDeviceToHost, s));
  LF_HIP(hipMemcpyAsync(f->stats_pinned, f->stats, sizeof(StepStats) * n, hipMemcpyDeviceToHost, s));
  return LF_OK;
}

lf_status chunk_tail(lf_fields* f, int64_t n, hipStream_t s) {
  LF_HIP(launch_reduce_parts(f->parts, n, f->stats, s));
  return chunk_tail_copies(f, n, s);
}

// what a captured chunk's kernels name: buffers, capacities, coefficient
// tables and which steps measure
static uint64_t graph_key(const lf_fields* f, int parity) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](uint64_t x) { h = (h ^ x) * 1099511628211ull; };
  mix((uint64_t)parity);
  mix((uint64_t)(uintptr_t)f->ovf[0]);
  mix((uint64_t)(uintptr_t)f->ovf[1]);
  mix((uint64_t)f->ovf_cap);
  mix((uint64_t)(uintptr_t)f->wide);
  mix((uint64_t)f->wide_cap);
  mix((uint64_t)(uintptr_t)f->wide_rows);
  mix((uint64_t)(uintptr_t)f->parts);
  mix((uint64_t)(uintptr_t)f->stats);
  mix((uint64_t)(uintptr_t)f->types);
  mix((uint64_t)(uintptr_t)f->coef);
  mix((uint64_t)f->n_types);
  mix((uint64_t)f->measure_all);
  mix((uint64_t)(uintptr_t)f->lell);
  mix((uint64_t)(uintptr_t)f->slice_cls);
  return h;
}

void drop_graphs(lf_fields* f) {
  for (int p = 0; p < 2; ++p) {
    if (f->graph[p]) (void)hipGraphExecDestroy(f->graph[p]);
    f->graph[p] = nullptr;
    f->graph_key[p] = 0;
  }
}

// the kernels of a chunk of n steps starting from the current buffer
static lf_status enqueue_chunk(lf_fields* f, int64_t n, hipStream_t s) {
  LF_HIP(launch_reset_flags(f->flags, f->parts, n, s));
  for (int64_t k = 0; k < n; ++k) LF_HIP(launch_step(chunk_step_args(f, k, n), s, nullptr, nullptr));
  LF_HIP(launch_reduce_parts(f->parts, n, f->stats, s));
  return LF_OK;
}

// a whole chunk from its captured graph (captured on first use)
static lf_status launch_chunk_graph(lf_fields* f, hipStream_t s) {
  const int p = f->cur & 1;
  const uint64_t key = graph_key(f, p);
  if (!f->graph[p] || f->graph_key[p] != key) {
    if (f->graph[p]) (void)hipGraphExecDestroy(f->graph[p]);
    f->graph[p] = nullptr;
    hipGraph_t g = nullptr;
    LF_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    lf_status st = enqueue_chunk(f, kMaxChunk, s);
    hipError_t e = hipStreamEndCapture(s, &g);
    if (st) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&f->graph[p], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      f->graph[p] = nullptr;
      return hip_fail(e, "hipGraphInstantiate");
    }
    f->graph_key[p] = key;
  }
  LF_HIP(hipGraphLaunch(f->graph[p], s));
  return LF_OK;
}

// Enqueues n steps on the context stream, then asynchronous copies of the
// failure flags and per-step counters and an event; does not wait.
lf_status step_issue(lf_fields* f, int64_t n) {
  LF_HIP(hipSetDevice(f->mesh->ctx->device));
  hipStream_t s = f->mesh->ctx->stream;
  if (f->reorder_every > 0 && f->steps >= f->next_reorder) {
    lf_status st = fields_reorder(f);
    if (st) return st;
    f->next_reorder = f->steps + f->reorder_every;
  }
  lf_status st = ensure_step_buffers(f, n);
  if (st) return st;
  if (f->use_graphs && n == kMaxChunk && f->timing <= 0 && s != nullptr) {
    st = launch_chunk_graph(f, s);
    if (st) return st;
    st = chunk_tail_copies(f, n, s);
    if (st) return st;
    LF_HIP(hipEventRecord(f->done_ev, s));
    f->pending = n;
    f->ev_issued = 0;
    return LF_OK;
  }
  LF_HIP(launch_reset_flags(f->flags, f->parts, n, s));
  size_t used = 0;
  for (int64_t k = 0; k < n; ++k) {
    StepArgs a = chunk_step_args(f, k, n);
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (f->timing > 0 && f->timing_ctr++ % f->timing == 0) {
      t0 = pool_event(f->ev0, used);
      t1 = pool_event(f->ev1, used);
      if (t0 && t1) ++used;
    }
    LF_HIP(launch_step(a, s, t0, t1));
  }
  st = chunk_tail(f, n, s);
  if (st) return st;
  LF_HIP(hipEventRecord(f->done_ev, s));
  f->pending = n;
  f->ev_issued = used;
  return LF_OK;
}

bool step_ready(lf_fields* f) {
  return f->pending == 0 || hipEventQuery(f->done_ev) == hipSuccess;
}

// Books a completed chunk of n steps from its flags and per-step counters
// (host copies): the steps before the first failed one count; storage that
// ran out is grown.  *remaining = steps that did not complete.
lf_status step_book(lf_fields* f, int64_t n, int64_t* remaining) {
  const StepFlags fl = *f->flags_host;
  // steps before the first failed one are complete; the later ones did nothing
  const int64_t ok = fl.poisoned ? std::min<int64_t>(fl.fail_step, n) : n;
  book_steps(f, f->stats_pinned, ok);
  *remaining = n - ok;
  if (fl.wide_seen && !f->wide_rows) {
    // rows touching more than kRowRegs layers occur: from the next chunk on
    // they are stepped after each step launch, one wavefront per row, so that
    // no wavefront steps many of them in turn
    LF_HIP(hipStreamSynchronize(f->mesh->ctx->stream));
    LF_HIP(dalloc(&f->wide_rows, f->mesh->n_v));
  }
  if (!fl.poisoned) return LF_OK;
  if (fl.poisoned & 2u) {
    clear_step_state(f);
    return fail(LF_ECAPACITY, "a vertex touches more than 64 layers");
  }
  if (fl.poisoned & 8u) {
    lf_status st = grow_wide(f);
    if (st) return st;
  }
  if (fl.poisoned & 1u) {
    lf_status st = grow(f, (int64_t)fl.need);
    if (st) return st;
  }
  return clear_step_state(f);
}

// Waits for the issued steps and books the completed ones.  *remaining is
// the number of issued steps that did not complete (storage was grown: issue
// them again).
lf_status step_complete(lf_fields* f, int64_t* remaining) {
  *remaining = 0;
  if (f->pending == 0) return LF_OK;
  LF_HIP(hipSetDevice(f->mesh->ctx->device));
  LF_HIP(hipEventSynchronize(f->done_ev));
  for (size_t k = 0; k < f->ev_issued; ++k) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, f->ev0[k], f->ev1[k]) == hipSuccess) {
      f->timed_ms += ms;
      f->timed_launches++;
    }
  }
  const int64_t n = f->pending;
  f->pending = 0;
  return step_book(f, n, remaining);
}

bool chunk_quiet(const lf_fields* f, int64_t n, double eps) {
  for (int64_t k = 0; k < n; ++k) {
    const StepStats& t = f->stats_pinned[k];
    if (t.changed != 0 || (double)bits_float(t.dmax) > eps) return false;
  }
  return n > 0;
}

}  // namespace lf

extern "C" {

lf_status lf_fields_set_coefficients(lf_fields* f, int32_t n_types, const int32_t* layer_types,
                                     const double* table) try {
  if (!f) return fail(LF_EINVAL, "NULL argument");
  LF_SETTLE(f);
  if (n_types < 0 || n_types > 65536) return fail(LF_EINVAL, "n_types out of range");
  if (n_types > 0 && (!layer_types || !table)) return fail(LF_EINVAL, "NULL argument");
  const int64_t n_r = (int64_t)f->n_s + 1, n_pairs = (int64_t)n_types * n_types;
  for (int64_t l = 0; n_types > 0 && l < n_r; ++l)
    if (layer_types[l] < 0 || layer_types[l] >= n_types) return fail(LF_EINVAL, "layer type out of range");
  std::vector<float4> tab;
  try {
    tab.resize((size_t)n_pairs);
  } catch (const std::bad_alloc&) {
    return fail(LF_ENOMEM, "coefficient table does not fit in host memory");
  }
  for (int64_t q = 0; q < n_pairs; ++q) {
    float v[3];
    for (int k = 0; k < 3; ++k) {
      v[k] = (float)table[3 * q + k];
      if (!std::isfinite(v[k])) return fail(LF_EINVAL, "coefficient not finite in float32");
    }
    tab[(size_t)q] = make_float4(v[0], v[1], v[2], 0.f);
  }
  LF_HIP(hipSetDevice(f->mesh->ctx->device));
  hipStream_t s = f->mesh->ctx->stream;
  // the steps already issued keep the old tables until they have run
  LF_HIP(hipStreamSynchronize(s));
  int32_t* types = nullptr;
  float4* coef = nullptr;
  if (n_types > 0) {
    hipError_t e = dalloc(&types, n_r);
    if (e == hipSuccess) e = dalloc(&coef, n_pairs);
    if (e == hipSuccess)
      e = hipMemcpyAsync(types, layer_types, sizeof(int32_t) * n_r, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(coef, tab.data(), sizeof(float4) * n_pairs, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      (void)hipFree(types);
      (void)hipFree(coef);
      return hip_fail(e, "coefficient tables");
    }
  }
  (void)hipFree(f->types);
  (void)hipFree(f->coef);
  f->types = types;
  f->coef = coef;
  f->n_types = n_types;
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_last_change(lf_fields* f, int64_t* changed_rows, double* max_delta) try {
  if (!f) return fail(LF_EINVAL, "NULL argument");
  LF_SETTLE(f);
  if (changed_rows) *changed_rows = (int64_t)f->last_changed;
  if (max_delta) *max_delta = (double)f->last_dmax;
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_step_until(lf_fields* f, int32_t max_steps, double eps, int32_t check_every,
                        int64_t* steps_done, int64_t* converged_at) try {
  if (!f || max_steps < 0 || check_every < 1 || check_every > kMaxChunk || !(eps >= 0))
    return fail(LF_EINVAL, "invalid argument");
  LF_SETTLE(f);
  int64_t done = 0, conv = 0;
  int grows = 0;
  f->measure_all = true;
  struct Restore {  // measures back to the last step of a chunk on every exit
    lf_fields* f;
    ~Restore() { f->measure_all = false; }
  } restore{f};
  while (done < max_steps && !conv) {
    const int64_t m = std::min<int64_t>((int64_t)max_steps - done, check_every);
    int64_t ok = 0;  // the chunk, replaying what storage growth interrupted
    while (ok < m) {
      lf_status st = step_issue(f, m - ok);
      if (st) return st;
      int64_t rem = 0;
      st = step_complete(f, &rem);
      if (st) return st;
      // a chunk is judged whole: any step of it that was not quiet, even one
      // before a replay, makes it not converged
      if (!chunk_quiet(f, m - ok - rem, eps)) conv = -1;
      ok += m - ok - rem;
      if (rem > 0 && ++grows > 32) return fail(LF_ECAPACITY, "field storage keeps overflowing");
    }
    done += m;
    conv = (conv == 0 && m == check_every) ? done : 0;
  }
  if (steps_done) *steps_done = done;
  if (converged_at) *converged_at = conv;
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

}  // extern "C"

namespace lf {

// steps n steps in chunks, each waited for and booked
static lf_status step_blocking(lf_fields* f, int64_t n) {
  int64_t left = n;
  int grows = 0;
  while (left > 0) {
    // chunks of at most kMaxChunk steps: the steps issued after a failed
    // one run for nothing, so a failure wastes at most one chunk
    const int64_t m = std::min<int64_t>(left, kMaxChunk);
    lf_status st = step_issue(f, m);
    if (st) return st;
    int64_t rem = 0;
    st = step_complete(f, &rem);
    if (st) return st;
    left -= m - rem;
    if (rem > 0 && ++grows > 32) return fail(LF_ECAPACITY, "field storage keeps overflowing");
  }
  return LF_OK;
}

lf_status fields_settle(lf_fields* f) {
  if (f->pending == 0 && f->async_left == 0) return LF_OK;
  int64_t rem = 0;
  lf_status st = step_complete(f, &rem);
  const int64_t left = rem + f->async_left;
  f->async_left = 0;
  if (st) return st;
  return step_blocking(f, left);
}

}  // namespace lf

extern "C" {

lf_status lf_step_async(lf_fields* f, int32_t n) try {
  if (!f || n < 0) return fail(LF_EINVAL, "invalid argument");
  LF_SETTLE(f);
  if (n == 0) return LF_OK;
  const int64_t m = std::min<int64_t>(n, kMaxChunk);
  lf_status st = step_issue(f, m);
  if (st) return st;
  f->async_left = n - m;
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_step(lf_fields* f, int32_t n) try {
  if (!f || n < 0) return fail(LF_EINVAL, "invalid argument");
  LF_SETTLE(f);
  return step_blocking(f, n);
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_fields_set_reorder(lf_fields* f, int32_t every, int32_t tile_rows,
                                int32_t classes) try {
  if (!f || every < 0 || tile_rows < 256 || tile_rows > kTileRows || tile_rows % 256 ||
      classes < 2 || classes > 4)
    return fail(LF_EINVAL, "invalid argument");
  LF_SETTLE(f);
  f->reorder_every = every;
  f->reorder_tile = tile_rows;
  f->reorder_classes = classes;
  if (every > 0) f->next_reorder = std::min<int64_t>(f->next_reorder, f->steps + every);
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_fields_reorders(lf_fields* f, int64_t* n) try {
  if (!f || !n) return fail(LF_EINVAL, "NULL argument");
  LF_SETTLE(f);
  *n = f->reorders;
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_fields_use_graphs(lf_fields* f, int32_t on) try {
  if (!f || (on != 0 && on != 1)) return fail(LF_EINVAL, "invalid argument");
  LF_SETTLE(f);
  LF_HIP(hipSetDevice(f->mesh->ctx->device));
  if (!on) drop_graphs(f);
  f->use_graphs = on == 1;
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_sync(lf_fields* f) try {
  if (!f) return fail(LF_EINVAL, "NULL argument");
  LF_SETTLE(f);
  LF_HIP(hipStreamSynchronize(f->mesh->ctx->stream));
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_fields_export(lf_fields* f, int64_t* nnz, int32_t* rowptr, int32_t* col, float* val,
                           int32_t is_dev) try {
  if (!f || !nnz) return fail(LF_EINVAL, "NULL argument");
  LF_SETTLE(f);
  *nnz = f->nnz;
  if (!rowptr && !col && !val) return LF_OK;
  if (!rowptr || !col || !val) return fail(LF_EINVAL, "rowptr, col and val must all be given");
  LF_HIP(hipSetDevice(f->mesh->ctx->device));
  hipStream_t s = f->mesh->ctx->stream;
  const int32_t n_v = f->mesh->n_v;
  const int32_t* up = nullptr;
  const Ent* ue = nullptr;
  lf_status st = fields_csr(f, &up, &ue);
  if (st) return st;
  if (is_dev) {
    LF_HIP(hipMemcpyAsync(rowptr, up, sizeof(int32_t) * (n_v + 1), hipMemcpyDeviceToDevice, s));
    LF_HIP(launch_split(ue, *nnz, col, val, s));
  } else {
    DevBuf<int32_t> dc;
    DevBuf<float> dv;
    LF_HIP(dc.alloc(*nnz));
    LF_HIP(dv.alloc(*nnz));
    LF_HIP(launch_split(ue, *nnz, dc.p, dv.p, s));
    LF_HIP(hipMemcpyAsync(rowptr, up, sizeof(int32_t) * (n_v + 1), hipMemcpyDeviceToHost, s));
    if (*nnz > 0) {
      LF_HIP(hipMemcpyAsync(col, dc.p, sizeof(int32_t) * *nnz, hipMemcpyDeviceToHost, s));
      LF_HIP(hipMemcpyAsync(val, dv.p, sizeof(float) * *nnz, hipMemcpyDeviceToHost, s));
    }
  }
  LF_HIP(hipStreamSynchronize(s));
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_fields_import(lf_fields* f, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                           const float* val, int32_t is_dev) try {
  if (!f || !rowptr || (nnz > 0 && (!col || !val)) || nnz < 0)
    return fail(LF_EINVAL, "invalid argument");
  LF_SETTLE(f);
  if (nnz > (1ll << 31) - 1) return fail(LF_EINVAL, "more than 2^31 entries");
  LF_HIP(hipSetDevice(f->mesh->ctx->device));
  hipStream_t s = f->mesh->ctx->stream;
  const int32_t n_v = f->mesh->n_v;
  DevBuf<int32_t> dp, dc, bad;
  DevBuf<float> dv;
  const int32_t* p = rowptr;
  const int32_t* c = col;
  const float* v = val;
  if (!is_dev) {
    if (rowptr[n_v] != nnz || rowptr[0] != 0) return fail(LF_EINVAL, "rowptr does not match nnz");
    for (int32_t i = 0; i < n_v; ++i)
      if (rowptr[i + 1] < rowptr[i]) return fail(LF_EINVAL, "rowptr is not monotone");
    LF_HIP(dp.alloc(n_v + 1));
    LF_HIP(dc.alloc(nnz));
    LF_HIP(dv.alloc(nnz));
    LF_HIP(hipMemcpyAsync(dp.p, rowptr, sizeof(int32_t) * (n_v + 1), hipMemcpyHostToDevice, s));
    if (nnz > 0) {
      LF_HIP(hipMemcpyAsync(dc.p, col, sizeof(int32_t) * nnz, hipMemcpyHostToDevice, s));
      LF_HIP(hipMemcpyAsync(dv.p, val, sizeof(float) * nnz, hipMemcpyHostToDevice, s));
    }
    p = dp.p;
    c = dc.p;
    v = dv.p;
  } else {
    int32_t last = -1;
    LF_HIP(hipMemcpyAsync(&last, rowptr + n_v, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    LF_HIP(hipStreamSynchronize(s));
    if (last != nnz) return fail(LF_EINVAL, "rowptr does not match nnz");
  }
  // validated into the CSR view, then converted to fixed-width rows in the
  // other buffer (the current fields stay intact on error)
  f->csr_valid = false;
  lf_status st = reserve_csr(f, nnz);
  if (st) return st;
  if (nnz > f->ovf_cap) {
    st = grow(f, nnz);
    if (st) return st;
  }
  LF_HIP(bad.alloc(1));
  LF_HIP(launch_fill_i32(bad.p, 1, 0, s));
  LF_HIP(launch_join_check(c, v, p, n_v, f->n_s + 1, nnz, f->uent, bad.p, s));
  int32_t hb = 0;
  LF_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  LF_HIP(hipStreamSynchronize(s));
  if (hb) return fail(LF_EINVAL, "imported fields are not canonical (code " + std::to_string(hb) + ")");
  LF_HIP(hipMemcpyAsync(f->uptr, p, sizeof(int32_t) * (n_v + 1), hipMemcpyDeviceToDevice, s));
  const int tgt = 1 - f->cur;
  LF_HIP(csr_to_ell(f->uptr, f->uent, f->inv, n_v, f->ell[tgt], f->ovf[tgt], s));
  f->cur = tgt;
  f->nnz = nnz;
  f->csr_valid = true;
  st = clear_step_state(f);
  if (st) return st;
  LF_HIP(hipStreamSynchronize(s));
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_labels(lf_fields* f, int32_t* labels, int32_t is_dev) try {
  if (!f || !labels) return fail(LF_EINVAL, "NULL argument");
  LF_SETTLE(f);
  LF_HIP(hipSetDevice(f->mesh->ctx->device));
  hipStream_t s = f->mesh->ctx->stream;
  const int32_t n_v = f->mesh->n_v;
  const int32_t* up = nullptr;
  const Ent* ue = nullptr;
  lf_status st = fields_csr(f, &up, &ue);
  if (st) return st;
  if (is_dev) {
    LF_HIP(launch_labels(up, ue, n_v, f->n_s, labels, s));
  } else {
    DevBuf<int32_t> d;
    LF_HIP(d.alloc(n_v));
    LF_HIP(launch_labels(up, ue, n_v, f->n_s, d.p, s));
    LF_HIP(hipMemcpyAsync(labels, d.p, sizeof(int32_t) * n_v, hipMemcpyDeviceToHost, s));
    LF_HIP(hipStreamSynchronize(s));
    return LF_OK;
  }
  LF_HIP(hipStreamSynchronize(s));
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_stats(lf_fields* f, int64_t* nnz_u, int64_t* skel, int64_t* steps, int64_t* empty,
                   int64_t* grows) try {
  if (!f) return fail(LF_EINVAL, "NULL argument");
  LF_SETTLE(f);
  LF_HIP(hipSetDevice(f->mesh->ctx->device));
  if (nnz_u) *nnz_u = f->nnz;
  if (skel) *skel = (int64_t)f->skel_total;
  if (steps) *steps = f->steps;
  if (empty) *empty = (int64_t)f->events_total;
  if (grows) *grows = f->grow_events;
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_traffic(lf_fields* f, int64_t* entries_in, int64_t* entries_out) try {
  if (!f) return fail(LF_EINVAL, "NULL argument");
  LF_SETTLE(f);
  if (entries_in) *entries_in = (int64_t)f->in_total;
  if (entries_out) *entries_out = (int64_t)f->out_total;
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_step_timing(lf_fields* f, int32_t enable, double* total_ms, int64_t* launches) try {
  if (!f) return fail(LF_EINVAL, "NULL argument");
  LF_SETTLE(f);
  if (total_ms) *total_ms = f->timed_ms;
  if (launches) *launches = f->timed_launches;
  if (enable >= 0) {
    if (enable && !f->timing) {
      f->timed_ms = 0.0;
      f->timed_launches = 0;
      f->timing_ctr = 0;
    }
    f->timing = enable;
  }
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

}  // extern "C"
