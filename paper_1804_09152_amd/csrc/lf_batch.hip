// Batches of independent meshes stepped by the same launches: the batch is
// the disjoint union of its meshes with per-mesh layer offsets and one
// shared base layer (see lf.h).
#include <string.h>

#include <new>
#include <string>
#include <vector>

#include "lf_internal.h"

struct lf_batch {
  lf_ctx* ctx;
  lf_mesh* mesh;
  lf_fields* fields;
  int32_t n;
  std::vector<int32_t> voff, nv, soff, ns;
  int32_t base;  // shared base layer
};

namespace lf {
namespace {

constexpr int kT = 256;

// rows [row0, row0 + nrows) of a batch's fields, renumbered to one mesh
__global__ void k_batch_extract(const int32_t* uptr, const Ent* uent, int32_t row0, int32_t nrows,
                                int32_t off, int32_t base, int32_t ns, int32_t* rp, int32_t* col,
                                float* val) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > nrows) return;
  const int32_t b0 = uptr[row0];
  rp[i] = uptr[row0 + i] - b0;
  if (i == nrows) return;
  for (int32_t p = uptr[row0 + i]; p < uptr[row0 + i + 1]; ++p) {
    const Ent e = uent[p];
    col[p - b0] = e.col == base ? ns : e.col - off;
    val[p - b0] = e.val;
  }
}

__global__ void k_batch_labels(const int32_t* lab, int32_t row0, int32_t nrows, int32_t off,
                               int32_t* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  const int32_t l = lab[row0 + i];
  out[i] = l < 0 ? -1 : l - off;
}

lf_status bfail(lf_status st, const std::string& m) {
  set_error(m);
  return st;
}

template <class T>
struct DBuf {
  T* p = nullptr;
  ~DBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(int64_t n) { return dalloc(&p, n); }
};

}  // namespace
}  // namespace lf

using namespace lf;

extern "C" {

lf_status lf_batch_create(lf_ctx* ctx, int32_t n, const double* const* V, const int32_t* n_v,
                          const int32_t* const* F, const int32_t* n_f, int32_t op,
                          const int32_t* const* seeds, const int32_t* n_s, const lf_params* P,
                          lf_batch** out) try {
  if (!ctx || n < 1 || !V || !n_v || !F || !n_f || !seeds || !n_s || !out)
    return bfail(LF_EINVAL, "invalid argument");
  *out = nullptr;
  int64_t tv = 0, tf = 0, ts = 0;
  for (int32_t m = 0; m < n; ++m) {
    if (!V[m] || !F[m] || !seeds[m] || n_v[m] < 3 || n_f[m] < 1 || n_s[m] < 1 || n_s[m] >= n_v[m])
      return bfail(LF_EINVAL, "mesh " + std::to_string(m) + " is invalid");
    tv += n_v[m];
    tf += n_f[m];
    ts += n_s[m];
  }
  if (tv >= kMaxVerts || tf > 4 * tv) return bfail(LF_EINVAL, "batch too large");
  lf_batch* b = new lf_batch();
  b->ctx = ctx;
  b->n = n;
  std::vector<double> Vc((size_t)(3 * tv));
  std::vector<int32_t> Fc((size_t)(3 * tf)), Sc((size_t)ts);
  int64_t vo = 0, fo = 0, so = 0;
  for (int32_t m = 0; m < n; ++m) {
    b->voff.push_back((int32_t)vo);
    b->nv.push_back(n_v[m]);
    b->soff.push_back((int32_t)so);
    b->ns.push_back(n_s[m]);
    memcpy(Vc.data() + 3 * vo, V[m], sizeof(double) * 3 * n_v[m]);
    for (int64_t k = 0; k < 3ll * n_f[m]; ++k) {
      const int32_t x = F[m][k];
      if (x < 0 || x >= n_v[m]) {
        delete b;
        return bfail(LF_EINVAL, "mesh " + std::to_string(m) + " has a vertex id out of range");
      }
      Fc[(size_t)(3 * fo + k)] = x + (int32_t)vo;
    }
    for (int32_t k = 0; k < n_s[m]; ++k) {
      const int32_t s = seeds[m][k];
      if (s < 0 || s >= n_v[m]) {
        delete b;
        return bfail(LF_EINVAL, "mesh " + std::to_string(m) + " has a seed out of range");
      }
      Sc[(size_t)(so + k)] = s + (int32_t)vo;
    }
    vo += n_v[m];
    fo += n_f[m];
    so += n_s[m];
  }
  b->base = (int32_t)ts;
  std::vector<int32_t> parts(b->voff);
  parts.push_back((int32_t)tv);
  lf_status st = lf::mesh_create(ctx, Vc.data(), (int32_t)tv, Fc.data(), (int32_t)tf, op,
                                 parts.data(), n, &b->mesh);
  if (st) {
    delete b;
    return st;
  }
  st = lf_fields_create(b->mesh, Sc.data(), (int32_t)ts, P, &b->fields);
  if (st) {
    lf_mesh_destroy(b->mesh);
    delete b;
    return st;
  }
  *out = b;
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_batch_destroy(lf_batch* b) try {
  if (!b) return LF_OK;
  lf_fields_destroy(b->fields);
  lf_mesh_destroy(b->mesh);
  delete b;
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_batch_fields(lf_batch* b, lf_fields** f) try {
  if (!b || !f) return bfail(LF_EINVAL, "NULL argument");
  *f = b->fields;
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_batch_export(lf_batch* b, int32_t m, int64_t* nnz, int32_t* rowptr, int32_t* col,
                          float* val) try {
  if (!b || !nnz || m < 0 || m >= b->n) return bfail(LF_EINVAL, "invalid argument");
  LF_SETTLE(b->fields);
  lf_fields* f = b->fields;
  LF_HIP(hipSetDevice(b->ctx->device));
  hipStream_t s = b->ctx->stream;
  const int32_t r0 = b->voff[m], nr = b->nv[m];
  const int32_t* up = nullptr;
  const Ent* ue = nullptr;
  lf_status st = fields_csr(f, &up, &ue);
  if (st) return st;
  int32_t lo = 0, hi = 0;
  LF_HIP(hipMemcpyAsync(&lo, up + r0, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  LF_HIP(hipMemcpyAsync(&hi, up + r0 + nr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  LF_HIP(hipStreamSynchronize(s));
  *nnz = hi - lo;
  if (!rowptr && !col && !val) return LF_OK;
  if (!rowptr || !col || !val) return bfail(LF_EINVAL, "rowptr, col and val must all be given");
  DBuf<int32_t> drp, dc;
  DBuf<float> dv;
  LF_HIP(drp.alloc(nr + 1));
  LF_HIP(dc.alloc(*nnz));
  LF_HIP(dv.alloc(*nnz));
  hipLaunchKernelGGL(k_batch_extract, dim3((nr + kT) / kT), dim3(kT), 0, s, up, ue, r0, nr, b->soff[m], b->base, b->ns[m], drp.p, dc.p, dv.p);
  LF_HIP(hipGetLastError());
  LF_HIP(hipMemcpyAsync(rowptr, drp.p, sizeof(int32_t) * (nr + 1), hipMemcpyDeviceToHost, s));
  if (*nnz > 0) {
    LF_HIP(hipMemcpyAsync(col, dc.p, sizeof(int32_t) * *nnz, hipMemcpyDeviceToHost, s));
    LF_HIP(hipMemcpyAsync(val, dv.p, sizeof(float) * *nnz, hipMemcpyDeviceToHost, s));
  }
  LF_HIP(hipStreamSynchronize(s));
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_batch_labels(lf_batch* b, int32_t m, int32_t* labels) try {
  if (!b || !labels || m < 0 || m >= b->n) return bfail(LF_EINVAL, "invalid argument");
  LF_SETTLE(b->fields);
  lf_fields* f = b->fields;
  LF_HIP(hipSetDevice(b->ctx->device));
  hipStream_t s = b->ctx->stream;
  const int32_t r0 = b->voff[m], nr = b->nv[m];
  const int32_t* up = nullptr;
  const Ent* ue = nullptr;
  lf_status st = fields_csr(f, &up, &ue);
  if (st) return st;
  DBuf<int32_t> all, part;
  LF_HIP(all.alloc(f->mesh->n_v));
  LF_HIP(part.alloc(nr));
  LF_HIP(launch_labels(up, ue, f->mesh->n_v, f->n_s, all.p, s));
  hipLaunchKernelGGL(k_batch_labels, dim3((nr + kT - 1) / kT), dim3(kT), 0, s, all.p, r0, nr,
                     b->soff[m], part.p);
  LF_HIP(hipGetLastError());
  LF_HIP(hipMemcpyAsync(labels, part.p, sizeof(int32_t) * nr, hipMemcpyDeviceToHost, s));
  LF_HIP(hipStreamSynchronize(s));
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

}  // extern "C"
