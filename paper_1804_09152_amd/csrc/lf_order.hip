// Re-ordering of the step's rows by work class.
//
// A wavefront's time is set by its most expensive row, and in the locality
// order almost every 64-row slice mixes rows inside a cell (one layer, and
// every neighbour holding that same single layer: the step leaves such a row
// at exactly {layer: 1}) with rows in and next to the bands between cells
// (the full merge and update).  Every few hundred steps the rows of each
// tile of kTileRows consecutive rows are re-ordered, stably, interior rows
// first; slices made only of interior rows are flagged, and the step kernel
// gives them a short path that checks the condition again and writes the row
// without merging (any slice whose check fails takes the full path, so the
// results do not depend on the order or on the flags).  Tiles keep rows near
// their neighbours (the tile is a patch of the locality order), so the L2
// still serves the neighbour rows.  The fields, their overflow area, the
// operator copy (slices, CSR and diagonal, every row keeping its entries in
// the mesh's order) and the vertex <-> row maps are permuted on the GPU.
#include <algorithm>
#include <new>

#include "lf_internal.h"

namespace lf {
namespace {

constexpr int kT = 256;
constexpr int kPerMax = kTileRows / kT;  // rows per thread in the tile ranking, at most

unsigned blocks_of(int64_t n, int t = kT) { return (unsigned)((n + t - 1) / t); }

// Work class of a row: 0 for an interior row (one inline entry of layer c,
// and every neighbour row one inline entry of layer c); otherwise 1, 2 or 3
// for at most 2, 3, or more distinct layers in the row and its neighbours
// (the number of slots the merge and update run over).  A row with entries
// beyond the slice width, or reading an overflow row, is class 3.
constexpr int kClasses = 4;

__global__ void k_classify(const EllRow* u, const Ent* lell, int32_t op_w, int32_t n_v,
                           int32_t n_classes, uint8_t* cls) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_v) return;
  const int sl = i / kSlice, lane = i % kSlice;
  const Ent* ops = lell + (int64_t)sl * op_w * kSlice + lane;
  int32_t seen[4];
  int n = 0;
  bool big = false;
  auto add_row = [&](const EllRow& r) {
    if (r.e[0].col == kOvfMark) {
      big = true;
      return;
    }
    for (int j = 0; j < kEll && r.e[j].col >= 0; ++j) {
      bool dup = false;
      for (int t = 0; t < n; ++t) dup = dup || seen[t] == r.e[j].col;
      if (dup) continue;
      if (n == 4) {
        big = true;
        return;
      }
      seen[n++] = r.e[j].col;
    }
  };
  const EllRow own = u[i];
  const int32_t c = own.e[0].col;
  bool in = c >= 0 && own.e[1].col < 0;
  add_row(own);
  for (int k = 0; k < op_w; ++k) {
    const Ent le = ops[k * kSlice];
    if (le.col < 0) continue;
    const EllRow nb = u[le.col];
    in = in && nb.e[0].col == c && nb.e[1].col < 0;
    add_row(nb);
  }
  if (op_w == kOpWidth && ops[(kOpWidth - 1) * kSlice].col >= 0) {
    in = false;
    big = true;
  }
  const int q = in ? 0 : (big || n >= 4) ? 3 : (n == 3 ? 2 : 1);
  cls[i] = (uint8_t)(q < n_classes ? q : n_classes - 1);
}

// new position of every row: per tile, the rows of class 0, then 1, 2, 3,
// each class in its current order (a stable counting sort per tile)
__global__ __launch_bounds__(kT) void k_tile_rank(const uint8_t* cls, int32_t n_v,
                                                  int32_t tile, int32_t* newpos) {
  // per thread, the counts of its rows of each class, 16 bits each
  __shared__ unsigned long long sh[kT];
  const int kPer = tile / kT;
  const int64_t t0 = (int64_t)blockIdx.x * tile;
  const int32_t tile_n = (int32_t)(n_v - t0 < tile ? n_v - t0 : tile);
  const int r0 = threadIdx.x * kPer;
  unsigned long long mine = 0;
  for (int q = 0; q < kPer; ++q) {
    const int r = r0 + q;
    if (r < tile_n) mine += 1ull << (16 * cls[t0 + r]);
  }
  sh[threadIdx.x] = mine;
  __syncthreads();
  for (int o = 1; o < kT; o <<= 1) {  // inclusive scan (Hillis-Steele)
    const unsigned long long y = threadIdx.x >= o ? sh[threadIdx.x - o] : 0ull;
    __syncthreads();
    sh[threadIdx.x] += y;
    __syncthreads();
  }
  const unsigned long long tot = sh[kT - 1];
  unsigned long long before = sh[threadIdx.x] - mine;
  int base[kClasses], at[kClasses];
  int acc = 0;
  for (int q = 0; q < kClasses; ++q) {
    base[q] = acc;
    acc += (int)((tot >> (16 * q)) & 0xffff);
    at[q] = (int)((before >> (16 * q)) & 0xffff);
  }
  for (int q = 0; q < kPer; ++q) {
    const int r = r0 + q;
    if (r >= tile_n) break;
    const int k = cls[t0 + r];
    newpos[t0 + r] = (int32_t)(t0 + base[k] + at[k]);
    ++at[k];
  }
}

// moves row k to newpos[k]: the order maps, the class and the fields row
__global__ void k_apply_order(const int32_t* newpos, const int32_t* perm_old, int32_t n_v,
                              const uint8_t* cls, const EllRow* u_old, int32_t* perm_new,
                              int32_t* inv_new, uint8_t* cls_new, EllRow* u_new) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_v) return;
  const int32_t p = newpos[k], v = perm_old[k];
  perm_new[p] = v;
  inv_new[v] = p;
  cls_new[p] = cls[k];
  u_new[p] = u_old[k];
}

// a slice is flagged when all of its rows are interior (rows past the last
// vertex count as interior); one wavefront per slice
__global__ __launch_bounds__(kSlice) void k_slice_flags(const uint8_t* cls, int32_t n_v,
                                                        uint8_t* flags) {
  const int i = blockIdx.x * kSlice + threadIdx.x;
  const bool in = i >= n_v || cls[i] == 0;
  const bool all = __all(in);
  if (threadIdx.x == 0) flags[blockIdx.x] = all ? 1 : 0;
}

template <class T>
struct Buf {
  T* p = nullptr;
  ~Buf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(int64_t n) { return dalloc(&p, n); }
  T* release() {
    T* q = p;
    p = nullptr;
    return q;
  }
};

}  // namespace

void fields_order_reset(lf_fields* f) {
  if (f->own_order) {
    (void)hipFree(const_cast<int32_t*>(f->perm));
    (void)hipFree(const_cast<int32_t*>(f->inv));
    (void)hipFree(const_cast<Ent*>(f->lell));
    (void)hipFree(const_cast<int32_t*>(f->slptr));
    (void)hipFree(const_cast<Ent*>(f->slent));
    (void)hipFree(const_cast<float*>(f->sldiag));
  }
  (void)hipFree(f->slice_cls);
  const lf_mesh* m = f->mesh;
  f->perm = m->perm;
  f->inv = m->inv;
  f->lell = m->lell;
  f->slptr = m->slptr;
  f->slent = m->slent;
  f->sldiag = m->sldiag;
  f->op_w = m->op_w;
  f->slice_cls = nullptr;
  f->own_order = false;
}

lf_status fields_reorder(lf_fields* f) {
  lf_mesh* m = f->mesh;
  const int32_t n_v = m->n_v, n_sl = m->n_slices;
  hipStream_t s = m->ctx->stream;
  LF_HIP(hipSetDevice(m->ctx->device));
  Buf<uint8_t> cls, cls_new, flags;
  Buf<int32_t> newpos, perm, inv;
  LF_HIP(cls.alloc(n_v));
  LF_HIP(cls_new.alloc(n_v));
  LF_HIP(flags.alloc(n_sl));
  LF_HIP(newpos.alloc(n_v));
  LF_HIP(perm.alloc(n_v));
  LF_HIP(inv.alloc(n_v));
  const int cur = f->cur;
  hipLaunchKernelGGL(k_classify, dim3(blocks_of(n_v)), dim3(kT), 0, s, f->ell[cur], f->lell,
                     f->op_w, n_v, f->reorder_classes, cls.p);
  LF_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_tile_rank, dim3(blocks_of(n_v, f->reorder_tile)), dim3(kT), 0, s, cls.p,
                     n_v, f->reorder_tile, newpos.p);
  LF_HIP(hipGetLastError());
  // the fields move to the other buffer, which becomes the current one; the
  // overflow area moves with them (rows keep their offsets)
  hipLaunchKernelGGL(k_apply_order, dim3(blocks_of(n_v)), dim3(kT), 0, s, newpos.p, f->perm, n_v,
                     cls.p, f->ell[cur], perm.p, inv.p, cls_new.p, f->ell[1 - cur]);
  LF_HIP(hipGetLastError());
  LF_HIP(hipMemcpyAsync(f->ovf[1 - cur], f->ovf[cur], sizeof(Ent) * f->ovf_cap,
                        hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(k_slice_flags, dim3((unsigned)n_sl), dim3(kSlice), 0, s, cls_new.p, n_v,
                     flags.p);
  LF_HIP(hipGetLastError());
  // the operator copy in the new order, from the mesh's CSR (every row keeps
  // its entries in the mesh's order, so every row sums the same terms in the
  // same order as before)
  int32_t* plptr = nullptr;
  Ent* plent = nullptr;
  float* pldiag = nullptr;
  LF_HIP(permute_operator(m->lptr, m->lent, m->ldiag, perm.p, inv.p, n_v, m->nnz_off, &plptr,
                          &plent, &pldiag, s));
  Ent* plell = nullptr;
  int32_t w = 0;
  hipError_t e = build_slices(plptr, plent, n_v, &plell, &w, s);
  if (e != hipSuccess) {
    (void)hipFree(plptr);
    (void)hipFree(plent);
    (void)hipFree(pldiag);
    return hip_fail(e, "re-ordered operator slices");
  }
  LF_HIP(hipStreamSynchronize(s));
  drop_graphs(f);
  if (f->own_order) {
    (void)hipFree(const_cast<int32_t*>(f->perm));
    (void)hipFree(const_cast<int32_t*>(f->inv));
    (void)hipFree(const_cast<Ent*>(f->lell));
    (void)hipFree(const_cast<int32_t*>(f->slptr));
    (void)hipFree(const_cast<Ent*>(f->slent));
    (void)hipFree(const_cast<float*>(f->sldiag));
  }
  (void)hipFree(f->slice_cls);
  f->perm = perm.release();
  f->inv = inv.release();
  f->lell = plell;
  f->slptr = plptr;
  f->slent = plent;
  f->sldiag = pldiag;
  f->op_w = w;
  f->slice_cls = flags.release();
  f->own_order = true;
  f->cur = 1 - cur;
  f->reorders++;
  // the step counters are per buffer parity: start both clean
  LF_HIP(launch_fill_i32((int32_t*)f->counters, 4, 0, s));
  LF_HIP(launch_reset_flags(f->flags, nullptr, 0, s));
  LF_HIP(hipStreamSynchronize(s));
  return LF_OK;
}

}  // namespace lf
