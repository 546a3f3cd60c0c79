// Setup-time kernels: mesh operator and its slices, field initialisation,
// scans, conversions between the fixed-width field rows and CSR, labels.
#include <algorithm>

#include "lf_internal.h"

namespace lf {

namespace {

constexpr int kT = 256;

inline unsigned blocks_for(int64_t n, int per = kT) {
  int64_t b = (n + per - 1) / per;
  return (unsigned)(b < 1 ? 1 : b);
}

// ---- fills -----------------------------------------------------------------

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---- initialisation (Algorithm 1, first line) --------------------------------

__global__ void k_scatter_owner(const int32_t* seeds, int32_t n_s, int32_t* owner) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n_s) owner[seeds[k]] = k;
}

// One ring of seed regions (Algorithm 1, first line: a seed and its
// neighbours): a vertex not yet in a region joins the lowest-index region
// among its neighbours' (n_s = none); the regions of the previous ring are
// read from own_in, the grown ones written to own_out.  Ring by ring this
// gives every vertex within r edges of a seed the lowest index among its
// nearest seeds, and a seed keeps itself.
__global__ void k_ring_grow(const int32_t* lptr, const Ent* lent, const int32_t* own_in,
                            int32_t* own_out, int32_t n_v, int32_t n_s) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_v) return;
  int32_t o = own_in[v];
  if (o == n_s)
    for (int32_t q = lptr[v]; q < lptr[v + 1]; ++q) o = min(o, own_in[lent[q].col]);
  own_out[v] = o;
}

// owner[v] = seed index of v, or n_s (the base layer) for unseeded vertices
// (fields rows are in the step's vertex order: row k holds vertex perm[k])
__global__ void k_init_fields(const int32_t* owner, const int32_t* perm, int32_t n_v, EllRow* u) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_v) {
    EllRow r;
    r.e[0] = Ent{owner[perm[i]], 1.0f};
#pragma unroll
    for (int j = 1; j < kEll; ++j) r.e[j] = Ent{-1, 0.f};
    u[i] = r;
  }
}

// ---- layouts: operator slices, fixed-width field rows <-> CSR -------------------

// largest off-diagonal count of any row
__global__ void k_max_degree(const int32_t* lptr, int32_t n_v, int32_t* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int d = i < n_v ? lptr[i + 1] - lptr[i] : 0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) d = max(d, __shfl_xor(d, o, 64));
  if ((threadIdx.x & 63) == 0 && d > 0) atomicMax(out, d);
}

__global__ void k_slice_fill(const int32_t* lptr, const Ent* lent, int32_t n_v, int32_t n_sl,
                             int32_t w, Ent* lell) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int sl = i / kSlice, lane = i % kSlice;
  if (sl >= n_sl) return;
  const int a = i < n_v ? lptr[i] : 0, n = i < n_v ? lptr[i + 1] - a : 0;
  for (int k = 0; k < w; ++k)
    lell[((int64_t)sl * w + k) * kSlice + lane] = k < n ? lent[a + k] : Ent{-1, 0.f};
}

// CSR row i (caller's vertex order) is fields row inv[i]
__global__ void k_ell_count(const EllRow* u, const int32_t* inv, int32_t n_v, int32_t* cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_v) return;
  const EllRow r = u[inv[i]];
  int n = 0;
  if (r.e[0].col == kOvfMark) {
    n = (int)ovf_dec(r.e[2].col);
  } else {
#pragma unroll
    for (int j = 0; j < kEll; ++j) n += r.e[j].col >= 0 ? 1 : 0;
  }
  cnt[i] = n;
}

__global__ void k_ell_fill(const EllRow* u, const Ent* ovf, const int32_t* inv, int32_t n_v,
                           const int32_t* uptr, Ent* uent) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_v) return;
  const EllRow r = u[inv[i]];
  const int32_t o = uptr[i], n = uptr[i + 1] - o;
  if (r.e[0].col == kOvfMark) {
    const Ent* src = ovf + ovf_dec(r.e[1].col);
    for (int j = 0; j < n; ++j) uent[o + j] = src[j];
  } else {
    for (int j = 0; j < n; ++j) uent[o + j] = r.e[j];
  }
}

__global__ void k_csr_to_ell(const int32_t* uptr, const Ent* uent, const int32_t* inv,
                             int32_t n_v, EllRow* u, Ent* ovf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_v) return;
  const int32_t a = uptr[i], n = uptr[i + 1] - a;
  EllRow r;
  if (n > kEll) {
    r.e[0] = Ent{kOvfMark, 0.f};
    r.e[1] = Ent{ovf_enc(a), 0.f};
    r.e[2] = Ent{ovf_enc(n), 0.f};
    for (int j = 0; j < n; ++j) ovf[a + j] = uent[a + j];
  } else {
#pragma unroll
    for (int j = 0; j < kEll; ++j) r.e[j] = j < n ? uent[a + j] : Ent{-1, 0.f};
  }
  u[inv[i]] = r;
}

// the step's operator: row k is vertex perm[k], columns renumbered through
// inv, entries kept in their order (so every row sums in the same order)
__global__ void k_perm_count(const int32_t* lptr, const int32_t* perm, int32_t n_v, int32_t* cnt) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n_v) cnt[k] = lptr[perm[k] + 1] - lptr[perm[k]];
}

__global__ void k_perm_fill(const int32_t* lptr, const Ent* lent, const float* ldiag,
                            const int32_t* perm, const int32_t* inv, int32_t n_v,
                            const int32_t* plptr, Ent* plent, float* pldiag) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_v) return;
  const int32_t v = perm[k], a = lptr[v], n = lptr[v + 1] - a, o = plptr[k];
  for (int j = 0; j < n; ++j) {
    const Ent e = lent[a + j];
    plent[o + j] = Ent{inv[e.col], e.val};
  }
  pldiag[k] = ldiag[v];
}

// ---- exclusive scan -------------------------------------------------------------
// three passes: per-block sums, one block scanning the block sums, per-block
// scan with its offset.  Blocks cover kScanItems elements.

constexpr int kScanPer = 4;
constexpr int kScanItems = kT * kScanPer;

__device__ __forceinline__ long long block_incl_scan(long long v, long long* sh) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const long long y = __shfl_up(v, o, 64);
    if (lane >= o) v += y;
  }
  if (lane == 63) sh[wid] = v;
  __syncthreads();
  long long off = 0;
  for (int w = 0; w < wid; ++w) off += sh[w];
  __syncthreads();
  return v + off;
}

__global__ __launch_bounds__(kT) void k_scan_sums(const int32_t* in, int64_t n, long long* sums) {
  __shared__ long long sh[kT / 64];
  const int64_t b0 = (int64_t)blockIdx.x * kScanItems;
  long long v = 0;
  for (int k = 0; k < kScanPer; ++k) {
    const int64_t j = b0 + (int64_t)threadIdx.x * kScanPer + k;
    if (j < n) v += in[j];
  }
  const long long incl = block_incl_scan(v, sh);
  if (threadIdx.x == kT - 1) sums[blockIdx.x] = incl;
}

__global__ __launch_bounds__(kT) void k_scan_sums_scan(long long* sums, int64_t nb) {
  __shared__ long long sh[kT / 64];
  __shared__ long long carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t c0 = 0; c0 < nb; c0 += kT) {
    const int64_t j = c0 + threadIdx.x;
    const long long v = j < nb ? sums[j] : 0;
    const long long incl = block_incl_scan(v, sh);
    const long long base = carry;
    if (j < nb) sums[j] = base + incl - v;  // exclusive
    __syncthreads();
    if (threadIdx.x == kT - 1) carry = base + incl;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kT) void k_scan_apply(const int32_t* in, int64_t n,
                                                  const long long* offs, int32_t* out) {
  __shared__ long long sh[kT / 64];
  const int64_t b0 = (int64_t)blockIdx.x * kScanItems;
  int32_t vals[kScanPer];
  long long v = 0;
  for (int k = 0; k < kScanPer; ++k) {
    const int64_t j = b0 + (int64_t)threadIdx.x * kScanPer + k;
    vals[k] = j < n ? in[j] : 0;
    v += vals[k];
  }
  const long long incl = block_incl_scan(v, sh);
  long long run = offs[blockIdx.x] + incl - v;
  for (int k = 0; k < kScanPer; ++k) {
    const int64_t j = b0 + (int64_t)threadIdx.x * kScanPer + k;
    if (j < n) out[j] = (int32_t)run;
    run += vals[k];
    if (j == n - 1) out[n] = (int32_t)run;
  }
}

// ---- operator (Section 3.2, Laplacian computation) ------------------------------

struct HalfEdge {
  int32_t col;
  int32_t face;
  double w;
};

__global__ void k_face_count(const int32_t* F, int32_t n_f, int32_t* cnt) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n_f) return;
  for (int k = 0; k < 3; ++k) atomicAdd(&cnt[F[3 * (int64_t)f + k]], 2);
}

// for every corner o of a face, the opposite edge (p, q) gets the corner's
// half cotangent (cotangent operator) or 1 (graph operator), both ways
__global__ void k_face_fill(const double* V, const int32_t* F, int32_t n_f, int op,
                            int32_t* cursor, HalfEdge* he, int32_t* bad) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n_f) return;
  const int32_t* c = F + 3 * (int64_t)f;
  for (int k = 0; k < 3; ++k) {
    const int32_t o = c[k], p = c[(k + 1) % 3], q = c[(k + 2) % 3];
    double w = 1.0;
    if (op == 1) {
      const double ux = V[3 * (int64_t)p] - V[3 * (int64_t)o];
      const double uy = V[3 * (int64_t)p + 1] - V[3 * (int64_t)o + 1];
      const double uz = V[3 * (int64_t)p + 2] - V[3 * (int64_t)o + 2];
      const double vx = V[3 * (int64_t)q] - V[3 * (int64_t)o];
      const double vy = V[3 * (int64_t)q + 1] - V[3 * (int64_t)o + 1];
      const double vz = V[3 * (int64_t)q + 2] - V[3 * (int64_t)o + 2];
      const double cx = uy * vz - uz * vy, cy = uz * vx - ux * vz, cz = ux * vy - uy * vx;
      const double s = sqrt(cx * cx + cy * cy + cz * cz);
      if (s == 0.0) { atomicOr(bad, 1); return; }
      w = 0.5 * (ux * vx + uy * vy + uz * vz) / s;
    }
    int32_t a = atomicAdd(&cursor[p], 1);
    he[a] = HalfEdge{q, f, w};
    a = atomicAdd(&cursor[q], 1);
    he[a] = HalfEdge{p, f, w};
  }
}

// per row: order the half-edges by (neighbour, face) so that the sum of the
// contributions of one edge has a fixed order, merge, and take the diagonal
// as minus the sum of the row (float64, in neighbour order)
__global__ void k_row_merge(const int32_t* tptr, HalfEdge* he, int32_t n_v, int op,
                            int32_t* ucnt, float* ldiag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_v) return;
  const int32_t a = tptr[i], b = tptr[i + 1];
  for (int32_t x = a + 1; x < b; ++x) {
    const HalfEdge h = he[x];
    int32_t y = x - 1;
    while (y >= a && (he[y].col > h.col || (he[y].col == h.col && he[y].face > h.face))) {
      he[y + 1] = he[y];
      --y;
    }
    he[y + 1] = h;
  }
  int32_t m = 0;
  double diag = 0.0;
  for (int32_t x = a; x < b;) {
    int32_t y = x;
    double s = 0.0;
    while (y < b && he[y].col == he[x].col) { s += he[y].w; ++y; }
    if (op == 0) s = 1.0;
    he[a + m] = HalfEdge{he[x].col, 0, s};
    diag -= s;
    ++m;
    x = y;
  }
  ucnt[i] = m;
  ldiag[i] = (float)diag;
}

__global__ void k_row_emit(const int32_t* tptr, const HalfEdge* he, const int32_t* lptr,
                           int32_t n_v, Ent* lent) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_v) return;
  const int32_t a = tptr[i], o = lptr[i], m = lptr[i + 1] - lptr[i];
  for (int32_t k = 0; k < m; ++k) lent[o + k] = Ent{he[a + k].col, (float)he[a + k].w};
}

// operator with the diagonal in its sorted place
__global__ void k_operator_export(const int32_t* lptr, const Ent* lent, const float* ldiag,
                                  int32_t n_v, int32_t* rowptr, int32_t* col, float* val) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_v) return;
  int32_t o = lptr[i] + i;
  rowptr[i] = o;
  if (i == n_v - 1) rowptr[n_v] = lptr[n_v] + n_v;
  if (!col) return;
  bool placed = false;
  for (int32_t q = lptr[i]; q < lptr[i + 1]; ++q) {
    if (!placed && lent[q].col > i) {
      col[o] = i; val[o] = ldiag[i]; ++o; placed = true;
    }
    col[o] = lent[q].col; val[o] = lent[q].val; ++o;
  }
  if (!placed) { col[o] = i; val[o] = ldiag[i]; }
}

// ---- field import / export --------------------------------------------------------

__global__ void k_split(const Ent* e, int64_t n, int32_t* col, float* val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) { col[i] = e[i].col; val[i] = e[i].val; }
}

// checks a caller's CSR for canonical form while packing it; bad != 0 on error
__global__ void k_join_check(const int32_t* col, const float* val, const int32_t* ptr,
                             int32_t n_v, int32_t n_r, int64_t nnz, Ent* out, int32_t* bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_v) return;
  const int32_t a = ptr[i], b = ptr[i + 1];
  if (i == 0 && a != 0) atomicOr(bad, 1);
  if (a < 0 || b < a || (int64_t)b > nnz) { atomicOr(bad, 2); return; }
  int32_t last = -1;
  for (int32_t p = a; p < b; ++p) {
    const int32_t c = col[p];
    const float v = val[p];
    if (c <= last || c >= n_r) atomicOr(bad, 4);
    if (!(v > 0.f && v <= 1.f)) atomicOr(bad, 8);
    last = c;
    out[p] = Ent{c, v};
  }
}

// ---- labels (sharp visualisation, Figure 10) -------------------------------------

__global__ void k_labels(const int32_t* uptr, const Ent* uent, int32_t n_v, int32_t n_s,
                         int32_t* labels) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_v) return;
  int32_t best = -1;
  float bv = 0.f;
  for (int32_t p = uptr[i]; p < uptr[i + 1]; ++p) {
    const Ent e = uent[p];
    if (e.col >= n_s) continue;  // the base layer is no cell
    if (best < 0 || e.val > bv) { best = e.col; bv = e.val; }
  }
  labels[i] = best;
}

// spreads the low 21 bits of x to every third bit
__device__ __forceinline__ unsigned long long spread3(unsigned long long x) {
  x &= 0x1fffffull;
  x = (x | (x << 32)) & 0x1f00000000ffffull;
  x = (x | (x << 16)) & 0x1f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

constexpr int kIdBits = 25;  // vertex ids below 2^25

// key of vertex v: its part (top part_bits bits), the interleaved positions
// quantised to axis_bits bits per axis in the part's box, then v
__global__ void k_morton_keys(const double* V, int32_t n_v, const int32_t* part_off,
                              int32_t n_parts, const double* box, int part_bits, int axis_bits,
                              unsigned long long* keys) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_v) return;
  int32_t lo = 0, hi = n_parts;  // the part holding v: part_off[lo] <= v < part_off[lo + 1]
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (part_off[mid] <= v) lo = mid;
    else hi = mid;
  }
  const double* b = box + 6 * (int64_t)lo;
  const double top = (double)((1u << axis_bits) - 1u);
  unsigned long long code = 0;
  for (int k = 0; k < 3; ++k) {
    const double ext = b[3 + k] - b[k];
    double t = ext > 0.0 ? (V[3 * (int64_t)v + k] - b[k]) / ext : 0.0;
    if (!(t >= 0.0)) t = 0.0;  // also NaN
    if (t > 1.0) t = 1.0;
    code |= spread3((unsigned long long)(t * top)) << k;
  }
  const unsigned long long part = part_bits ? (unsigned long long)lo << (64 - part_bits) : 0ull;
  keys[v] = part | (code << kIdBits) | (unsigned long long)v;
}

__global__ void k_order_from_keys(const unsigned long long* keys, int32_t n_v, int32_t* perm,
                                  int32_t* inv) {
  const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_v) return;
  const int32_t v = (int32_t)(keys[k] & ((1ull << kIdBits) - 1ull));
  perm[k] = v;
  inv[v] = k;
}

}  // namespace

hipError_t locality_order(const double* V, int32_t n_v, const int32_t* part_off, int32_t n_parts,
                          const double* box, int32_t* perm, int32_t* inv, hipStream_t s) {
  // 64 bits: part, 3 axes, vertex id
  int part_bits = 0;
  while ((1ll << part_bits) < n_parts) ++part_bits;
  const int axis_bits = std::max(1, std::min(21, (64 - kIdBits - part_bits) / 3));
  int64_t N = 1;
  while (N < n_v) N <<= 1;
  unsigned long long* keys = nullptr;
  int32_t* d_off = nullptr;
  double* d_box = nullptr;
  hipError_t e = dalloc(&keys, N);
  if (e == hipSuccess) e = dalloc(&d_off, (int64_t)n_parts + 1);
  if (e == hipSuccess) e = dalloc(&d_box, 6ll * n_parts);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_off, part_off, sizeof(int32_t) * (n_parts + 1), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_box, box, sizeof(double) * 6 * n_parts, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_morton_keys, dim3(blocks_for(n_v)), dim3(kT), 0, s, V, n_v, d_off, n_parts,
                       d_box, part_bits, axis_bits, keys);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = sort_keys_u64(keys, n_v, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_order_from_keys, dim3(blocks_for(n_v)), dim3(kT), 0, s, keys, n_v, perm,
                       inv);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // before the buffers are freed
  (void)hipFree(keys);
  (void)hipFree(d_off);
  (void)hipFree(d_box);
  return e;
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n)), dim3(kT), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(n)), dim3(kT), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_scatter_owner(const int32_t* seeds, int32_t n_s, int32_t* owner,
                                hipStream_t s) {
  if (n_s <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_owner, dim3(blocks_for(n_s)), dim3(kT), 0, s, seeds, n_s, owner);
  return hipGetLastError();
}
hipError_t launch_ring_grow(const int32_t* lptr, const Ent* lent, const int32_t* own_in,
                           int32_t* own_out, int32_t n_v, int32_t n_s, hipStream_t s) {
  hipLaunchKernelGGL(k_ring_grow, dim3(blocks_for(n_v)), dim3(kT), 0, s, lptr, lent, own_in,
                     own_out, n_v, n_s);
  return hipGetLastError();
}
hipError_t launch_init_fields(const int32_t* owner, const int32_t* perm, int32_t n_v, EllRow* u,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_init_fields, dim3(blocks_for(n_v)), dim3(kT), 0, s, owner, perm, n_v, u);
  return hipGetLastError();
}

int64_t scan_tmp_elems(int64_t n) { return (n + kScanItems - 1) / kScanItems + 1; }

hipError_t exclusive_scan(const int32_t* in, int32_t* out, int64_t n, long long* tmp,
                          hipStream_t s) {
  if (n <= 0) return hipMemsetAsync(out, 0, sizeof(int32_t), s);
  const int64_t nb = (n + kScanItems - 1) / kScanItems;
  hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(kT), 0, s, in, n, tmp);
  hipLaunchKernelGGL(k_scan_sums_scan, dim3(1), dim3(kT), 0, s, tmp, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kT), 0, s, in, n, tmp, out);
  return hipGetLastError();
}

hipError_t build_operator(const double* V, const int32_t* F, int32_t n_v, int32_t n_f, int op,
                          int32_t** lptr_out, Ent** lent_out, float** ldiag_out,
                          int64_t* nnz_off, int* bad_face, hipStream_t s) {
  hipError_t e;
  int32_t *cnt = nullptr, *tptr = nullptr, *cursor = nullptr, *ucnt = nullptr, *lptr = nullptr,
          *bad = nullptr;
  long long* tmp = nullptr;
  HalfEdge* he = nullptr;
  Ent* lent = nullptr;
  float* ldiag = nullptr;
  int32_t total = 0, h_bad = 0;
  *bad_face = 0;
#define TRY(x)                   \
  do {                           \
    e = (x);                     \
    if (e != hipSuccess) goto fail; \
  } while (0)
  TRY(dalloc(&cnt, n_v));
  TRY(dalloc(&tptr, n_v + 1));
  TRY(dalloc(&cursor, n_v + 1));
  TRY(dalloc(&ucnt, n_v));
  TRY(dalloc(&lptr, n_v + 1));
  TRY(dalloc(&bad, 1));
  TRY(dalloc(&tmp, scan_tmp_elems(n_v)));
  TRY(dalloc(&ldiag, n_v));
  TRY(hipMemsetAsync(cnt, 0, sizeof(int32_t) * n_v, s));
  TRY(hipMemsetAsync(bad, 0, sizeof(int32_t), s));
  hipLaunchKernelGGL(k_face_count, dim3(blocks_for(n_f)), dim3(kT), 0, s, F, n_f, cnt);
  TRY(hipGetLastError());
  TRY(exclusive_scan(cnt, tptr, n_v, tmp, s));
  TRY(hipMemcpyAsync(cursor, tptr, sizeof(int32_t) * (n_v + 1), hipMemcpyDeviceToDevice, s));
  TRY(hipMemcpyAsync(&total, tptr + n_v, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  TRY(hipStreamSynchronize(s));
  TRY(dalloc(&he, total));
  hipLaunchKernelGGL(k_face_fill, dim3(blocks_for(n_f)), dim3(kT), 0, s, V, F, n_f, op, cursor,
                     he, bad);
  TRY(hipGetLastError());
  TRY(hipMemcpyAsync(&h_bad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  TRY(hipStreamSynchronize(s));
  if (h_bad) { *bad_face = 1; e = hipSuccess; goto fail; }
  hipLaunchKernelGGL(k_row_merge, dim3(blocks_for(n_v)), dim3(kT), 0, s, tptr, he, n_v, op, ucnt,
                     ldiag);
  TRY(hipGetLastError());
  TRY(exclusive_scan(ucnt, lptr, n_v, tmp, s));
  TRY(hipMemcpyAsync(&total, lptr + n_v, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  TRY(hipStreamSynchronize(s));
  TRY(dalloc(&lent, total));
  hipLaunchKernelGGL(k_row_emit, dim3(blocks_for(n_v)), dim3(kT), 0, s, tptr, he, lptr, n_v, lent);
  TRY(hipGetLastError());
  TRY(hipStreamSynchronize(s));
  hipFree(cnt); hipFree(tptr); hipFree(cursor); hipFree(ucnt); hipFree(bad); hipFree(tmp);
  hipFree(he);
  *lptr_out = lptr;
  *lent_out = lent;
  *ldiag_out = ldiag;
  *nnz_off = total;
  return hipSuccess;
fail:
  hipFree(cnt); hipFree(tptr); hipFree(cursor); hipFree(ucnt); hipFree(bad); hipFree(tmp);
  hipFree(he); hipFree(lptr); hipFree(lent); hipFree(ldiag);
  return e;
#undef TRY
}

hipError_t build_slices(const int32_t* lptr, const Ent* lent, int32_t n_v, Ent** lell,
                        int32_t* width, hipStream_t s) {
  *lell = nullptr;
  const int32_t n_sl = (n_v + kSlice - 1) / kSlice;
  int32_t* dmax = nullptr;
  hipError_t e = dalloc(&dmax, 1);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(kT), 0, s, dmax, (int64_t)1, 0);
    hipLaunchKernelGGL(k_max_degree, dim3(blocks_for(n_v)), dim3(kT), 0, s, lptr, n_v, dmax);
    e = hipGetLastError();
  }
  int32_t d = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&d, dmax, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(dmax);
  const int32_t w = d < kOpWidth ? d : kOpWidth;
  if (e == hipSuccess) e = dalloc(lell, (int64_t)n_sl * kSlice * (w > 0 ? w : 1));
  if (e == hipSuccess && w > 0) {
    hipLaunchKernelGGL(k_slice_fill, dim3(blocks_for((int64_t)n_sl * kSlice)), dim3(kT), 0, s,
                       lptr, lent, n_v, n_sl, w, *lell);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipFree(*lell);
    *lell = nullptr;
  }
  *width = w;
  return e;
}

hipError_t ell_to_csr_ptr(const EllRow* u, const int32_t* inv, int32_t n_v, int32_t* counts,
                          int32_t* uptr, long long* tmp, hipStream_t s) {
  hipLaunchKernelGGL(k_ell_count, dim3(blocks_for(n_v)), dim3(kT), 0, s, u, inv, n_v, counts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return exclusive_scan(counts, uptr, n_v, tmp, s);
}

hipError_t ell_to_csr_fill(const EllRow* u, const Ent* ovf, const int32_t* inv, int32_t n_v,
                           const int32_t* uptr, Ent* uent, hipStream_t s) {
  hipLaunchKernelGGL(k_ell_fill, dim3(blocks_for(n_v)), dim3(kT), 0, s, u, ovf, inv, n_v, uptr,
                     uent);
  return hipGetLastError();
}

hipError_t csr_to_ell(const int32_t* uptr, const Ent* uent, const int32_t* inv, int32_t n_v,
                      EllRow* u, Ent* ovf, hipStream_t s) {
  hipLaunchKernelGGL(k_csr_to_ell, dim3(blocks_for(n_v)), dim3(kT), 0, s, uptr, uent, inv, n_v, u,
                     ovf);
  return hipGetLastError();
}

hipError_t permute_operator(const int32_t* lptr, const Ent* lent, const float* ldiag,
                            const int32_t* perm, const int32_t* inv, int32_t n_v, int64_t nnz,
                            int32_t** plptr, Ent** plent, float** pldiag, hipStream_t s) {
  *plptr = nullptr;
  *plent = nullptr;
  *pldiag = nullptr;
  int32_t* cnt = nullptr;
  long long* tmp = nullptr;
  hipError_t e = dalloc(&cnt, n_v);
  if (e == hipSuccess) e = dalloc(&tmp, scan_tmp_elems(n_v));
  if (e == hipSuccess) e = dalloc(plptr, n_v + 1);
  if (e == hipSuccess) e = dalloc(plent, nnz);
  if (e == hipSuccess) e = dalloc(pldiag, n_v);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_perm_count, dim3(blocks_for(n_v)), dim3(kT), 0, s, lptr, perm, n_v, cnt);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = exclusive_scan(cnt, *plptr, n_v, tmp, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_perm_fill, dim3(blocks_for(n_v)), dim3(kT), 0, s, lptr, lent, ldiag,
                       perm, inv, n_v, *plptr, *plent, *pldiag);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(cnt);
  (void)hipFree(tmp);
  if (e != hipSuccess) {
    (void)hipFree(*plptr);
    (void)hipFree(*plent);
    (void)hipFree(*pldiag);
    *plptr = nullptr;
    *plent = nullptr;
    *pldiag = nullptr;
  }
  return e;
}

hipError_t launch_split(const Ent* e, int64_t n, int32_t* col, float* val, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_split, dim3(blocks_for(n)), dim3(kT), 0, s, e, n, col, val);
  return hipGetLastError();
}
hipError_t launch_join_check(const int32_t* col, const float* val, const int32_t* ptr,
                             int32_t n_v, int32_t n_r, int64_t nnz, Ent* out, int32_t* bad,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_join_check, dim3(blocks_for(n_v)), dim3(kT), 0, s, col, val, ptr, n_v, n_r,
                     nnz, out, bad);
  return hipGetLastError();
}
hipError_t launch_operator_export(const int32_t* lptr, const Ent* lent, const float* ldiag,
                                  int32_t n_v, int32_t* rowptr, int32_t* col, float* val,
                                  hipStream_t s) {
  hipLaunchKernelGGL(k_operator_export, dim3(blocks_for(n_v)), dim3(kT), 0, s, lptr, lent, ldiag,
                     n_v, rowptr, col, val);
  return hipGetLastError();
}
hipError_t launch_labels(const int32_t* uptr, const Ent* uent, int32_t n_v, int32_t n_s,
                         int32_t* labels, hipStream_t s) {
  hipLaunchKernelGGL(k_labels, dim3(blocks_for(n_v)), dim3(kT), 0, s, uptr, uent, n_v, n_s, labels);
  return hipGetLastError();
}

}  // namespace lf
