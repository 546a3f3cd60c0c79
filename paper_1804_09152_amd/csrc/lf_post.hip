// Lloyd-like re-seeding and dual-mesh extraction (Section 5) on gfx950.
//
// Both run once per Lloyd round, not per time step.  Geometry is float64.
// Every result is deterministic: per-cell sums are accumulated in 64-bit
// fixed point (integer atomics are order independent), minima use integer
// atomics on order-preserving keys, and sets of cell pairs are built in hash
// tables and then sorted.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "lf_internal.h"

namespace lf {

namespace {

constexpr int kT = 256;
constexpr unsigned long long kEmpty = ~0ull;

inline unsigned nblk(int64_t n) {
  const int64_t b = (n + kT - 1) / kT;
  return (unsigned)(b < 1 ? 1 : b);
}

// ---- generic helpers ---------------------------------------------------------

__global__ void k_fill64(unsigned long long* p, int64_t n, unsigned long long v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// one compare-exchange stage of a bitonic sort over n (a power of two) keys
__global__ void k_bitonic(unsigned long long* a, int64_t n, int64_t k, int64_t j) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t l = i ^ j;
  if (l <= i) return;
  const unsigned long long x = a[i], y = a[l];
  const bool up = (i & k) == 0;
  if (up ? (x > y) : (x < y)) {
    a[i] = y;
    a[l] = x;
  }
}

// The stages of the same network whose partners lie within one chunk of C
// keys (C a power of two, at most kSortChunk), run by one block in LDS:
// with k = 0 every stage of k = 2..C (the chunk sorted in the direction
// the network gives it), otherwise the steps j = C/2..1 of stage k > C.
// Same compare-exchanges in the same order as the one-stage kernel.
constexpr int kSortChunk = 2048;
// rounds of an iteration to a fixed point launched per read of its flag
constexpr int kCheckEvery = 16;
__global__ __launch_bounds__(1024) void k_bitonic_local(unsigned long long* a, int64_t C, int64_t k) {
  __shared__ unsigned long long sh[kSortChunk];
  const int64_t base = (int64_t)blockIdx.x * C;
  for (int64_t t = threadIdx.x; t < C; t += blockDim.x) sh[t] = a[base + t];
  __syncthreads();
  auto stage = [&](int64_t kk, int64_t j) {
    for (int64_t t = threadIdx.x; t < C / 2; t += blockDim.x) {
      const int64_t i = 2 * j * (t / j) + (t % j), l = i + j;
      const bool up = ((base + i) & kk) == 0;
      const unsigned long long x = sh[i], y = sh[l];
      if (up ? (x > y) : (x < y)) {
        sh[i] = y;
        sh[l] = x;
      }
    }
    __syncthreads();
  };
  if (k == 0) {
    for (int64_t kk = 2; kk <= C; kk <<= 1)
      for (int64_t j = kk >> 1; j > 0; j >>= 1) stage(kk, j);
  } else {
    for (int64_t j = C >> 1; j > 0; j >>= 1) stage(k, j);
  }
  for (int64_t t = threadIdx.x; t < C; t += blockDim.x) a[base + t] = sh[t];
}

// sorts keys[0..n) ascending in place; keys has room for next_pow2(n)
hipError_t sort_u64(unsigned long long* keys, int64_t n, hipStream_t s) {
  if (n <= 1) return hipSuccess;
  int64_t N = 1;
  while (N < n) N <<= 1;
  if (N > n) hipLaunchKernelGGL(k_fill64, dim3(nblk(N - n)), dim3(kT), 0, s, keys + n, N - n, kEmpty);
  const int64_t C = std::min<int64_t>(N, kSortChunk);
  const dim3 lg((unsigned)(N / C)), lb((unsigned)std::min<int64_t>(C / 2, 1024));
  hipLaunchKernelGGL(k_bitonic_local, lg, lb, 0, s, keys, C, (int64_t)0);
  for (int64_t k = 2 * C; k <= N; k <<= 1) {
    for (int64_t j = k >> 1; j >= C; j >>= 1)
      hipLaunchKernelGGL(k_bitonic, dim3(nblk(N)), dim3(kT), 0, s, keys, N, k, j);
    hipLaunchKernelGGL(k_bitonic_local, lg, lb, 0, s, keys, C, k);
  }
  return hipGetLastError();
}

int64_t pow2_at_least(int64_t n) {
  int64_t N = 1;
  while (N < n) N <<= 1;
  return N;
}

__device__ __forceinline__ unsigned long long hash64(unsigned long long x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ull;
  x ^= x >> 33;
  return x;
}

// insert into an open-addressing set of `cap` (power of two) slots
__device__ __forceinline__ void set_insert(unsigned long long* tab, int64_t cap,
                                           unsigned long long key, int* overflow) {
  unsigned long long h = hash64(key) & (unsigned long long)(cap - 1);
  for (int64_t probe = 0; probe < cap; ++probe) {
    const unsigned long long old = atomicCAS(&tab[h], kEmpty, key);
    if (old == kEmpty || old == key) return;
    h = (h + 1) & (unsigned long long)(cap - 1);
  }
  atomicOr(overflow, 1);
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// the keys of a hash set, in any order (they are sorted next): one atomic
// per wavefront reserves the wavefront's run of the output
__global__ void k_set_extract(const unsigned long long* tab, int64_t cap, unsigned long long* out,
                              unsigned long long* count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned long long k = i < cap ? tab[i] : kEmpty;
  const bool has = k != kEmpty;
  const unsigned long long mask = __ballot(has);
  const int lane = (int)(threadIdx.x & 63);
  unsigned long long base = 0;
  if (lane == 0 && mask) base = atomicAdd(count, (unsigned long long)__popcll(mask));
  base = __shfl(base, 0, 64);
  if (has) out[base + __popcll(mask & ((1ull << lane) - 1ull))] = k;
}

__device__ __forceinline__ bool bsearch_u64(const unsigned long long* a, int64_t n,
                                            unsigned long long key, int64_t* at) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  *at = lo;
  return lo < n && a[lo] == key;
}

__device__ __forceinline__ bool bsearch_i32(const int32_t* a, int32_t lo, int32_t hi, int32_t key) {
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return a[lo] == key && lo >= 0;
}

// value of layer c at vertex v (0 when absent)
__device__ __forceinline__ float u_at(const int32_t* uptr, const Ent* uent, int32_t v, int32_t c) {
  for (int32_t p = uptr[v]; p < uptr[v + 1]; ++p)
    if (uent[p].col == c) return uent[p].val;
  return 0.f;
}

// The distinct cells of a face whose value passes `thr` (strictly positive
// when ge is false, >= thr when ge is true) at one of its vertices; a cell
// is reported once, at the first vertex of the face holding it.
template <class Fn>
__device__ __forceinline__ void face_cells(const int32_t* F, int64_t f, const int32_t* uptr,
                                           const Ent* uent, int32_t n_s, float thr, bool ge,
                                           Fn fn) {
  int32_t v[3] = {F[3 * f], F[3 * f + 1], F[3 * f + 2]};
  for (int k = 0; k < 3; ++k) {
    for (int32_t p = uptr[v[k]]; p < uptr[v[k] + 1]; ++p) {
      const Ent e = uent[p];
      if (e.col >= n_s) continue;
      if (ge ? !(e.val >= thr) : !(e.val > 0.f)) continue;
      bool seen = false;
      for (int kk = 0; kk < k && !seen; ++kk)
        for (int32_t pp = uptr[v[kk]]; pp < uptr[v[kk] + 1]; ++pp)
          if (uent[pp].col == e.col && (ge ? uent[pp].val >= thr : uent[pp].val > 0.f)) {
            seen = true;
            break;
          }
      if (!seen) fn(e.col);
    }
  }
}

struct Vec3 {
  double x, y, z;
};
__device__ __forceinline__ Vec3 vload(const double* V, int32_t i) {
  return Vec3{V[3 * (int64_t)i], V[3 * (int64_t)i + 1], V[3 * (int64_t)i + 2]};
}
__device__ __forceinline__ Vec3 vsub(Vec3 a, Vec3 b) { return Vec3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ Vec3 vcross(Vec3 a, Vec3 b) {
  return Vec3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ double vdot(Vec3 a, Vec3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// ---- Lloyd-like re-seeding -------------------------------------------------------

struct CellSums {
  unsigned long long a, bx, by, bz, nx, ny, nz;  // fixed point, two's complement
};

__device__ __forceinline__ unsigned long long fx(double v, double scale) {
  return (unsigned long long)__double2ll_rn(v * scale);
}
__device__ __forceinline__ double unfx(unsigned long long v, double scale) {
  return (double)(long long)v / scale;
}

// largest face area and coordinate magnitude (non-negative doubles order
// like their bit patterns)
// largest face area and largest |coordinate| (non-negative doubles, so their
// bit patterns order like the values): reduced per wavefront, one atomic each
__global__ void k_bounds(const double* V, const int32_t* F, int32_t n_f, unsigned long long* amax,
                         unsigned long long* xmax) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long a = 0, x = 0;
  if (f < n_f) {
    const Vec3 p0 = vload(V, F[3 * (int64_t)f]), p1 = vload(V, F[3 * (int64_t)f + 1]),
               p2 = vload(V, F[3 * (int64_t)f + 2]);
    const Vec3 c = vcross(vsub(p1, p0), vsub(p2, p0));
    const double area = 0.5 * sqrt(vdot(c, c));
    double m = 0.0;
    const Vec3 ps[3] = {p0, p1, p2};
    for (int k = 0; k < 3; ++k)
      m = fmax(m, fmax(fabs(ps[k].x), fmax(fabs(ps[k].y), fabs(ps[k].z))));
    a = (unsigned long long)__double_as_longlong(area);
    x = (unsigned long long)__double_as_longlong(m);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long ya = __shfl_xor(a, o, 64), yx = __shfl_xor(x, o, 64);
    a = ya > a ? ya : a;
    x = yx > x ? yx : x;
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(amax, a);
    atomicMax(xmax, x);
  }
}

// per face: area, area * barycentre and area * unit normal, added to every
// cell having a vertex of the face in its support
__global__ void k_lloyd_accum(const double* V, const int32_t* F, int32_t n_f, const int32_t* uptr,
                              const Ent* uent, int32_t n_s, double scale, CellSums* acc) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n_f) return;
  const Vec3 p0 = vload(V, F[3 * (int64_t)f]), p1 = vload(V, F[3 * (int64_t)f + 1]),
             p2 = vload(V, F[3 * (int64_t)f + 2]);
  const Vec3 c = vcross(vsub(p1, p0), vsub(p2, p0));
  const double area = 0.5 * sqrt(vdot(c, c));
  const unsigned long long ia = fx(area, scale);
  const unsigned long long ibx = fx(area * (p0.x + p1.x + p2.x) / 3.0, scale);
  const unsigned long long iby = fx(area * (p0.y + p1.y + p2.y) / 3.0, scale);
  const unsigned long long ibz = fx(area * (p0.z + p1.z + p2.z) / 3.0, scale);
  const unsigned long long inx = fx(0.5 * c.x, scale), iny = fx(0.5 * c.y, scale),
                           inz = fx(0.5 * c.z, scale);
  face_cells(F, f, uptr, uent, n_s, 0.f, false, [&](int32_t cell) {
    CellSums* s = acc + cell;
    atomicAdd(&s->a, ia);
    atomicAdd(&s->bx, ibx);
    atomicAdd(&s->by, iby);
    atomicAdd(&s->bz, ibz);
    atomicAdd(&s->nx, inx);
    atomicAdd(&s->ny, iny);
    atomicAdd(&s->nz, inz);
  });
}

struct CellLine {
  Vec3 ctr, dir;
  int32_t valid;
  int32_t pad;
};

__global__ void k_lloyd_lines(const CellSums* acc, int32_t n_s, double scale, CellLine* lines,
                              unsigned long long* best_s, int32_t* best_f) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_s) return;
  const CellSums s = acc[c];
  const double A = unfx(s.a, scale);
  const Vec3 N = Vec3{unfx(s.nx, scale), unfx(s.ny, scale), unfx(s.nz, scale)};
  const double nn = sqrt(vdot(N, N));
  CellLine L;
  L.valid = (A > 0.0 && nn > 0.0) ? 1 : 0;
  L.pad = 0;
  L.ctr = L.valid ? Vec3{unfx(s.bx, scale) / A, unfx(s.by, scale) / A, unfx(s.bz, scale) / A}
                  : Vec3{0, 0, 0};
  L.dir = L.valid ? Vec3{N.x / nn, N.y / nn, N.z / nn} : Vec3{0, 0, 1};
  lines[c] = L;
  best_s[c] = kEmpty;
  best_f[c] = 0x7fffffff;
}

// line o + s d against triangle (p0, p1, p2), closed edges (Moller-Trumbore)
__device__ __forceinline__ bool line_hit(Vec3 o, Vec3 d, Vec3 p0, Vec3 p1, Vec3 p2, double* s) {
  const Vec3 e1 = vsub(p1, p0), e2 = vsub(p2, p0);
  const Vec3 h = vcross(d, e2);
  const double det = vdot(e1, h);
  if (det == 0.0) return false;
  const double inv = 1.0 / det;
  const Vec3 t = vsub(o, p0);
  const double u = inv * vdot(t, h);
  const Vec3 q = vcross(t, e1);
  const double v = inv * vdot(d, q);
  *s = inv * vdot(e2, q);
  return u >= 0.0 && v >= 0.0 && 1.0 - u - v >= 0.0;
}

// a hit of a cell's line on one of its faces
struct HitRec {
  unsigned long long key;  // |s| as bits (non-negative doubles order like their bits)
  int32_t cell, face;
};

// pass 0: smallest |s| per cell, and every hit appended to `hits` (while it
// has room); pass 1: lowest face id among the hits at the smallest |s|, by a
// second walk over all faces, needed only when the list overflowed
__global__ void k_lloyd_hits(const double* V, const int32_t* F, int32_t n_f, const int32_t* uptr,
                             const Ent* uent, int32_t n_s, const CellLine* lines,
                             unsigned long long* best_s, int32_t* best_f, int pass, HitRec* hits,
                             unsigned int* n_hits, int64_t hit_cap) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n_f) return;
  if (pass == 1 && (int64_t)*n_hits <= hit_cap) return;  // the list holds every hit
  const Vec3 p0 = vload(V, F[3 * (int64_t)f]), p1 = vload(V, F[3 * (int64_t)f + 1]),
             p2 = vload(V, F[3 * (int64_t)f + 2]);
  face_cells(F, f, uptr, uent, n_s, 0.f, false, [&](int32_t cell) {
    const CellLine L = lines[cell];
    if (!L.valid) return;
    double s = 0.0;
    if (!line_hit(L.ctr, L.dir, p0, p1, p2, &s)) return;
    const unsigned long long key = (unsigned long long)__double_as_longlong(fabs(s));
    if (pass == 0) {
      atomicMin(&best_s[cell], key);
      const unsigned int at = atomicAdd(n_hits, 1u);
      if ((int64_t)at < hit_cap) hits[at] = HitRec{key, cell, f};
    } else if (key == best_s[cell]) {
      atomicMin(&best_f[cell], f);
    }
  });
}

// pass 1 from the list of hits (when it holds them all)
__global__ void k_lloyd_hit_faces(const HitRec* hits, const unsigned int* n_hits, int64_t hit_cap,
                                  const unsigned long long* best_s, int32_t* best_f) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)*n_hits;
  if (n > hit_cap || k >= n) return;
  const HitRec h = hits[k];
  if (h.key == best_s[h.cell]) atomicMin(&best_f[h.cell], h.face);
}

// the hit face's vertex nearest the hit point becomes the candidate seed
__global__ void k_lloyd_pick(const double* V, const int32_t* F, int32_t n_s, const CellLine* lines,
                             const int32_t* best_f, const int32_t* old, int32_t* cand,
                             int32_t* status) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_s) return;
  const int32_t f = best_f[c];
  if (f == 0x7fffffff) {
    cand[c] = old[c];
    status[c] = 1;
    return;
  }
  const CellLine L = lines[c];
  const int32_t* fv = F + 3 * (int64_t)f;
  const Vec3 p0 = vload(V, fv[0]), p1 = vload(V, fv[1]), p2 = vload(V, fv[2]);
  double s = 0.0;
  line_hit(L.ctr, L.dir, p0, p1, p2, &s);
  const Vec3 h = Vec3{L.ctr.x + s * L.dir.x, L.ctr.y + s * L.dir.y, L.ctr.z + s * L.dir.z};
  int32_t bv = -1;
  double bd = 0.0;
  const Vec3 ps[3] = {p0, p1, p2};
  for (int k = 0; k < 3; ++k) {
    const Vec3 dv = vsub(ps[k], h);
    const double dd = vdot(dv, dv);
    if (bv < 0 || dd < bd || (dd == bd && fv[k] < bv)) {
      bd = dd;
      bv = fv[k];
    }
  }
  cand[c] = bv;
  status[c] = 0;
}

// collision rounds: a cell that stays claims its seed first (key c), movers
// follow by cell id (key n_s + c); losers go back to their old seed
__global__ void k_owner_reset(const int32_t* cand, const int32_t* old, int32_t n_s, int32_t* owner) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_s) return;
  owner[cand[c]] = 0x7fffffff;
  owner[old[c]] = 0x7fffffff;
}
__global__ void k_owner_claim(const int32_t* cand, const int32_t* old, int32_t n_s, int32_t* owner) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_s) return;
  atomicMin(&owner[cand[c]], cand[c] == old[c] ? c : n_s + c);
}
__global__ void k_owner_check(int32_t* cand, const int32_t* old, int32_t n_s, const int32_t* owner,
                              int32_t* status, int32_t* changed) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_s) return;
  const int32_t key = cand[c] == old[c] ? c : n_s + c;
  if (owner[cand[c]] != key) {
    cand[c] = old[c];
    status[c] = 2;
    *changed = 1;
  }
}

// ---- dual mesh -------------------------------------------------------------------

// thresholded cells of a vertex (at most four values >= 0.25 can share a
// row summing to at most one, but any count is handled)
__global__ void k_dual_count(const int32_t* F, int32_t n_f, int32_t n_v, const int32_t* uptr,
                             const Ent* uent, int32_t n_s, float tau,
                             unsigned long long* counts /* [2] */) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long cv = 0, ct = 0;
  if (t < n_v) {
    long long k = 0;
    for (int32_t p = uptr[t]; p < uptr[t + 1]; ++p)
      k += (uent[p].col < n_s && uent[p].val >= tau) ? 1 : 0;
    if (k > 1) cv = (unsigned long long)(k * (k - 1) / 2);
  }
  if (t < n_f) {
    long long k = 0;
    face_cells(F, t, uptr, uent, n_s, tau, true, [&](int32_t) { ++k; });
    if (k > 1) ct = (unsigned long long)(k * (k - 1) / 2);
  }
  // one atomic per wavefront and counter
  cv = wave_sum_u64(cv);
  ct = wave_sum_u64(ct);
  if ((threadIdx.x & 63) == 0) {
    if (cv) atomicAdd(&counts[0], cv);
    if (ct) atomicAdd(&counts[1], ct);
  }
}

// A_v: pairs of cells above tau at one vertex; A_t: pairs of cells above tau
// on one face (the logical products Phibar Phibar^T and (Phibar Mbar)(Phibar Mbar)^T)
__global__ void k_dual_pairs(const int32_t* F, int32_t n_f, int32_t n_v, const int32_t* uptr,
                             const Ent* uent, int32_t n_s, float tau, unsigned long long* tv,
                             int64_t cap_v, unsigned long long* tt, int64_t cap_t, int* ovf) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned long long NS = (unsigned long long)n_s;
  if (t < n_v) {
    for (int32_t a = uptr[t]; a < uptr[t + 1]; ++a) {
      if (!(uent[a].col < n_s && uent[a].val >= tau)) continue;
      for (int32_t b = a + 1; b < uptr[t + 1]; ++b) {
        if (!(uent[b].col < n_s && uent[b].val >= tau)) continue;
        set_insert(tv, cap_v, (unsigned long long)uent[a].col * NS + uent[b].col, ovf);
      }
    }
  }
  if (t < n_f) {
    int32_t cells[32];
    int k = 0;
    face_cells(F, t, uptr, uent, n_s, tau, true, [&](int32_t c) {
      if (k < 32) cells[k] = c;
      ++k;
    });
    if (k > 32) {
      atomicOr(ovf, 2);
      return;
    }
    for (int a = 0; a < k; ++a)
      for (int b = 0; b < k; ++b)
        if (cells[a] < cells[b]) set_insert(tt, cap_t, (unsigned long long)cells[a] * NS + cells[b], ovf);
  }
}

__global__ void k_mark_absent(const unsigned long long* kt, int64_t nt, const unsigned long long* kv,
                              int64_t nv, int32_t* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nt) return;
  int64_t at;
  flag[i] = bsearch_u64(kv, nv, kt[i], &at) ? 0 : 1;
}

__global__ void k_compact_u64(const unsigned long long* in, const int32_t* flag, const int32_t* pos,
                              int64_t n, unsigned long long* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && flag[i]) out[pos[i]] = in[i];
}

// tau-isoline of a field on a face as a segment in barycentric coordinates
// (weights of corners 1 and 2); false when the face is not crossed
__device__ __forceinline__ bool iso_seg(const double f[3], double tau, double seg[4]) {
  const bool in0 = f[0] >= tau, in1 = f[1] >= tau, in2 = f[2] >= tau;
  if (in0 == in1 && in1 == in2) return false;
  const bool in[3] = {in0, in1, in2};
  int m = 0;
  for (int e = 0; e < 3; ++e) {
    const int a = e, b = (e + 1) % 3;
    if (in[a] == in[b]) continue;
    const double t = (tau - f[a]) / (f[b] - f[a]);
    double w[3] = {0.0, 0.0, 0.0};
    w[a] = 1.0 - t;
    w[b] = t;
    seg[2 * m] = w[1];
    seg[2 * m + 1] = w[2];
    ++m;
  }
  return m == 2;
}

__device__ __forceinline__ double orient(const double* a, const double* b, const double* c) {
  return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]);
}
__device__ __forceinline__ bool in_box(const double* a, const double* b, const double* c) {
  return fmin(a[0], b[0]) <= c[0] && c[0] <= fmax(a[0], b[0]) && fmin(a[1], b[1]) <= c[1] &&
         c[1] <= fmax(a[1], b[1]);
}
// closed segments P, Q intersect
__device__ __forceinline__ bool segs_cross(const double* P, const double* Q) {
  const double* p0 = P;
  const double* p1 = P + 2;
  const double* q0 = Q;
  const double* q1 = Q + 2;
  const double d1 = orient(q0, q1, p0), d2 = orient(q0, q1, p1);
  const double d3 = orient(p0, p1, q0), d4 = orient(p0, p1, q1);
  if (((d1 > 0 && d2 < 0) || (d1 < 0 && d2 > 0)) && ((d3 > 0 && d4 < 0) || (d3 < 0 && d4 > 0)))
    return true;
  if (d1 == 0 && in_box(q0, q1, p0)) return true;
  if (d2 == 0 && in_box(q0, q1, p1)) return true;
  if (d3 == 0 && in_box(p0, p1, q0)) return true;
  if (d4 == 0 && in_box(p0, p1, q1)) return true;
  return false;
}

// candidates confirmed by an isoline crossing on a face they share
__global__ void k_cand_faces(const int32_t* F, int32_t n_f, const int32_t* uptr, const Ent* uent,
                             int32_t n_s, float tau, const unsigned long long* kc, int64_t nc,
                             int32_t* conf) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n_f || nc == 0) return;
  int32_t cells[32];
  int k = 0;
  face_cells(F, f, uptr, uent, n_s, tau, true, [&](int32_t c) {
    if (k < 32) cells[k] = c;
    ++k;
  });
  k = k < 32 ? k : 32;
  const int32_t* fv = F + 3 * (int64_t)f;
  for (int a = 0; a < k; ++a)
    for (int b = 0; b < k; ++b) {
      if (!(cells[a] < cells[b])) continue;
      int64_t at;
      const unsigned long long key = (unsigned long long)cells[a] * n_s + cells[b];
      if (!bsearch_u64(kc, nc, key, &at)) continue;
      double fp[3], fq[3], sp[4], sq[4];
      for (int j = 0; j < 3; ++j) {
        fp[j] = (double)u_at(uptr, uent, fv[j], cells[a]);
        fq[j] = (double)u_at(uptr, uent, fv[j], cells[b]);
      }
      if (iso_seg(fp, (double)tau, sp) && iso_seg(fq, (double)tau, sq) && segs_cross(sp, sq))
        atomicOr(&conf[at], 1);
    }
}

// symmetric CSR from sorted unique keys p*n+q (both directions present)
__global__ void k_keys_rowptr(const unsigned long long* keys, int64_t nk, int32_t n, int32_t* rowptr,
                              int32_t* col) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nk) col[i] = (int32_t)(keys[i] % (unsigned long long)n);
  if (i <= n) {
    int64_t at;
    bsearch_u64(keys, nk, (unsigned long long)i * n, &at);
    rowptr[i] = (int32_t)at;
  }
}

__device__ __forceinline__ bool adj(const int32_t* rp, const int32_t* col, int32_t p, int32_t q) {
  int32_t lo = rp[p], hi = rp[p + 1];
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (col[mid] < q) lo = mid + 1;
    else hi = mid;
  }
  return lo < rp[p + 1] && col[lo] == q;
}

// manifold rule: a confirmed candidate whose cells share two or more A_v
// neighbours is dropped
__global__ void k_cand_state(const unsigned long long* kc, int64_t nc, int32_t n_s,
                             const int32_t* conf, const int32_t* vrp, const int32_t* vcol,
                             int32_t* state) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc) return;
  if (!conf[i]) {
    state[i] = 0;
    return;
  }
  const int32_t p = (int32_t)(kc[i] / n_s), q = (int32_t)(kc[i] % n_s);
  int32_t a = vrp[p], b = vrp[q], shared = 0;
  while (a < vrp[p + 1] && b < vrp[q + 1]) {
    if (vcol[a] == vcol[b]) { ++shared; ++a; ++b; }
    else if (vcol[a] < vcol[b]) ++a;
    else ++b;
  }
  state[i] = shared >= 2 ? 2 : 1;
}

// both directions of each unordered key, into out[2*i], out[2*i+1]
__global__ void k_both_dirs(const unsigned long long* k, int64_t n, int32_t n_s,
                            unsigned long long* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const unsigned long long p = k[i] / n_s, q = k[i] % n_s;
  out[2 * i] = p * n_s + q;
  out[2 * i + 1] = q * n_s + p;
}

__global__ void k_kept_keys(const unsigned long long* kc, const int32_t* state, int64_t nc,
                            unsigned long long* out, unsigned long long* count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nc && state[i] == 1) out[atomicAdd(count, 1ull)] = kc[i];
}

// 3-cliques i<j<k of the curated adjacency, counted then written in order
__global__ void k_tri_count(const int32_t* rp, const int32_t* col, int32_t n, int32_t* cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t c = 0;
  for (int32_t a = rp[i]; a < rp[i + 1]; ++a) {
    const int32_t j = col[a];
    if (j <= i) continue;
    for (int32_t b = a + 1; b < rp[i + 1]; ++b)
      if (adj(rp, col, j, col[b])) ++c;
  }
  cnt[i] = c;
}
__global__ void k_tri_fill(const int32_t* rp, const int32_t* col, int32_t n, const int32_t* off,
                           int32_t* tri) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t o = off[i];
  for (int32_t a = rp[i]; a < rp[i + 1]; ++a) {
    const int32_t j = col[a];
    if (j <= i) continue;
    for (int32_t b = a + 1; b < rp[i + 1]; ++b) {
      const int32_t k = col[b];
      if (adj(rp, col, j, k)) {
        tri[3 * o] = i;
        tri[3 * o + 1] = j;
        tri[3 * o + 2] = k;
        ++o;
      }
    }
  }
}

// a cell with exactly three mutually adjacent neighbours j<k<l: the triangle
// (j,k,l) covers it and is removed
__global__ void k_spurious(const int32_t* rp, const int32_t* col, int32_t n, const int32_t* tri,
                           int64_t nt, int32_t* keep) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || rp[i + 1] - rp[i] != 3) return;
  const int32_t j = col[rp[i]], k = col[rp[i] + 1], l = col[rp[i] + 2];
  if (!(adj(rp, col, j, k) && adj(rp, col, k, l) && adj(rp, col, j, l))) return;
  int64_t lo = 0, hi = nt;
  while (lo < hi) {  // triangles are in lexicographic order
    const int64_t mid = (lo + hi) >> 1;
    const int32_t* t = tri + 3 * mid;
    const bool less = t[0] < j || (t[0] == j && (t[1] < k || (t[1] == k && t[2] < l)));
    if (less) lo = mid + 1;
    else hi = mid;
  }
  if (lo < nt && tri[3 * lo] == j && tri[3 * lo + 1] == k && tri[3 * lo + 2] == l) keep[lo] = 0;
}

__global__ void k_compact_tri(const int32_t* tri, const int32_t* keep, const int32_t* pos,
                              int64_t nt, int32_t* out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt || !keep[t]) return;
  const int64_t o = pos[t];
  out[3 * o] = tri[3 * t];
  out[3 * o + 1] = tri[3 * t + 1];
  out[3 * o + 2] = tri[3 * t + 2];
}

// edge keys (lo*n_s+hi)*(nt+1)+t of every triangle edge
__global__ void k_edge_keys(const int32_t* tri, int64_t nt, int32_t n_s, unsigned long long* keys) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  for (int e = 0; e < 3; ++e) {
    const int32_t x = tri[3 * t + e], y = tri[3 * t + (e + 1) % 3];
    const unsigned long long lo = x < y ? x : y, hi = x < y ? y : x;
    keys[3 * t + e] = (lo * n_s + hi) * (unsigned long long)(nt + 1) + t;
  }
}

// across[3t+e] = the triangle sharing edge e of t when exactly two share it
__global__ void k_edge_links(const unsigned long long* keys, int64_t nk, int64_t nt, int32_t n_s,
                             const int32_t* tri, int32_t* across, unsigned long long* nonmanifold) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nk) return;
  const unsigned long long T = (unsigned long long)(nt + 1);
  const unsigned long long e = keys[i] / T;
  if (i > 0 && keys[i - 1] / T == e) return;  // first of its group handles it
  int64_t j = i;
  while (j < nk && keys[j] / T == e) ++j;
  if (j - i > 2) atomicAdd(nonmanifold, 1ull);
  if (j - i != 2) return;
  const int64_t f0 = keys[i] % T, f1 = keys[i + 1] % T;
  const int32_t lo = (int32_t)(e / n_s), hi = (int32_t)(e % n_s);
  for (int s = 0; s < 3; ++s) {
    int32_t x = tri[3 * f0 + s], y = tri[3 * f0 + (s + 1) % 3];
    if ((x == lo && y == hi) || (x == hi && y == lo)) across[3 * f0 + s] = (int32_t)f1;
    x = tri[3 * f1 + s];
    y = tri[3 * f1 + (s + 1) % 3];
    if ((x == lo && y == hi) || (x == hi && y == lo)) across[3 * f1 + s] = (int32_t)f0;
  }
}

// components of the edge-adjacency graph by minimum-label propagation
// Components of the dual triangles across manifold edges, by union-find:
// every hook puts the larger root under the smaller one with a
// compare-and-swap, so parents only decrease, every walk up a tree ends,
// and the root of a component is its lowest triangle id.  One pass hooks
// every edge, a second one points every triangle at its root.
__device__ __forceinline__ int32_t cc_root(int32_t* parent, int32_t v) {
  int32_t cur = parent[v];
  if (cur != v) {
    int32_t prev = v, next;
    while (cur > (next = parent[cur])) {  // path halving; next < cur < prev
      parent[prev] = next;
      prev = cur;
      cur = next;
    }
  }
  return cur;
}

__global__ void k_cc_hook(const int32_t* across, int32_t* parent, int64_t nt) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  int32_t a = cc_root(parent, (int32_t)t);
  for (int e = 0; e < 3; ++e) {
    const int32_t g = across[3 * t + e];
    if (g < 0) continue;
    int32_t b = cc_root(parent, g);
    while (a != b) {
      // a failed swap returns the node's new, lower parent: climb to it
      if (a < b) {
        const int32_t r = atomicCAS(&parent[b], b, a);
        if (r == b) break;
        b = r;
      } else {
        const int32_t r = atomicCAS(&parent[a], a, b);
        if (r == a) break;
        a = r;
      }
    }
  }
}

__global__ void k_cc_final(int32_t* parent, int64_t nt) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nt) parent[t] = cc_root(parent, (int32_t)t);
}

__global__ void k_comp_init(int32_t* label, int64_t nt) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nt) label[t] = (int32_t)t;
}

// area-weighted normals at seed vertices (faces touching a seed)
__global__ void k_seed_normals(const double* V, const int32_t* F, int32_t n_f, const int32_t* owner,
                               int32_t n_s, double* vn) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n_f) return;
  const int32_t* fv = F + 3 * (int64_t)f;
  const int32_t ow[3] = {owner[fv[0]], owner[fv[1]], owner[fv[2]]};
  if (ow[0] >= n_s && ow[1] >= n_s && ow[2] >= n_s) return;  // no seed: no geometry read
  const Vec3 c = vcross(vsub(vload(V, fv[1]), vload(V, fv[0])), vsub(vload(V, fv[2]), vload(V, fv[0])));
  for (int k = 0; k < 3; ++k) {
    const int32_t o = ow[k];
    if (o < n_s) {
      atomicAdd(&vn[3 * (int64_t)o], c.x);
      atomicAdd(&vn[3 * (int64_t)o + 1], c.y);
      atomicAdd(&vn[3 * (int64_t)o + 2], c.z);
    }
  }
}

// roots: the lowest triangle of each component, turned to agree with the
// summed normals at its three seeds
__global__ void k_orient_roots(const int32_t* tri, const int32_t* label, int64_t nt,
                               const double* V, const int32_t* seeds, const double* vn,
                               int32_t* otri, int32_t* level) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  int32_t a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
  if (label[t] != t) {
    level[t] = -1;
    return;
  }
  const Vec3 x0 = vload(V, seeds[a]), x1 = vload(V, seeds[b]), x2 = vload(V, seeds[c]);
  const Vec3 n = vcross(vsub(x1, x0), vsub(x2, x0));
  const Vec3 r = Vec3{vn[3 * a] + vn[3 * b] + vn[3 * c], vn[3 * a + 1] + vn[3 * b + 1] + vn[3 * c + 1],
                      vn[3 * a + 2] + vn[3 * b + 2] + vn[3 * c + 2]};
  if (vdot(n, r) < 0.0) {
    const int32_t s = b;
    b = c;
    c = s;
  }
  otri[3 * t] = a;
  otri[3 * t + 1] = b;
  otri[3 * t + 2] = c;
  level[t] = 0;
}

// one breadth-first level: an unoriented triangle next to one oriented at
// the previous level (the lowest such neighbour) takes the opposite edge
// direction
__global__ void k_orient_level(const int32_t* tri, const int32_t* across, int64_t nt, int32_t lev,
                               int32_t* otri, int32_t* level, int32_t* changed) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt || level[t] >= 0) return;
  int32_t par = -1;
  for (int e = 0; e < 3; ++e) {
    const int32_t g = across[3 * t + e];
    if (g >= 0 && level[g] == lev - 1 && (par < 0 || g < par)) par = g;
  }
  if (par < 0) return;
  // the shared edge as the parent traverses it: x -> y; t takes y -> x
  const int32_t* op = otri + 3 * (int64_t)par;
  const int32_t a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
  for (int s = 0; s < 3; ++s) {
    const int32_t x = op[s], y = op[(s + 1) % 3];
    const bool hx = (x == a || x == b || x == c), hy = (y == a || y == b || y == c);
    if (hx && hy) {
      const int32_t z = a ^ b ^ c ^ x ^ y;
      otri[3 * t] = y;
      otri[3 * t + 1] = x;
      otri[3 * t + 2] = z;
      level[t] = lev;
      *changed = 1;
      return;
    }
  }
}

// pairs of edge-adjacent oriented triangles that traverse their shared edge
// the same way
__global__ void k_orient_conflicts(const int32_t* otri, const int32_t* across, int64_t nt,
                                   unsigned long long* conflicts) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  for (int s = 0; s < 3; ++s) {
    const int32_t x = otri[3 * t + s], y = otri[3 * t + (s + 1) % 3];
    for (int e = 0; e < 3; ++e) {
      const int32_t g = across[3 * t + e];
      if (g <= t) continue;
      const int32_t* og = otri + 3 * (int64_t)g;
      bool hx = false, hy = false, same = false;
      for (int r = 0; r < 3; ++r) {
        hx |= og[r] == x;
        hy |= og[r] == y;
        same |= (og[r] == x && og[(r + 1) % 3] == y);
      }
      if (hx && hy && same) atomicAdd(conflicts, 1ull);
    }
  }
}

}  // namespace

hipError_t sort_keys_u64(unsigned long long* keys, int64_t n, hipStream_t s) {
  return sort_u64(keys, n, s);
}

}  // namespace lf

// ---- state kept for inspection ---------------------------------------------------

struct DualState {
  std::vector<int32_t> av_rp, av_col, at_rp, at_col, ad_rp, ad_col;
  std::vector<int32_t> cand, cand_state, tri;
  long long n_removed = 0, n_conflict = 0, n_nonmanifold = 0;
};

namespace lf {

void dual_release(lf_fields* f) {
  delete f->dual;
  f->dual = nullptr;
}

namespace {

lf_status fail(lf_status st, const std::string& msg) {
  set_error(msg);
  return st;
}

template <class T>
struct Buf {
  T* p = nullptr;
  ~Buf() {
    if (p) hipFree(p);
  }
  hipError_t alloc(int64_t n) {
    if (p) (void)hipFree(p);
    p = nullptr;
    return dalloc(&p, n);
  }
};

// LF_TEST_SMALL_TABLES=1 starts the growable tables of the post-processing
// (cell-pair sets, the list of line hits) with tiny capacities, so that a
// test can run their fallback paths on ordinary inputs
bool small_tables() {
  const char* e = getenv("LF_TEST_SMALL_TABLES");
  return e && e[0] == '1';
}

template <class T>
hipError_t to_host(std::vector<T>& v, const T* d, int64_t n, hipStream_t s) {
  v.resize((size_t)std::max<int64_t>(n, 0));
  if (n <= 0) return hipSuccess;
  return hipMemcpyAsync(v.data(), d, sizeof(T) * n, hipMemcpyDeviceToHost, s);
}

// sorted unique keys of a hash set -> device array `out` (capacity pow2)
lf_status set_to_sorted(unsigned long long* tab, int64_t cap, Buf<unsigned long long>& out,
                        int64_t* n, hipStream_t s) {
  Buf<unsigned long long> cnt;
  LF_HIP(cnt.alloc(1));
  LF_HIP(hipMemsetAsync(cnt.p, 0, sizeof(unsigned long long), s));
  LF_HIP(out.alloc(cap));
  hipLaunchKernelGGL(k_set_extract, dim3(nblk(cap)), dim3(kT), 0, s, tab, cap, out.p, cnt.p);
  LF_HIP(hipGetLastError());
  unsigned long long h = 0;
  LF_HIP(hipMemcpyAsync(&h, cnt.p, sizeof(h), hipMemcpyDeviceToHost, s));
  LF_HIP(hipStreamSynchronize(s));
  *n = (int64_t)h;
  LF_HIP(sort_u64(out.p, *n, s));
  return LF_OK;
}

// symmetric CSR (n+1 pointers) from sorted unordered keys p*n+q, p<q
lf_status sym_csr(const unsigned long long* k, int64_t nk, int32_t n, Buf<int32_t>& rp,
                  Buf<int32_t>& col, hipStream_t s) {
  Buf<unsigned long long> both;
  LF_HIP(both.alloc(pow2_at_least(2 * nk + 1)));
  if (nk > 0) hipLaunchKernelGGL(k_both_dirs, dim3(nblk(nk)), dim3(kT), 0, s, k, nk, n, both.p);
  LF_HIP(sort_u64(both.p, 2 * nk, s));
  LF_HIP(rp.alloc(n + 1));
  LF_HIP(col.alloc(2 * nk + 1));
  hipLaunchKernelGGL(k_keys_rowptr, dim3(nblk(std::max<int64_t>(2 * nk, n + 1))), dim3(kT), 0, s,
                     both.p, 2 * nk, n, rp.p, col.p);
  LF_HIP(hipGetLastError());
  return LF_OK;
}

}  // namespace
}  // namespace lf

using namespace lf;

extern "C" {

lf_status lf_lloyd_reseed(lf_fields* f, int32_t* seeds_out, int32_t* status_out) try {
  if (!f || !seeds_out) return fail(LF_EINVAL, "NULL argument");
  LF_SETTLE(f);
  lf_mesh* m = f->mesh;
  LF_HIP(hipSetDevice(m->ctx->device));
  hipStream_t s = m->ctx->stream;
  const int32_t n_s = f->n_s, n_f = m->n_f;
  const int32_t* uptr = nullptr;
  const Ent* uent = nullptr;
  {
    lf_status st = fields_csr(f, &uptr, &uent);
    if (st) return st;
  }
  Buf<unsigned long long> bounds, best_s;
  Buf<CellSums> acc;
  Buf<CellLine> lines;
  Buf<int32_t> best_f, cand, old, status, owner, changed;
  LF_HIP(bounds.alloc(2));
  LF_HIP(acc.alloc(n_s));
  LF_HIP(lines.alloc(n_s));
  LF_HIP(best_s.alloc(n_s));
  LF_HIP(best_f.alloc(n_s));
  LF_HIP(cand.alloc(n_s));
  LF_HIP(old.alloc(n_s));
  LF_HIP(status.alloc(n_s));
  LF_HIP(owner.alloc(m->n_v));
  LF_HIP(changed.alloc(1));
  LF_HIP(hipMemsetAsync(acc.p, 0, sizeof(CellSums) * n_s, s));
  LF_HIP(hipMemcpyAsync(old.p, f->seeds.data(), sizeof(int32_t) * n_s, hipMemcpyHostToDevice, s));
  if (m->amax < 0.0) {  // a property of the mesh: measured once
    LF_HIP(hipMemsetAsync(bounds.p, 0, 2 * sizeof(unsigned long long), s));
    hipLaunchKernelGGL(k_bounds, dim3(nblk(n_f)), dim3(kT), 0, s, m->V, m->F, n_f, bounds.p,
                       bounds.p + 1);
    LF_HIP(hipGetLastError());
    unsigned long long hb[2] = {0, 0};
    LF_HIP(hipMemcpyAsync(hb, bounds.p, sizeof(hb), hipMemcpyDeviceToHost, s));
    LF_HIP(hipStreamSynchronize(s));
    memcpy(&m->amax, &hb[0], sizeof(double));
    memcpy(&m->xmax, &hb[1], sizeof(double));
  }
  const double amax = m->amax, xmax = m->xmax;
  // fixed-point scale: the largest possible per-cell sum stays below 2^62
  const double bound = std::max(1e-300, (double)n_f * amax * (xmax + 1.0));
  const double scale = std::ldexp(1.0, 62 - (int)std::ceil(std::log2(bound)));
  hipLaunchKernelGGL(k_lloyd_accum, dim3(nblk(n_f)), dim3(kT), 0, s, m->V, m->F, n_f, uptr, uent, n_s,
                     scale, acc.p);
  hipLaunchKernelGGL(k_lloyd_lines, dim3(nblk(n_s)), dim3(kT), 0, s, acc.p, n_s, scale, lines.p,
                     best_s.p, best_f.p);
  // hits are few (a handful per cell): the second pass walks their list,
  // and the walk over all faces runs only if the list overflowed
  const int64_t hit_cap = small_tables() ? 1 : 8ll * n_s + 4096;
  Buf<HitRec> hits;
  Buf<unsigned int> n_hits;
  LF_HIP(hits.alloc(hit_cap));
  LF_HIP(n_hits.alloc(1));
  LF_HIP(hipMemsetAsync(n_hits.p, 0, sizeof(unsigned int), s));
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1)
      hipLaunchKernelGGL(k_lloyd_hit_faces, dim3(nblk(hit_cap)), dim3(kT), 0, s, hits.p, n_hits.p,
                         hit_cap, best_s.p, best_f.p);
    hipLaunchKernelGGL(k_lloyd_hits, dim3(nblk(n_f)), dim3(kT), 0, s, m->V, m->F, n_f, uptr, uent,
                       n_s, lines.p, best_s.p, best_f.p, pass, hits.p, n_hits.p, hit_cap);
  }
  hipLaunchKernelGGL(k_lloyd_pick, dim3(nblk(n_s)), dim3(kT), 0, s, m->V, m->F, n_s, lines.p,
                     best_f.p, old.p, cand.p, status.p);
  LF_HIP(hipGetLastError());
  for (int round = 0; round <= n_s; ++round) {
    LF_HIP(hipMemsetAsync(changed.p, 0, sizeof(int32_t), s));
    hipLaunchKernelGGL(k_owner_reset, dim3(nblk(n_s)), dim3(kT), 0, s, cand.p, old.p, n_s, owner.p);
    hipLaunchKernelGGL(k_owner_claim, dim3(nblk(n_s)), dim3(kT), 0, s, cand.p, old.p, n_s, owner.p);
    hipLaunchKernelGGL(k_owner_check, dim3(nblk(n_s)), dim3(kT), 0, s, cand.p, old.p, n_s, owner.p,
                       status.p, changed.p);
    LF_HIP(hipGetLastError());
    int32_t hc = 0;
    LF_HIP(hipMemcpyAsync(&hc, changed.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    LF_HIP(hipStreamSynchronize(s));
    if (!hc) break;
  }
  LF_HIP(hipMemcpyAsync(seeds_out, cand.p, sizeof(int32_t) * n_s, hipMemcpyDeviceToHost, s));
  if (status_out)
    LF_HIP(hipMemcpyAsync(status_out, status.p, sizeof(int32_t) * n_s, hipMemcpyDeviceToHost, s));
  LF_HIP(hipStreamSynchronize(s));
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_lloyd(lf_fields* f, int32_t rounds, int32_t steps_per_round, int32_t* seeds_out) try {
  if (!f || rounds < 0 || steps_per_round < 0) return fail(LF_EINVAL, "invalid argument");
  LF_SETTLE(f);
  std::vector<int32_t> seeds((size_t)f->n_s);
  for (int32_t r = 0; r < rounds; ++r) {
    lf_status st = lf_lloyd_reseed(f, seeds.data(), nullptr);
    if (!st) st = lf_fields_reset(f, seeds.data());
    if (!st) st = lf_step(f, steps_per_round);
    if (st) return st;
  }
  if (seeds_out) return lf_fields_seeds(f, seeds_out);
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_dual_mesh(lf_fields* f, double tau, int64_t* n_tri, int32_t* tris, int64_t* adj_nnz,
                       int32_t* adj_rowptr, int32_t* adj_col) try {
  if (!f || !n_tri || !adj_nnz) return fail(LF_EINVAL, "NULL argument");
  LF_SETTLE(f);
  if (!(tau > 0.0 && tau <= 1.0)) return fail(LF_EINVAL, "tau must be in (0, 1]");
  lf_mesh* m = f->mesh;
  // a repeated call with output buffers returns the previous result
  if ((tris || adj_rowptr || adj_col) && f->dual && f->dual->ad_rp.size() == (size_t)f->n_s + 1) {
    DualState* d = f->dual;
    *n_tri = (int64_t)d->tri.size() / 3;
    *adj_nnz = (int64_t)d->ad_col.size();
    if (tris) memcpy(tris, d->tri.data(), sizeof(int32_t) * d->tri.size());
    if (adj_rowptr) memcpy(adj_rowptr, d->ad_rp.data(), sizeof(int32_t) * d->ad_rp.size());
    if (adj_col) memcpy(adj_col, d->ad_col.data(), sizeof(int32_t) * d->ad_col.size());
    return LF_OK;
  }
  LF_HIP(hipSetDevice(m->ctx->device));
  hipStream_t s = m->ctx->stream;
  const int32_t n_s = f->n_s, n_f = m->n_f, n_v = m->n_v;
  const float ftau = (float)tau;
  const int32_t* uptr = nullptr;
  const Ent* uent = nullptr;
  {
    lf_status st = fields_csr(f, &uptr, &uent);
    if (st) return st;
  }
  const int64_t nmax = std::max<int64_t>(n_v, n_f);

  // A_v and A_t as hash sets of cell pairs.  A cell meets a handful of
  // others, so the tables start at 16 slots per cell (a low load for any
  // ordinary partition); a table that fills up (bit 1) is sized again from
  // the exact number of pair incidences, which always suffices.
  Buf<unsigned long long> counts, tv, tt, kv, kt;
  Buf<int> ovf;
  LF_HIP(ovf.alloc(1));
  int64_t cap_v = small_tables() ? 16 : pow2_at_least(std::max<int64_t>(1024, 16ll * n_s));
  int64_t cap_t = cap_v;
  for (int attempt = 0;; ++attempt) {
    LF_HIP(tv.alloc(cap_v));
    LF_HIP(tt.alloc(cap_t));
    LF_HIP(hipMemsetAsync(ovf.p, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_fill64, dim3(nblk(cap_v)), dim3(kT), 0, s, tv.p, cap_v, kEmpty);
    hipLaunchKernelGGL(k_fill64, dim3(nblk(cap_t)), dim3(kT), 0, s, tt.p, cap_t, kEmpty);
    hipLaunchKernelGGL(k_dual_pairs, dim3(nblk(nmax)), dim3(kT), 0, s, m->F, n_f, n_v, uptr, uent,
                       n_s, ftau, tv.p, cap_v, tt.p, cap_t, ovf.p);
    LF_HIP(hipGetLastError());
    int hov = 0;
    LF_HIP(hipMemcpyAsync(&hov, ovf.p, sizeof(int), hipMemcpyDeviceToHost, s));
    LF_HIP(hipStreamSynchronize(s));
    if (hov & 2) return fail(LF_ECAPACITY, "more than 32 cells above tau on one face");
    if (!(hov & 1)) break;
    if (attempt > 0) return fail(LF_ECAPACITY, "cell-pair tables overflowed");
    LF_HIP(counts.alloc(2));
    LF_HIP(hipMemsetAsync(counts.p, 0, 2 * sizeof(unsigned long long), s));
    hipLaunchKernelGGL(k_dual_count, dim3(nblk(nmax)), dim3(kT), 0, s, m->F, n_f, n_v, uptr, uent,
                       n_s, ftau, counts.p);
    LF_HIP(hipGetLastError());
    unsigned long long hc[2];
    LF_HIP(hipMemcpyAsync(hc, counts.p, sizeof(hc), hipMemcpyDeviceToHost, s));
    LF_HIP(hipStreamSynchronize(s));
    cap_v = pow2_at_least(std::max<int64_t>(1024, 2 * (int64_t)hc[0]));
    cap_t = pow2_at_least(std::max<int64_t>(1024, 2 * (int64_t)hc[1]));
  }
  int64_t nv = 0, nt = 0;
  lf_status st = set_to_sorted(tv.p, cap_v, kv, &nv, s);
  if (st) return st;
  st = set_to_sorted(tt.p, cap_t, kt, &nt, s);
  if (st) return st;

  // candidates: A_t pairs absent from A_v, in key order
  Buf<int32_t> flag, pos, conf, cstate;
  Buf<long long> tmp;
  Buf<unsigned long long> kc;
  LF_HIP(flag.alloc(nt + 1));
  LF_HIP(pos.alloc(nt + 1));
  LF_HIP(tmp.alloc(scan_tmp_elems(nt + 1)));
  if (nt > 0)
    hipLaunchKernelGGL(k_mark_absent, dim3(nblk(nt)), dim3(kT), 0, s, kt.p, nt, kv.p, nv, flag.p);
  LF_HIP(exclusive_scan(flag.p, pos.p, nt, tmp.p, s));
  int32_t nc32 = 0;
  LF_HIP(hipMemcpyAsync(&nc32, pos.p + nt, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  LF_HIP(hipStreamSynchronize(s));
  const int64_t nc = nc32;
  LF_HIP(kc.alloc(nc + 1));
  LF_HIP(conf.alloc(nc + 1));
  LF_HIP(cstate.alloc(nc + 1));
  if (nt > 0)
    hipLaunchKernelGGL(k_compact_u64, dim3(nblk(nt)), dim3(kT), 0, s, kt.p, flag.p, pos.p, nt, kc.p);
  LF_HIP(hipMemsetAsync(conf.p, 0, sizeof(int32_t) * (nc + 1), s));
  hipLaunchKernelGGL(k_cand_faces, dim3(nblk(n_f)), dim3(kT), 0, s, m->F, n_f, uptr, uent, n_s, ftau,
                     kc.p, nc, conf.p);
  LF_HIP(hipGetLastError());

  // A_v CSR, candidate verdicts (shared-neighbour rule), curated adjacency
  Buf<int32_t> vrp, vcol, trp, tcol, drp, dcol;
  st = sym_csr(kv.p, nv, n_s, vrp, vcol, s);
  if (st) return st;
  st = sym_csr(kt.p, nt, n_s, trp, tcol, s);
  if (st) return st;
  if (nc > 0)
    hipLaunchKernelGGL(k_cand_state, dim3(nblk(nc)), dim3(kT), 0, s, kc.p, nc, n_s, conf.p, vrp.p,
                       vcol.p, cstate.p);
  Buf<unsigned long long> kd, kcount;
  LF_HIP(kd.alloc(pow2_at_least(nv + nc + 1)));
  LF_HIP(kcount.alloc(1));
  if (nv > 0)
    LF_HIP(hipMemcpyAsync(kd.p, kv.p, sizeof(unsigned long long) * nv, hipMemcpyDeviceToDevice, s));
  LF_HIP(hipMemsetAsync(kcount.p, 0, sizeof(unsigned long long), s));
  if (nc > 0)
    hipLaunchKernelGGL(k_kept_keys, dim3(nblk(nc)), dim3(kT), 0, s, kc.p, cstate.p, nc, kd.p + nv,
                       kcount.p);
  unsigned long long hk = 0;
  LF_HIP(hipMemcpyAsync(&hk, kcount.p, sizeof(hk), hipMemcpyDeviceToHost, s));
  LF_HIP(hipStreamSynchronize(s));
  const int64_t nd = nv + (int64_t)hk;
  LF_HIP(sort_u64(kd.p, nd, s));
  st = sym_csr(kd.p, nd, n_s, drp, dcol, s);
  if (st) return st;

  // triangles: 3-cliques, spurious ones removed
  Buf<int32_t> tcnt, toff, tri, keep, kpos, tri2;
  LF_HIP(tcnt.alloc(n_s));
  LF_HIP(toff.alloc(n_s + 1));
  Buf<long long> tmp2;
  LF_HIP(tmp2.alloc(scan_tmp_elems(n_s + 1)));
  hipLaunchKernelGGL(k_tri_count, dim3(nblk(n_s)), dim3(kT), 0, s, drp.p, dcol.p, n_s, tcnt.p);
  LF_HIP(exclusive_scan(tcnt.p, toff.p, n_s, tmp2.p, s));
  int32_t nt0 = 0;
  LF_HIP(hipMemcpyAsync(&nt0, toff.p + n_s, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  LF_HIP(hipStreamSynchronize(s));
  LF_HIP(tri.alloc(3ll * nt0 + 3));
  LF_HIP(keep.alloc(nt0 + 1));
  LF_HIP(kpos.alloc(nt0 + 1));
  hipLaunchKernelGGL(k_tri_fill, dim3(nblk(n_s)), dim3(kT), 0, s, drp.p, dcol.p, n_s, toff.p, tri.p);
  LF_HIP(launch_fill_i32(keep.p, nt0, 1, s));
  hipLaunchKernelGGL(k_spurious, dim3(nblk(n_s)), dim3(kT), 0, s, drp.p, dcol.p, n_s, tri.p, nt0,
                     keep.p);
  Buf<long long> tmp3;
  LF_HIP(tmp3.alloc(scan_tmp_elems(nt0 + 1)));
  LF_HIP(exclusive_scan(keep.p, kpos.p, nt0, tmp3.p, s));
  int32_t ntk = 0;
  LF_HIP(hipMemcpyAsync(&ntk, kpos.p + nt0, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  LF_HIP(hipStreamSynchronize(s));
  LF_HIP(tri2.alloc(3ll * ntk + 3));
  if (nt0 > 0)
    hipLaunchKernelGGL(k_compact_tri, dim3(nblk(nt0)), dim3(kT), 0, s, tri.p, keep.p, kpos.p, nt0,
                       tri2.p);

  // orientation
  const int64_t T = ntk;
  Buf<unsigned long long> ek, nonman, conflicts;
  Buf<int32_t> across, label, level, otri, chg;
  Buf<double> vn;
  LF_HIP(ek.alloc(pow2_at_least(3 * T + 1)));
  LF_HIP(across.alloc(3 * T + 1));
  LF_HIP(label.alloc(T + 1));
  LF_HIP(level.alloc(T + 1));
  LF_HIP(otri.alloc(3 * T + 3));
  LF_HIP(chg.alloc(1));
  LF_HIP(nonman.alloc(1));
  LF_HIP(conflicts.alloc(1));
  LF_HIP(vn.alloc(3ll * n_s));
  LF_HIP(hipMemsetAsync(nonman.p, 0, sizeof(unsigned long long), s));
  LF_HIP(hipMemsetAsync(conflicts.p, 0, sizeof(unsigned long long), s));
  LF_HIP(hipMemsetAsync(vn.p, 0, sizeof(double) * 3 * n_s, s));
  LF_HIP(launch_fill_i32(across.p, 3 * T + 1, -1, s));
  if (T > 0) {
    hipLaunchKernelGGL(k_edge_keys, dim3(nblk(T)), dim3(kT), 0, s, tri2.p, T, n_s, ek.p);
    LF_HIP(sort_u64(ek.p, 3 * T, s));
    hipLaunchKernelGGL(k_edge_links, dim3(nblk(3 * T)), dim3(kT), 0, s, ek.p, 3 * T, T, n_s, tri2.p,
                       across.p, nonman.p);
    // component labels: the lowest triangle id of each component
    hipLaunchKernelGGL(k_comp_init, dim3(nblk(T)), dim3(kT), 0, s, label.p, T);
    hipLaunchKernelGGL(k_cc_hook, dim3(nblk(T)), dim3(kT), 0, s, across.p, label.p, T);
    hipLaunchKernelGGL(k_cc_final, dim3(nblk(T)), dim3(kT), 0, s, label.p, T);
    LF_HIP(launch_fill_i32(f->owner, n_v, n_s, s));
    LF_HIP(hipMemcpyAsync(f->d_seeds, f->seeds.data(), sizeof(int32_t) * n_s, hipMemcpyHostToDevice, s));
    LF_HIP(launch_scatter_owner(f->d_seeds, n_s, f->owner, s));
    hipLaunchKernelGGL(k_seed_normals, dim3(nblk(n_f)), dim3(kT), 0, s, m->V, m->F, n_f, f->owner,
                       n_s, vn.p);
    hipLaunchKernelGGL(k_orient_roots, dim3(nblk(T)), dim3(kT), 0, s, tri2.p, label.p, T, m->V,
                       f->d_seeds, vn.p, otri.p, level.p);
    // breadth-first levels; a level past the last one assigns nothing, so the
    // host reads the flag once per kCheckEvery levels
    for (int32_t lev = 1; lev <= T; lev += kCheckEvery) {
      LF_HIP(hipMemsetAsync(chg.p, 0, sizeof(int32_t), s));
      for (int32_t q = 0; q < kCheckEvery; ++q)
        hipLaunchKernelGGL(k_orient_level, dim3(nblk(T)), dim3(kT), 0, s, tri2.p, across.p, T,
                           lev + q, otri.p, level.p, chg.p);
      int32_t h = 0;
      LF_HIP(hipMemcpyAsync(&h, chg.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      LF_HIP(hipStreamSynchronize(s));
      if (!h) break;
    }
    hipLaunchKernelGGL(k_orient_conflicts, dim3(nblk(T)), dim3(kT), 0, s, otri.p, across.p, T,
                       conflicts.p);
    LF_HIP(hipGetLastError());
  }

  // results to the host
  DualState* d = f->dual ? f->dual : new DualState();
  f->dual = d;
  LF_HIP(to_host(d->av_rp, vrp.p, n_s + 1, s));
  LF_HIP(hipStreamSynchronize(s));
  LF_HIP(to_host(d->av_col, vcol.p, d->av_rp[n_s], s));
  LF_HIP(to_host(d->at_rp, trp.p, n_s + 1, s));
  LF_HIP(hipStreamSynchronize(s));
  LF_HIP(to_host(d->at_col, tcol.p, d->at_rp[n_s], s));
  LF_HIP(to_host(d->ad_rp, drp.p, n_s + 1, s));
  LF_HIP(hipStreamSynchronize(s));
  LF_HIP(to_host(d->ad_col, dcol.p, d->ad_rp[n_s], s));
  std::vector<unsigned long long> hkc;
  LF_HIP(to_host(hkc, kc.p, nc, s));
  LF_HIP(to_host(d->cand_state, cstate.p, nc, s));
  LF_HIP(to_host(d->tri, otri.p, 3 * T, s));
  unsigned long long hn = 0, hcf = 0;
  LF_HIP(hipMemcpyAsync(&hn, nonman.p, sizeof(hn), hipMemcpyDeviceToHost, s));
  LF_HIP(hipMemcpyAsync(&hcf, conflicts.p, sizeof(hcf), hipMemcpyDeviceToHost, s));
  LF_HIP(hipStreamSynchronize(s));
  d->cand.resize(2 * nc);
  for (int64_t i = 0; i < nc; ++i) {
    d->cand[2 * i] = (int32_t)(hkc[i] / n_s);
    d->cand[2 * i + 1] = (int32_t)(hkc[i] % n_s);
  }
  d->n_removed = nt0 - ntk;
  d->n_nonmanifold = (long long)hn;
  d->n_conflict = (long long)hcf;
  *n_tri = T;
  *adj_nnz = (int64_t)d->ad_col.size();
  if (tris) memcpy(tris, d->tri.data(), sizeof(int32_t) * d->tri.size());
  if (adj_rowptr) memcpy(adj_rowptr, d->ad_rp.data(), sizeof(int32_t) * d->ad_rp.size());
  if (adj_col) memcpy(adj_col, d->ad_col.data(), sizeof(int32_t) * d->ad_col.size());
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_dual_matrix(lf_fields* f, int32_t which, int64_t* nnz, int32_t* rowptr, int32_t* col) try {
  if (!f || !nnz || (which != 0 && which != 1)) return fail(LF_EINVAL, "invalid argument");
  LF_SETTLE(f);
  if (!f->dual) return fail(LF_EINVAL, "no dual mesh computed yet");
  const std::vector<int32_t>& rp = which == 0 ? f->dual->av_rp : f->dual->at_rp;
  const std::vector<int32_t>& c = which == 0 ? f->dual->av_col : f->dual->at_col;
  *nnz = (int64_t)c.size();
  if (rowptr) memcpy(rowptr, rp.data(), sizeof(int32_t) * rp.size());
  if (col) memcpy(col, c.data(), sizeof(int32_t) * c.size());
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

lf_status lf_dual_candidates(lf_fields* f, int64_t* n_cand, int32_t* pairs, int32_t* state) try {
  if (!f || !n_cand) return fail(LF_EINVAL, "invalid argument");
  LF_SETTLE(f);
  if (!f->dual) return fail(LF_EINVAL, "no dual mesh computed yet");
  *n_cand = (int64_t)f->dual->cand_state.size();
  if (pairs) memcpy(pairs, f->dual->cand.data(), sizeof(int32_t) * f->dual->cand.size());
  if (state) memcpy(state, f->dual->cand_state.data(), sizeof(int32_t) * f->dual->cand_state.size());
  return LF_OK;
} catch (const std::bad_alloc&) {
  return lf::host_oom();
}

}  // extern "C"
