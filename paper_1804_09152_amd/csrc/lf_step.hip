// One explicit Euler step of the layered-field method on gfx950.
//
// The step of Algorithm 1 (Section 3.2) for every vertex i, in the row form
// U = Phi^T (rows = vertices, columns = layers):
//   lam_l = L_t(l, i) = sum_u L(i, u) U(u, l)                 (SpGEMM row)
//   S     = { l : phi_l > 0  or  (phi_l == 0 and lam_l > 0) } (rows of interest)
//   v_j   = clamp(phi_j + dt * d_j, 0, 1) for j in S          (update)
//   v    /= sum_S v ; entries below theta dropped             (normalise, prune)
// d_j is the triple sum of Algorithm 1 with the coefficient matrices a, w, e;
// with one value per matrix (and the base-layer coupling described in the
// header) the sums over k and l collapse to per-row totals, so each entry
// costs O(1) once the row totals are known:
//   T = sum_S lam, P_C = sum_{cells in S} phi, R_C = sum_{cells in S} sqrt(phi)
//   Q_j = a/2 (T - lam_j) + w (P_C - phi_j)            (w term for cells only)
//   G_j = e (R_C - sqrt phi_j) + e sqrt(phi_base)      (cell; base term if in S)
//   G_b = -e R_C                                       (base)
//   d_j = -(mu/n) (n Q_j - sum_k Q_k - sqrt(phi_j) G_j)
// which is equation (11) with the alternate inner sum of equation (15).
//
// Design: one thread per vertex row, 256 rows per tile.  The row's union of
// layers (its own row and the rows of its mesh neighbours, typically 1-4
// layers) is accumulated in registers (8 slots); a row with more layers
// takes a slower path with 64 slots in a global-memory workspace row (the
// kernel uses no private memory).  Nothing but U and
// the operator is read, nothing but the next U is written: the field
// Laplacian and the rows of interest never leave the chip.  The output is
// compacted in the same pass: a block-wide scan of the per-row counts and a
// decoupled look-back over tiles (tile order taken from an atomic ticket, so
// every tile a thread waits on is already running) give each row its offset.
#include <hip/hip_ext.h>

#include "lf_internal.h"

namespace lf {

namespace {

// tile status word: [63:62] flag, [61:31] rows-of-interest prefix, [30:0] entry prefix
constexpr unsigned long long kFlagAgg = 1ull << 62;
constexpr unsigned long long kFlagPre = 2ull << 62;
constexpr unsigned long long kLow31 = (1ull << 31) - 1;
constexpr unsigned long long kNoFlag = ~(3ull << 62);
constexpr unsigned kSpinLimit = 1u << 22;

__device__ __forceinline__ unsigned long long ld_status(unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_status(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// square root of a field value in [0, 1]: the hardware instruction (within
// one unit in the last place), not the correctly rounded library sequence
__device__ __forceinline__ float root(float x) { return __builtin_amdgcn_sqrtf(x); }

template <int K>
struct RowBuf {
  int col[K];
  float phi[K];
  float lam[K];
  float out[K];
};

template <int K>
struct MaskT {
  using type = unsigned long long;
};
template <>
struct MaskT<kRowRegs> {
  using type = unsigned int;
};

// Closed-form update of one row's active layers.  Slots s < cnt hold the
// row's union of layers (col, phi = U(i,col), lam = field Laplacian).
// out[s] receives the normalised kept value or -1.
template <int K, bool UNROLL, class B>
__device__ __forceinline__ void row_update(B& r, int cnt, const StepConsts& c, int& n_keep,
                                           int& n_skel, int& ev) {
  using M = typename MaskT<K>::type;
  M act = 0;
  int n = 0, nC = 0;
  bool hb = false;
  float sqb = 0.f, T = 0.f, PC = 0.f, RC = 0.f, Pall = 0.f, Rall = 0.f;
// unrolled: stop at the wavefront's largest slot count (slots at and above
// cnt keep out = -1, set by the caller); runtime loop for the wide path
#define LF_SLOTS                                  \
  _Pragma("unroll") for (int s = 0; s < K; ++s)   \
    if (!__any(s < cnt)) break;                   \
    else
#define LF_SLOTS_RT _Pragma("unroll 1") for (int s = 0; s < K; ++s)
  if constexpr (UNROLL) {
    LF_SLOTS {
      r.out[s] = -1.f;
      if (s < cnt) {
        const float ph = r.phi[s];
        if (ph > 0.f || (ph == 0.f && r.lam[s] > 0.f)) {
          act |= (M)1 << s;
          ++n;
          T += r.lam[s];
          const float sq = root(ph);
          Pall += ph;
          Rall += sq;
          if (r.col[s] == c.n_s) { hb = true; sqb = sq; }
          else { ++nC; PC += ph; RC += sq; }
        }
      }
    }
  } else {
    LF_SLOTS_RT {
      r.out[s] = -1.f;
      if (s < cnt) {
        const float ph = r.phi[s];
        if (ph > 0.f || (ph == 0.f && r.lam[s] > 0.f)) {
          act |= (M)1 << s;
          ++n;
          T += r.lam[s];
          const float sq = root(ph);
          Pall += ph;
          Rall += sq;
          if (r.col[s] == c.n_s) { hb = true; sqb = sq; }
          else { ++nC; PC += ph; RC += sq; }
        }
      }
    }
  }
  n_skel = n;
  n_keep = 0;
  ev = 0;
  if (n == 0) return;
  const float ha = 0.5f * c.a;
  const float fn = (float)n;
  const float sumQ = (c.base_mode == 0)
                         ? ha * (float)(n - 1) * T + c.w * (float)(nC - 1) * PC
                         : ha * (float)(n - 1) * T + c.w * (float)(n - 1) * Pall;
  const float mun = c.mu / fn;
  const float gb = hb ? c.e * sqb : 0.f;
  float V = 0.f;
  auto upd = [&](int s) {
    const float ph = r.phi[s], la = r.lam[s];
    const float sq = root(ph);
    const bool base = r.col[s] == c.n_s;
    float Q, G;
    if (c.base_mode == 0) {
      Q = ha * (T - la) + (base ? 0.f : c.w * (PC - ph));
      G = base ? -c.e * RC : c.e * (RC - sq) + gb;
    } else {
      Q = ha * (T - la) + c.w * (Pall - ph);
      G = c.e * (Rall - sq);
    }
    const float d = -mun * (fn * Q - sumQ - sq * G);
    float v = ph + c.dt * d;
    if (v > 1.f) v = 1.f;
    if (v <= 0.f) v = 0.f;
    r.out[s] = v;
    V += v;
  };
  if constexpr (UNROLL) {
    LF_SLOTS if ((act >> s) & 1) upd(s);
  } else {
    LF_SLOTS_RT if ((act >> s) & 1) upd(s);
  }
  if (!(V > 0.f)) {
    ev = 1;
    if constexpr (UNROLL) {
      LF_SLOTS r.out[s] = -1.f;
    } else {
      LF_SLOTS_RT r.out[s] = -1.f;
    }
    return;
  }
  int k = 0;
  // one division per row; a single active layer normalises to exactly 1
  const float inv = 1.f / V;
  auto fin = [&](int s) {
    const float o = n == 1 ? 1.f : r.out[s] * inv;
    const bool keep = o > 0.f && o >= c.theta;
    r.out[s] = keep ? o : -1.f;
    k += keep ? 1 : 0;
  };
  if constexpr (UNROLL) {
    LF_SLOTS if ((act >> s) & 1) fin(s);
  } else {
    LF_SLOTS_RT if ((act >> s) & 1) fin(s);
  }
  n_keep = k;
#undef LF_SLOTS
#undef LF_SLOTS_RT
}

// ---- register path --------------------------------------------------------

// The slot loops below stop at the wavefront's largest slot count (a uniform
// branch), and are otherwise straight-line selects: no early exits, so the
// register arrays stay in place instead of being copied per control path.
#define LF_FOR_USED_SLOTS(bound)                   \
  _Pragma("unroll") for (int s = 0; s < kRowRegs; ++s) \
    if (!__any(s < (bound))) break;                 \
    else

__device__ __forceinline__ void put_regs(RowBuf<kRowRegs>& r, int slot, int c, float ph, float la) {
#pragma unroll
  for (int s = 0; s < kRowRegs; ++s) {
    const bool m = s == slot;
    r.col[s] = m ? c : r.col[s];
    r.phi[s] = m ? ph : r.phi[s];
    r.lam[s] = m ? la : r.lam[s];
  }
}

// adds w*x into layer c (a new slot when c is not held yet); ovf when the
// row needs more than kRowRegs slots
__device__ __forceinline__ void add_regs(RowBuf<kRowRegs>& r, int& cnt, bool& ovf, int c, float w,
                                         float x) {
  bool found = false;
  LF_FOR_USED_SLOTS(cnt) {
    const bool m = r.col[s] == c;
    r.lam[s] = m ? fmaf(w, x, r.lam[s]) : r.lam[s];
    found = found || m;
  }
  if (!found) {
    const bool ins = cnt < kRowRegs;
    const float wx = w * x;
    LF_FOR_USED_SLOTS(cnt + 1) {
      const bool m = ins && s == cnt;
      r.col[s] = m ? c : r.col[s];
      r.lam[s] = m ? wx : r.lam[s];
    }
    ovf = ovf || !ins;
    cnt += ins ? 1 : 0;
  }
}

constexpr int kNbPre = 8;  // neighbours whose rows are prefetched

// Gathers row i: its own layers (lam starts at L_ii * phi) and then, in the
// operator's column order, every neighbour row scaled by L(i,u).  The loads
// are issued in four independent rounds (row bounds; operator row; the
// neighbours' row bounds; the first two entries of the own row and of every
// neighbour row) so that a thread keeps about twenty loads in flight
// instead of walking a chain of dependent ones.  The accumulation order is
// fixed: own row, then neighbour by neighbour, each row in layer order.
__device__ __forceinline__ bool gather_regs(RowBuf<kRowRegs>& r, int& cnt, int i,
                                            const StepArgs& A) {
#pragma unroll
  for (int s = 0; s < kRowRegs; ++s) { r.col[s] = -1; r.phi[s] = 0.f; r.lam[s] = 0.f; }
  cnt = 0;
  const int p0 = A.uptr_in[i], p1 = A.uptr_in[i + 1];
  const int q0 = A.lptr[i], q1 = A.lptr[i + 1];
  const float dg = A.ldiag[i];
  int nu[kNbPre];
  float nw[kNbPre];
#pragma unroll
  for (int k = 0; k < kNbPre; ++k) {
    const bool ok = q0 + k < q1;
    const Ent le = ok ? A.lent[q0 + k] : Ent{-1, 0.f};
    nu[k] = le.col;
    nw[k] = le.val;
  }
  int na[kNbPre], nb[kNbPre];
#pragma unroll
  for (int k = 0; k < kNbPre; ++k) {
    na[k] = nu[k] >= 0 ? A.uptr_in[nu[k]] : 0;
    nb[k] = nu[k] >= 0 ? A.uptr_in[nu[k] + 1] : 0;
  }
  const Ent o0 = p0 < p1 ? A.uent_in[p0] : Ent{-1, 0.f};
  const Ent o1 = p0 + 1 < p1 ? A.uent_in[p0 + 1] : Ent{-1, 0.f};
  const Ent o2 = p0 + 2 < p1 ? A.uent_in[p0 + 2] : Ent{-1, 0.f};
  Ent e0[kNbPre], e1[kNbPre], e2[kNbPre];
#pragma unroll
  for (int k = 0; k < kNbPre; ++k) {
    e0[k] = na[k] < nb[k] ? A.uent_in[na[k]] : Ent{-1, 0.f};
    e1[k] = na[k] + 1 < nb[k] ? A.uent_in[na[k] + 1] : Ent{-1, 0.f};
    e2[k] = na[k] + 2 < nb[k] ? A.uent_in[na[k] + 2] : Ent{-1, 0.f};
  }
  if (p1 - p0 > kRowRegs) return false;
  // own row: slots 0, 1, 2 in layer order (lam starts at L_ii * phi)
  if (p0 < p1) { r.col[0] = o0.col; r.phi[0] = o0.val; r.lam[0] = dg * o0.val; }
  if (p0 + 1 < p1) { r.col[1] = o1.col; r.phi[1] = o1.val; r.lam[1] = dg * o1.val; }
  if (p0 + 2 < p1) { r.col[2] = o2.col; r.phi[2] = o2.val; r.lam[2] = dg * o2.val; }
  cnt = min(p1 - p0, 3);
  for (int p = p0 + 3; p < p1; ++p) {
    const Ent e = A.uent_in[p];
    put_regs(r, cnt, e.col, e.val, dg * e.val);
    ++cnt;
  }
  bool ovf = false;
#pragma unroll
  for (int k = 0; k < kNbPre; ++k) {
    if (na[k] < nb[k]) add_regs(r, cnt, ovf, e0[k].col, nw[k], e0[k].val);
    if (na[k] + 1 < nb[k]) add_regs(r, cnt, ovf, e1[k].col, nw[k], e1[k].val);
    if (na[k] + 2 < nb[k]) add_regs(r, cnt, ovf, e2[k].col, nw[k], e2[k].val);
    for (int p = na[k] + 3; p < nb[k]; ++p) {
      const Ent e = A.uent_in[p];
      add_regs(r, cnt, ovf, e.col, nw[k], e.val);
    }
  }
  for (int q = q0 + kNbPre; q < q1; ++q) {  // vertices of degree above kNbPre
    const Ent le = A.lent[q];
    const int a0 = A.uptr_in[le.col], a1 = A.uptr_in[le.col + 1];
    for (int p = a0; p < a1; ++p) {
      const Ent e = A.uent_in[p];
      add_regs(r, cnt, ovf, e.col, le.val, e.val);
    }
  }
  return !ovf;
}

// ---- wide path (rows touching more than kRowRegs layers) ----------------------

// Same arithmetic in the same order as the register path, with kRowWide
// slots in a global-memory workspace row.  Returns the number of kept
// entries (0 and *ovf set when the row touches more than kRowWide layers).
__device__ __forceinline__ int wide_row(int i, const StepArgs* A, WideRow* r, int* n_skel, int* ev,
                                     int* ovf) {
  int cnt = 0;
  *n_skel = 0;
  *ev = 0;
  const float dg = A->ldiag[i];
  for (int p = A->uptr_in[i]; p < A->uptr_in[i + 1]; ++p) {
    if (cnt == kRowWide) { *ovf = 1; return 0; }
    const Ent e = A->uent_in[p];
    r->col[cnt] = e.col;
    r->phi[cnt] = e.val;
    r->lam[cnt] = dg * e.val;
    ++cnt;
  }
  for (int q = A->lptr[i]; q < A->lptr[i + 1]; ++q) {
    const Ent le = A->lent[q];
    for (int p = A->uptr_in[le.col]; p < A->uptr_in[le.col + 1]; ++p) {
      const Ent e = A->uent_in[p];
      int s = 0;
      while (s < cnt && r->col[s] != e.col) ++s;
      if (s < cnt) {
        r->lam[s] = fmaf(le.val, e.val, r->lam[s]);
      } else {
        if (cnt == kRowWide) { *ovf = 1; return 0; }
        r->col[cnt] = e.col;
        r->phi[cnt] = 0.f;
        r->lam[cnt] = le.val * e.val;
        ++cnt;
      }
    }
  }
  for (int s = cnt; s < kRowWide; ++s) { r->col[s] = -1; r->phi[s] = 0.f; r->lam[s] = 0.f; }
  int n_keep = 0;
  row_update<kRowWide, false>(*r, cnt, A->c, n_keep, *n_skel, *ev);
  r->cnt = cnt;
  r->n_keep = n_keep;
  return n_keep;
}

// kept entries of a wide row, in ascending layer order
__device__ __forceinline__ void wide_write(const WideRow* r, Ent* dst) {
  int last = -1;
  for (int k = 0; k < r->n_keep; ++k) {
    int best = -1;
    for (int s = 0; s < r->cnt; ++s)
      if (r->out[s] > 0.f && r->col[s] > last && (best < 0 || r->col[s] < r->col[best])) best = s;
    dst[k] = Ent{r->col[best], r->out[best]};
    last = r->col[best];
  }
}

// marks this step (and so every later one of the call) as not done
__device__ __forceinline__ void step_failed(const StepArgs& A, unsigned bit) {
  atomicOr(&A.flags->poisoned, bit);
  atomicMin(&A.flags->fail_step, A.step_idx);
}

__device__ __forceinline__ int wave_incl_scan(int x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

__global__ __launch_bounds__(kBlock) void k_step(StepArgs A) {
  __shared__ int s_tile;
  __shared__ int s_wave[kBlock / 64];
  __shared__ unsigned long long s_excl;
  const int tid = threadIdx.x;
  if (tid == 0) {
    const unsigned pois =
        __hip_atomic_load(&A.flags->poisoned, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_tile = pois ? -1 : (int)atomicAdd(A.ticket, 1u);
  }
  __syncthreads();
  const int tile = s_tile;
  if (tile < 0) return;  // an earlier step overflowed: nothing to do
  if (tid == 0) {
    A.status_next[tile] = 0ull;
    if (tile == 0) {
      *A.ticket_next = 0u;
      *A.wide_ctr_next = 0u;
    }
  }
  const int i = tile * kBlock + tid;

  RowBuf<kRowRegs> r;
  int cnt = 0, n_keep = 0, n_skel = 0, ev = 0, rowovf = 0;
  int wide = -1;  // workspace slot of a wide row
#pragma unroll
  for (int s = 0; s < kRowRegs; ++s) r.out[s] = -1.f;
  if (i < A.n_v) {
    if (gather_regs(r, cnt, i, A)) {
      row_update<kRowRegs, true>(r, cnt, A.c, n_keep, n_skel, ev);
    } else {
      const unsigned slot = atomicAdd(A.wide_ctr, 1u);
      if (slot < (unsigned)A.wide_cap) {
        wide = (int)slot;
        n_keep = wide_row(i, &A, A.wide + slot, &n_skel, &ev, &rowovf);
        if (rowovf) step_failed(A, 2u);
      } else {
        step_failed(A, 8u);  // the step is replayed with more slots
      }
    }
  }
  if (ev) atomicAdd(&A.stats->events, 1ull);

  // block scan of (kept entries, rows-of-interest size), packed 16/16
  const int x = n_keep | (n_skel << 16);
  int incl = wave_incl_scan(x);
  const int wid = tid >> 6, lane = tid & 63;
  if (lane == 63) s_wave[wid] = incl;
  __syncthreads();
  int woff = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) {
    const int v = s_wave[w];
    woff += (w < wid) ? v : 0;
    tot += v;
  }
  incl += woff;

  // decoupled look-back over tiles, one wavefront reading 64 predecessors
  // per probe: lane k looks at tile (tile - 1 - k - 64 m)
  if (tid < 64) {
    const unsigned long long agg =
        ((unsigned long long)(tot >> 16) << 31) | (unsigned long long)(tot & 0xffff);
    unsigned long long excl = 0;
    if (tile == 0) {
      if (lane == 0) st_status(&A.status[0], kFlagPre | agg);
    } else {
      if (lane == 0) st_status(&A.status[tile], kFlagAgg | agg);
      int j0 = tile - 1;
      unsigned spins = 0;
      bool timed_out = false;
      for (;;) {
        const int j = j0 - lane;
        unsigned long long v;
        for (;;) {
          // before tile 0 there is nothing: read as a prefix of zero
          v = j >= 0 ? ld_status(&A.status[j]) : kFlagPre;
          if (!__any((v >> 62) == 0)) break;
          if (++spins > kSpinLimit) { timed_out = true; break; }
          __builtin_amdgcn_s_sleep(1);
        }
        if (timed_out) {
          if (lane == 0) step_failed(A, 4u);
          break;
        }
        const unsigned long long pre = __ballot((v >> 62) == 2);
        const int first = pre ? __ffsll((unsigned long long)pre) - 1 : 64;
        unsigned long long c = lane <= first ? (v & kNoFlag) : 0ull;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
        excl += c;
        if (pre) break;
        j0 -= 64;
      }
      if (lane == 0) st_status(&A.status[tile], kFlagPre | (excl + agg));
    }
    if (lane == 0) s_excl = excl;
  }
  __syncthreads();
  const unsigned long long ex = s_excl;
  const long long ex_count = (long long)(ex & kLow31);
  const long long ex_skel = (long long)(ex >> 31);
  const long long base = ex_count + (long long)((incl - x) & 0xffff);

  if (i < A.n_v) {
    A.uptr_out[i + 1] = (int)(base + n_keep);
    if (base + n_keep <= A.cap) {
      Ent* dst = A.uent_out + base;
      if (wide < 0) {
#pragma unroll
        for (int s = 0; s < kRowRegs; ++s) {
          if (!__any(s < cnt)) break;
          if (r.out[s] > 0.f) {
            int rank = 0;
#pragma unroll
            for (int t = 0; t < kRowRegs; ++t) {
              if (!__any(t < cnt)) break;
              rank += (r.out[t] > 0.f && r.col[t] < r.col[s]) ? 1 : 0;
            }
            dst[rank] = Ent{r.col[s], r.out[s]};
          }
        }
      } else if (!rowovf) {
        wide_write(A.wide + wide, dst);
      }
    }
  }
  if (tile == 0 && tid == 0) A.uptr_out[0] = 0;
  if (tile == A.n_tiles - 1 && tid == 0) {
    const long long total = ex_count + (tot & 0xffff);
    const long long skel = ex_skel + (tot >> 16);
    if (total > A.cap) {
      atomicMax(&A.flags->need, (unsigned long long)total);
      step_failed(A, 1u);
    }
    A.stats->skel = (unsigned long long)skel;
    A.stats->out = (unsigned long long)total;
    A.stats->in = (unsigned long long)A.uptr_in[A.n_v];
  }
}

__global__ void k_reset_flags(StepFlags* f, StepStats* st, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0) {
    f->poisoned = 0;
    f->fail_step = 0xffffffffu;
    f->need = 0;
  }
  if (st && k < n) st[k] = StepStats{0, 0, 0, 0};
}

}  // namespace

hipError_t launch_step(const StepArgs& a, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
  if (t0 && t1) {
    hipExtLaunchKernelGGL(k_step, dim3(a.n_tiles), dim3(kBlock), 0, s, t0, t1, 0, a);
  } else {
    hipLaunchKernelGGL(k_step, dim3(a.n_tiles), dim3(kBlock), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_reset_flags(StepFlags* f, StepStats* st, int n, hipStream_t s) {
  const int nb = n > 0 ? (n + 255) / 256 : 1;
  hipLaunchKernelGGL(k_reset_flags, dim3(nb), dim3(256), 0, s, f, st, n);
  return hipGetLastError();
}

}  // namespace lf
