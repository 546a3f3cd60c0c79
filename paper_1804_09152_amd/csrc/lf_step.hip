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
// Design: one wavefront per slice of 64 consecutive rows, one thread per
// row.  The fields are held in fixed-width rows of three entries (24 bytes;
// longer rows, rare, live in an overflow area), so a
// row's output position is known before the step: no compaction scan, no
// ordering between wavefronts.  The operator slice is stored column-major,
// so the k-th neighbours of the 64 rows are one contiguous 512-byte load
// whose address follows from the wavefront's index alone.
// A row's data arrive in two dependent rounds (its own row, diagonal and
// operator entries; then the rows of its neighbours); the union of layers
// (typically 1-4) is accumulated in 8 register slots; a row with more
// layers, or reading an overflow row, takes a slower path with 64 slots in a
// global-memory workspace row (the kernel uses no private memory).  Nothing
// but U and the operator is read and nothing but the next U is written: the
// field Laplacian and the rows of interest never leave the chip.
#include <hip/hip_ext.h>

#include "lf_internal.h"

namespace lf {

namespace {

// square root of a field value in [0, 1]: the hardware instruction (within
// one unit in the last place), not the correctly rounded library sequence
__device__ __forceinline__ float root(float x) { return __builtin_amdgcn_sqrtf(x); }

template <int K>
struct RowBuf {
  int col[K];
  float phi[K];
  float lam[K];  // field Laplacian; after the update, the output value
};

// output value of slot s: in registers it replaces the field Laplacian,
// which is dead once the slot is updated; the workspace row keeps both
template <int K>
__device__ __forceinline__ float& out_of(RowBuf<K>& r, int s) { return r.lam[s]; }
__device__ __forceinline__ float& out_of(WideRow& r, int s) { return r.out[s]; }

template <int K>
struct MaskT {
  using type = unsigned long long;
};
template <>
struct MaskT<kRowRegs> {
  using type = unsigned int;
};

// Coefficients {a, w, e} of the ordered pair of layers (j, l), j != l, with
// types tj, tl: the table entry; in base_mode 0 a pair with the base carries
// no w, and the base's e against a cell is negated (the scalar reading of
// the base, one table entry per pair of types).
__device__ __forceinline__ float4 pair_coef(const StepConsts& c, int tj, int tl, bool jb,
                                            bool lb) {
  float4 k = c.tab[(int64_t)tj * c.n_types + tl];
  if (c.base_mode == 0 && (jb || lb)) {
    k.y = 0.f;
    if (jb) k.z = -k.z;
  }
  return k;
}

// The update of one slot j of a row from the row totals (TYPED = false):
//   Q_j = a/2 (T - lam_j) + w (P_C - phi_j)             (w term for cells only)
//   G_j = e (R_C - sqrt phi_j) + e sqrt(phi_base)       (cell; base term if in S)
//   G_b = -e R_C                                        (base)
//   v_j = clamp(phi_j - dt (mu/n) (n Q_j - sum Q - sqrt(phi_j) G_j), 0, 1)
// (base_mode 1: every layer a cell of the sums over all of S, no base term).
struct RowTotals {
  float ha, fn, sumQ, mun, gb, T, PC, RC, Pall, Rall;
};
__device__ __forceinline__ RowTotals row_totals(int n, int nC, bool hb, float sqb, float T,
                                                float PC, float RC, float Pall, float Rall,
                                                const StepConsts& c) {
  RowTotals t;
  t.ha = 0.5f * c.a;
  t.fn = (float)n;
  t.sumQ = (c.base_mode == 0) ? t.ha * (float)(n - 1) * T + c.w * (float)(nC - 1) * PC
                              : t.ha * (float)(n - 1) * T + c.w * (float)(n - 1) * Pall;
  t.mun = c.mu / t.fn;
  t.gb = hb ? c.e * sqb : 0.f;
  t.T = T;
  t.PC = PC;
  t.RC = RC;
  t.Pall = Pall;
  t.Rall = Rall;
  return t;
}
__device__ __forceinline__ float slot_update(float ph, float la, int col, const RowTotals& t,
                                             const StepConsts& c) {
  const float sq = root(ph);
  const bool base = col == c.n_s;
  float Q, G;
  if (c.base_mode == 0) {
    Q = t.ha * (t.T - la) + (base ? 0.f : c.w * (t.PC - ph));
    G = base ? -c.e * t.RC : c.e * (t.RC - sq) + t.gb;
  } else {
    Q = t.ha * (t.T - la) + c.w * (t.Pall - ph);
    G = c.e * (t.Rall - sq);
  }
  const float d = -t.mun * (t.fn * Q - t.sumQ - sq * G);
  float v = ph + c.dt * d;
  if (v > 1.f) v = 1.f;
  if (v <= 0.f) v = 0.f;
  return v;
}

// Update of one row's active layers.  Slots s < cnt hold the row's union of
// layers (col, phi = U(i,col), lam = field Laplacian); ub is the
// wavefront's largest cnt in the register path (UNROLL), unused in the wide
// path.  out_of(r, s) receives the normalised kept value, or -1 (or 0 in
// register slots beyond ub).  TYPED = false: one value per coefficient
// matrix, the sums over layers collapse to row totals (closed form above).
// TYPED: per-pair coefficients from the layer types,
//   Q_j = sum_{l != j} (a_jl lam_l / 2 + w_jl phi_l),
//   G_j = sum_{k != j} e_jk sqrt(phi_k),
//   d_j = -(mu/n) (n Q_j - sum_k Q_k - sqrt(phi_j) G_j),
// the same sums of Algorithm 1 with the pairs spelled out (O(n^2) per row).
template <int K, bool UNROLL, bool TYPED, class B>
__device__ __forceinline__ void row_update(B& r, int cnt, int ub, const StepConsts& c,
                                           int& n_keep, int& n_skel, int& ev) {
  int n = 0, nC = 0;
  bool hb = false;
  float sqb = 0.f, T = 0.f, PC = 0.f, RC = 0.f, Pall = 0.f, Rall = 0.f;
// unrolled: stop at the wavefront's largest slot count ub, a uniform value
// (register slots at and above the row's count hold no layer and phi = lam =
// 0, so they are never active); runtime loop over the workspace row for the
// wide path.  The first loop marks every inactive slot by phi = -1 for the
// later ones.
#define LF_SLOTS                                  \
  _Pragma("unroll") for (int s = 0; s < K; ++s)   \
    if (s >= ub) break;                           \
    else
#define LF_SLOTS_RT _Pragma("unroll 1") for (int s = 0; s < K; ++s)
  if constexpr (UNROLL) {
    LF_SLOTS {
      const float ph = r.phi[s];
      const bool a = ph > 0.f || (ph == 0.f && r.lam[s] > 0.f);
      r.phi[s] = a ? ph : -1.f;  // an inactive slot is marked by phi = -1
      if (a) {
        ++n;
        T += r.lam[s];
        const float sq = root(ph);
        Pall += ph;
        Rall += sq;
        if (r.col[s] == c.n_s) { hb = true; sqb = sq; }
        else { ++nC; PC += ph; RC += sq; }
      }
    }
  } else {
    LF_SLOTS_RT {
      if (s < cnt) {
        const float ph = r.phi[s];
        const bool a = ph > 0.f || (ph == 0.f && r.lam[s] > 0.f);
        r.phi[s] = a ? ph : -1.f;  // an inactive slot is marked by phi = -1
        if (a) {
          ++n;
          T += r.lam[s];
          const float sq = root(ph);
          Pall += ph;
          Rall += sq;
          if (r.col[s] == c.n_s) { hb = true; sqb = sq; }
          else { ++nC; PC += ph; RC += sq; }
        }
      } else {
        r.phi[s] = -1.f;  // the workspace slots past the row's count: inactive too
      }
    }
  }
  n_skel = n;
  n_keep = 0;
  ev = 0;
  if (n == 0) {
    if constexpr (UNROLL) {
      LF_SLOTS out_of(r, s) = -1.f;
    } else {
      LF_SLOTS_RT out_of(r, s) = -1.f;
    }
    return;
  }
  const RowTotals t = row_totals(n, nC, hb, sqb, T, PC, RC, Pall, Rall, c);
  const float fn = t.fn, mun = t.mun;
  float V = 0.f;
  auto upd = [&](int s) {
    const float v = slot_update(r.phi[s], r.lam[s], r.col[s], t, c);
    out_of(r, s) = v;
    V += v;
  };
  if constexpr (TYPED) {
    // inner loops over the other active slots l
#define LF_INNER                                                  \
  _Pragma("unroll") for (int l = 0; l < (UNROLL ? K : 1); ++l)    \
    if (l >= ub) break;                                           \
    else
#define LF_INNER_RT for (int l = 0; l < cnt; ++l)
    // n Q_j - sqrt(phi_j) G_j per slot: registers in the register path, the workspace row's
    // output slots (overwritten by the value below) in the wide path
    float qbuf[UNROLL ? K : 1];
    auto q_at = [&](int s) -> float& {
      if constexpr (UNROLL) return qbuf[s];
      else return out_of(r, s);
    };
    // the slots' types and square roots: computed once into registers in
    // the register path
    int tbuf[UNROLL ? K : 1];
    float sbuf[UNROLL ? K : 1];
    if constexpr (UNROLL) {
      LF_SLOTS {
        tbuf[s] = r.phi[s] >= 0.f ? c.types[r.col[s]] : 0;
        sbuf[s] = root(r.phi[s]);
      }
    }
    auto type_of = [&](int s) {
      if constexpr (UNROLL) return tbuf[s];
      else return c.types[r.col[s]];
    };
    auto sqrt_of = [&](int s) {
      if constexpr (UNROLL) return sbuf[s];
      else return root(r.phi[s]);
    };
    // Q_s and G_s in one pass over the other active slots (one table read
    // per ordered pair); what d_s needs besides the sum of all Q is kept
    // per slot: n Q_s - sqrt(phi_s) G_s
    auto qg_of = [&](int s) {
      const int ts = type_of(s);
      const bool sb = r.col[s] == c.n_s;
      float Q = 0.f, G = 0.f;
      auto term = [&](int l) {
        if (l == s || !(r.phi[l] >= 0.f)) return;
        const float4 k = pair_coef(c, ts, type_of(l), sb, r.col[l] == c.n_s);
        Q += 0.5f * k.x * r.lam[l] + k.y * r.phi[l];
        G += k.z * sqrt_of(l);
      };
      if constexpr (UNROLL) {
        LF_INNER term(l);
      } else {
        LF_INNER_RT term(l);
      }
      return float2{Q, G};
    };
#undef LF_INNER
#undef LF_INNER_RT
    float sQ = 0.f;
    auto pass_q = [&](int s) {
      const float2 qg = qg_of(s);
      q_at(s) = fn * qg.x - sqrt_of(s) * qg.y;
      sQ += qg.x;
    };
    auto pass_v = [&](int s) {
      float v = r.phi[s] + c.dt * (-mun * (q_at(s) - sQ));
      if (v > 1.f) v = 1.f;
      if (v <= 0.f) v = 0.f;
      out_of(r, s) = v;
      V += v;
    };
    if constexpr (UNROLL) {
      LF_SLOTS if (r.phi[s] >= 0.f) pass_q(s);
      LF_SLOTS if (r.phi[s] >= 0.f) pass_v(s); else out_of(r, s) = -1.f;
    } else {
      LF_SLOTS_RT if (r.phi[s] >= 0.f) pass_q(s);
      LF_SLOTS_RT if (r.phi[s] >= 0.f) pass_v(s); else out_of(r, s) = -1.f;
    }
  } else if constexpr (UNROLL) {
    LF_SLOTS if (r.phi[s] >= 0.f) upd(s); else out_of(r, s) = -1.f;
  } else {
    LF_SLOTS_RT if (r.phi[s] >= 0.f) upd(s); else out_of(r, s) = -1.f;
  }
  if (!(V > 0.f)) {
    ev = 1;
    if constexpr (UNROLL) {
      LF_SLOTS out_of(r, s) = -1.f;
    } else {
      LF_SLOTS_RT out_of(r, s) = -1.f;
    }
    return;
  }
  int k = 0;
  // one division per row; a single active layer normalises to exactly 1
  const float inv = 1.f / V;
  auto fin = [&](int s) {
    const float o = n == 1 ? 1.f : out_of(r, s) * inv;
    const bool keep = o > 0.f && o >= c.theta;
    out_of(r, s) = keep ? o : -1.f;
    k += keep ? 1 : 0;
  };
  if constexpr (UNROLL) {
    LF_SLOTS if (r.phi[s] >= 0.f) fin(s);
  } else {
    LF_SLOTS_RT if (r.phi[s] >= 0.f) fin(s);
  }
  n_keep = k;
#undef LF_SLOTS
#undef LF_SLOTS_RT
}

// ---- register path --------------------------------------------------------

constexpr int kNoLayer = -2147483647 - 1;  // layer of an empty register slot

// whether the predicate holds on some active lane of the wavefront (the
// ballot's mask is the compare's own result, with no re-materialisation)
__device__ __forceinline__ bool wave_any(bool p) { return __builtin_amdgcn_ballot_w64(p) != 0; }

// The slot loops below stop at the wavefront's largest slot count (a uniform
// branch), and are otherwise straight-line selects: no early exits, so the
// register arrays stay in place instead of being copied per control path.
#define LF_FOR_USED_SLOTS(bound)                   \
  _Pragma("unroll") for (int s = 0; s < kRowRegs; ++s) \
    if (!wave_any(s < (bound))) break;              \
    else

// adds w*x into layer c (a new slot when c is not held yet); ovf when the
// row needs more than kRowRegs slots.  For the rare entries met under
// divergent control (overflow rows, operator rows beyond the slice).
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

// the wavefront's largest slot count, from every lane's count
__device__ __forceinline__ int wave_slots(int cnt) {
  int ub = 0;
#pragma unroll
  for (int s = 0; s < kRowRegs; ++s) ub += wave_any(cnt > s) ? 1 : 0;
  return ub;
}

constexpr int kXcds = 8;   // accelerator dies of the MI355X, each with its own L2
constexpr int kWideBlocks = 2048;  // wavefronts of a k_wide launch (rows beyond: in turn)
#ifndef LF_WIN
#define LF_WIN 3
#endif
constexpr int kWin = LF_WIN;  // neighbour rows in flight

__device__ __forceinline__ bool is_ovf(const Ent& e) { return e.col == kOvfMark; }

// row v of U_t: a 32-bit byte offset from the buffer's base (rows are 32
// bytes and a field buffer stays far below 4 GiB), so that the load adds
// the offset to the base in the address unit instead of in 64-bit vector
// arithmetic
__device__ __forceinline__ EllRow row_at(const EllRow* base, int v) {
  return *reinterpret_cast<const EllRow*>(reinterpret_cast<const char*>(base) +
                                          (uint32_t)v * (uint32_t)sizeof(EllRow));
}

// entries of a row of U_t
struct RowView {
  const Ent* p;
  int n;
};

// the entries of an overflow row (bounds-checked, so that a row written by
// a failed step reads as empty)
__device__ __forceinline__ RowView ovf_view(const StepArgs& A, const EllRow& u) {
  const long long o = ovf_dec(u.e[1].col), n = ovf_dec(u.e[2].col);
  if (o < 0 || n < 0 || o + n > A.ovf_cap) return RowView{A.ovf_in, 0};
  return RowView{A.ovf_in + o, (int)n};
}

// entries of row u of U_t: inline, or in the overflow area
__device__ __forceinline__ RowView row_view(const StepArgs* A, int u) {
  const Ent* e = A->u_in[u].e;
  if (is_ovf(e[0])) return ovf_view(*A, A->u_in[u]);
  int n = 0;
  while (n < kEll && e[n].col >= 0) ++n;
  return RowView{e, n};
}

// One inline neighbour row (up to kEll entries, ascending layers, filled
// from entry 0) scaled by w, merged by every lane at once.  `ub` is the
// wavefront's largest slot count, kept in a scalar register and updated from
// the lanes that open a slot, so the slot loops cost no vector compare for
// their bound; it must stay uniform, so this is called only in
// wavefront-uniform control flow.  One pass over the slots searches for all
// of the row's entries (its entries are distinct layers, so at most one
// matches a slot; a slot that none matches gets fma(w, 0, lam), which leaves
// it unchanged); then each entry no slot holds opens one, in entry order --
// the same sums and slot order as add_regs called once per entry.  key[j]
// is the layer of entry j, or a negative value on a lane where entry j does
// not take part: a negative key opens no slot and matches none (slots hold
// layers >= 0, empty ones kNoLayer; an overflow header's column that equals
// kNoLayer carries the value 0, so its match adds nothing).  Which entries
// the slots hold is kept as wavefront masks (ballots) in scalar registers.
// NV: the entries that take part on some lane.
template <int NV>
__device__ __forceinline__ void add_row_wave(RowBuf<kRowRegs>& r, int& cnt, int& ub, bool& ovf,
                                             const int (&key)[kEll], const float (&x)[kEll],
                                             float w) {
  // found[j]: the lanes whose entry j is held by a slot (or takes no part),
  // as a wavefront mask in scalar registers
  unsigned long long found[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) found[j] = __builtin_amdgcn_ballot_w64(key[j] < 0);
  const unsigned long long lanes = __builtin_amdgcn_read_exec();
  // a row's entries fill from entry 0: none takes part where entry 0 does not
  if ((lanes & ~found[0]) == 0ull) return;
#pragma unroll
  for (int s = 0; s < kRowRegs; ++s) {
    if (s >= ub) break;
    float xs = 0.f;
#pragma unroll
    for (int j = NV - 1; j >= 0; --j) {
      const bool m = r.col[s] == key[j];
      xs = m ? x[j] : xs;
      found[j] |= __builtin_amdgcn_ballot_w64(m);
    }
    r.lam[s] = fmaf(w, xs, r.lam[s]);
  }
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const unsigned long long nf = lanes & ~found[j];
    if (nf == 0ull) continue;
    const unsigned long long im = nf & __builtin_amdgcn_ballot_w64(cnt < kRowRegs);
    const bool ins = __builtin_amdgcn_inverse_ballot_w64(im);
    const float wx = w * x[j];
#pragma unroll
    for (int s = 0; s < kRowRegs; ++s) {
      if (s > ub) break;
      const bool m = ins && s == cnt;
      r.col[s] = m ? key[j] : r.col[s];
      r.lam[s] = m ? wx : r.lam[s];
    }
    if (nf & ~im) ovf = ovf || __builtin_amdgcn_inverse_ballot_w64(nf & ~im);
    ub += (im & __builtin_amdgcn_ballot_w64(cnt == ub)) ? 1 : 0;  // cnt <= ub on every lane
    cnt += ins ? 1 : 0;
  }
}

// Row i's gather into register slots: its own layers (lam starts at L_ii *
// phi) and then every neighbour row scaled by L(i,u), each row in layer
// order.  The neighbour rows stream through a window of kWin rows (the row
// of neighbour k + kWin is requested before neighbour k is merged, so a few
// loads stay in flight without holding every neighbour row in registers),
// in the operator's column order.  A row kept in the overflow area (a
// neighbour's, then the own row) is merged after the others, from there, so
// that only the lanes that meet one wait for its extra load rounds (the
// slots need no order: the output is ranked by layer).  Returns kGatherOk,
// or kGatherWide when the row touches more than kRowRegs layers.
constexpr int kGatherOk = 0, kGatherWide = 1;

__device__ __forceinline__ int gather_regs(RowBuf<kRowRegs>& r, int& cnt, int& ub, int& n_in,
                                           const int i, const bool live, const Ent* ops,
                                           const StepArgs& A) {
  // Every lane runs the gather (a lane past the last row, live false, reads
  // row 0 and adds nothing), so that the slot bound stays wavefront-uniform.
#pragma unroll
  for (int s = 0; s < kRowRegs; ++s) { r.col[s] = kNoLayer; r.phi[s] = 0.f; r.lam[s] = 0.f; }
  cnt = 0;
  const int ic = live ? i : 0;
  const EllRow own = row_at(A.u_in, ic);
  const float dg = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(A.ldiag) +
                                                   (uint32_t)ic * 4u);
  // entries of U_t in this row (for the counters)
  n_in = 0;
#pragma unroll
  for (int j = 0; j < kEll; ++j) n_in += own.e[j].col >= 0 ? 1 : 0;
  const bool own_ovf = live && is_ovf(own.e[0]);
  if (own_ovf) n_in = (int)ovf_dec(own.e[2].col);
  if (!live) n_in = 0;
  // operator entries: lanes past the last row hold {-1, 0} in the slice
  Ent le[kOpWidth];
#pragma unroll
  for (int k = 0; k < kOpWidth; ++k)
    le[k] = k < A.op_w ? ops[k * kSlice] : Ent{-1, 0.f};
  EllRow win[kWin];
#pragma unroll
  for (int k = 0; k < kWin; ++k) win[k] = row_at(A.u_in, le[k].col >= 0 ? le[k].col : A.n_v);
  bool ovf = false;
  // the entries of an overflow row, scaled by w
  auto merge_ovf = [&](const EllRow& u, float w) {
    const RowView v = ovf_view(A, u);
    for (int p = 0; p < v.n; ++p) add_regs(r, cnt, ovf, v.p[p].col, w, v.p[p].val);
  };
  // own row: slots 0..kEll-1 in layer order (an overflow row is merged
  // last; its header's columns are negative)
#pragma unroll
  for (int j = 0; j < kEll; ++j) {
    if (live && own.e[j].col >= 0) {
      r.col[j] = own.e[j].col;
      r.phi[j] = own.e[j].val;
      r.lam[j] = dg * own.e[j].val;
      cnt = j + 1;
    }
  }
  ub = wave_slots(cnt);
  // neighbours in the slice whose rows are overflow rows: neighbour k at bit
  // nk - 1 - k (one doubling add per neighbour)
  unsigned onb = 0;
  int nk = 0;
#pragma unroll
  for (int k = 0; k < kOpWidth; ++k) {
    if (k >= A.op_w) break;
    const EllRow u = win[k % kWin];
    if (k + kWin < kOpWidth && k + kWin < A.op_w)
      win[k % kWin] = row_at(A.u_in, le[k + kWin].col >= 0 ? le[k + kWin].col : A.n_v);
    onb = onb + onb + (is_ovf(u.e[0]) ? 1u : 0u);
    nk = k + 1;
    // a missing neighbour reads the empty row (layers -1) and an overflow
    // row's header has negative columns: neither matches a slot (an empty
    // slot holds kNoLayer) and neither opens one
    int key[kEll];
    float x[kEll];
#pragma unroll
    for (int j = 0; j < kEll; ++j) {
      key[j] = u.e[j].col;
      x[j] = u.e[j].val;
    }
    add_row_wave<kEll>(r, cnt, ub, ovf, key, x, le[k].val);
  }
  // the rare entries, under divergent control: the slot bound is counted
  // again afterwards
  const bool tail = A.op_w == kOpWidth && le[kOpWidth - 1].col >= 0;  // rows beyond the slices
  if (wave_any(tail || onb != 0u || own_ovf)) {
    if (tail) {
      for (int q = A.lptr[i] + kOpWidth; q < A.lptr[i + 1]; ++q) {
        const Ent l = A.lent[q];
        if (l.col < 0) continue;
        const EllRow u = row_at(A.u_in, l.col);
        if (is_ovf(u.e[0])) {
          merge_ovf(u, l.val);
          continue;
        }
#pragma unroll
        for (int j = 0; j < kEll; ++j)
          if (u.e[j].col >= 0) add_regs(r, cnt, ovf, u.e[j].col, l.val, u.e[j].val);
      }
    }
    while (onb) {  // the overflow rows among the slice's neighbours, in column order
      const int b = 31 - __builtin_clz(onb);
      const int k = nk - 1 - b;
      onb &= ~(1u << b);
      const Ent l = ops[k * kSlice];
      merge_ovf(row_at(A.u_in, l.col), l.val);
    }
    if (own_ovf) {  // own entries: add L_ii * phi and set phi of their slots
      const RowView o = ovf_view(A, row_at(A.u_in, i));
      for (int p = 0; p < o.n; ++p) {
        const Ent e = o.p[p];
        add_regs(r, cnt, ovf, e.col, dg, e.val);
#pragma unroll
        for (int t = 0; t < kRowRegs; ++t) r.phi[t] = r.col[t] == e.col ? e.val : r.phi[t];
      }
    }
    ub = wave_slots(cnt);
  }
  return ovf ? kGatherWide : kGatherOk;
}

// ---- wide path (many layers, or overflow rows) --------------------------------



// Same arithmetic in the same order as the register path, with kRowWide
// slots in a global-memory workspace row.  Returns the number of kept
// entries (0 and *ovf set when the row touches more than kRowWide layers).
template <bool TYPED>
__device__ __forceinline__ int wide_row(int i, const Ent* ops, const StepArgs* A, WideRow* r,
                                        int* n_skel, int* ev, int* ovf) {
  int cnt = 0;
  *n_skel = 0;
  *ev = 0;
  const float dg = A->ldiag[i];
  const RowView o = row_view(A, i);
  for (int p = 0; p < o.n; ++p) {
    if (cnt == kRowWide) { *ovf = 1; return 0; }
    const Ent e = o.p[p];
    r->col[cnt] = e.col;
    r->phi[cnt] = e.val;
    r->lam[cnt] = dg * e.val;
    ++cnt;
  }
  const int q0 = A->lptr[i], deg = A->lptr[i + 1] - q0;
  for (int k = 0; k < deg; ++k) {
    const Ent le = k < A->op_w ? ops[k * kSlice] : A->lent[q0 + k];
    if (le.col < 0) continue;
    const RowView v = row_view(A, le.col);
    for (int p = 0; p < v.n; ++p) {
      const Ent e = v.p[p];
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
  row_update<kRowWide, false, TYPED>(*r, cnt, cnt, A->c, n_keep, *n_skel, *ev);
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

// marks this step (and so every later one of the chunk) as not done
__device__ __forceinline__ void step_failed(const StepArgs& A, unsigned bit) {
  atomicOr(&A.flags->poisoned, bit);
  atomicMin(&A.flags->fail_step, A.step_idx);
}

// Sum over the wavefront, complete in lane 63 only: a scan within each row
// of 16 lanes by DPP row shifts, then the row totals carried on by DPP row
// broadcasts (lane 15 into row 1 and lane 47 into row 3; then lane 31 into
// rows 2 and 3).  Lanes shifted in from outside a row, and rows left out by
// the row mask, add 0.  Needs every lane active.
__device__ __forceinline__ unsigned dpp_sum63(unsigned x) {
  x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, true);  // row_shr:1
  x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, true);  // row_shr:2
  x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, true);  // row_shr:4
  x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, true);  // row_shr:8
  x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return x;
}
// the same for the maximum of non-negative floats (ordered as their bits)
__device__ __forceinline__ unsigned dpp_max63(unsigned x) {
  auto mx = [](unsigned a, unsigned b) { return a > b ? a : b; };
  x = mx(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, true));
  x = mx(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, true));
  x = mx(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, true));
  x = mx(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, true));
  x = mx(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false));
  x = mx(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false));
  return x;
}

__device__ __forceinline__ int wave_sum(int x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Change of the row in this step (convergence measures): changed = 1 when
// its label (argmax over the cell layers, lowest layer on ties) or its set of
// layers at or above tau differs, and dmax = the largest
// |U_{t+1}(i,l) - U_t(i,l)| over the layers of either step.  phi is the old
// value (0 if absent), o the new one (<= 0 if absent).
struct ChangeAcc {
  int lo = -1, ln = -1;  // old and new label
  float vo = 0.f, vn = 0.f;
  bool tau_diff = false;
  float dmax = 0.f;
  __device__ __forceinline__ void add(int c, float phi, float o, const StepConsts& k) {
    tau_diff = tau_diff || ((phi >= k.tau) != (o >= k.tau));
    dmax = fmaxf(dmax, fabsf((o > 0.f ? o : 0.f) - phi));
    if (c >= 0 && c < k.n_s) {
      if (phi > 0.f && (lo < 0 || phi > vo || (phi == vo && c < lo))) { lo = c; vo = phi; }
      if (o > 0.f && (ln < 0 || o > vn || (o == vn && c < ln))) { ln = c; vn = o; }
    }
  }
  __device__ __forceinline__ int changed() const { return (tau_diff || lo != ln) ? 1 : 0; }
};

// after the update, lam holds the kept output value or a value <= 0
// (slots at and above the row's count hold layer -1 and take no part; ub is
// the wavefront's largest count)
__device__ __forceinline__ void row_change(const RowBuf<kRowRegs>& r, int ub,
                                           const StepConsts& k, int& changed, float& dmax) {
  ChangeAcc a;
#pragma unroll
  for (int s = 0; s < kRowRegs; ++s) {
    if (s >= ub) break;
    a.add(r.col[s], fmaxf(r.phi[s], 0.f), r.lam[s], k);
  }
  changed = a.changed();
  dmax = a.dmax;
}

__device__ __forceinline__ void wide_change(const WideRow* r, const StepConsts& k, int& changed,
                                            float& dmax) {
  ChangeAcc a;
  for (int s = 0; s < r->cnt; ++s) a.add(r->col[s], fmaxf(r->phi[s], 0.f), r->out[s], k);
  changed = a.changed();
  dmax = a.dmax;
}

__device__ __forceinline__ float wave_max(float x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmaxf(x, __shfl_xor(x, o, 64));
  return x;
}

// ---- rows touching more than kRowRegs layers, one wavefront per row ----------

// Lane masks (one bit per lane of the wavefront, in scalar registers) and
// the value of a register on one lane.
using Mask = unsigned long long;
__device__ __forceinline__ Mask ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ __forceinline__ bool lane_in(Mask m) { return __builtin_amdgcn_inverse_ballot_w64(m); }
__device__ __forceinline__ int lane_i32(int x, int s) { return __builtin_amdgcn_readlane(x, s); }
__device__ __forceinline__ float lane_f32(float x, int s) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), s));
}

struct WideResult {
  int n_keep, n_skel, ev, changed;
  float dmax;
};

// A row touching more than kRowRegs layers, stepped by the whole wavefront:
// lane s holds the row's slot s (up to kRowWide = 64 slots, one per lane).
// The neighbourhood is merged in a fixed order (own entries, then each
// neighbour row in the operator's column order, each row in layer order; a
// slot already holding the layer takes fma(L(i,u), U(u,l), lam), a new layer
// opens the next slot); the row totals and the normalisation sum run over
// the slots in slot order, as in the register path, and each slot's update
// runs on its own lane.  i: the row (its operator entries are column
// i / kSlice's operator slice).  Called with every lane active (all values
// below that do not depend on the lane are uniform); writes the row, inline
// or in the overflow area.
template <bool TYPED>
__device__ __forceinline__ WideResult wide_row_wave(const StepArgs& A, const int i) {
  const int lane = threadIdx.x;
  const Ent* ops = A.lell + (int64_t)(i / kSlice) * A.op_w * kSlice + i % kSlice;
  WideResult res{0, 0, 0, 0, 0.f};
  int col = -1;  // slot `lane`: layer, U_t value, field Laplacian
  float phi = 0.f, lam = 0.f;
  int cnt = 0;
  bool full = false;  // more than kRowWide layers
  const float dg = A.ldiag[i];
  // adds x scaled by wgt into layer c (a new slot when no lane holds it)
  auto add = [&](int c, float wgt, float x) {
    const Mask m = ballot(col == c);
    if (m != 0) {
      if (lane_in(m)) lam = fmaf(wgt, x, lam);
    } else if (cnt == kRowWide) {
      full = true;
    } else {
      if (lane == cnt) {
        col = c;
        phi = 0.f;
        lam = wgt * x;
      }
      ++cnt;
    }
  };
  // The neighbours' operator entries and rows are loaded one neighbour per
  // lane, and a neighbour row kept in the overflow area has its first kPre
  // entries loaded by its lane too, all before the own row is merged; the
  // merge then runs in the fixed order on values already in registers (a
  // longer overflow row reads the rest from memory).
  constexpr int kPre = 6;
  const int q0 = A.lptr[i], deg = A.lptr[i + 1] - q0;
  for (int k0 = 0; k0 == 0 || k0 < deg; k0 += kSlice) {
    const int k = k0 + lane;
    Ent le{-1, 0.f};
    if (k < deg) le = k < A.op_w ? ops[k * kSlice] : A.lent[q0 + k];
    EllRow u;
#pragma unroll
    for (int j = 0; j < kEll; ++j) u.e[j] = Ent{-1, 0.f};
    if (le.col >= 0) u = row_at(A.u_in, le.col);
    int pre_n = 0;
    Ent pre[kPre];
#pragma unroll
    for (int p = 0; p < kPre; ++p) pre[p] = Ent{-1, 0.f};
    if (le.col >= 0 && u.e[0].col == kOvfMark) {
      const RowView v = ovf_view(A, u);
      pre_n = v.n;
#pragma unroll
      for (int p = 0; p < kPre; ++p)
        if (p < v.n) pre[p] = v.p[p];
    }
    if (k0 == 0) {  // own entries first: distinct layers
      const RowView own = row_view(&A, i);
      for (int p = 0; p < own.n; ++p) {
        if (cnt == kRowWide) {
          full = true;
          break;
        }
        const Ent e = own.p[p];
        if (lane == cnt) {
          col = e.col;
          phi = e.val;
          lam = dg * e.val;
        }
        ++cnt;
      }
    }
    const int kn = deg - k0 < kSlice ? deg - k0 : kSlice;
    for (int q = 0; q < kn && !full; ++q) {
      const int nb = lane_i32(le.col, q);
      if (nb < 0) continue;
      const float wgt = lane_f32(le.val, q);
      if (lane_i32(u.e[0].col, q) == kOvfMark) {
        const int n = lane_i32(pre_n, q);
#pragma unroll
        for (int p = 0; p < kPre; ++p) {
          if (p >= n || full) break;
          add(lane_i32(pre[p].col, q), wgt, lane_f32(pre[p].val, q));
        }
        if (n > kPre) {
          const RowView v = row_view(&A, nb);
          for (int p = kPre; p < v.n && !full; ++p) add(v.p[p].col, wgt, v.p[p].val);
        }
        continue;
      }
#pragma unroll
      for (int j = 0; j < kEll; ++j) {
        const int c = lane_i32(u.e[j].col, q);
        if (c < 0 || full) break;
        add(c, wgt, lane_f32(u.e[j].val, q));
      }
    }
    if (full) break;
  }
  Ent* row = A.u_out[i].e;
  if (full) {  // the step fails; the row is written empty
    if (lane == 0) step_failed(A, 2u);
    if (lane < kEll) row[lane] = Ent{-1, 0.f};
    return res;
  }
  // rows of interest and row totals, over the slots in slot order
  const bool act = lane < cnt && (phi > 0.f || (phi == 0.f && lam > 0.f));
  const float sq = root(phi);
  const Mask am = ballot(act);
  int n = 0, nC = 0;
  bool hb = false;
  float sqb = 0.f, T = 0.f, PC = 0.f, RC = 0.f, Pall = 0.f, Rall = 0.f;
  for (int s = 0; s < cnt; ++s) {
    if (!((am >> s) & 1)) continue;
    const float ph_s = lane_f32(phi, s), sq_s = lane_f32(sq, s);
    ++n;
    T += lane_f32(lam, s);
    Pall += ph_s;
    Rall += sq_s;
    if (lane_i32(col, s) == A.c.n_s) { hb = true; sqb = sq_s; }
    else { ++nC; PC += ph_s; RC += sq_s; }
  }
  res.n_skel = n;
  float out = -1.f;
  if (n > 0) {
    const RowTotals t = row_totals(n, nC, hb, sqb, T, PC, RC, Pall, Rall, A.c);
    float v;
    if constexpr (TYPED) {
      const int ty = A.c.types[act ? col : 0];
      const bool sb = col == A.c.n_s;
      float Q = 0.f, G = 0.f;
      for (int l = 0; l < cnt; ++l) {
        if (!((am >> l) & 1)) continue;
        const int col_l = lane_i32(col, l);
        const float4 k = pair_coef(A.c, ty, A.c.types[col_l], sb, col_l == A.c.n_s);
        if (lane != l) {
          Q += 0.5f * k.x * lane_f32(lam, l) + k.y * lane_f32(phi, l);
          G += k.z * lane_f32(sq, l);
        }
      }
      const float q = t.fn * Q - sq * G;
      float sQ = 0.f;
      for (int s = 0; s < cnt; ++s)
        if ((am >> s) & 1) sQ += lane_f32(Q, s);
      v = phi + A.c.dt * (-t.mun * (q - sQ));
      if (v > 1.f) v = 1.f;
      if (v <= 0.f) v = 0.f;
    } else {
      v = slot_update(phi, lam, col, t, A.c);
    }
    float V = 0.f;
    for (int s = 0; s < cnt; ++s)
      if ((am >> s) & 1) V += lane_f32(v, s);
    if (!(V > 0.f)) {
      res.ev = 1;
    } else {
      // one division per row; a single active layer normalises to exactly 1
      const float inv = 1.f / V;
      const float o = n == 1 ? 1.f : v * inv;
      out = act && o > 0.f && o >= A.c.theta ? o : -1.f;
    }
  }
  if (A.measure) {
    ChangeAcc a;
    for (int s = 0; s < cnt; ++s) a.add(lane_i32(col, s), lane_f32(phi, s), lane_f32(out, s), A.c);
    res.changed = a.changed();
    res.dmax = a.dmax;
  }
  // kept entries in ascending layer order
  const Mask km = ballot(out > 0.f);
  const int n_keep = __builtin_popcountll(km);
  res.n_keep = n_keep;
  int rank = 0;
  for (int s = 0; s < cnt; ++s)
    if ((km >> s) & 1) rank += lane_i32(col, s) < col ? 1 : 0;
  if (n_keep > kEll) {
    unsigned o32 = 0;
    if (lane == 0) o32 = atomicAdd(A.ovf_ctr, (unsigned)n_keep);
    const long long o = (long long)(unsigned)__builtin_amdgcn_readfirstlane((int)o32);
    const bool fits = o + n_keep <= A.ovf_cap;
    if (lane == 0 && !fits) {
      atomicMax(&A.flags->need, (unsigned long long)(o + n_keep));
      step_failed(A, 1u);  // the step is replayed with a larger area
    }
    if (lane == 0) row[0] = Ent{kOvfMark, 0.f};
    if (lane == 1) row[1] = Ent{ovf_enc(fits ? o : 0), 0.f};
    if (lane == 2) row[2] = Ent{ovf_enc(fits ? n_keep : 0), 0.f};
    if (fits && lane_in(km)) A.ovf_out[o + rank] = Ent{col, out};
  } else {
    if (lane_in(km)) row[rank] = Ent{col, out};
    if (lane >= n_keep && lane < kEll) row[lane] = Ent{-1, 0.f};
  }
  return res;
}

// kept register-path entries in ascending layer order at dst[0..n_keep)
// (ub: the wavefront's largest slot count)
__device__ __forceinline__ void write_regs(const RowBuf<kRowRegs>& r, int ub, Ent* dst) {
#pragma unroll
  for (int s = 0; s < kRowRegs; ++s) {
    if (s >= ub) break;
    if (r.lam[s] > 0.f) {
      int rank = 0;
#pragma unroll
      for (int t = 0; t < kRowRegs; ++t) {
        if (t >= ub) break;
        rank += (r.lam[t] > 0.f && r.col[t] < r.col[s]) ? 1 : 0;
      }
      dst[rank] = Ent{r.col[s], r.lam[s]};
    }
  }
}

// kept register-path entries (at most kEll) as one fixed-width row
__device__ __forceinline__ EllRow row_regs(const RowBuf<kRowRegs>& r, int ub) {
  EllRow o;
#pragma unroll
  for (int p = 0; p < kEll; ++p) o.e[p] = Ent{-1, 0.f};
#pragma unroll
  for (int s = 0; s < kRowRegs; ++s) {
    if (s >= ub) break;
    int rank = 0;
#pragma unroll
    for (int t = 0; t < kRowRegs; ++t) {
      if (t >= ub) break;
      rank += (r.lam[t] > 0.f && r.col[t] < r.col[s]) ? 1 : 0;
    }
    const bool kept = r.lam[s] > 0.f;
#pragma unroll
    for (int p = 0; p < kEll; ++p) {
      const bool m = kept && rank == p;
      o.e[p].col = m ? r.col[s] : o.e[p].col;
      o.e[p].val = m ? r.lam[s] : o.e[p].val;
    }
  }
  return o;
}

// A slice flagged interior: when every row still holds one layer c and every
// neighbour row that same single layer, the update of each row is exact and
// trivial -- S = {c}, n = 1, every term of d_c cancels, and the normalised
// value is 1 -- so the rows are written as {c: 1} with the counters and
// change measures the full path would give (one row of interest, one entry
// in and out).  Returns false, having written nothing, when some row of the
// slice no longer qualifies; the caller then takes the full path.
__device__ __forceinline__ bool interior_slice(const StepArgs& A, const int sl,
                                               const unsigned poisoned) {
  const int lane = threadIdx.x;
  const int i = sl * kSlice + lane;
  bool ok = true;
  int32_t c = -1;
  float ph = 0.f;
  if (i < A.n_v) {
    // the first two entries of the own row and of each neighbour row
    const Ent* own = reinterpret_cast<const Ent*>(reinterpret_cast<const char*>(A.u_in) +
                                                  (uint32_t)i * (uint32_t)sizeof(EllRow));
    const Ent e0 = own[0], e1 = own[1];
    c = e0.col;
    ph = e0.val;
    ok = c >= 0 && e1.col < 0;
    const Ent* ops = A.lell + (int64_t)sl * A.op_w * kSlice + lane;
#pragma unroll
    for (int k = 0; k < kOpWidth; ++k) {
      if (k >= A.op_w) break;
      const Ent le = ops[k * kSlice];
      if (le.col >= 0) {
        const Ent* nb = reinterpret_cast<const Ent*>(reinterpret_cast<const char*>(A.u_in) +
                                                     (uint32_t)le.col * (uint32_t)sizeof(EllRow));
        ok = ok && nb[0].col == c && nb[1].col < 0;
      }
    }
    // entries beyond the slice width are not checked here
    if (A.op_w == kOpWidth && ops[(kOpWidth - 1) * kSlice].col >= 0) ok = false;
  }
  if (!__all(ok)) return false;
  if (poisoned) return true;  // as the full path: a failed chunk writes nothing
  if (sl == 0 && lane == 0) {
    *A.ovf_ctr_next = 0u;
    *A.wide_ctr_next = 0u;
  }
  int rows = 0, changed = 0;
  float dmax = 0.f;
  if (i < A.n_v) {
    EllRow o;
    o.e[0] = Ent{c, 1.0f};
#pragma unroll
    for (int p = 1; p < kEll; ++p) o.e[p] = Ent{-1, 0.f};
    *reinterpret_cast<EllRow*>(reinterpret_cast<char*>(A.u_out) +
                               (uint32_t)i * (uint32_t)sizeof(EllRow)) = o;
    rows = 1;
    if (A.measure) {
      ChangeAcc a;
      a.add(c, ph, 1.0f, A.c);
      changed = a.changed();
      dmax = a.dmax;
    }
  }
  const int n = wave_sum(rows), ch = A.measure ? wave_sum(changed) : 0;
  const float dm = A.measure ? wave_max(dmax) : 0.f;
  if (lane == 0) {
    StepStats* P = A.parts + (sl & (kParts - 1));
    atomicAdd(&P->skel, (unsigned long long)n);
    atomicAdd(&P->out, (unsigned long long)n);
    atomicAdd(&P->in, (unsigned long long)n);
    if (ch) atomicAdd(&P->changed, (unsigned long long)ch);
    if (dm > 0.f) atomicMax(&P->dmax, (unsigned long long)__float_as_uint(dm));
  }
  return true;
}

// One wavefront's slice sl of one step of the fields described by A.
// TYPED: per-pair coefficients (a separate instance, so that the scalar
// step keeps its registers).
template <bool TYPED>
__device__ __forceinline__ void step_slice(const StepArgs& A, const int sl) {
  const int lane = threadIdx.x;
  // Whether an earlier step of the chunk failed: the flag is set by atomics
  // in an earlier launch, and a scalar load sees it (caches are made
  // coherent between launches).  It is loaded here and tested after the
  // gather, which only reads, so that its latency overlaps the first loads.
  const unsigned poisoned =
      *(const __attribute__((address_space(4))) unsigned int*)&A.flags->poisoned;
  const int i = sl * kSlice + lane;
  if (A.slice_cls && A.slice_cls[sl] && interior_slice(A, sl, poisoned)) return;

  RowBuf<kRowRegs> r;
  int cnt = 0, ub = 0, n_keep = 0, n_skel = 0, n_in = 0, ev = 0, rowovf = 0, changed = 0;
  float dmax = 0.f;
  int wide = -1;  // workspace slot of a wide row
  bool deferred = false;  // a wide row left to k_wide
  // this row's operator entries: column-major in the wavefront's slice
  const Ent* ops = A.lell + (int64_t)sl * A.op_w * kSlice + lane;
  const bool in_regs = gather_regs(r, cnt, ub, n_in, i, i < A.n_v, ops, A) == kGatherOk;
  // An earlier step of the chunk failed: write nothing (no row, no overflow
  // entry, no workspace slot, no counter), so that the last good fields (the
  // input of the failed step, which this step would overwrite) survive for
  // the replay.
  if (poisoned) return;
  if (sl == 0 && lane == 0) {
    *A.ovf_ctr_next = 0u;
    *A.wide_ctr_next = 0u;
  }
  if (i < A.n_v) {
    if (in_regs) {
      row_update<kRowRegs, true, TYPED>(r, cnt, ub, A.c, n_keep, n_skel, ev);
      if (A.measure) row_change(r, ub, A.c, changed, dmax);
    } else if (A.wide_rows) {
      // stepped after this launch by k_wide, one wavefront per row
      A.wide_rows[atomicAdd(A.wide_ctr, 1u)] = i;
      deferred = true;
    } else {
      atomicOr(&A.flags->wide_seen, 1u);
      const unsigned slot = atomicAdd(A.wide_ctr, 1u);
      if (slot < (unsigned)A.wide_cap) {
        wide = (int)slot;
        n_keep = wide_row<TYPED>(i, ops, &A, A.wide + slot, &n_skel, &ev, &rowovf);
        if (rowovf) {
          step_failed(A, 2u);
          n_keep = 0;
        } else {
          if (A.measure) wide_change(A.wide + slot, A.c, changed, dmax);
        }
      } else {
        step_failed(A, 8u);  // the step is replayed with more slots
      }
    }
    // the row: inline, or in the overflow area of U_{t+1}
    Ent* row = A.u_out[i].e;
    Ent* dst = row;
    if (deferred) {
      dst = nullptr;
    } else if (n_keep > kEll) {
      const long long o = (long long)atomicAdd(A.ovf_ctr, (unsigned)n_keep);
      const bool fits = o + n_keep <= A.ovf_cap;
      if (!fits) {
        atomicMax(&A.flags->need, (unsigned long long)(o + n_keep));
        step_failed(A, 1u);  // the step is replayed with a larger area
      }
      row[0] = Ent{kOvfMark, 0.f};
      row[1] = Ent{ovf_enc(fits ? o : 0), 0.f};
      row[2] = Ent{ovf_enc(fits ? n_keep : 0), 0.f};
      dst = fits ? A.ovf_out + o : nullptr;
    } else if (wide < 0) {
      // the whole row from registers: 24-byte stores, contiguous across the
      // wavefront
      *reinterpret_cast<EllRow*>(reinterpret_cast<char*>(A.u_out) +
                                 (uint32_t)i * (uint32_t)sizeof(EllRow)) = row_regs(r, ub);
      dst = nullptr;
    } else {
      for (int p = n_keep; p < kEll; ++p) row[p] = Ent{-1, 0.f};
    }
    if (dst) {
      if (wide < 0) write_regs(r, ub, dst);
      else if (!rowovf) wide_write(A.wide + wide, dst);
    }
  }
  // counters of the slice, added into one of kParts slots; per row at most
  // 64 rows of interest and kept entries, so a wavefront's sums fit 16 bits
  // and travel packed; the totals are complete in the last lane
  const unsigned so = dpp_sum63((unsigned)n_skel | ((unsigned)n_keep << 16)),
                 in = dpp_sum63((unsigned)n_in),
                 ec = dpp_sum63((unsigned)ev | ((unsigned)changed << 16));
  const float dm = A.measure ? __uint_as_float(dpp_max63(__float_as_uint(dmax))) : 0.f;
  if (lane == kSlice - 1) {
    StepStats* P = A.parts + (sl & (kParts - 1));
    atomicAdd(&P->skel, (unsigned long long)(so & 0xffff));
    atomicAdd(&P->out, (unsigned long long)(so >> 16));
    atomicAdd(&P->in, (unsigned long long)in);
    if (ec & 0xffff) atomicAdd(&P->events, (unsigned long long)(ec & 0xffff));
    if (ec >> 16) atomicAdd(&P->changed, (unsigned long long)(ec >> 16));
    if (dm > 0.f) atomicMax(&P->dmax, (unsigned long long)__float_as_uint(dm));
  }
}

// XCD-aware block order: workgroups are dealt to the 8 XCDs round-robin, so
// XCD x runs blocks x, x + 8, ...; giving it the contiguous slices
// [x * per, (x+1) * per) of n keeps neighbouring rows (close in the step's
// vertex order) in one L2
__device__ __forceinline__ int xcd_slice(int n) {
  const int per = (n + kXcds - 1) / kXcds;
  return (int)(blockIdx.x % kXcds) * per + (int)(blockIdx.x / kXcds);
}

// Scalar registers bound the step kernel's residency on gfx950: with the 104
// the compiler would use, six wavefronts per SIMD are resident (6,144 on
// 1,024 SIMDs, measured with per-wavefront clock stamps), with 78 eight;
// capped at 88, seven (the vector registers, at most 72, allow seven).  The
// cap costs a few scalar values kept in vector-register lanes instead.
#define LF_STEP_REGS __attribute__((amdgpu_waves_per_eu(4), amdgpu_num_sgpr(88)))

template <bool TYPED>
__global__ __launch_bounds__(kSlice) LF_STEP_REGS void k_step(StepArgs A) {
  const int sl = xcd_slice(A.n_slices);
  if (sl >= A.n_slices) return;
  step_slice<TYPED>(A, sl);
}

// p as a pointer into the global address space (from its integer value, so
// that the compiler does not fold the conversion away)
template <class T>
__device__ __forceinline__ T* to_global(T* p) {
  return (T*)(__attribute__((address_space(1))) T*)(uintptr_t)p;
}

// One step of several independent field objects in one launch: their slices
// follow one another (job j owns slices [first[j], first[j+1]) of the
// launch, first[n_jobs] = total), each with its own arguments G[j]; the XCD
// order runs over the whole launch.
template <bool TYPED>
__global__ __launch_bounds__(kSlice) LF_STEP_REGS void k_step_group(
    const StepArgs* __restrict__ G, const int32_t* __restrict__ first, int32_t n_jobs) {
  const int total = first[n_jobs];
  const int g = xcd_slice(total);
  if (g >= total) return;
  int lo = 0, hi = n_jobs - 1;  // the last job whose first slice is <= g
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  // the job's arguments, every pointer rebuilt in the global address space
  // (pointers read from memory are generic to the compiler, which would then
  // use flat accesses, and a flat access also waits on the LDS counter)
  StepArgs a = G[lo];
  a.lell = to_global(a.lell);
  a.lptr = to_global(a.lptr);
  a.lent = to_global(a.lent);
  a.ldiag = to_global(a.ldiag);
  a.u_in = to_global(a.u_in);
  a.u_out = to_global(a.u_out);
  a.ovf_in = to_global(a.ovf_in);
  a.ovf_out = to_global(a.ovf_out);
  a.ovf_ctr = to_global(a.ovf_ctr);
  a.ovf_ctr_next = to_global(a.ovf_ctr_next);
  a.c.types = to_global(a.c.types);
  a.c.tab = to_global(a.c.tab);
  a.wide = to_global(a.wide);
  a.wide_ctr = to_global(a.wide_ctr);
  a.wide_ctr_next = to_global(a.wide_ctr_next);
  a.flags = to_global(a.flags);
  a.parts = to_global(a.parts);
  a.slice_cls = to_global(a.slice_cls);
  a.wide_rows = to_global(a.wide_rows);
  step_slice<TYPED>(a, g - first[lo]);
}

// The rows a k_step launch left to it (wide_rows[0 .. *wide_ctr)), each
// stepped by one wavefront; their counters join the step's partial slots.
// Nothing is done when an earlier step of the chunk failed.
template <bool TYPED>
__global__ __launch_bounds__(kSlice) void k_wide(StepArgs A) {
  if (*(const __attribute__((address_space(4))) unsigned int*)&A.flags->poisoned) return;
  const unsigned n = *A.wide_ctr;
  for (unsigned q = blockIdx.x; q < n; q += gridDim.x) {
    const WideResult o = wide_row_wave<TYPED>(A, A.wide_rows[q]);
    if (threadIdx.x == 0) {
      StepStats* P = A.parts + (q & (kParts - 1));
      atomicAdd(&P->skel, (unsigned long long)o.n_skel);
      atomicAdd(&P->out, (unsigned long long)o.n_keep);
      if (o.ev) atomicAdd(&P->events, (unsigned long long)o.ev);
      if (o.changed) atomicAdd(&P->changed, (unsigned long long)o.changed);
      if (o.dmax > 0.f) atomicMax(&P->dmax, (unsigned long long)__float_as_uint(o.dmax));
    }
  }
}

__global__ void k_reset_flags(StepFlags* f, StepStats* parts, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0) {
    f->poisoned = 0;
    f->fail_step = 0xffffffffu;
    f->need = 0;
    f->wide_seen = 0;
  }
  if (parts && k < n) parts[k] = StepStats{0, 0, 0, 0, 0, 0};
}

// one block per step: sums the kParts partial counters (maximum for dmax)
__global__ __launch_bounds__(kParts) void k_reduce_parts(const StepStats* parts,
                                                         StepStats* out) {
  constexpr int kF = 6;
  __shared__ unsigned long long sh[kF][kParts / 64];
  const StepStats p = parts[(int64_t)blockIdx.x * kParts + threadIdx.x];
  unsigned long long v[kF] = {p.skel, p.out, p.in, p.events, p.changed, p.dmax};
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kF; ++q) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const unsigned long long y = __shfl_xor(v[q], o, 64);
      v[q] = q == kF - 1 ? (y > v[q] ? y : v[q]) : v[q] + y;
    }
    if (lane == 0) sh[q][wid] = v[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t[kF] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < kF; ++q)
#pragma unroll
      for (int w = 0; w < kParts / 64; ++w)
        t[q] = q == kF - 1 ? (sh[q][w] > t[q] ? sh[q][w] : t[q]) : t[q] + sh[q][w];
    out[blockIdx.x] = StepStats{t[0], t[1], t[2], t[3], t[4], t[5]};
  }
}

}  // namespace

hipError_t launch_step(const StepArgs& a, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
  const dim3 grid((unsigned)(kXcds * ((a.n_slices + kXcds - 1) / kXcds)));
  if (a.wide_rows) {  // the step kernel, then its wide rows (timed together)
    hipError_t e = (t0 && t1) ? hipEventRecord(t0, s) : hipSuccess;
    if (e != hipSuccess) return e;
    if (a.c.n_types > 0) hipLaunchKernelGGL(k_step<true>, grid, dim3(kSlice), 0, s, a);
    else hipLaunchKernelGGL(k_step<false>, grid, dim3(kSlice), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const dim3 wgrid((unsigned)(a.n_v < kWideBlocks ? a.n_v : kWideBlocks));
    if (a.c.n_types > 0) hipLaunchKernelGGL(k_wide<true>, wgrid, dim3(kSlice), 0, s, a);
    else hipLaunchKernelGGL(k_wide<false>, wgrid, dim3(kSlice), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return (t0 && t1) ? hipEventRecord(t1, s) : hipSuccess;
  }
  if (t0 && t1) {
    if (a.c.n_types > 0) hipExtLaunchKernelGGL(k_step<true>, grid, dim3(kSlice), 0, s, t0, t1, 0, a);
    else hipExtLaunchKernelGGL(k_step<false>, grid, dim3(kSlice), 0, s, t0, t1, 0, a);
  } else {
    if (a.c.n_types > 0) hipLaunchKernelGGL(k_step<true>, grid, dim3(kSlice), 0, s, a);
    else hipLaunchKernelGGL(k_step<false>, grid, dim3(kSlice), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_step_group(const StepArgs* G, const int32_t* first, int32_t n_jobs,
                             int32_t total_slices, bool typed, hipStream_t s) {
  if (n_jobs <= 0 || total_slices <= 0) return hipSuccess;
  const dim3 grid((unsigned)(kXcds * ((total_slices + kXcds - 1) / kXcds)));
  if (typed) hipLaunchKernelGGL(k_step_group<true>, grid, dim3(kSlice), 0, s, G, first, n_jobs);
  else hipLaunchKernelGGL(k_step_group<false>, grid, dim3(kSlice), 0, s, G, first, n_jobs);
  return hipGetLastError();
}

hipError_t launch_reset_flags(StepFlags* f, StepStats* parts, int64_t n, hipStream_t s) {
  const int64_t m = parts ? n * kParts : 0;
  const unsigned nb = m > 0 ? (unsigned)((m + 255) / 256) : 1u;
  hipLaunchKernelGGL(k_reset_flags, dim3(nb), dim3(256), 0, s, f, parts, m);
  return hipGetLastError();
}

hipError_t launch_reduce_parts(const StepStats* parts, int64_t n, StepStats* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_parts, dim3((unsigned)n), dim3(kParts), 0, s, parts, out);
  return hipGetLastError();
}

}  // namespace lf
