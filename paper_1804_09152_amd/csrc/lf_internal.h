// Internal declarations of the gfx950 layered-field library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "lf.h"

namespace lf {

// One stored entry of a sparse row: column id and value, one 8-byte load.
struct __attribute__((aligned(8))) Ent {
  int32_t col;
  float val;
};

constexpr int kBlock = 256;      // rows per tile of the step kernel
constexpr int kRowRegs = 8;      // layers per row held in registers
constexpr int kRowWide = 64;     // row limit of the wide (spill) path
constexpr int kMaxVerts = 1 << 25;

// Device-side step status.  Written by the step kernels, read by the host
// once per lf_step call.
struct StepFlags {
  unsigned int poisoned;   // bit 0 capacity, bit 1 row limit, bit 2 look-back timeout,
                           // bit 3 wide-row workspace exhausted
  unsigned int fail_step;  // index (within the call) of the first failed step
  unsigned long long need; // entries needed by a step that overflowed
};

// Per-step counters, written for step k of an lf_step call at stats[k]: the
// host adds up those of the steps that completed.
struct StepStats {
  unsigned long long skel;    // sum of |rows of interest|
  unsigned long long out;     // nnz(U_{t+1})
  unsigned long long in;      // nnz(U_t)
  unsigned long long events;  // columns whose normalisation sum was zero
};

struct StepConsts {
  float a, w, e, mu, dt, theta;
  int32_t base_mode;
  int32_t n_s;
};

// Workspace of one row touching more than kRowRegs layers (global memory, so
// that the step kernel itself needs no private memory).
struct WideRow {
  int32_t col[kRowWide];
  float phi[kRowWide];
  float lam[kRowWide];
  float out[kRowWide];
  int32_t cnt, n_keep, pad0, pad1;
};

struct StepArgs {
  const int32_t* lptr;  // off-diagonal operator rows
  const Ent* lent;
  const float* ldiag;
  const int32_t* uptr_in;
  const Ent* uent_in;
  int32_t* uptr_out;
  Ent* uent_out;
  int32_t n_v;
  int32_t n_tiles;
  long long cap;
  StepConsts c;
  unsigned long long* status;       // tile status of this step
  unsigned long long* status_next;  // cleared here for the next step
  unsigned int* ticket;
  unsigned int* ticket_next;
  WideRow* wide;                   // workspace slots for wide rows
  int32_t wide_cap;
  int32_t pad_;
  unsigned int* wide_ctr;          // slots taken in this step
  unsigned int* wide_ctr_next;     // cleared here for the next step
  StepFlags* flags;
  StepStats* stats;                // this step's counters
  uint32_t step_idx;               // index of this step within the call
  uint32_t pad2_;
};

// error handling -----------------------------------------------------------
void set_error(const std::string& msg);
lf_status hip_fail(hipError_t e, const char* what);
#define LF_HIP(call)                                       \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return lf::hip_fail(e_, #call);  \
  } while (0)

// launchers (each defined next to its kernels) ------------------------------
hipError_t launch_step(const StepArgs& a, hipStream_t s, hipEvent_t t0, hipEvent_t t1);
// clears the failure flags and the first n per-step counters
hipError_t launch_reset_flags(StepFlags* f, StepStats* st, int n, hipStream_t s);
hipError_t launch_init_fields(const int32_t* owner, int32_t n_v, int32_t* uptr, Ent* uent,
                              hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s);
hipError_t launch_scatter_owner(const int32_t* seeds, int32_t n_s, int32_t* owner, hipStream_t s);

// exclusive scan of n int32 counts into out[0..n] (out[n] = total); tmp must
// hold scan_tmp_elems(n) int64
int64_t scan_tmp_elems(int64_t n);
hipError_t exclusive_scan(const int32_t* in, int32_t* out, int64_t n, long long* tmp,
                          hipStream_t s);

// operator build (a1)
hipError_t build_operator(const double* V, const int32_t* F, int32_t n_v, int32_t n_f, int op,
                          int32_t** lptr, Ent** lent, float** ldiag, int64_t* nnz_off,
                          int* bad_face, hipStream_t s);

hipError_t launch_split(const Ent* e, int64_t n, int32_t* col, float* val, hipStream_t s);
hipError_t launch_join_check(const int32_t* col, const float* val, const int32_t* ptr,
                             int32_t n_v, int32_t n_r, int64_t nnz, Ent* out, int32_t* bad,
                             hipStream_t s);
hipError_t launch_operator_export(const int32_t* lptr, const Ent* lent, const float* ldiag,
                                  int32_t n_v, int32_t* rowptr, int32_t* col, float* val,
                                  hipStream_t s);
hipError_t launch_labels(const int32_t* uptr, const Ent* uent, int32_t n_v, int32_t n_s,
                         int32_t* labels, hipStream_t s);

// releases the dual-mesh state of a field object
void dual_release(lf_fields* f);

// asynchronous stepping: issue n steps; poll; book them (remaining > 0 when
// storage had to grow and those steps must be issued again)
lf_status step_issue(lf_fields* f, int64_t n);
bool step_ready(lf_fields* f);
lf_status step_complete(lf_fields* f, int64_t* remaining);

// device allocation helpers
template <class T>
hipError_t dalloc(T** p, int64_t n) {
  *p = nullptr;
  if (n <= 0) n = 1;
  return hipMalloc((void**)p, (size_t)n * sizeof(T));
}

}  // namespace lf

struct lf_ctx {
  int32_t device;
  hipStream_t stream;
  bool own_stream;
};

struct lf_mesh {
  lf_ctx* ctx;
  int32_t n_v, n_f, op;
  double* V;        // device float64 positions
  int32_t* F;       // device triangles
  int32_t* lptr;    // off-diagonal operator, CSR
  lf::Ent* lent;
  float* ldiag;     // diagonal of the operator
  int64_t nnz_off;
  std::vector<double> Vh;  // host copies for small host-side geometry needs
  std::vector<int32_t> Fh;
};

struct DualState;  // defined with the dual-mesh kernels

struct lf_fields {
  lf_mesh* mesh;
  int32_t n_s;
  lf_params P;
  std::vector<int32_t> seeds;
  int32_t* d_seeds;
  int32_t* owner;              // scratch n_v
  int32_t* uptr[2];
  lf::Ent* uent[2];
  int64_t cap;
  int cur;
  unsigned long long* status[2];
  unsigned int* tickets;       // 4 counters: tile tickets and wide-row slots, per parity
  lf::WideRow* wide;
  int32_t wide_cap;
  lf::StepFlags* flags;
  lf::StepFlags* flags_host;   // pinned
  lf::StepStats* stats;        // per-step counters of one call
  int64_t stats_cap;
  lf::StepStats* stats_pinned; // their host copy
  int64_t stats_pinned_cap;
  int64_t pending;             // steps issued and not yet booked
  hipEvent_t done_ev;          // recorded after the copies of an issued chunk
  size_t ev_issued;            // timing events used by the issued chunk
  int32_t n_tiles;
  // totals over completed steps
  long long steps, grow_events;
  unsigned long long skel_total, out_total, in_total, events_total;
  // timing
  bool timing;
  std::vector<hipEvent_t> ev0, ev1;
  size_t ev_used;
  double timed_ms;
  long long timed_launches;
  DualState* dual;
};
