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

constexpr int kSlice = 64;      // rows per operator slice = one wavefront of the step kernel
constexpr int kEll = 3;         // field entries per row held inline
constexpr int kRowRegs = 8;     // layers per row held in registers
constexpr int kRowWide = 64;    // row limit of the wide (spill) path
constexpr int kMaxVerts = 1 << 25;
constexpr int kParts = 256;     // partial-sum slots of the per-step counters
constexpr int32_t kOvfMark = -2;  // first column of a row kept in the overflow area
constexpr int64_t kMaxChunk = 256;  // steps lf_step issues before it books them
constexpr int kTileRows = 4096;     // rows per re-ordering tile (64 slices)

// One row of the fields in fixed-width form: up to kEll entries, ascending
// layers, unused slots {-1, 0}.  A row with more entries keeps them in the
// overflow area: e[0] = {kOvfMark, 0}, e[1].col = ~offset, e[2].col = ~count
// (bit-inverted, so negative: no column of a header reads as a layer), values
// 0.  The field buffers hold one row more than the mesh has vertices: row n_v
// is an empty row, never written, that stands in for missing neighbours.
struct __attribute__((aligned(8))) EllRow {
  Ent e[kEll];
};
__host__ __device__ inline int32_t ovf_enc(int64_t v) { return ~(int32_t)v; }
__host__ __device__ inline int64_t ovf_dec(int32_t c) { return (int64_t)~c; }

// The operator's off-diagonal entries for the step, in slices of kSlice
// rows stored column-major with one width w for all slices: entry k < w of
// row i at ((i / kSlice) * w + k) * kSlice + i % kSlice, shorter rows padded
// with {-1, 0}.  w = min(largest row, kOpWidth); a longer row keeps its
// entries from w on in the CSR copy (lptr / lent), in the same order.
constexpr int kOpWidth = 8;

// Device-side step status.  Written by the step kernels, read by the host
// once per issued chunk of steps.
struct StepFlags {
  unsigned int poisoned;   // bit 0 overflow area full, bit 1 row limit, bit 2 unused,
                           // bit 3 wide-row workspace exhausted
  unsigned int fail_step;  // index (within the chunk) of the first failed step
  unsigned long long need; // overflow entries needed by a step that ran out
  unsigned int wide_seen;  // a row touching more than kRowRegs layers was stepped inline
  unsigned int pad_;
};

// Per-step counters: each step adds its partial sums into kParts slots
// (spread to keep atomics on one address few); a reduction kernel folds them
// into one StepStats per step, and the host adds those of completed steps.
struct StepStats {
  unsigned long long skel;     // sum of |rows of interest|
  unsigned long long out;      // nnz(U_{t+1})
  unsigned long long in;       // nnz(U_t)
  unsigned long long events;   // columns whose normalisation sum was zero
  unsigned long long changed;  // rows whose label or set of layers >= tau changed
  unsigned long long dmax;     // max |U_{t+1} - U_t| (float bits; non-negative, so the
                               // integer maximum is the float maximum)
};

struct StepConsts {
  float a, w, e, mu, dt, theta;
  int32_t base_mode;
  int32_t n_s;
  float tau;  // threshold of the rows' tau pattern (convergence measure)
  // per-pair coefficients (0: the scalars a, w, e): type of every layer and
  // {a, w, e, 0} of every pair of types, row-major
  int32_t n_types;
  const int32_t* types;
  const float4* tab;
};

// Workspace of one row touching more than kRowRegs layers, or reading a row
// kept in the overflow area (global memory, so that the step kernel itself
// needs no private memory).
struct WideRow {
  int32_t col[kRowWide];
  float phi[kRowWide];
  float lam[kRowWide];
  float out[kRowWide];
  int32_t cnt, n_keep, pad0, pad1;
};

struct StepArgs {
  const Ent* lell;                 // operator slices (see kOpWidth)
  const int32_t* lptr;             // operator CSR rows (entries beyond the slices)
  const Ent* lent;
  const float* ldiag;              // operator diagonal
  const EllRow* u_in;              // fields U_t
  EllRow* u_out;                   // fields U_{t+1}
  const Ent* ovf_in;               // overflow area of U_t
  Ent* ovf_out;                    // overflow area of U_{t+1}
  long long ovf_cap;               // entries of either overflow area
  unsigned int* ovf_ctr;           // overflow entries taken in this step
  unsigned int* ovf_ctr_next;      // cleared here for the next step
  int32_t n_v;
  int32_t n_slices;
  int32_t op_w;                    // slice width w
  int32_t pad0_;
  StepConsts c;
  WideRow* wide;                   // workspace slots for wide rows
  int32_t wide_cap;
  int32_t pad_;
  unsigned int* wide_ctr;          // slots taken in this step
  unsigned int* wide_ctr_next;     // cleared here for the next step
  StepFlags* flags;
  StepStats* parts;                // kParts partial sums of this step
  uint32_t step_idx;               // index of this step within the chunk
  uint32_t measure;                // compute the convergence measures of this step
  // per slice: 1 when every row of the slice was an interior row (one layer,
  // and every neighbour the same single layer) at the last re-ordering; such
  // slices check that it still holds and then skip the merge and update
  // (nullptr: no slice is tried)
  const uint8_t* slice_cls;
  // rows touching more than kRowRegs layers: nullptr, each stepped by its
  // own lane with a workspace slot; else (capacity n_v) their list, stepped
  // after the launch by k_wide, one wavefront per row (wide_ctr counts it)
  int32_t* wide_rows;
};

// error handling -----------------------------------------------------------
void set_error(const std::string& msg);
lf_status hip_fail(hipError_t e, const char* what);
// a host allocation failed inside an entry point: LF_ENOMEM, nothing thrown
// across the C ABI
lf_status host_oom();
#define LF_HIP(call)                                       \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return lf::hip_fail(e_, #call);  \
  } while (0)

// launchers (each defined next to its kernels) ------------------------------
hipError_t launch_step(const StepArgs& a, hipStream_t s, hipEvent_t t0, hipEvent_t t1);
// one step of n_jobs field objects in one launch: device arrays G[n_jobs] of
// their arguments and first[n_jobs + 1] of their first slices in the launch
// (first[n_jobs] = total_slices); all scalar (typed = false) or all with
// per-pair coefficients (typed = true)
hipError_t launch_step_group(const StepArgs* G, const int32_t* first, int32_t n_jobs,
                             int32_t total_slices, bool typed, hipStream_t s);
// clears the failure flags and n steps' partial counters (n * kParts slots)
hipError_t launch_reset_flags(StepFlags* f, StepStats* parts, int64_t n, hipStream_t s);
// folds the partial counters of n steps into one StepStats per step
hipError_t launch_reduce_parts(const StepStats* parts, int64_t n, StepStats* out, hipStream_t s);
hipError_t launch_init_fields(const int32_t* owner, const int32_t* perm, int32_t n_v, EllRow* u,
                              hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s);
hipError_t launch_scatter_owner(const int32_t* seeds, int32_t n_s, int32_t* owner, hipStream_t s);
// one ring of seed regions over the operator's off-diagonal pattern (caller's
// vertex order)
hipError_t launch_ring_grow(const int32_t* lptr, const Ent* lent, const int32_t* own_in,
                            int32_t* own_out, int32_t n_v, int32_t n_s, hipStream_t s);

// exclusive scan of n int32 counts into out[0..n] (out[n] = total); tmp must
// hold scan_tmp_elems(n) int64
int64_t scan_tmp_elems(int64_t n);
hipError_t exclusive_scan(const int32_t* in, int32_t* out, int64_t n, long long* tmp,
                          hipStream_t s);

// operator build (a1)
hipError_t build_operator(const double* V, const int32_t* F, int32_t n_v, int32_t n_f, int op,
                          int32_t** lptr, Ent** lent, float** ldiag, int64_t* nnz_off,
                          int* bad_face, hipStream_t s);

// operator CSR (off-diagonal) -> slices of one width (kOpWidth at most)
hipError_t build_slices(const int32_t* lptr, const Ent* lent, int32_t n_v, Ent** lell,
                        int32_t* width, hipStream_t s);
// The step works in its own vertex order (a locality-preserving order chosen
// at mesh creation): fields row k and step-operator row k belong to vertex
// perm[k]; vertex v is row inv[v].  Everything at the boundary (CSR view,
// import, seeds, labels) is in the caller's order.
// fields: fixed-width rows (+ overflow area) -> CSR in the caller's order
// (uptr must hold n_v + 1, uent the entry count); counts int32 n_v
// scratch, tmp scan_tmp_elems(n_v)
hipError_t ell_to_csr_ptr(const EllRow* u, const int32_t* inv, int32_t n_v, int32_t* counts,
                          int32_t* uptr, long long* tmp, hipStream_t s);
hipError_t ell_to_csr_fill(const EllRow* u, const Ent* ovf, const int32_t* inv, int32_t n_v,
                           const int32_t* uptr, Ent* uent, hipStream_t s);
// canonical CSR (caller's order) -> fixed-width rows; rows longer than kEll
// keep their entries at their CSR offsets in ovf (which holds at least nnz
// entries)
hipError_t csr_to_ell(const int32_t* uptr, const Ent* uent, const int32_t* inv, int32_t n_v,
                      EllRow* u, Ent* ovf, hipStream_t s);
// sorts keys[0..n) ascending in place (bitonic network; keys has room for
// the next power of two of n, padded with ~0)
hipError_t sort_keys_u64(unsigned long long* keys, int64_t n, hipStream_t s);
// The step's vertex order: within each part [part_off[p], part_off[p+1])
// (host array), vertices sorted along a Morton curve of their positions in
// the part's bounding box (host box[6 p .. 6 p + 5]: lo xyz, hi xyz), ties by
// vertex id.  V is the device copy of the positions; perm (row -> vertex)
// and inv (vertex -> row) are device arrays of n_v.
hipError_t locality_order(const double* V, int32_t n_v, const int32_t* part_off, int32_t n_parts,
                          const double* box, int32_t* perm, int32_t* inv, hipStream_t s);
// the operator in the step's order (rows permuted, columns renumbered,
// entries of a row in their original order)
hipError_t permute_operator(const int32_t* lptr, const Ent* lent, const float* ldiag,
                            const int32_t* perm, const int32_t* inv, int32_t n_v, int64_t nnz,
                            int32_t** plptr, Ent** plent, float** pldiag, hipStream_t s);

hipError_t launch_split(const Ent* e, int64_t n, int32_t* col, float* val, hipStream_t s);
hipError_t launch_join_check(const int32_t* col, const float* val, const int32_t* ptr,
                             int32_t n_v, int32_t n_r, int64_t nnz, Ent* out, int32_t* bad,
                             hipStream_t s);
hipError_t launch_operator_export(const int32_t* lptr, const Ent* lent, const float* ldiag,
                                  int32_t n_v, int32_t* rowptr, int32_t* col, float* val,
                                  hipStream_t s);
hipError_t launch_labels(const int32_t* uptr, const Ent* uent, int32_t n_v, int32_t n_s,
                         int32_t* labels, hipStream_t s);

// lf_mesh_create with the vertex order of the step chosen per part: the
// vertices of part p are [part_off[p], part_off[p+1]) (a batch keeps each
// mesh's rows together)
lf_status mesh_create(lf_ctx* ctx, const double* V, int32_t n_v, const int32_t* F, int32_t n_f,
                      int32_t op, const int32_t* part_off, int32_t n_parts, lf_mesh** out);

// releases the dual-mesh state of a field object
void dual_release(lf_fields* f);

// CSR view of the current fields (rebuilt after steps); valid until the
// next step, reset or import
lf_status fields_csr(lf_fields* f, const int32_t** uptr, const Ent** uent);

// asynchronous stepping: issue n steps; poll; book them (remaining > 0 when
// storage had to grow and those steps must be issued again).  Steps issued
// after a failed one still run (on well-formed data) and are discarded, so
// callers keep n modest.
lf_status step_issue(lf_fields* f, int64_t n);
bool step_ready(lf_fields* f);
lf_status step_complete(lf_fields* f, int64_t* remaining);
// completes what lf_step_async left in flight or to run (books the issued
// chunk, steps again what had to be replayed, runs the rest); every entry
// point that reads or changes the fields calls it first
lf_status fields_settle(lf_fields* f);
#define LF_SETTLE(f)                               \
  do {                                             \
    lf_status s_ = lf::fields_settle(f);           \
    if (s_ != LF_OK) return s_;                    \
  } while (0)
// whether all of the first n steps booked by the last step_complete were
// quiet: no row changed its label or its layers at or above tau, and no
// value moved by more than eps
bool chunk_quiet(const lf_fields* f, int64_t n, double eps);
// device bytes a mesh / a field object holds (their allocations, as sized now)
int64_t mesh_bytes(const lf_mesh* m);
int64_t fields_bytes(const lf_fields* f);
// per-step counters, their host copies and the chunk event for chunks of up
// to n steps
lf_status ensure_step_buffers(lf_fields* f, int64_t n);
// arguments of step k of a chunk of n steps starting at the current buffer
StepArgs chunk_step_args(lf_fields* f, int64_t k, int64_t n);
// after a chunk of n steps: fold the counters and copy them and the flags to
// the host (stream s)
lf_status chunk_tail(lf_fields* f, int64_t n, hipStream_t s);
// books a completed chunk of n steps from the host copies (see step_complete)
lf_status step_book(lf_fields* f, int64_t n, int64_t* remaining);
// releases the captured chunk graphs of a field object
void drop_graphs(lf_fields* f);
// re-orders the step's rows: within tiles of kTileRows rows, interior rows
// first; the fields, the operator copy and the order maps are permuted
lf_status fields_reorder(lf_fields* f);
// the fields' order arrays back to the mesh's (frees owned ones)
void fields_order_reset(lf_fields* f);
// step arguments over the fields' own buffers for a step that reads the
// buffer of the given parity (the caller sets parts, step_idx and measure)
StepArgs step_args(lf_fields* f, int parity);
// books the first ok of the per-step counters st[]: totals, current buffer,
// entry count and change measures of the last booked step
void book_steps(lf_fields* f, const StepStats* st, int64_t ok);

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
  int32_t* lptr;    // off-diagonal operator, CSR, caller's vertex order
  lf::Ent* lent;
  float* ldiag;     // diagonal of the operator
  int64_t nnz_off;
  int32_t* perm;    // step order: row k is vertex perm[k]
  int32_t* inv;     // vertex v is row inv[v]
  int32_t* slptr;   // the operator in the step's order
  lf::Ent* slent;
  float* sldiag;
  lf::Ent* lell;    // the same off-diagonal entries in slices of kSlice rows
  int32_t op_w;     // their width
  int32_t n_slices;
  // largest face area and largest |coordinate| (the Lloyd sums' fixed-point
  // scale); measured on the first re-seeding, < 0 before
  double amax = -1.0, xmax = -1.0;
};

struct DualState;  // defined with the dual-mesh kernels

struct lf_fields {
  lf_mesh* mesh;
  int32_t n_s;
  lf_params P;
  std::vector<int32_t> seeds;
  std::vector<int32_t> region_owner;  // initial regions: owner of every vertex (empty: seeds)
  int32_t rings = 0;           // seeds grown by this many rings at (re-)initialisation
  // the step's row order: the mesh's (locality order) until the first
  // re-ordering, then the fields' own (owned = true): within tiles of
  // kTileRows rows, the interior rows first (see StepArgs::slice_cls)
  const int32_t* perm = nullptr;  // row k is vertex perm[k]
  const int32_t* inv = nullptr;   // vertex v is row inv[v]
  const lf::Ent* lell = nullptr;  // operator slices, CSR and diagonal in this order
  const int32_t* slptr = nullptr;
  const lf::Ent* slent = nullptr;
  const float* sldiag = nullptr;
  int32_t op_w = 0;
  uint8_t* slice_cls = nullptr;   // owned (nullptr before the first re-ordering)
  bool own_order = false;
  int32_t reorder_every = 0;      // steps between re-orderings (0: never)
  int32_t reorder_tile = lf::kTileRows;  // rows per tile (a multiple of 256, at most kTileRows)
  int32_t reorder_classes = 4;    // work classes the tiles are sorted into (2..4)
  int64_t next_reorder = 128;     // step count at which the next one happens
  int64_t reorders = 0;
  // list of the rows touching more than kRowRegs layers in a step (n_v
  // entries; allocated once a step has met one: from then on such rows are
  // stepped by k_wide after each step launch)
  int32_t* wide_rows = nullptr;
  int32_t* d_seeds;
  int32_t* owner;              // scratch n_v
  lf::EllRow* ell[2];          // fields, double-buffered
  lf::Ent* ovf[2];             // their overflow areas
  int64_t ovf_cap;
  int cur;
  int64_t nnz;                 // entries of the current fields
  unsigned int* counters;      // 4: overflow and wide-row counters, per parity
  lf::WideRow* wide;
  int32_t wide_cap;
  lf::StepFlags* flags;
  lf::StepFlags* flags_host;   // pinned
  lf::StepStats* parts;        // kParts partial counters per step of a chunk
  lf::StepStats* stats;        // folded per-step counters of a chunk
  int64_t stats_cap;           // steps either holds
  lf::StepStats* stats_pinned; // host copy of stats
  int64_t stats_pinned_cap;
  int64_t pending;             // steps issued and not yet booked
  int64_t async_left = 0;      // steps of lf_step_async not issued yet (run when settled)
  hipEvent_t done_ev;          // recorded after the copies of an issued chunk
  size_t ev_issued;            // timing events used by the issued chunk
  // CSR view of the current fields, for export and post-processing
  int32_t* uptr;
  lf::Ent* uent;
  int64_t csr_cap;
  bool csr_valid;
  long long* scan_tmp;         // scan_tmp_elems(n_v)
  // totals over completed steps
  long long steps, grow_events;
  unsigned long long skel_total, out_total, in_total, events_total;
  unsigned long long last_changed;  // change made by the last completed step
  float last_dmax;
  bool measure_all;  // convergence measures on every step (else on the last of a chunk)
  // per-pair coefficients (n_types 0: the scalar constants)
  int32_t n_types;
  int32_t* types;    // n_s + 1
  float4* coef;      // n_types * n_types
  // chunks of kMaxChunk steps replayed from a captured graph (kernels only),
  // one per starting buffer; rebuilt when a buffer they name changes
  bool use_graphs = false;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  uint64_t graph_key[2] = {0, 0};
  // timing
  int32_t timing;             // time every timing-th step launch (0: off)
  int64_t timing_ctr;         // step launches issued while timing
  std::vector<hipEvent_t> ev0, ev1;
  double timed_ms;
  long long timed_launches;
  DualState* dual;
};
