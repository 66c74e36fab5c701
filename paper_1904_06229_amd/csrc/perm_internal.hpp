// Host-side interface between the C-ABI runtime (perm_host.cpp) and the
// kernel sources.  Plain structs and launch functions; no torch types.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace perm {

constexpr int kWave = 64;
constexpr int kBlock = 256;  // 4 waves per workgroup, one per SIMD
constexpr int kWavesPerBlock = kBlock / kWave;

constexpr int kMaxN = 64;
constexpr int kMaxBatchedN = 32;

// Status codes written by the staging kernels (same values as perm_status).
constexpr int32_t kStOk = 0;
constexpr int32_t kStInval = 1;
constexpr int32_t kStRange = 2;
constexpr int32_t kStNonFinite = 3;

// One walk launch: chunks [first, first + nchunks) of length 2^b, i.e.
// Gray indices [first * 2^b, (first + nchunks) * 2^b).  b = 0 walks single
// terms (used for unaligned range ends).
struct WalkArgs {
  const double* staged;   // +A then -A, column-major, ld = n (complex: pairs)
  const double* rowabs;   // n values 1/2 sum_j |a_ij| (drift normalisation)
  const int32_t* status;  // staging status; nonzero -> the walk does nothing
  uint64_t first;
  uint64_t nchunks;
  uint64_t ntasks;        // wave tasks: 2 * ceil(nchunks / 128)
  int32_t b;
  int32_t drift;          // 1: compute the chunk-end drift
  void* partials;         // per workgroup: dd (2 doubles), complex dd (4), or u128 (2 words)
  double* drift_part;     // per workgroup
};

// Result record written by the finishing kernel, copied to the host.
struct DevResult {
  double v[4];        // re hi, re lo, im hi, im lo (raw sum S, before 2(-1)^n and unscaling)
  uint64_t iw[2];     // 0/1 path: sum_g (-1)^(g+1) prod r_i modulo 2^128
  double drift;       // max drift (or -1)
  int32_t status;
  int32_t exp_sum;    // sum of row-scaling exponents
  double bound;       // 0/1 path: log2 accumulator bound
  int32_t variant;    // 0/1 path: 1 if the pair-shared walk ran
  int32_t ones0;      // 0/1 path: ones in the staged column 0
  uint64_t ticks;     // one-launch path: wall-clock ticks from the first workgroup's
                      // start to the result (0 elsewhere)
  uint32_t done;      // one-launch path: set to 1 after every other field is written
  uint32_t pad;
};

enum Kind { kReal = 0, kComplex = 1, kInt01 = 2 };

// Device buffers of one single-matrix call (stage, walks, finish), carved out
// of one block of device memory; see carve_call_buffers for the layout.
struct CallBuffers {
  int32_t* status = nullptr;   // staging status words
  int32_t* rowexp = nullptr;   // row-scaling exponents (kMaxN)
  double* bound = nullptr;     // 0/1 path: log2 accumulator bound
  DevResult* dres = nullptr;   // device result record
  double* rowabs = nullptr;    // kMaxN row norms (drift normalisation)
  double* staged = nullptr;    // +A then -A: 4 kMaxN^2 doubles (complex)
  void* partials = nullptr;    // max_parts slots of 32 bytes
  double* drift = nullptr;     // max_parts doubles
  int max_parts = 0;
  DevResult* hres = nullptr;      // pinned host record, or null: the record is copied back
  DevResult* hres_dev = nullptr;  // hres as the device addresses it
  hipEvent_t ev_start = nullptr;  // events around the walks, or null: no kernel timing
  hipEvent_t ev_stop = nullptr;
  int cu_count = 256;
  // one-launch path (small real and complex permanents); null: not available
  double* fused_slots = nullptr;  // kFusedMaxBlocks slots of kFusedSlotDoubles
  uint32_t* counter = nullptr;    // finished workgroups; zero between calls
  uint64_t* t0 = nullptr;         // earliest workgroup start; all ones between calls
  int wall_khz = 0;               // rate of the device wall clock
};

constexpr size_t call_align(size_t x) { return (x + 255) / 256 * 256; }

// Byte offsets of the sub-buffers; index 8 is the total size.
constexpr size_t call_buffer_offset(int part, int max_parts) {
  const size_t sz[8] = {64,
                        sizeof(int32_t) * kMaxN,
                        64,
                        sizeof(DevResult),
                        sizeof(double) * kMaxN,
                        sizeof(double) * 4 * kMaxN * kMaxN,
                        32 * (size_t)max_parts,
                        sizeof(double) * (size_t)max_parts};
  size_t off = 0;
  for (int k = 0; k < part; ++k) off = call_align(off + sz[k]);
  return off;
}

constexpr size_t call_buffer_bytes(int max_parts) { return call_buffer_offset(8, max_parts); }

inline void carve_call_buffers(char* base, int max_parts, CallBuffers* b) {
  b->status = (int32_t*)(base + call_buffer_offset(0, max_parts));
  b->rowexp = (int32_t*)(base + call_buffer_offset(1, max_parts));
  b->bound = (double*)(base + call_buffer_offset(2, max_parts));
  b->dres = (DevResult*)(base + call_buffer_offset(3, max_parts));
  b->rowabs = (double*)(base + call_buffer_offset(4, max_parts));
  b->staged = (double*)(base + call_buffer_offset(5, max_parts));
  b->partials = (void*)(base + call_buffer_offset(6, max_parts));
  b->drift = (double*)(base + call_buffer_offset(7, max_parts));
  b->max_parts = max_parts;
}

// Each walk family is built as two translation units (n <= 32 and n > 32);
// the launch_walk_* dispatchers in perm_host.cpp pick one by n.
hipError_t launch_walk_real_lo(int n, int mode, bool drift, const WalkArgs& a, int grid,
                               hipStream_t s);
hipError_t launch_walk_real_hi(int n, int mode, bool drift, const WalkArgs& a, int grid,
                               hipStream_t s);
hipError_t launch_walk_complex_lo(int n, int mode, bool drift, const WalkArgs& a, int grid,
                                  hipStream_t s);
hipError_t launch_walk_complex_hi(int n, int mode, bool drift, const WalkArgs& a, int grid,
                                  hipStream_t s);
hipError_t launch_walk_int01_lo(int n, bool drift, int variant, const WalkArgs& a, int grid,
                                hipStream_t s);
hipError_t launch_walk_int01_hi(int n, bool drift, int variant, const WalkArgs& a, int grid,
                                hipStream_t s);
// 0/1 walk variant 0: plain exact walk; 1: the pair-shared walk where the
// staging kernel's status[1] allows it, the plain walk otherwise (decided on
// the device, in one launch).
// Smallest pair_rows (n/3) for which the pair-shared 0/1 walk is built.
constexpr int kInt01PairMinRows = 3;

// One-launch permanent of a small real or complex matrix: every workgroup
// stages its own copy, walks its chunks, and the last one to finish adds the
// partials in workgroup order (kern_fused.hip).
constexpr int kFusedMaxN = 24;
constexpr int kFusedMaxBlocks = 512;
constexpr int kFusedSlotDoubles = 2 * 2 * kFusedMaxN * kFusedMaxN;  // +A, -A, complex

struct FusedArgs {
  const double* A;        // caller's matrix, column-major, leading dimension ld
  int32_t ld;
  int32_t row_scaling;
  double* slots;          // per workgroup: its staged +A then -A (ld = n)
  uint64_t slot_stride;   // doubles between workgroup slots
  uint64_t ntasks;        // wave tasks of the aligned chunks of [0, 2^(n-1))
  uint64_t nchunks;
  int32_t b;              // log2 chunk length (>= 1)
  int32_t pad;
  double* partials;       // 4 doubles per workgroup
  uint32_t* counter;      // zero on entry; set back to zero by the last workgroup
  uint64_t* t0;           // all ones on entry; set back by the last workgroup
  DevResult* res;         // result record
};

hipError_t launch_fused(bool cplx, int n, int mode, const FusedArgs& a, int grid, hipStream_t s);

// Staging: validate A, choose row exponents, write +A/-A (0/1: +2A/-2A).
// 0/1 input with pair_rows > 0: the matrix is permuted (sparsest column
// first, its nonzero rows on top, then rows by ascending degree) and status[1]
// is set to 1 when the pair-shared walk with that many dynamic rows is exact.
hipError_t launch_stage(int kind, const void* A, int n, int ld, int row_scaling, int range_check,
                        int pair_rows, double* staged, double* rowabs, int32_t* rowexp,
                        int32_t* status, double* bound, hipStream_t s);

// The per-workgroup partials as the caller's records (perm_opts.partials_out).
hipError_t launch_export_partials(int kind, const void* partials, const double* drift_part,
                                  int want_drift, int nparts, const int32_t* rowexp, int n,
                                  double* out, hipStream_t s);

// Fixed-order sum of the per-workgroup partials into a DevResult.
hipError_t launch_finish(int kind, const void* partials, int nparts, const double* drift_part,
                         int want_drift, const int32_t* status, const int32_t* rowexp, int n,
                         const double* bound, DevResult* res, hipStream_t s);

// ---------------------------------------------------------------- batched ----

// One queue item: 64 lane chunks of one matrix (wave task `task` of its body).
struct BatchItem {
  int32_t mat;     // matrix index
  int32_t n;
  int32_t b;       // log2 chunk length
  int32_t pad;
  uint64_t task;   // wave task within the matrix (see task_chunk)
  uint64_t nchunks;
};

struct BatchArgs {
  const double* staged;      // staged matrices (per matrix: +A then -A)
  const int64_t* st_off;     // offset of matrix m's staged block (doubles)
  const int32_t* mstatus;    // per-matrix staging status
  const BatchItem* items;    // sorted by size, largest first
  double* slots;             // 4 doubles per item
};

hipError_t launch_batched_stage(int is_complex, const double* A, const int64_t* d_off,
                                const int32_t* d_n, int count, int row_scaling, double* staged,
                                const int64_t* st_off, int32_t* rowexp_sum, int32_t* mstatus,
                                hipStream_t s);
// Items [item0, item0 + nitems), all of size n, by the size's own kernel.
hipError_t launch_batched_size(int is_complex, int mode, int n, const BatchArgs& a,
                               uint64_t item0, uint64_t nitems, int grid, hipStream_t s);
hipError_t launch_batched_finish(const double* slots, const int64_t* item_first,
                                 const int32_t* item_count, const int32_t* d_n,
                                 const int32_t* rowexp_sum, const int32_t* mstatus, int count,
                                 double* d_out, int32_t* d_status, hipStream_t s);
// Resident workgroups per CU of size n's batched kernel.
int batched_walk_blocks_per_cu(int is_complex, int mode, int n);

// ------------------------------------------------------ mixed-radix sums ----
// Ryser-type sums whose column sets are enumerated digit by digit: repeated
// columns (Eq. ryser2; perm_repeated) and the restricted sets of sparse
// matrices (App. B; perm_sparse).  Digit k has radix r_k and takes values
// f_k in reflected mixed-radix Gray order (digit 0 fastest), so one step
// changes one digit by one and adds or removes one column:
//   kind 0 (a column with multiplicity m): value f adds f * c, weight
//          (-1)^f C(m, f); one column (`size` 1);
//   kind 1 (a block of `size` columns that the set must meet): value v
//          stands for the nonempty subset gray(v + 1) of the block's columns,
//          weight (-1)^|subset|.
// The signed weights of every digit value sit in one table (omega).  A chunk
// is one run of the first b digits through all L = r_0...r_{b-1} values;
// inside it the changed digit, its direction and the inner weight depend only
// on the step and the chunk's parity (tables tin/toff), and the lane -> chunk
// map gives all lanes of a wave one parity.

constexpr int kRepBinomStride = kMaxN + 1;  // largest radix of a kind-0 digit (m <= 64)
constexpr int kMixMaxLog2Chunk = 14;        // L <= 2^14
constexpr int kSparseMaxBlock = 12;         // blocks of more columns do not restrict
constexpr int kMixMaxOmega = kMaxN * 4096;  // omega table entries

struct MixDigits {
  int32_t R;              // digits
  int32_t ncols;          // staged columns (sum of the sizes)
  int32_t kind[kMaxN];
  int32_t radix[kMaxN];
  int32_t first[kMaxN];   // first staged column of the digit
  int32_t size[kMaxN];    // staged columns of the digit
  int32_t mult[kMaxN];    // kind 0: multiplicity m
  int32_t src[kMaxN];     // staged column c is source column src[c]
  int32_t cmult[kMaxN];   // copies of staged column c in the matrix (row-norm weight)
  int32_t row[kMaxN];     // staged row i is source row row[i]
};

// Device copy of the digit description, read with scalar loads by the walk:
// per digit its radix, kind and omega offset; per staged column the digit it
// belongs to and its bit within the digit's subset (0 for kind 0).
enum { kDigRadix = 0, kDigKind = 1, kDigWofs = 2, kDigColDigit = 3, kDigColBit = 4, kDigFields = 5 };

struct MixArgs {
  const double* staged;   // [+cols | 0] [-cols | 0] (n x (ncols+1) each), then two start columns
  const double* omega;    // signed weight of every digit value
  const double* tin;      // 2 x L: signed weight of the inner digits at step s (parity 0, 1)
  const int32_t* toff;    // 2 x L: offset (doubles) into staged of the column added after
                          // step s; the last step adds the zero column
  const int32_t* dig;     // kDigFields x kMaxN digit fields
  const uint64_t* qabs;   // Q_k = r_0 ... r_{k-1}, k = 0..R
  const int32_t* status;  // staging status; nonzero -> the walk does nothing
  uint64_t first;         // first chunk (walk) or first Gray index (single terms)
  uint64_t nchunks;
  uint64_t ntasks;        // 2 * ceil(nchunks / 128)
  int32_t R, b, L, ncols;
  int32_t outer_col;      // first staged column of digit b (the first outer digit)
  int32_t pad;
  void* partials;         // per workgroup: dd (real) or complex dd
};

// in_kind: 0 real doubles, 1 complex pairs, 2 bytes (0/1 data, staged as doubles).
hipError_t launch_mix_stage(int in_kind, const void* A, int n, int ld, const MixDigits& dg,
                            int b, int L, int row_scaling, double* staged, double* omega,
                            double* tin, int32_t* toff, int32_t* dig, uint64_t* qabs,
                            int32_t* rowexp, int32_t* status, hipStream_t s);
// single: every lane sums one term (Gray indices first .. first + nchunks - 1).
// exact (real only; 0/1 data with weights +-1, L <= 2^10): 128-bit integer
// partials instead of double-double ones.  groups (exact chunk walk only):
// 0 multiplies the rows in groups of int01_group_rows(n), valid for any 0/1
// matrix; 1..kMixMaxRowGroups splits the staged rows into that many equal
// groups (ceil(n / groups) rows, the last shorter), which the caller has
// checked keep every group's product of row degrees below 2^50.
constexpr int kMixExactMaxLog2Chunk = 10;
constexpr int kMixMaxRowGroups = 4;
hipError_t launch_mix_walk_real_lo(int n, bool single, bool exact, int groups, const MixArgs& a,
                                   int grid, hipStream_t s);
hipError_t launch_mix_walk_real_hi(int n, bool single, bool exact, int groups, const MixArgs& a,
                                   int grid, hipStream_t s);
hipError_t launch_mix_walk_complex_lo(int n, bool single, bool exact, int groups,
                                      const MixArgs& a, int grid, hipStream_t s);
hipError_t launch_mix_walk_complex_hi(int n, bool single, bool exact, int groups,
                                      const MixArgs& a, int grid, hipStream_t s);

// App. B greedypartition on the device.  Trial 0 takes the lowest row index
// among rows of least degree; trials 1.. break ties with a counter-based hash
// of (seed, trial, step); the trial with the fewest column sets wins (lowest
// trial on ties).
struct SparsePart {
  int32_t status;         // 0, or 1 when a row is zero (per = 0)
  int32_t nblocks;
  int32_t ntail;
  int32_t trial;          // winning trial
  int32_t cols[kMaxN];    // blocks in selection order (columns ascending), then T ascending
  int32_t bsize[kMaxN];
  double log2_terms;      // log2 of 2^|T| prod (2^|S| - 1)
  double log2_degprod;    // log2 prod_i (nonzeros of row i)
  double bregman;         // sum_i log2(d_i!) / d_i: log2 of Bregman's bound on |per| (0/1 data)
  int32_t deg[kMaxN];     // d_i, the nonzeros of row i
};

hipError_t launch_sparse_partition(int in_kind, const void* A, int n, int ld, int trials,
                                   uint64_t seed, SparsePart* out, hipStream_t s);

// ------------------------------------------------------------------ band ----
// App. C transfer matrix (perm_band): one wavefront per matrix, four per workgroup.
constexpr int kBandMaxK = 5;  // rank tables of 2^(2k+1) masks in LDS

struct BandArgs {
  const double* A;        // matrices back to back (column-major, ld = n; complex pairs)
  const int64_t* off;     // element offset (doubles) of matrix m
  const int32_t* n;       // sizes
  int32_t count;
  int32_t pad;
  double* out;            // 4 doubles per matrix
  int32_t* status;        // per matrix (may be null)
};

hipError_t launch_band(bool cplx, int k, const BandArgs& a, int grid, hipStream_t s);
// Workgroups of band_kernel<k> resident on one CU (occupancy query).
int band_blocks_per_cu(bool cplx, int k);

// Rows per exactly-multiplied group in the 0/1 walk: the largest k with
// n^k < 2^50 (|2 w_i| <= n, so a group's product stays below 2^50).
constexpr int int01_group_rows(int n) {
  if (n <= 1) return 1;
  int k = 0;
  double p = 1.0;
  while (p * n < 1125899906842624.0) {
    p *= n;
    ++k;
  }
  return k;
}

}  // namespace perm
