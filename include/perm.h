/*
 * perm.h -- exact matrix permanents on AMD Instinct MI355X (gfx950).
 *
 * The library evaluates the permanent of a dense n x n real, complex or 0/1
 * matrix (Lundow & Markstrom, Sec. I, Eq. per) with the half-range,
 * Gray-code-ordered form of Ryser's inclusion-exclusion (Sec. II.A: Ryser's
 * formula, Eq. ryser, visited in Gray order and halved by pinning the last
 * column; App. A: distribute, Gray unranking, nextset, subpermanent,
 * permanent).  In the notation of App. A, for the Gray code x = gray(g) of a
 * term index g in [0, 2^(n-1)),
 *
 *     w_i(x) = a_{i,n} - 1/2 sum_{j=1..n} a_{ij} + sum_{j<n, x_j=1} a_{ij},
 *     S      = sum_g (-1)^(g+1) prod_i w_i(gray(g)),
 *     per(A) = 2 (-1)^n S.
 *
 * Conventions shared by every entry point:
 *   - Matrices are caller-owned DEVICE memory, column-major with leading
 *     dimension ld >= n: a(i,j) = A[i + j*ld].  Complex matrices are
 *     interleaved (re, im) doubles: a(i,j) = A[2(i+j*ld)] + i A[2(i+j*ld)+1].
 *     Since per(A) = per(A^T), a row-major caller may pass its array as is.
 *   - `stream` is a hipStream_t (NULL = the default stream).  All work is
 *     enqueued on it.  Single-matrix calls return a host value once the result
 *     is complete: they wait for that stream, or, on the one-launch path of
 *     small real and complex permanents, for the result record the kernel
 *     writes into pinned host memory as its last act; perm_batched only
 *     enqueues and returns at once.
 *   - No pointer is kept after a call returns.  Library-owned device
 *     workspace (staged matrix, partial sums, item plans) is allocated lazily per
 *     device and kept until perm_release().
 *   - Calls may overlap (several host threads, several streams):
 *       perm_real, perm_complex, perm_int01, perm_partial each lease a
 *       workspace of their own for the length of the call (a new one is
 *       allocated when all are busy), so overlapping calls run concurrently;
 *       perm_repeated*, perm_sparse*, perm_band take turns on one device (the
 *       next call enters once the previous one has returned and its stream has
 *       drained); perm_batched keeps one plan per device and orders its reuse
 *       by stream: a call on another stream first waits, on the device, for the
 *       previous call's work.
 *     perm_release() must not overlap any other call.
 *   - Errors are reported only through the returned status; on error the
 *     outputs are left untouched.  perm_last_error() has a text message.
 *   - n = 0 gives per = 1 (the empty product).  n <= 64.
 */
#ifndef PERM_H
#define PERM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PERM_OK = 0,
  PERM_EINVAL = 1,     /* bad n, ld, option, range, or (0/1 path) an entry not 0 or 1 */
  PERM_ERANGE = 2,     /* 0/1 path: the exact result might not fit 128 bits (see perm_int01) */
  PERM_ENONFINITE = 3, /* a NaN or infinity in A */
  PERM_ENOMEM = 4,     /* device or pinned host allocation failed */
  PERM_EHIP = 5,       /* HIP runtime error (text in perm_last_error) */
  PERM_ENOTIMPL = 6    /* option combination not provided */
} perm_status;

/* Arithmetic of the Gray walk (App. A, subpermanent; Sec. II.B, Precision). */
typedef enum {
  PERM_FP64_DD = 0,  /* FP64 row sums and products, per-lane double-double sum (default;
                        the analogue of the paper's Kahan / double-quad summation) */
  PERM_FP64 = 1,     /* FP64 row sums, products and plain FP64 sum (the paper's "double") */
  PERM_SPLIT_F32 = 2 /* FP64 row sums, FP32 products, double-double sum */
} perm_precision;

/* Options.  A zeroed struct (or NULL) selects the defaults. */
typedef struct {
  int32_t precision;      /* perm_precision; ignored by perm_int01 */
  int32_t log2_chunk;     /* Gray terms per lane chunk = 2^log2_chunk; 0 = automatic.
                             Every chunk's row sums are formed afresh from A, so this
                             bounds the walk's drift.  Max 24 (0/1 path: 10). */
  int32_t drift_check;    /* 1: at every chunk end re-form the row sums from A and report
                             the largest |w_walked - w_fresh| / (1/2 sum_j |a_ij|) */
  int32_t no_row_scaling; /* 1: do not scale rows by powers of two (scaling is exact and
                             undone at the end; it keeps FP32 products in range) */
  int32_t blocks;         /* workgroups of the walk kernel; 0 = automatic (8 per CU) */
  int32_t use_graph;      /* perm_batched: replay a captured HIP graph when the same
                             arguments come again (1) or launch directly (0) */
  int32_t partials_cap;   /* records available at partials_out (0 when it is NULL) */
  int32_t reserved;       /* must be 0 */
  double* partials_out;   /* optional DEVICE array (perm_real, perm_complex, perm_int01,
                             perm_partial, perm_partial_noalloc): the partial sums the
                             final sum is taken over -- one record per workgroup of the
                             walk launches, in the order they are added (the paper keeps
                             such an array before its final compensated sum, Sec. II.B).
                             Record k = 5 doubles: re_hi, re_lo, im_hi, im_lo of the
                             workgroup's double-double sum of its terms (in the sign
                             convention of perm_partial, scaled back to A itself; 0/1
                             input: words 0 and 1 hold the low and high 64 bits of its
                             two's-complement 128-bit integer sum of prod_i 2w_i, words 2
                             and 3 are 0), then the largest row-sum drift of its chunks
                             (drift_check; -1 otherwise).  perm_result.parts = the number
                             of records.  Too small a partials_cap is PERM_EINVAL.  The
                             array is filled on `stream` before the call returns.  Other
                             entry points reject it (PERM_ENOTIMPL) */
} perm_opts;

/* Result of a single-matrix call. */
typedef struct {
  double re_hi, re_lo;   /* real part as the unevaluated sum re_hi + re_lo */
  double im_hi, im_lo;   /* imaginary part (0 for real and 0/1 input) */
  uint64_t int_lo;       /* 0/1 path: exact value, two's-complement 128-bit (low word) */
  int64_t int_hi;        /*                                              (high word) */
  double max_drift;      /* drift_check: largest relative row-sum drift; otherwise -1 */
  uint64_t terms;        /* Gray terms summed */
  uint64_t chunks;       /* lane chunks walked (including single-term ragged ends) */
  int32_t log2_chunk;    /* chunk length used */
  int32_t blocks;        /* workgroups of the main walk launch */
  float kernel_ms;       /* duration of the walk launches, from HIP events on `stream`;
                            on the one-launch path (walk_variant 1 of perm_real and
                            perm_complex) the device wall clock from the first workgroup's
                            start to the result */
  float total_ms;        /* perm_real, perm_complex, perm_int01, perm_partial: wall time of
                            the call on the host, from entry until the result is in host
                            memory.  perm_repeated*, perm_sparse*: HIP events on `stream`
                            from staging to the result */
  int32_t walk_variant;  /* perm_int01: 2 if the banded pair walk ran, 1 if the pair-shared
                            walk ran, else 0.  perm_real,
                            perm_complex: 1 if the one-launch path ran (n <= 24 with
                            default blocks and no drift check: staging, walk and the
                            fixed-order sum in one kernel), else 0.  perm_sparse
                            with PERM_DT_INT01: the row groups of the exact product (1..4),
                            or 0 for the size-only grouping.  Otherwise 0 */
  int32_t col0_nonzeros; /* 0/1 path, pair-shared or banded walk: ones in the column flipped
                            between the two terms of every pair; otherwise 0 */
  int32_t parts;         /* partial sums the result was added from (the records written
                            to opts->partials_out when it is given) */
  int32_t pad;
} perm_result;

/*
 * perm_real -- per(A) of a real n x n matrix (FP64 input).
 *   dA      device pointer, column-major, leading dimension ld >= max(n,1).
 *   out     host pointer; value in re_hi + re_lo (relative error of the default
 *           precision: about 1e-15..1e-11, depending on the cancellation among the
 *           terms).
 * Errors: PERM_EINVAL (n < 0, n > 64, ld < n, bad opts), PERM_ENONFINITE, PERM_EHIP.
 */
perm_status perm_real(const double* dA, int n, int ld, const perm_opts* opts,
                      perm_result* out, void* stream);

/*
 * perm_complex -- per(A) of a complex n x n matrix (interleaved complex128).
 *   Value in (re_hi + re_lo) + i (im_hi + im_lo).  Errors as perm_real.
 */
perm_status perm_complex(const double* dA, int n, int ld, const perm_opts* opts,
                         perm_result* out, void* stream);

/*
 * perm_int01 -- exact per(A) of a 0/1 matrix (one byte per entry, each 0 or 1).
 *   The walk keeps the doubled row sums r_i = 2 w_i, which are small integers,
 *   and sums sum_g (-1)^(g+1) prod_i r_i = (-1)^n 2^(n-1) per(A) exactly modulo
 *   2^128 (the row sums are exact integers held in FP64 registers; products are
 *   formed exactly in row groups whose bound stays below 2^50 and combined with
 *   error-free transformations into 51-bit integer bins).  The result is exact
 *   when 2^(n-1) per(A) < 2^127; the library checks the sufficient condition
 *   (n-1) + sum_i log2(d_i!)/d_i < 127 (Bregman's bound, d_i = row sums) on the
 *   device before the walk and returns PERM_ERANGE otherwise (always passes for
 *   n <= 28).  Value in int_lo/int_hi; re_hi + re_lo holds its nearest double pair.
 *   Rows and columns are permuted first (the permanent does not change): the
 *   column with the fewest ones becomes the most frequently flipped one, its
 *   nonzero rows come first.  When that column has at most n/3 ones and those
 *   n/3 rows' sums multiply to less than 2^50, the two terms of every pair
 *   share the product of the other rows and one exact combination
 *   (walk_variant = 1): about 40% fewer operations per term for 0/1 matrices
 *   of density 1/2.  The column with the fewest ones outside those rows then
 *   becomes the column flipped after every other pair, the rows with a one
 *   there follow, up to (n - n/3)/2 rows; when it has at most that many ones
 *   there and those rows' sums, and the remaining rows' sums, each multiply to
 *   less than 2^50, the product of the remaining rows is shared by two pairs
 *   and that flip skips them (walk_variant = 2): about 10% fewer again.
 * Errors: PERM_EINVAL (sizes, or an entry other than 0/1), PERM_ERANGE, PERM_EHIP.
 */
perm_status perm_int01(const uint8_t* dA, int n, int ld, const perm_opts* opts,
                       perm_result* out, void* stream);

/* Element types for perm_partial. */
typedef enum { PERM_DT_REAL = 0, PERM_DT_COMPLEX = 1, PERM_DT_INT01 = 2 } perm_dtype;

/*
 * perm_partial -- the paper's subpermanent (App. A) over an explicit range:
 *   S = sum_{g=start}^{start+count-1} (-1)^(g+1) prod_i w_i(gray(g)),
 *   0 <= start, start + count <= 2^(n-1), n >= 1.  No final factor 2(-1)^n and
 *   no row-scaling factor is applied: the value refers to A itself.  For
 *   PERM_DT_INT01 the integer form sum_g (-1)^(g+1) prod_i (2 w_i) is returned
 *   exactly modulo 2^128 in int_lo/int_hi (= 2^n S; no range check is made).
 *   Ranges need not be aligned; unaligned ends are summed one term per lane.
 *   Splitting [0, 2^(n-1)) into pieces and adding the partials gives the
 *   permanent (how the range would be divided between devices).
 */
perm_status perm_partial(int dtype, const void* dA, int n, int ld, uint64_t start,
                         uint64_t count, const perm_opts* opts, perm_result* out,
                         void* stream);

/*
 * perm_partial_noalloc -- perm_partial for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, ranges, result and errors as perm_partial,
 * but the call allocates nothing (no hipMalloc, hipFree, pinned host memory or
 * events): its staging copy, partial sums and result record live in a fixed
 * array of device memory inside the library (370 KiB per device, held
 * until the process ends), and the record is copied into `out` before the call
 * returns (it waits for `stream`).  kernel_ms is 0 (no events); total_ms is the
 * host wall time of the call.
 *   Limit: each walk launch uses at most PERM_NOALLOC_MAX_BLOCKS workgroups
 *   (0 = min(8 per CU, that limit), the same grid as perm_partial on a device of
 *   at most 256 CUs, so the two give identical bits there); opts->blocks above
 *   it is rejected with PERM_EINVAL.
 *   All calls on one device share that array and it keeps the last call's
 *   contents (each call writes every part it reads): calls that overlap on one
 *   device (several host threads or streams) race, and the caller must
 *   serialise them.  Calls on different devices are independent.
 */
#define PERM_NOALLOC_MAX_BLOCKS 2048
perm_status perm_partial_noalloc(int dtype, const void* dA, int n, int ld, uint64_t start,
                                 uint64_t count, const perm_opts* opts, perm_result* out,
                                 void* stream);

/*
 * perm_combine -- App. A, permanent: per(A) = 2 (-1)^n sum_k S_k from the
 * partial sums S_k of perm_partial over ranges that together cover
 * [0, 2^(n-1)) once (any cut into pieces, e.g. equal slices run one after
 * another, resumed from a checkpoint, or run on several devices).  Host only.
 *   dtype, n  as given to perm_partial.
 *   parts     HOST array of `count` results of perm_partial, in the order of
 *             their ranges; the sum is taken in exactly that order, so a given
 *             cut always gives the same bits.
 *   out       the permanent: re_hi + re_lo (+ i (im_hi + im_lo)), the sum of the
 *             parts' double-double values by accurate double-double additions, then
 *             multiplied by 2(-1)^n (exact).  PERM_DT_INT01: the parts' 128-bit
 *             integers are added modulo 2^128; the total is (-1)^n 2^(n-1) per(A),
 *             and per(A) is returned exactly in int_lo/int_hi (with its nearest
 *             double pair in re_hi + re_lo) provided 2^(n-1) per(A) < 2^127
 *             (check perm_int01_bound on the row sums first: the partial sums
 *             carry no range check).  terms, chunks, kernel_ms and total_ms are the
 *             parts' sums, max_drift their maximum; log2_chunk and blocks those
 *             of parts[0].
 * Errors: PERM_EINVAL (NULL pointers, bad dtype or n, count < 1, parts whose
 *   term counts do not add up to 2^(n-1), or 0/1 parts whose total is not a
 *   multiple of 2^(n-1), i.e. not the whole sum of one matrix).
 */
perm_status perm_combine(int dtype, int n, const perm_result* parts, int count,
                         perm_result* out);

/*
 * perm_batched -- permanents of many independent matrices (the random-matrix
 * studies of Secs. III-VI compute many independent permanents).
 *   dA       device array holding the matrices back to back; matrix m starts at
 *            element offset h_offset[m] (in doubles) and is column-major with
 *            ld = n_m (complex: interleaved pairs, offset still in doubles).
 *   h_n      HOST array of the sizes, 1 <= n_m <= 32.
 *   h_offset HOST array of offsets.
 *   count    number of matrices (0 is allowed and does nothing).
 *   d_out    device array, 4 doubles per matrix: re_hi, re_lo, im_hi, im_lo.
 *   d_status device array of count int32 (may be NULL): PERM_OK or PERM_ENONFINITE.
 * Work is bucketed by n (largest first), cut into wave-sized items of
 * 2^log2_chunk-term lane chunks (per-n lengths from the autotuner unless
 * opts->log2_chunk is set); each size runs as one persistent launch of that
 * size's kernel, the waves taking its items round-robin (items of one size cost
 * the same).  Enqueued on `stream`; returns without waiting.
 */
perm_status perm_batched(const double* dA, const int32_t* h_n, const int64_t* h_offset,
                         int count, int is_complex, const perm_opts* opts, double* d_out,
                         int32_t* d_status, void* stream);

/*
 * perm_autotune -- time candidate chunk lengths for the batched path on
 * synthetic matrices of each size in [n_lo, n_hi] (1 <= n_lo <= n_hi <= 32) and
 * keep the fastest per size for later perm_batched calls.  A chunk length 2^b
 * fixes the lanes per matrix: 2^(n-1-b) lanes, one chunk each, in wave items of
 * 64; the cache file lists both.  If cache_path is not
 * NULL the table is also written there as JSON (and perm_batched reads it back
 * when PERM_AUTOTUNE_CACHE names that file).  Waits for `stream`.
 */
perm_status perm_autotune(int is_complex, int n_lo, int n_hi, const char* cache_path,
                          void* stream);

/*
 * perm_repeated -- per(A) of an n x n matrix whose columns repeat (Sec. II.A,
 * Eq. ryser2): A has mult[k] copies of column k of C (k < R, sum mult = n), in
 * any order.  With f ranging over the vectors 0 <= f_k <= mult[k],
 *
 *     per(A) = (-1)^n sum_f (-1)^(f_1+...+f_R) prod_k C(mult[k], f_k)
 *                          prod_i sum_k f_k c_ik,
 *
 * prod_k (mult[k] + 1) terms instead of 2^(n-1).  Repeated rows: per(A) =
 * per(A^T), so pass the distinct rows as the columns of C.
 *   dC      device pointer to C, n x R, column-major with leading dimension
 *           ld >= n (dtype PERM_DT_REAL: doubles; PERM_DT_COMPLEX: interleaved
 *           pairs).  PERM_DT_INT01 is not accepted (pass 0/1 data as doubles).
 *   mult    HOST array of R multiplicities, each >= 1, summing to n.
 *   1 <= R <= n <= 64 and prod_k (mult[k] + 1) <= 2^63.
 *   The vectors f are walked in reflected mixed-radix Gray order (digit k =
 *   f_k, digit 0 changing fastest), so every step changes one f_k by +-1 and
 *   adds or subtracts one column of C.  A lane walks a chunk that runs the
 *   first b digits through all their values (L = (mult[0]+1)...(mult[b-1]+1)
 *   terms, b chosen so that L <= 2^log2_chunk, automatic when 0, at most 2^14);
 *   out->log2_chunk reports b.  Precision: PERM_FP64_DD only; drift_check is
 *   not provided (PERM_ENOTIMPL).  Row scaling as for perm_real.
 * Errors: PERM_EINVAL (sizes, multiplicities, options), PERM_ENONFINITE,
 *   PERM_ENOTIMPL, PERM_EHIP.
 */
perm_status perm_repeated(int dtype, const double* dC, int n, int R, int ld,
                          const int32_t* mult, const perm_opts* opts, perm_result* out,
                          void* stream);

/*
 * perm_repeated_partial -- the sum of Eq. ryser2 over Gray indices
 * [start, start + count) of that order, without the factor (-1)^n:
 *   sum_{g} (-1)^(sum f) prod_k C(mult[k], f_k) prod_i sum_k f_k c_ik,  f = f(g),
 * start + count <= prod_k (mult[k] + 1).  Ranges need not be aligned to chunks.
 * Arguments and errors as perm_repeated.
 */
perm_status perm_repeated_partial(int dtype, const double* dC, int n, int R, int ld,
                                  const int32_t* mult, uint64_t start, uint64_t count,
                                  const perm_opts* opts, perm_result* out, void* stream);

/*
 * perm_sparse -- per(A) of a sparse n x n matrix by the restricted Ryser sum of
 * App. B (greedypartition, sparsepermanent).  A set J of columns can give a
 * nonzero term of Eq. ryser only if every row has a nonzero entry in J.
 * greedypartition repeatedly takes a remaining row of least degree, makes its
 * set of nonzero columns a block S_l, and drops every remaining row whose set
 * meets S_l.  The sum then runs only over the J that meet every block: a
 * nonempty subset of each S_l times any subset of the other columns T.
 * 2^|T| prod_l (2^|S_l| - 1) terms instead of 2^n; the value is per(A) exactly
 * (only zero terms are dropped).  Blocks of more than 12 columns do not restrict
 * (their columns join T).
 *   dtype   PERM_DT_REAL, PERM_DT_COMPLEX or PERM_DT_INT01 (bytes 0/1, any nonzero
 *           byte value is taken as an integer entry).
 *   dA      device matrix, column-major, ld >= n, 1 <= n <= 64.
 *   trials  1: the greedy takes the lowest row index among rows of least degree.
 *           2..256: trial 0 as before, trials 1.. break ties at random (a
 *           counter-based hash of seed, trial and step), and the partition with the
 *           fewest column sets is used (the paper's randomised variant).
 *   The sets are walked in reflected mixed-radix Gray order: one digit per block
 *   (radix 2^|S_l| - 1, value v standing for the subset gray(v + 1) of the block's
 *   columns in ascending order), in selection order, then one radix-2 digit per
 *   column of T (ascending); every step adds or removes one column.
 *   out->terms is the number of sets; log2_chunk reports the inner digits.
 *   PERM_DT_INT01: exact.  The row sums are integers; every product is formed
 *   exactly in row groups and summed in 51-bit integer bins folded into a 128-bit
 *   integer (as perm_int01; chunks of at most 2^10 terms).  A row sum is at most
 *   the row's degree d_i, so the rows are dealt into the fewest (1..4) equal groups
 *   whose products of degrees stay below 2^50 (out->walk_variant); when none
 *   fits, groups of the largest k rows with n^k < 2^50, as in perm_int01.  The
 *   result (int_lo/int_hi, and its nearest double pair in re_hi + re_lo) is exact
 *   when |per| < 2^127; the library checks Bregman's bound sum_i log2(d_i!)/d_i < 127
 *   and returns PERM_ERANGE otherwise.  A zero row gives 0.
 * Errors: PERM_EINVAL, PERM_ENONFINITE, PERM_ERANGE, PERM_ENOTIMPL (options other
 *   than log2_chunk <= 14, blocks, no_row_scaling), PERM_EHIP.
 */
perm_status perm_sparse(int dtype, const void* dA, int n, int ld, int trials, uint64_t seed,
                        const perm_opts* opts, perm_result* out, void* stream);

/*
 * perm_sparse_partial -- the raw sum of Eq. ryser's terms (-1)^|J| prod_i sum_{j in J}
 * a_ij over Gray indices [start, start + count) of that enumeration, without the
 * factor (-1)^n; start + count <= out->terms of perm_sparse.  0/1 input gives the
 * exact integer sum modulo 2^128 in int_lo/int_hi (no range check).  Arguments as
 * perm_sparse.
 */
perm_status perm_sparse_partial(int dtype, const void* dA, int n, int ld, int trials,
                                uint64_t seed, uint64_t start, uint64_t count,
                                const perm_opts* opts, perm_result* out, void* stream);

/*
 * perm_sparse_partition -- the partition perm_sparse would use: block_of_col (HOST,
 * n entries) gets the block index of every column in selection order, -1 for T;
 * *nblocks the number of blocks; *terms the number of column sets.  Waits for
 * `stream`.  PERM_EINVAL also when A has a zero row.
 */
perm_status perm_sparse_partition(int dtype, const void* dA, int n, int ld, int trials,
                                  uint64_t seed, int32_t* block_of_col, int32_t* nblocks,
                                  uint64_t* terms, void* stream);

/*
 * perm_band -- permanents of band matrices (a_ij = 0 whenever |i - j| > k) by
 * the transfer matrix of App. C (bandpermanent), one wavefront per matrix.
 *   per(A) is the sum of the coefficients of prod_i (sum_j a_ij x_j) with every
 *   x_j^2 = 0; after row i the variable of column i-k-1 is set to 1, so only
 *   the monomials over columns i-k..i+k are kept, and of those only the ones with
 *   min(i+1, k+1) columns can reach the end (at most binom(2k+1, k+1) of them).
 *   O(n * binom(2k+1, k+1) * k) operations per matrix, no inclusion-exclusion and so
 *   no cancellation beyond that of the entries themselves.
 *   dtype    PERM_DT_REAL or PERM_DT_COMPLEX.
 *   dA       device array, matrices back to back; matrix m starts at element offset
 *            h_offset[m] (in doubles) and is column-major with ld = n_m (complex:
 *            interleaved pairs).  Entries with |i - j| > k are not read: the result is
 *            the permanent of the band part.
 *   h_n      HOST array of sizes, 1 <= n_m <= 65536; h_offset HOST array of offsets.
 *   k        0 <= k <= 5 (the coefficients and the 2^(2k+1)-entry rank table live in LDS).
 *   d_out    device array, 4 doubles per matrix: re_hi, re_lo, im_hi, im_lo (each row is
 *            scaled by a power of two during the product and the scale is restored at the
 *            end; values beyond the double range come back as +-inf).
 *   d_status device array of count int32 (may be NULL): PERM_OK or PERM_ENONFINITE.
 * Options: only `blocks` (workgroups of four wavefronts, one matrix per wavefront at a
 * time; 0 = as many as fit on the device at once, from the occupancy of the kernel for k,
 * and no more than the batch needs).  Waits for `stream`.
 * Errors: PERM_EINVAL, PERM_ENOTIMPL (other options), PERM_ENOMEM, PERM_EHIP.
 */
perm_status perm_band(int dtype, const double* dA, const int32_t* h_n, const int64_t* h_offset,
                      int count, int k, const perm_opts* opts, double* d_out, int32_t* d_status,
                      void* stream);

/* Chunk plan for a Gray-index range, computed on the host (no GPU needed). */
typedef struct {
  int32_t log2_chunk;      /* L = 2^log2_chunk */
  uint64_t head_start, head_count;   /* unaligned leading terms, one term per lane */
  uint64_t body_first_chunk;         /* body = chunks [first, first+body_chunks) of length L */
  uint64_t body_chunks;
  uint64_t tail_start, tail_count;   /* unaligned trailing terms */
  uint64_t body_tasks;               /* wave tasks (64 lanes each) covering the body */
} perm_plan_info;

/*
 * perm_plan -- the decomposition the library uses for [start, start+count) at
 * size n (App. A distribute, with power-of-two aligned chunks instead of m
 * equal parts).  log2_chunk = 0 picks automatically; is_int01 caps it at 10.
 * Returns PERM_EINVAL for an invalid range.  Host only.
 */
perm_status perm_plan(int n, uint64_t start, uint64_t count, int log2_chunk, int is_int01,
                      perm_plan_info* out);

/*
 * perm_int01_bound -- log2 of the 0/1 path's accumulator bound,
 * (n-1) + sum_i log2(d_i!)/d_i for row sums d_i (rows with d_i = 0 make the
 * permanent 0 and the bound 0).  Host only; the device check uses the same rule.
 */
double perm_int01_bound(const int32_t* row_degrees, int n);

const char* perm_strerror(perm_status s);  /* static text for a status */
const char* perm_last_error(void);         /* text of the last failure on this thread */
const char* perm_version(void);
void perm_release(void);                   /* free library-owned workspace on all devices */

#ifdef __cplusplus
}
#endif

#endif /* PERM_H */
