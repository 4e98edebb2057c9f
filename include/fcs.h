/*
 * fcs.h -- C ABI of the MI355X (gfx950) fast count sketch library, libfcs.so.
 *
 * The operations follow Cao and Liu, "Efficient Tensor Contraction via Fast
 * Count Sketch" (arXiv 2106.13062):
 *   - Definition 4 and the general-tensor formula of Section 3.2: the FCS of
 *     a tensor T of order N is the count sketch of vec(T) under the implicit
 *     long hash pair H = sum_n h_n(i_n), S = prod_n s_n(i_n); it has
 *     J~ = sum_n J_n - N + 1 entries.
 *   - Section 3.1: for a CP tensor [[lambda; U_0..U_{N-1}]] the same sketch is
 *     sum_r lambda_r F^-1(prod_n F(CS_n(U_n)(:, r))) with zero-padded FFTs.
 *   - Section 3.3 (Proposition 1) and Section 4: sketched contractions are
 *     inner products of sketches made with the same hash functions, and the
 *     estimate is the median over D independent sketches; T(I, u, v) uses the
 *     FFT form of Section 4.1.
 *
 * Conventions for every entry point
 *   - Indices are 0-based: h_n(i) is in [0, J_n), bins are in [0, J~).
 *   - Dense tensors are vec(T): mode 0 varies fastest (the paper's
 *     column-major vec); a C-contiguous array of shape (I_{N-1}, ..., I_0)
 *     is exactly that.
 *   - Device pointers are HIP device addresses of the current device; host
 *     pointers are ordinary process memory.  Every pointer argument says
 *     which it is.
 *   - The library never allocates or frees device memory.  Hash tables and
 *     workspaces are caller-owned device buffers whose sizes the library
 *     reports (fcs_plan_table_bytes, fcs_workspace_bytes).  Plans are small
 *     host objects owned by the caller until fcs_plan_destroy.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls are asynchronous on that stream unless stated otherwise; the
 *     library keeps no pointer beyond the work it enqueued.
 *   - Every argument is validated before anything is enqueued; on any error
 *     the call returns a non-zero fcs_status, enqueues nothing and leaves
 *     every output untouched.  fcs_last_error() then describes the problem.
 *     A failed kernel launch returns FCS_EDEVICE.  No exception crosses the
 *     ABI.
 *   - A bound plan is read-only and may be used from several streams at
 *     once; concurrent calls need separate workspaces.
 *   - Both operands of any sketched contraction must come from the same plan
 *     (same seed, shapes and hash lengths): Proposition 1 compares sketches
 *     made with identical hash functions.
 */
#ifndef FCS_H
#define FCS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* exported symbols of libfcs.so (the library is built with hidden default
 * visibility) */
#if defined(__GNUC__) || defined(__clang__)
#define FCS_API __attribute__((visibility("default")))
#else
#define FCS_API
#endif

#define FCS_MAX_ORDER 8      /* largest supported order N                  */
#define FCS_MAX_D 64         /* largest number of independent sketches D   */
#define FCS_MAX_FFT 16384    /* largest LDS-resident FFT size P            */
#define FCS_PROBE_MAX_WINDOW 10000  /* largest window of fcs_probe_lds_atomics */

typedef enum {
    FCS_OK = 0,
    FCS_EINVAL = 1,          /* bad argument (shape, pointer, size, mode)   */
    FCS_ENOMEM = 2,          /* caller buffer smaller than required         */
    FCS_EADMIT = 3,          /* request over the serving admission cap (the
                                serving layer reports it; no call here
                                returns it)                                 */
    FCS_EDEVICE = 4,         /* a HIP call or kernel launch failed          */
    FCS_EUNSUPPORTED = 5     /* valid request outside this build's limits   */
} fcs_status;

typedef struct fcs_plan *fcs_plan_t;

/* Plan description (Definition 4): order N, mode sizes I_n, hash lengths
 * J_n, D independent sketches and the seed of all hash pairs.
 *   N      1..FCS_MAX_ORDER
 *   I      host array of N sizes, each >= 1, product < 2^62
 *   J      host array of N hash lengths, each >= 1, J~ < 2^31
 *   D      1..FCS_MAX_D
 *   seed   64-bit seed of the hash family (see fcs_plan_bind)
 *   L      transform length of the CP / spectral paths; 0 lets the plan
 *          choose.  A caller value must be >= J~ and of the form Q * P with
 *          P a power of two in [256, FCS_MAX_FFT] and 1 <= Q <= 64.  The
 *          paper pads to J~ points (Section 3.1); any L >= J~ gives the same
 *          linear convolution, so L only changes rounding. */
typedef struct {
    int32_t N;
    const int64_t *I;
    const int64_t *J;
    int32_t D;
    uint64_t seed;
    int64_t L;
} fcs_plan_desc;

/* Validate a description and build a host plan (no device work).
 * out: host pointer receiving the plan.  Errors: FCS_EINVAL, FCS_EUNSUPPORTED. */
FCS_API fcs_status fcs_plan_create(const fcs_plan_desc *desc, fcs_plan_t *out);

/* Plan of the higher-order count sketch of Definition 3 (the comparison
 * sketch of Section 2.2): HCS(T)[j_0, ..., j_{N-1}] sums S T over the
 * multi-indices with h_n(i_n) = j_n for every n, a J_0 x ... x J_{N-1}
 * tensor.  Its hash pairs are those of the sketch plan with the same
 * description (same seed, I_n and J_n), with h_n scaled by the mixed-radix
 * stride prod_{m<n} J_m: then sum_n h_n(i_n) is the flattened index of
 * (h_0(i_0), ..., h_{N-1}(i_{N-1})) with mode 0 fastest, and every call that
 * takes a plan computes the higher-order count sketch instead, flattened to
 * J~ = prod_n J_n entries: fcs_sketch_dense / _coo for general tensors,
 * fcs_sketch_cp for CP tensors (the outer products of the rank-1 form are
 * exactly the linear convolution of the scaled mode sketches),
 * fcs_decompress (entry = S HCS[h_0, ..., h_{N-1}], median over D),
 * fcs_contract_inner.  fcs_plan_export returns the scaled hash values.
 * Errors: as fcs_plan_create; FCS_EUNSUPPORTED when prod_n J_n >= 2^31 - 1. */
FCS_API fcs_status fcs_plan_create_hcs(const fcs_plan_desc *desc, fcs_plan_t *out);

/* Bytes of device memory fcs_plan_bind needs for hash and twiddle tables. */
FCS_API size_t fcs_plan_table_bytes(fcs_plan_t plan);

/* Fill the plan's tables into caller device memory `dev_tables` (at least
 * fcs_plan_table_bytes bytes, 256-byte aligned) on `stream`, and attach that
 * memory to the plan.  The buffer must stay allocated and unmodified while
 * the plan is used.  Hash pairs: for sketch d and mode n,
 *   key = mix(mix(seed) + d * 2^16 + n),  y = mix(key + i),
 *   h_n(i) = ((y >> 32) * J_n) >> 32,     s_n(i) = (y & 1) ? -1 : +1,
 * where mix is the SplitMix64 output function (Steele, Lea, Flood 2014);
 * the paper asks only for 2-wise independent pairs (Definitions 1-4).
 * Layout of the tables (each part starting at a 256-byte boundary): the
 * packed hash words, uint32 [D][sum_n I_n] (bit 31 = sign s = -1, bits
 * 0..30 = h_n(i)); the twiddles exp(-2 pi i k / P), float2 [P]; the
 * twiddles exp(-2 pi i k / L), float2 [L]; then the inverse hash lists.
 * Twiddles are evaluated in single precision (exact integer reduction of
 * the angle to an octant, sincospif there; about 1.5 ulp at worst, exact
 * at the quarter turns).
 * Errors: FCS_EINVAL (null or misaligned buffer), FCS_EDEVICE. */
FCS_API fcs_status fcs_plan_bind(fcs_plan_t plan, void *dev_tables, void *stream);

/* Copy hash pair (h_n, s_n) of sketch d from the bound device tables to host
 * arrays h_host[I_n] and s_host[I_n].  Synchronises `stream`.
 * Errors: FCS_EINVAL (unbound plan, d or n out of range), FCS_EDEVICE. */
FCS_API fcs_status fcs_plan_export(fcs_plan_t plan, int32_t d, int32_t n,
                           int32_t *h_host, int8_t *s_host, void *stream);

/* Lane order of the dense scatter (a performance detail of fcs_sketch_dense,
 * exposed for inspection and tests; host computation, no device use, on a
 * created plan, bound or not).  The dense kernel adds the sketches in groups
 * of *group_size and streams rows of mode 0 in 256-column segments, one wave
 * of 64 lanes per segment, each lane holding one 16-byte block (4 columns).
 * For group g, segment s and lane l, out[(g * segs + s) * 64 + l] is the
 * block that lane loads within the segment's set of 4 segments (1024
 * columns), where segs = ceil(I_0 / 256); the blocks of a set are a
 * permutation over its waves, chosen to spread the LDS banks of the
 * group's bins.  fcs_plan_dense_order_bytes gives the size of `out` (0 when
 * the plan keeps the plain order); group_size may be NULL.
 * Errors: FCS_EINVAL (null plan or output, `bytes` too small). */
FCS_API size_t fcs_plan_dense_order_bytes(fcs_plan_t plan);
FCS_API fcs_status fcs_plan_dense_order(fcs_plan_t plan, uint8_t *out, size_t bytes, int32_t *group_size);

/* Sizes of the plan: J~ (sketch length), L = Q * P (transform length), P
 * (FFT size) and Q (number of length-P slices of the transform).  Any output
 * pointer may be NULL. */
FCS_API fcs_status fcs_plan_info(fcs_plan_t plan, int64_t *Jtilde, int64_t *L,
                         int64_t *P, int32_t *Q);

/* Number of spectrum entries (complex) per sketch in the `spec` layout used
 * by fcs_sketch_cp, fcs_sketch_spectrum and fcs_contract_free_mode:
 * (floor(Q/2) + 1) * P.  spec[d][q][k] = X_d[Q*k + q], X_d the L-point DFT
 * (unnormalised, e^{-2 pi i jk/L}) of sketch d zero-padded to L, for
 * q = 0..floor(Q/2), k = 0..P-1; the other frequencies follow from X_d being
 * the transform of a real sequence. */
FCS_API int64_t fcs_plan_spec_len(fcs_plan_t plan);

/* Release a plan (host memory only; the caller still owns dev_tables). */
FCS_API fcs_status fcs_plan_destroy(fcs_plan_t plan);

/* Workspace operations. */
enum {
    FCS_OP_DENSE = 0,        /* fcs_sketch_dense                            */
    FCS_OP_COO = 1,          /* fcs_sketch_coo                              */
    FCS_OP_CP = 2,           /* fcs_sketch_cp with rank R                   */
    FCS_OP_INNER = 3,        /* fcs_contract_inner                          */
    FCS_OP_FREE_MODE = 4,    /* fcs_contract_free_mode with P pairs         */
    FCS_OP_SPECTRUM = 5,     /* fcs_sketch_spectrum                         */
    FCS_OP_KRON = 6,         /* fcs_sketch_kron                             */
    FCS_OP_CONTRACTION = 7,  /* fcs_sketch_contraction, R = shared length   */
    FCS_OP_FULL = 8          /* fcs_contract_full with P tuples             */
};

/* Device workspace bytes an operation needs (R: CP rank, or the shared index
 * length of a contraction; P: vector pairs; ignored where irrelevant).  Returns 0 for an invalid operation. */
FCS_API size_t fcs_workspace_bytes(fcs_plan_t plan, int32_t op, int64_t R, int64_t P);

/* Dense sketch, general-tensor formula of Section 3.2, all D sketches in one
 * pass over T.
 *   T    device, float, prod_n I_n entries in vec order (mode 0 fastest)
 *   out  device, float, D x J~ row-major; overwritten
 *   ws   device workspace of ws_bytes >= fcs_workspace_bytes(FCS_OP_DENSE),
 *        4-byte aligned.  On return (stream order) its first two 32-bit
 *        words count the row blocks that were redone in the exact pass
 *        (first launch pass: full groups of sketches, second: the tail
 *        group); the rest is scratch.
 * Precision: each row block is sketched first in 32-bit fixed point at a
 * scale from its sampled leading rows, and that pass is kept only when no
 * entry left the fixed-point range and the modelled rounding error of every
 * sketch window is at most 3e-6 of the window's norm (at most 5.2e-6 in
 * the worst case over the rounding, in expectation over the hash signs).
 * Otherwise the block is redone at a scale from its own root mean square,
 * which bounds the expected relative error by 2^-18 (3.8e-6) of the
 * block's 2-norm for any finite input; entries far above the root mean
 * square are then added as float atomics, and NaN / Inf propagate.  Float
 * sums are accumulated in a scheduling-dependent order, so results may
 * differ between runs by rounding; integer-valued inputs whose partial sums
 * stay below 2^24 are exact.  Errors: FCS_EINVAL, FCS_ENOMEM, FCS_EDEVICE. */
FCS_API fcs_status fcs_sketch_dense(fcs_plan_t plan, const float *T, float *out,
                            void *ws, size_t ws_bytes, void *stream);

/* COO sketch: the same formula over nnz coordinates; repeated coordinates
 * add (the sketch is linear).
 *   idx  device, int32, N x nnz mode-major (idx[n*nnz + k] = i_n of entry k),
 *        each in [0, I_n)
 *   val  device, float, nnz values
 *   out  device, float, D x J~; overwritten
 * nnz = 0 gives a zero sketch.  Indices are trusted: out-of-range indices
 * are undefined behaviour (validate on the host if they are untrusted).
 * Precision: an entry is summed in 32-bit fixed point (with every wrap of a
 * bin carried exactly) only when rounding moves it by at most 2^-17 of its
 * own magnitude; other entries are added as float atomics, so the expected
 * relative error from rounding is at most 2^-17 (7.6e-6) for any input.
 * Errors: FCS_EINVAL, FCS_ENOMEM, FCS_EDEVICE. */
FCS_API fcs_status fcs_sketch_coo(fcs_plan_t plan, int64_t nnz, const int32_t *idx,
                          const float *val, float *out, void *ws,
                          size_t ws_bytes, void *stream);

/* CP sketch, Section 3.1: per-mode count sketch of every factor column,
 * zero-padded L-point FFT, mode-wise product, sum over the R ranks weighted
 * by lambda, inverse FFT, truncation to J~.
 *   R       rank >= 0 (R = 0 gives a zero sketch)
 *   U       host array of N device pointers; U[n] is the I_n x R factor
 *           stored column-major (column r is U[n][r*I_n .. r*I_n + I_n))
 *   lambda  device, float, R weights, or NULL for all ones
 *   out     device, float, D x J~; overwritten (may be NULL if spec is set)
 *   spec    device, float2 (re, im), D x fcs_plan_spec_len, or NULL; receives
 *           the spectrum of each sketch in the layout of fcs_plan_spec_len
 *   ws      device workspace of at least fcs_workspace_bytes(FCS_OP_CP, R)
 *           bytes: chunk partial spectra, slice terms and the maxima
 *           max_i |U_n(i, r)| of the factor columns
 * Precision: a count sketch of hash length J_n <= P is summed exactly in
 * 64-bit fixed point scaled to its column maximum (each entry truncated by
 * less than 2^(ceil(log2 I_n) - 61) times that maximum), then rounded once
 * to float; a column holding NaN or Inf is summed in float instead.  Longer
 * hashes (folded onto P positions) are float sums in bucket order.  The
 * transforms, products and rank sums are float.
 * Errors: FCS_EINVAL, FCS_ENOMEM, FCS_EUNSUPPORTED, FCS_EDEVICE. */
FCS_API fcs_status fcs_sketch_cp(fcs_plan_t plan, int64_t R, const float *const *U,
                         const float *lambda, float *out, float *spec,
                         void *ws, size_t ws_bytes, void *stream);

/* Allocation-free variant of fcs_sketch_cp, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, results and
 * errors as fcs_sketch_cp except the workspace: the chunk partial spectra,
 * slice terms and column maxima live in a device array of FCS_NOALLOC_SCRATCH_BYTES
 * inside the library (one per device, held until the process ends).  When
 * the partials of fcs_sketch_cp's rank chunks would not fit, fewer chunks
 * are used (the rank sums then group differently, a rounding-level
 * difference); a call whose slice terms and column maxima exceed the array fails with
 * FCS_ENOMEM before anything is enqueued.  The call makes no allocation.
 * All calls on one device share its array: calls that overlap on a device
 * (concurrent streams or threads) race and must be serialised by the
 * caller. */
#define FCS_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
FCS_API fcs_status fcs_sketch_cp_noalloc(fcs_plan_t plan, int64_t R, const float *const *U,
                                 const float *lambda, float *out, float *spec, void *stream);

/* Kronecker product compression, Section 4.3: the FCS of A (x) B viewed as
 * the order-4 tensor T[i0, i1, i2, i3] = A[i0, i1] B[i2, i3] (modes of the
 * plan: 0, 1 index A, 2, 3 index B).  Computed as the linear convolution of
 * the order-2 sketches of A and B (FCS is a convolution of mode sketches),
 * each summed exactly in 64-bit fixed point from the float entries (the
 * largest magnitude of a matrix maps into [2^(B-1), 2^B) with
 * B = min(40, 62 - ceil(log2 of its entry count)), so rounding moves the
 * sketch by at most sqrt(entries) 2^-B of its norm), then transformed,
 * multiplied and inverted in float.  Bins that do not fit in LDS (more than
 * about 20000) are kept in the workspace; a matrix with at most four
 * entries per bin on average is then summed with float atomics instead (a
 * bin's few entries in an order that is not fixed).  A plan with more than
 * two stored slices (Q > 4) computes the sketch as fcs_sketch_contraction
 * with Lc = 1, whose tiles spread the slices over workgroups.
 *   plan  order-4 plan
 *   A     device, float, I_0 x I_1 column-major (vec(A))
 *   B     device, float, I_2 x I_3 column-major
 *   out   device, float, D x J~; overwritten (may be NULL if spec is set)
 *   spec  device, float2, D x fcs_plan_spec_len, or NULL
 *   ws    device workspace of ws_bytes >= fcs_workspace_bytes(FCS_OP_KRON)
 * A matrix with a non-finite entry gives a NaN sketch.
 * Errors: FCS_EINVAL, FCS_ENOMEM, FCS_EUNSUPPORTED, FCS_EDEVICE. */
FCS_API fcs_status fcs_sketch_kron(fcs_plan_t plan, const float *A, const float *B,
                           float *out, float *spec, void *ws, size_t ws_bytes,
                           void *stream);

/* Full contraction T(v_0, ..., v_{N-1}), a vector at every mode, for P
 * vector tuples at once (Section 4.1; T(u,u,u) of the power method).  Per
 * sketch d, est_{d,p} = <y_d, FCS_d(v_{0,p} o ... o v_{N-1,p})>, the
 * inner-product estimate of Proposition 1 with a rank-1 tensor, evaluated
 * from the spectra by Parseval without forming the rank-1 sketch:
 * (1/L) times the sum over the transform of X_d conj(prod_n F(CS_n(v_n)))
 * (float products, sums in double); out[p] = median over d (mean of the
 * middle pair for even D).
 *   spec   device, float2, D x fcs_plan_spec_len (fcs_sketch_cp or
 *          fcs_sketch_spectrum of the sketched tensor)
 *   P      number of vector tuples >= 0 (P = 0 does nothing)
 *   vecs   host array of N device pointers, vecs[n] P x I_n row-major float
 *   out    device, double, P medians
 *   per_d  device, double, P x D per-sketch estimates, or NULL; when NULL,
 *          ws of ws_bytes >= fcs_workspace_bytes(FCS_OP_FULL, 0, P) holds
 *          them (8-byte aligned)
 * Errors: FCS_EINVAL, FCS_ENOMEM, FCS_EUNSUPPORTED, FCS_EDEVICE. */
FCS_API fcs_status fcs_contract_full(fcs_plan_t plan, const float *spec, int64_t P,
                                     const float *const *vecs, double *out, double *per_d,
                                     void *ws, size_t ws_bytes, void *stream);

/* Tensor contraction compression, Section 4.3: the FCS of
 * C[i0, i1, i2, i3] = sum_l A[i0, i1, l] B[l, i2, i3] without forming C.  By
 * linearity it is the sum over l of the Kronecker-product sketches of the
 * slices A(:,:,l) and B(l,:,:); the spectra of the slice products are summed
 * over l before one inverse transform per slice.  Each slice's order-2
 * sketch is summed as in fcs_sketch_kron.
 *   plan  order-4 plan; modes 0, 1 index A's first two modes, 2, 3 B's last
 *         two
 *   Lc    length of the shared index, 1 .. 2^20 (Lc = 1: the Kronecker
 *         product of A(:,:,0) and B(0,:,:))
 *   A     device, float, I_0 x I_1 x Lc column-major (mode 0 fastest)
 *   B     device, float, Lc x I_2 x I_3 column-major (the shared index
 *         fastest, so each slice B(l,:,:) is read with stride Lc)
 *   out   device, float, D x J~; overwritten (may be NULL if spec is set)
 *   spec  device, float2, D x fcs_plan_spec_len, or NULL
 *   ws    device workspace of ws_bytes >=
 *         fcs_workspace_bytes(FCS_OP_CONTRACTION, R = Lc), 16-byte aligned
 * A slice with a non-finite entry gives a NaN sketch.
 * Errors: FCS_EINVAL, FCS_ENOMEM, FCS_EUNSUPPORTED, FCS_EDEVICE. */
FCS_API fcs_status fcs_sketch_contraction(fcs_plan_t plan, int64_t Lc, const float *A,
                                          const float *B, float *out, float *spec, void *ws,
                                          size_t ws_bytes, void *stream);

/* Decompression, Section 4.3 (the rule stated there for the Kronecker
 * product and the contraction, applied at any order): per sketch d, entry i
 * of the recovered tensor is S_d(i) y_d[H_d(i)] with H_d = sum_n h_n(i_n)
 * and S_d = prod_n s_n(i_n); out holds the median over the D sketches (mean
 * of the middle pair for even D, formed in double and rounded once), so for
 * odd D every entry equals one of its D estimates exactly.
 *   y      device, float, D x J~ finite sketches of this plan
 *   order  host array of N mode indices, the output's layout from the
 *          fastest-varying mode outwards, or NULL for vec order (0, 1, ...,
 *          N-1).  A (x) B of fcs_sketch_kron as the (I_0 I_2) x (I_1 I_3)
 *          column-major matrix is order = {2, 0, 3, 1}
 *   out    device, float, prod_n I_n entries; overwritten (16-byte
 *          alignment and I_order[0] % 4 == 0 give vector stores)
 * The call allocates nothing and needs no workspace.  D <= 32, every I_n
 * < 2^31.
 * Errors: FCS_EINVAL (null pointer, misalignment, order not a permutation),
 * FCS_EUNSUPPORTED (D > 32, sizes out of range), FCS_EDEVICE. */
FCS_API fcs_status fcs_decompress(fcs_plan_t plan, const float *y, const int32_t *order,
                                  float *out, void *stream);

/* Spectrum of existing sketches (for contractions of dense or COO sketches):
 *   y     device, float, D x J~
 *   spec  device, float2, D x fcs_plan_spec_len; overwritten
 * Errors: FCS_EINVAL, FCS_ENOMEM, FCS_EUNSUPPORTED, FCS_EDEVICE. */
FCS_API fcs_status fcs_sketch_spectrum(fcs_plan_t plan, const float *y, float *spec,
                               void *ws, size_t ws_bytes, void *stream);

/* Sketched inner product, Proposition 1 and Section 4: per sketch d,
 * ip_d = sum_j a[d][j] b[d][j] (float inputs, products and sums in double),
 * and the median over d (mean of the two middle values for even D).
 *   a, b    device, float, D x J~ (sketches from the same plan)
 *   median  device, double, 1 value
 *   per_d   device, double, D values, or NULL
 * Errors: FCS_EINVAL, FCS_ENOMEM, FCS_EDEVICE. */
FCS_API fcs_status fcs_contract_inner(fcs_plan_t plan, const float *a, const float *b,
                              double *median, double *per_d, void *ws,
                              size_t ws_bytes, void *stream);

/* The same for any D sketches of `len` entries each (a, b: D x len, e.g.
 * tensor sketches from fcs_ts_fold); ws needs 8 D bytes (rounded up to 256)
 * when per_d is NULL.  Errors: FCS_EINVAL, FCS_ENOMEM, FCS_EDEVICE. */
FCS_API fcs_status fcs_inner_median(int32_t D, int64_t len, const float *a, const float *b,
                            double *median, double *per_d, void *ws, size_t ws_bytes,
                            void *stream);

/* Tensor sketch of Definition 2 (the comparison sketch of Section 2.2)
 * under the plan's hash pairs, from a fast count sketch y of the same tensor
 * and plan: with every J_n = J the tensor sketch's bin is the fast count
 * sketch's bin modulo J, so ts[d][k] = sum over m = k (mod J) of y[d][m]
 * (Section 3, item 2).  Folds the sketch of any input (dense, COO, CP).
 *   y   device, float, D x J~
 *   ts  device, float, D x J; overwritten
 * Errors: FCS_EINVAL (null pointers, unequal J_n, a higher-order count
 * sketch plan), FCS_EDEVICE. */
FCS_API fcs_status fcs_ts_fold(fcs_plan_t plan, const float *y, float *ts, void *stream);

/* T(I, u, v)-type contraction, Section 4.1: the identity at mode
 * `free_mode` and a vector at every other mode.  For each sketch d and pair
 * p, z = F^-1(X_d prod_{n != free} conj(F(CS_n(v_{n,p})))) and
 * est_{d,p}(i) = s_free(i) z(h_free(i)); out[p][i] = median over d.
 *   spec       device, float2, D x fcs_plan_spec_len (from fcs_sketch_cp or
 *              fcs_sketch_spectrum of the sketched tensor)
 *   free_mode  0..N-1
 *   P          number of vector tuples >= 0
 *   vecs       host array of N device pointers; vecs[free_mode] is ignored
 *              (may be NULL), vecs[n] is P x I_n row-major float
 *   out        device, double, P x I_free row-major
 *   ws         device workspace of at least fcs_workspace_bytes(FCS_OP_FREE_MODE,
 *              0, P) bytes (z, the per-sketch estimates, the vector maxima
 *              and norm exponents)
 * The count sketches of the vectors are formed as in fcs_sketch_cp (64-bit
 * fixed point scaled to each vector's maximum for J_n <= P; two vectors
 * share one transform on the conjugate-symmetric slices).
 * Errors: FCS_EINVAL, FCS_ENOMEM, FCS_EUNSUPPORTED, FCS_EDEVICE. */
FCS_API fcs_status fcs_contract_free_mode(fcs_plan_t plan, const float *spec,
                                  int32_t free_mode, int64_t P,
                                  const float *const *vecs, double *out,
                                  void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Batched uneven sketches: many CP and Kronecker sketch computations, each
 * with its own plan (order, sizes, hash lengths, D, seed), run by persistent
 * kernels (one per FFT size class) that take work tiles from a queue,
 * longest first; fcs_batch_run can capture all of them into one hipGraph
 * and replay it.  Results equal those of fcs_sketch_cp / fcs_sketch_kron on
 * each item alone (up to float summation order).
 * ------------------------------------------------------------------------ */
enum { FCS_ITEM_CP = 0, FCS_ITEM_KRON = 1 };

typedef struct {
    fcs_plan_t plan;          /* bound plan of this item; must outlive the batch */
    int32_t kind;             /* FCS_ITEM_CP or FCS_ITEM_KRON                   */
    int64_t R;                /* CP rank >= 0 (ignored for KRON)                */
    const float *const *U;    /* host array of device pointers: CP: N factors as
                                 for fcs_sketch_cp; KRON: {A, B} as for
                                 fcs_sketch_kron (read when the batch is created) */
    const float *lambda;      /* CP: device, R weights, or NULL for all ones   */
    float *out;               /* device, D x J~, or NULL if spec is set        */
    float *spec;              /* device, float2 D x fcs_plan_spec_len, or NULL */
} fcs_batch_item;

typedef struct {
    int32_t tile_ffts;        /* target forward FFTs per CP tile (ranks x modes);
                                 0 = 32                                          */
    int32_t wg_per_cu[7];     /* persistent workgroups per compute unit for the
                                 FFT sizes 2^8 .. 2^14; 0 = as many as LDS allows
                                 (at most 8)                                    */
    int32_t no_pack[7];       /* per FFT size class: nonzero = one transform per
                                 mode on every slice; 0 = two modes share one
                                 transform on the conjugate-symmetric slices
                                 (q = 0 and, Q even, Q/2), as fcs_sketch_cp    */
} fcs_batch_config;

typedef struct fcs_batch *fcs_batch_t;

/* Host only: validates every item, splits the work into tiles and lays out
 * the workspace.  cfg may be NULL (defaults).  Output and factor pointers
 * are captured here.  Errors: FCS_EINVAL, FCS_EUNSUPPORTED. */
FCS_API fcs_status fcs_batch_create(const fcs_batch_item *items, int64_t count,
                            const fcs_batch_config *cfg, fcs_batch_t *out);

/* Device workspace bytes (descriptors, tile queues, counters, partial
 * spectra, Kronecker factor sketches). */
FCS_API size_t fcs_batch_workspace_bytes(fcs_batch_t batch);

/* Tiles of the batch and the persistent grid of each FFT size class
 * (grids: 7 entries or NULL). */
FCS_API fcs_status fcs_batch_info(fcs_batch_t batch, int64_t *tiles, int32_t *grids);

/* Copies the descriptors and tile lists into ws (device, 256-byte aligned,
 * ws_bytes >= fcs_batch_workspace_bytes) and clears the counters; waits for
 * the copies (synchronises `stream`).  Call again after moving to another
 * workspace.  Errors: FCS_EINVAL, FCS_ENOMEM, FCS_EDEVICE. */
FCS_API fcs_status fcs_batch_prepare(fcs_batch_t batch, void *ws, size_t ws_bytes,
                             void *stream);

/* Computes every item into its out / spec on `stream`.  use_graph != 0
 * captures the launches into a hipGraph on the first call (per workspace)
 * and replays it; 0 launches the class kernels directly.  ws must be the
 * prepared workspace; runs of one batch must not overlap in time.
 * Errors: FCS_EINVAL, FCS_ENOMEM, FCS_EUNSUPPORTED, FCS_EDEVICE. */
FCS_API fcs_status fcs_batch_run(fcs_batch_t batch, void *ws, size_t ws_bytes,
                         int32_t use_graph, void *stream);

FCS_API fcs_status fcs_batch_destroy(fcs_batch_t batch);

/* ---------------------------------------------------------------------------
 * Small dense steps of the decomposition drivers (the robust tensor power
 * method of Section 4.1.1 and alternating least squares of Section 4.1.2),
 * on sketch-sized data, asynchronous on `stream`; norms in double.
 * ------------------------------------------------------------------------- */

/* out[r][:] = in[r][:] / ||in[r][:]||_2 for P rows of n entries (row-major);
 * exactly one of in64 (double) and in32 (float) is given; out is float;
 * norms (device, double, P values) may be NULL.  A zero row stays zero.
 * Errors: FCS_EINVAL, FCS_EDEVICE. */
FCS_API fcs_status fcs_normalize_rows(int64_t P, int64_t n, const double *in64, const float *in32,
                              float *out, double *norms, void *stream);

/* The power method's choice among starts: j = the first index of the
 * largest of vals[0..P) (NaN never wins), then row_out[0..n) = rows[j][:]
 * (rows: P x n float, row-major) and, where given, *val_out = (float)
 * vals[j], *val64_out = vals[j], *index_out = j (all device pointers).
 * Errors: FCS_EINVAL, FCS_EDEVICE. */
FCS_API fcs_status fcs_select_max(int64_t P, const double *vals, int64_t n, const float *rows,
                          float *row_out, float *val_out, double *val64_out,
                          int32_t *index_out, void *stream);

/* y += a x for n floats (deflation of a sketch or spectrum by a rank-1
 * term).  Errors: FCS_EINVAL, FCS_EDEVICE. */
FCS_API fcs_status fcs_axpy(int64_t n, float a, const float *x, float *y, void *stream);

/* One ALS factor update: with G the Hadamard product over the other modes
 * of F_m F_m^T (R x R, double; F_m = others[m], R x Iother[m] float
 * row-major, i.e. the factor's columns as rows), solve G X = Mt (Mt: R x In
 * double, the mode's unfolding times the Khatri-Rao product of the other
 * factors, transposed) by Cholesky, then lam[r] = ||X[r][:]||_2 and
 * Ft_out[r][:] = X[r][:] / lam[r] (float, R x In).  ws: device workspace of
 * fcs_als_workspace_bytes(R, In) bytes.  G must be positive definite (a
 * non-positive pivot gives NaN outputs).  Errors: FCS_EINVAL, FCS_ENOMEM,
 * FCS_EUNSUPPORTED (R > 90), FCS_EDEVICE. */
FCS_API size_t fcs_als_workspace_bytes(int32_t R, int64_t In);
FCS_API fcs_status fcs_als_update(int32_t R, int64_t In, const double *Mt, int32_t nother,
                          const float *const *others, const int64_t *Iother, float *Ft_out,
                          double *lam, void *ws, size_t ws_bytes, void *stream);

/* Measurement probe, not an operation of the paper: the cost of the LDS
 * atomics of the dense scatter (Section 3.2) alone, for comparison with
 * fcs_sketch_dense on the same grid.  `blocks` workgroups of 1024 threads
 * each add rows x 1024 columns x 4 windows of ones into four LDS windows of
 * `window` 32-bit bins, bin h_d(c) + o_d(row) of window d, with 32-bit LDS
 * atomics and no other memory traffic: h_d(c) in [0, span) from a counter
 * hash of `seed` (pattern 0: random column bins, the bank conflicts of
 * random hashes) or the 64 lanes of every atomic on consecutive bins
 * (pattern 1: no bank conflicts); o_d(row) in [0, window - span],
 * wave-uniform.  Every workgroup writes the sum of its bins, rows * 4096, to
 * sink[block] (device, `blocks` uint32).  Asynchronous on `stream`.
 * Errors: FCS_EINVAL (blocks < 1, rows outside [1, 2^20), pattern not 0 or
 * 1, span < 1024, span > window, window > FCS_PROBE_MAX_WINDOW, null sink),
 * FCS_EDEVICE. */
FCS_API fcs_status fcs_probe_lds_atomics(int32_t blocks, int32_t rows, int32_t window, int32_t span,
                                 int32_t pattern, uint32_t seed, uint32_t *sink, void *stream);

/* Text of a status code (static storage). */
FCS_API const char *fcs_status_str(fcs_status status);

/* Description of the last error raised on the calling thread (static or
 * thread-local storage; empty when the last call succeeded). */
FCS_API const char *fcs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FCS_H */
