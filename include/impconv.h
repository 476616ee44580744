/*
 * impconv.h -- C ABI of libimpconv: implicitly dealiased convolutions on
 * AMD Instinct MI355X (gfx950).
 *
 * The operations are those of J. C. Bowman and M. Roberts, "Efficient
 * dealiased convolutions without padding" (SIAM J. Sci. Comput., 2011):
 * linear (non-cyclic) convolution sums computed from size-N FFTs of
 * residue-split, twiddle-shifted subsequences instead of from explicitly
 * zero-padded size-2N (complex, 1/2 rule) or size-3N (centered Hermitian,
 * 2/3 rule) transforms.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Data pointers (f, g, e, h, work) are DEVICE pointers owned by the caller.
 *   Complex values are interleaved (re, im): complex64 = 2 x float,
 *   complex128 = 2 x double (the layout of torch.complex64/complex128).
 *   Arrays are C-contiguous, last axis stride 1.
 * - The result is the exact (unnormalized) convolution sum, as defined per
 *   entry point below; only the summation order differs from the definition.
 * - Work arrays are separate from the data and provided by the caller
 *   (Sec. 1: decoupling data and work memory); query their size with the
 *   *_workspace functions.  A size of 0 means work may be NULL.
 * - All work is enqueued on `stream` (a hipStream_t; NULL = default stream).
 *   Nothing synchronizes; device-side faults surface at the caller's next
 *   synchronization.
 * - Inputs are read only.  The output h may be an input itself (h == f, g
 *   or e) when the two arrays have the same extent, e.g. M = 1: the paper's
 *   in-place form (an input given as h is overwritten by the result).  Any
 *   other overlap of h with an input is IMPCONV_E_ARG.
 * - The library allocates no data-sized memory.  On first use on a device it
 *   allocates ~12 MB of twiddle tables (impconv_init); call impconv_init()
 *   outside any stream capture before capturing calls into a hipGraph.
 * - Every argument check happens on the host before any launch.  Errors:
 *     IMPCONV_E_ARG        null pointer, bad kind/dtype/flags, overlapping h
 *     IMPCONV_E_SIZE       m < 1, batch < 0, M < 1, bad storage extents
 *     IMPCONV_E_WORKSPACE  work_bytes smaller than the queried size
 *     IMPCONV_E_ALIGN      pointer not aligned to its complex element size
 *     IMPCONV_E_UNSUPPORTED a size beyond what this build implements
 *     IMPCONV_E_HIP        a HIP call failed (text in impconv_last_error())
 *   No exception crosses the ABI.  impconv_last_error() is thread-local.
 * - Any m >= 1 is accepted.  The kernels use FFT sizes N = the next power of
 *   two >= m (even N for the Hermitian rule); inputs read as zero beyond m,
 *   which leaves every output k < m unchanged.
 */
#ifndef IMPCONV_H
#define IMPCONV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum impconv_status {
    IMPCONV_OK = 0,
    IMPCONV_E_ARG = 1,
    IMPCONV_E_SIZE = 2,
    IMPCONV_E_WORKSPACE = 3,
    IMPCONV_E_ALIGN = 4,
    IMPCONV_E_UNSUPPORTED = 5,
    IMPCONV_E_HIP = 6
} impconv_status;

typedef enum impconv_dtype { IMPCONV_C64 = 0, IMPCONV_C128 = 1 } impconv_dtype;

typedef enum impconv_kind {
    IMPCONV_COMPLEX = 0,   /* origin at index 0, 1/2 padding rule (Sec. 2.1, 3.1, 3.4) */
    IMPCONV_HERMITIAN = 1, /* centered Hermitian, 2/3 padding rule (Sec. 2.3, 3.2, 3.4) */
    IMPCONV_TERNARY = 2    /* centered Hermitian ternary (Sec. 4) */
} impconv_kind;

/* Flag bits. */
#define IMPCONV_EXPLICIT_PADDED (1u << 0) /* comparator: explicitly zero-padded FFT convolution */
#define IMPCONV_REV_F (1u << 1)           /* complex 1D: read f reversed, f'_k = f_{m-1-k} */
#define IMPCONV_CONJ_G (1u << 2)          /* complex 1D: read g conjugated */
#define IMPCONV_REV_OUT (1u << 3)         /* complex 1D: write h reversed */
#define IMPCONV_NO_SYMMETRIZE (1u << 4)   /* Hermitian nD: trust the k_last = 0 plane (see conv2d) */
#define IMPCONV_HERMITIAN_ADJOINT (1u << 5) /* Hermitian 1D/nD: vector-Jacobian product edits (see below) */
#define IMPCONV_EXPLICIT_PRUNED (1u << 6) /* with EXPLICIT_PADDED: skip all-zero transforms, fuse padding */
#define IMPCONV_COMPENSATED (1u << 7)     /* complex64 complex convolutions: compensated twiddle products */
#define IMPCONV_ONE_STREAM (1u << 8)      /* ragged batches, 3D: every launch in order on `stream` alone */

/* Version as 10000*major + 100*minor + patch. */
int impconv_version(void);

/* Static description of a status code. */
const char* impconv_status_string(int status);

/* Text of the last error raised on the calling thread ("" if none). */
const char* impconv_last_error(void);

/* Create the twiddle tables of the current HIP device and resolve the
 * device address of the work memory of impconv_conv2d_noalloc there
 * (idempotent, thread-safe, synchronous).  Every other entry point calls the
 * table part implicitly; impconv_conv2d_noalloc requires it to have run on
 * its device. */
impconv_status impconv_init(void);

/* ----------------------------------------------------------------------
 * 1D convolutions.  Layout: f, g are [batch][M][m], h is [batch][m]; the
 * M axis is the dot-product width of Sec. 3.3 (f*g read as sum_i f_i*g_i).
 * work may be NULL when impconv_conv1d_workspace reports 0 bytes.
 * ---------------------------------------------------------------------- */

/* Workspace bytes for a 1D call of the given kind (flags as for the call). */
impconv_status impconv_conv1d_workspace(int kind, int dtype, int64_t batch, int64_t M, int64_t m,
                                        uint32_t flags, size_t* bytes);

/* Complex 1D convolution, Sec. 2.1 (fftpadBackward / fftpadForward / cconv):
 *   h_k = sum_{i<M} sum_{p=0}^{k} f'_{i,p} g'_{i,k-p},   k = 0..m-1,
 * with f' = f (or f reversed under IMPCONV_REV_F) and g' = g (or conj g under
 * IMPCONV_CONJ_G); IMPCONV_REV_OUT stores h_{m-1-k} at index k.  These three
 * flags express the adjoint: dL/df = REV_OUT(conv(REV_F(dL/dh), CONJ_G(g))).
 * With IMPCONV_EXPLICIT_PADDED the same sum is computed by the conventional
 * method (inputs copied zero-padded to 2N in work, size-2N cyclic FFT
 * convolution, output cropped); REV/CONJ flags are not accepted with it.
 * With IMPCONV_EXPLICIT_PRUNED as well, the padding is fused into the loads
 * instead (one size-2N cyclic convolution per row reads f and g, zero beyond
 * m, and writes the first m outputs; no workspace).
 * The implicit method takes the general p/q rule of Sec. 2.4 where it needs
 * clearly fewer transforms (see impconv_conv1d_complex_pq).  Lengths whose
 * power-of-two size exceeds 8192 otherwise run as three passes (column FFTs,
 * row convolutions, column FFTs); the first such call for a given size
 * creates that size's column twiddle table (synchronously, outside any
 * graph capture).
 * IMPCONV_COMPENSATED (implicit method, m <= 8192): in complex64 every
 * product by a root of unity -- residue shifts, FFT stage twiddles,
 * recombination -- is formed from the FP32 rounding h of the FP64 value and
 * the FP32 rounding l of the remainder, a h + a l, which removes the
 * twiddles' own representation error (at about twice the cost of each
 * twiddle product); the 1/2 rule is used.  No effect in complex128. */
impconv_status impconv_conv1d_complex(int dtype, int64_t batch, int64_t M, int64_t m,
                                      const void* f, const void* g, void* h, void* work,
                                      size_t work_bytes, uint32_t flags, void* stream);

/* Complex 1D convolution (the sum above) with the general p/q padding of
 * Sec. 2.4: the inputs, zero beyond m, are taken as P = ceil(m / np) blocks
 * of np values and implicitly padded to q np with q = ceil((2m - 1) / np),
 * q np >= 2m - 1, so that no cyclic wrap-around reaches k < m; q residue
 * transforms of size np per input replace the two of size 2^ceil(log2 m) of
 * the 1/2 rule.  np: a power of two with P in {2, 3} and np <= 4096
 * (complex64) or 2048 (complex128); np >= m (power of two <= 8192) runs the
 * 1/2 rule at size np; np = 0 the automatic choice of impconv_conv1d_complex,
 * which takes the p/q rule wherever its transform volume is clearly smaller
 * (m up to 12288 / 6144 in one pass); np = 2^ceil(log2 m) above 8192 the
 * multi-pass 1/2 rule.  Flags as for impconv_conv1d_complex (not
 * IMPCONV_EXPLICIT_PADDED).  Workspace: impconv_conv1d_complex_pq_workspace
 * (0 except for the multi-pass rule).  Other np: E_SIZE. */
impconv_status impconv_conv1d_complex_pq(int dtype, int64_t batch, int64_t M, int64_t m, int64_t np,
                                         const void* f, const void* g, void* h, void* work,
                                         size_t work_bytes, uint32_t flags, void* stream);

impconv_status impconv_conv1d_complex_pq_workspace(int dtype, int64_t batch, int64_t M, int64_t m, int64_t np,
                                                   size_t* bytes);

/* The rule impconv_conv1d_complex takes for length m: *np = 0 for the 1/2
 * rule at N = 2^ceil(log2 m) (*p = 1, *q = 2), else the p/q block size,
 * blocks and residues. */
impconv_status impconv_conv1d_complex_rule(int dtype, int64_t m, int64_t* np, int* p, int* q);

/* Centered Hermitian 1D convolution, Sec. 2.3 (2/3 rule, Fourier size 3N):
 * f, g hold the non-negative wavenumbers 0..m-1 of fields with
 * U_{-k} = conj U_k; Im f_0 and Im g_0 are ignored.
 *   h_k = sum_{i<M} sum_{p=k-m+1}^{m-1} f_{i,p} g_{i,k-p},   k = 0..m-1.
 * IMPCONV_EXPLICIT_PADDED: conventional comparator (half spectra copied into
 * a real-FFT buffer of size 2^ceil(log2(3m-2)), physical-space product).
 * IMPCONV_HERMITIAN_ADJOINT gives the vector-Jacobian product: for a real
 * loss L of h and gh = dL/dRe h + i dL/dIm h, the gradient with respect to
 * the stored half of f is conv1d_hermitian(gh', g) with gh'_0 = 2 Re gh_0 and
 * its entry 0 halved and real (the coupling f_{-p} = conj f_p folds the
 * negative wavenumbers into the positive ones); this flag applies exactly
 * those two edits, on load of the first input and on store.  Not accepted
 * with IMPCONV_EXPLICIT_PADDED. */
impconv_status impconv_conv1d_hermitian(int dtype, int64_t batch, int64_t M, int64_t m,
                                        const void* f, const void* g, void* h, void* work,
                                        size_t work_bytes, uint32_t flags, void* stream);

/* Centered Hermitian ternary 1D convolution, Sec. 4 (Fourier size 4N):
 * f, g, e are [batch][m] Hermitian halves (Im of entry 0 ignored);
 *   h_k = sum_{p,q,r in [-m+1, m-1], p+q+r=k} f_p g_q e_r,   k = 0..m-1.
 * IMPCONV_EXPLICIT_PADDED: conventional comparator (half spectra copied into
 * real-FFT buffers of length 2^ceil(log2(4m-3)), physical-space triple
 * product; m <= 4096). */
impconv_status impconv_conv1d_ternary(int dtype, int64_t batch, int64_t m, const void* f,
                                      const void* g, const void* e, void* h, void* work,
                                      size_t work_bytes, uint32_t flags, void* stream);

/* Profiling mode (off by default; not for use under stream capture): when
 * enabled, every kernel launch of the library is bracketed by two hipEvents
 * on its stream.  impconv_timing_report waits for them, writes a JSON array
 * of per-kernel aggregates {"name","count","total_ms","min_ms","max_ms"} to
 * buf (NUL-terminated, truncated to cap bytes), clears the records and
 * returns the length of the full report. */
void impconv_timing_enable(int on);
size_t impconv_timing_report(char* buf, size_t cap);

/* ----------------------------------------------------------------------
 * 2D / 3D convolutions (Secs. 3.1-3.4).  m[d] = logical modes per axis,
 * n[d] = storage extent per axis.  f, g are [batch][M][n0][n1](...[n2]),
 * h is [batch][n0][n1](...[n2]).
 *   IMPCONV_COMPLEX:   n[d] = m[d];  h_k = sum_i sum_{0<=p<=k} f_{i,p} g_{i,k-p}
 *                      for 0 <= k_d < m_d (componentwise).
 *   IMPCONV_HERMITIAN: leading axes centered, n[d] in {2m[d]-1, 2m[d]},
 *                      wavenumber k at index k + n[d] - m[d] (with n = 2m the
 *                      index-0 slot is a zero slot); last axis = Hermitian
 *                      half, n in {m, m+1}, wavenumber k at index k (index m
 *                      a zero slot).  h_k = sum_i sum_{p in B, k-p in B}
 *                      f_{i,p} g_{i,k-p} over the box B = prod [-m_d+1, m_d-1],
 *                      k_last >= 0, the full fields defined by
 *                      U_{-k} = conj U_k.  The k_last = 0 hyperplane is made
 *                      Hermitian on load (concluding remarks of the paper):
 *                      its authoritative half is the one whose first nonzero
 *                      leading wavenumber is positive, the other half is read
 *                      as its conjugate mirror and the origin as real.  With
 *                      IMPCONV_NO_SYMMETRIZE the plane is read as its
 *                      Hermitian projection (U_k + conj U_{-k}) / 2 instead
 *                      (identical for already-symmetric input).  Zero slots
 *                      of h are written as 0.
 * IMPCONV_COMPLEX also accepts IMPCONV_REV_F / IMPCONV_CONJ_G /
 * IMPCONV_REV_OUT as in 1D, each reversal applying to every axis within
 * m[d] (the adjoint: dL/df = REV_OUT(conv(REV_F(dL/dh), CONJ_G(g)))).
 * IMPCONV_HERMITIAN accepts IMPCONV_HERMITIAN_ADJOINT (not with
 * IMPCONV_NO_SYMMETRIZE or IMPCONV_EXPLICIT_PADDED), the vector-Jacobian
 * product: for a real loss L of h and gh = dL/dRe h + i dL/dIm h, the
 * gradient with respect to the stored half of f is the Hermitian
 * convolution of Gamma with g, where Gamma = gh off the k_last = 0
 * hyperplane and gh_k + conj gh_{-k} on it (both halves), followed on that
 * hyperplane by zero for the entries the symmetrization overwrites and the
 * origin halved and real.  The flag makes the first outer pass load f as
 * Gamma and the last outer pass apply the edits; pass gh as f.
 * IMPCONV_COMPLEX also accepts IMPCONV_COMPENSATED (implicit method; as in
 * 1D: compensated twiddle products in the complex64 column passes and rows;
 * the column passes then run one workgroup per tile).
 * IMPCONV_HERMITIAN with IMPCONV_EXPLICIT_PADDED (2D and 3D): the
 * conventional 2/3-rule comparator -- every centered axis zero padded to the
 * power of two P >= 3m - 2 (wavenumber k at index k mod P), the last axis to
 * the real length 2 NC >= 3m - 2, full-size complex FFTs along the centered
 * axes, real cyclic products (with the M-dot) along the last axis, inverse
 * FFTs, crop; it reads the k_last = 0 hyperplane as its Hermitian projection
 * (pass symmetric input to compare with the implicit path).  Workspace
 * 2 * batch * M * prod(P) * (NC + 1) complex values; 3m - 2 <= 4096 on the
 * centered axes and <= 16384 on the last.  With IMPCONV_EXPLICIT_PRUNED as
 * well: the same transforms without those of all-zero columns.
 * IMPCONV_EXPLICIT_PADDED (2D complex): the conventional comparator --
 * inputs copied into zero-padded 2N0 x 2N1 work arrays, full-size FFTs along
 * both axes, product, inverse, crop (m[d] <= 2048).  With
 * IMPCONV_EXPLICIT_PRUNED as well: the pruned comparator -- the same padded
 * transform sizes with the zero padding fused into the loads, no transform
 * of an all-zero column and the crop fused into the last store (work
 * 2 * batch * M * 2N0 * m1 complex values).
 * IMPCONV_EXPLICIT_PADDED (3D complex): the same comparator in 3D -- inputs
 * copied into zero-padded 2N0 x 2N1 x 2N2 arrays, full-size FFTs along all
 * three axes, product, inverse, crop (work 2 * batch * M * 8 N0 N1 N2
 * complex values; m0, m1 <= 2048, m2 <= 4096).  With
 * IMPCONV_EXPLICIT_PRUNED: padding fused into the loads, x transforms of the
 * m1 x m2 data columns only, y transforms of the m2 data columns, inverse
 * transforms of the cropped rows only, the last one writing h (work
 * 2 * batch * M * 4 N0 N1 * m2 complex values).
 * 3D: the y backward pass, the rows and the y forward pass run over chunks
 * of the (batch, x residue) planes; the rows and y forward pass of one chunk
 * run on the device's first auxiliary stream (the one of the ragged
 * batches, created once per device) while the caller's stream runs the y
 * backward pass of the next chunk, forked and joined by events (capturable;
 * the same threading caveat as for ragged batches applies).  With
 * IMPCONV_ONE_STREAM every launch runs in order on `stream`, with the same
 * kernels and bitwise the same result.
 * Outer axes support m[d] <= 4096 in this build; the innermost axis
 * m <= 8192 (complex) or m <= 16384 (Hermitian).
 * ---------------------------------------------------------------------- */
impconv_status impconv_convnd_workspace(int kind, int dtype, int ndim, const int64_t* m,
                                        const int64_t* n, int64_t batch, int64_t M,
                                        uint32_t flags, size_t* bytes);

impconv_status impconv_conv2d(int kind, int dtype, int64_t batch, int64_t M, const int64_t* m,
                              const int64_t* n, const void* f, const void* g, void* h,
                              void* work, size_t work_bytes, uint32_t flags, void* stream);

impconv_status impconv_conv3d(int kind, int dtype, int64_t batch, int64_t M, const int64_t* m,
                              const int64_t* n, const void* f, const void* g, void* h,
                              void* work, size_t work_bytes, uint32_t flags, void* stream);

/* Allocation-free form of impconv_conv2d, for callers that cannot allocate
 * device memory: code under hipGraph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, results, flags and errors as
 * impconv_conv2d, without work / work_bytes: the work arrays live in a fixed
 * region of device memory that belongs to the library's device code (one per
 * device, impconv_noalloc_capacity() bytes = 64 MiB, held until the process
 * ends).  The call allocates and frees nothing; it only enqueues kernels on
 * `stream`.
 *  - impconv_init() must have run on the current device first (it resolves
 *    the region's address); otherwise IMPCONV_E_ARG.
 *  - A convolution whose impconv_convnd_workspace exceeds the capacity is
 *    IMPCONV_E_WORKSPACE (e.g. complex64 complex 2D: 4 * batch * M *
 *    2^ceil(log2 m0) * m1 * 8 bytes must be <= 64 MiB).
 *  - Every call on a device shares that device's region and leaves its last
 *    contents there (nothing in the region needs to start at zero: each
 *    kernel writes the work it reads).  Calls that can overlap in time on one
 *    device -- on different streams, or from different threads without
 *    ordering between their streams -- race on the region and give wrong
 *    results: order them on one stream. */
impconv_status impconv_conv2d_noalloc(int kind, int dtype, int64_t batch, int64_t M, const int64_t* m,
                                      const int64_t* n, const void* f, const void* g, void* h,
                                      uint32_t flags, void* stream);

/* Bytes of work memory available to impconv_conv2d_noalloc on each device. */
size_t impconv_noalloc_capacity(void);

/* 2D centered Hermitian ternary convolution, Sec. 4 (tconv2): f, g, e and h
 * are [batch][n0][n1] in the 2D Hermitian storage of impconv_conv2d
 * (x centered, n0 in {2m0-1, 2m0}; y the Hermitian half, n1 in {m1, m1+1}),
 *   h_k = sum_{p, q in B, k-p-q in B} f_p g_q e_{k-p-q},
 * k in B = [-m0+1, m0-1] x [-m1+1, m1-1] with k_y >= 0, the full fields
 * defined by U_{-k} = conj U_k.  The k_y = 0 line is symmetrized on load as
 * in impconv_conv2d (IMPCONV_NO_SYMMETRIZE: its Hermitian projection);
 * zero slots of h are written as 0.  The x axis uses the ternary rule (two
 * residues of the centered transform padded to 4 N0', N0' = 2^ceil(log2 m0),
 * transforms of size 2 N0'), every row the 1D ternary convolution.  Workspace
 * (impconv_convnd_workspace with kind IMPCONV_TERNARY, ndim 2, M = 1):
 * 8 * batch * 2 N0' * n1 complex values.  This build: m0 <= 4096 in
 * complex64, 2048 in complex128; m1 <= 8192; E_UNSUPPORTED beyond.
 * IMPCONV_EXPLICIT_PADDED: the conventional comparator -- f, g, e copied into
 * zero-padded [4 N0'][2 N1' + 1] arrays (x wavenumbers wrapped modulo 4 N0'),
 * full-size complex FFTs along x, real cyclic triple products of length
 * 4 N1' along y, inverse x FFT, crop; it reads the k_y = 0 line as its
 * Hermitian projection (m0 <= 4096 in complex64, 1024 in complex128;
 * m1 <= 4096; workspace
 * 3 * batch * 4 N0' * (2 N1' + 1) complex values).  IMPCONV_EXPLICIT_PRUNED
 * as well: the all-zero columns k_y >= m1 are not transformed. */
impconv_status impconv_conv2d_ternary(int dtype, int64_t batch, const int64_t* m, const int64_t* n,
                                      const void* f, const void* g, const void* e, void* h,
                                      void* work, size_t work_bytes, uint32_t flags, void* stream);

/* ----------------------------------------------------------------------
 * Ragged batch of complex 1D convolutions of uneven lengths (Sec. 2.1 sum
 * per pair).  Pair j has length m_host[j] >= 1 and occupies elements
 * offset_host[j] .. offset_host[j] + m_host[j] - 1 of the packed f, g and h
 * arrays (pairs must not overlap).  The plan copies the descriptors to the
 * device once (synchronously, at creation) and groups pairs by FFT size;
 * executing it launches nothing but kernels, so it may be captured in a
 * hipGraph.  The fused size classes (N <= 8192; complex128: N <= 4096) run
 * together in one persistent launch by default: items of as many pairs of
 * one class as fill a 512-thread workgroup, numbered longest class first,
 * are taken from an atomic counter by one workgroup per compute unit until
 * none is left; the counter occupies the first 256 bytes of the workspace
 * and is cleared by a one-thread kernel at the start of every execution
 * (so work must be 16-byte aligned, and executions that may overlap on the
 * GPU need distinct workspaces).  impconv_ragged_plan_set_fused or the
 * autotuner may choose one launch per class instead.  The size classes
 * (the queue launch counting as one) run concurrently: the device has three
 * auxiliary streams (default priority) and events, created with its first
 * ragged plan and kept until the process ends (shared by all plans of the
 * device); execute forks them from `stream` with an event and joins them
 * back into it -- also when a launch fails part way -- so all work of the
 * call is ordered after what `stream` had queued and before what it queues
 * next; each class with N > 8192 uses a region of the workspace of its own.
 * Calls from several host threads are serialized while they enqueue (a
 * mutex of the plan and one of the device's auxiliary streams); executions
 * that may overlap on the GPU need distinct workspaces.  While one thread
 * captures an execution, no other thread may execute a ragged plan on the
 * same device without IMPCONV_ONE_STREAM (the auxiliary streams are part of
 * the capture until it ends).  Only impconv_ragged_plan_autotune and
 * impconv_ragged_plan_set_fused change a plan (its schedule, never its
 * results' definition); call them while no execution of the plan is
 * pending.  REV_F / CONJ_G / REV_OUT apply per pair
 * as in impconv_conv1d_complex.  IMPCONV_ONE_STREAM runs the size classes one
 * after another on `stream` alone (no fork or join; the auxiliary streams
 * stay idle) with the same kernels, so its results are bitwise those of the
 * concurrent form: for callers that want every launch on their stream, and
 * for timing each kernel without the classes overlapping.
 * ---------------------------------------------------------------------- */
typedef struct impconv_ragged_plan impconv_ragged_plan;

impconv_status impconv_ragged_plan_create(int dtype, int64_t npairs, const int64_t* m_host,
                                          const int64_t* offset_host, impconv_ragged_plan** plan);
impconv_status impconv_ragged_workspace(const impconv_ragged_plan* plan, size_t* bytes);
impconv_status impconv_ragged_execute(const impconv_ragged_plan* plan, const void* f,
                                      const void* g, void* h, void* work, size_t work_bytes,
                                      uint32_t flags, void* stream);
/* Destroying a plan first waits (on the host) for the plan's earlier eager
 * executions to finish -- each execution records a completion event on its
 * stream, and destruction waits for the last one of every stream -- since
 * their kernels read the plan's descriptor arrays; it waits for nothing
 * else on the device and destroys no stream.  A graph captured from a plan
 * must not be launched after the plan is destroyed.  NULL is accepted. */
impconv_status impconv_ragged_plan_destroy(impconv_ragged_plan* plan);

/* Autotuner of the plan's schedule, timed on zero-filled temporary arrays
 * of the plan's packed extent (three executions per candidate after one
 * warm-up, on `stream`):
 *  - four-step classes (N > 8192): every supported split N = N1 x N2
 *    (16 <= N2 <= 4096, 16 <= N1 <= 8192), which sets the FFT sizes and
 *    radices of their row and column passes;
 *  - classes in the work queue: both supported values per thread E (the row
 *    kernels' choice and half of it), which set the radices and the pairs
 *    per item, each timed as a queue launch of that class alone;
 *  - then the fused classes as one queue launch against one launch per
 *    class, keeping the faster.
 * Each class's winner is recorded in the process-wide schedule cache under
 * (architecture, variant "fourstep" or "fused", dtype, N); a class whose
 * key is already there takes the recorded choice without being timed
 * (impconv_ragged_plan_schedule reports "source": "cache").  The call
 * allocates and frees device memory (3 x extent elements plus the
 * workspace size) and synchronizes the stream: call it outside graph
 * capture, while no execution of the plan is pending.  Results of a tuned
 * plan equal those of the untuned one up to rounding.  Errors: E_ARG (null
 * plan, other device), E_HIP (allocation, launch or timing failure; the
 * plan keeps its previous schedule for the classes not yet tuned). */
impconv_status impconv_ragged_plan_autotune(impconv_ragged_plan* plan, void* stream);

/* Fixes how the plan's fused classes run: queue = 1 one persistent
 * work-queue launch, 0 one launch of the fused row kernel per class; elems
 * = values per thread in the queue for every queued class that supports it
 * (the row kernels' choice or half of it), 0 = the row kernels' choice.
 * Copies the queue's class table to the device (synchronous): call it
 * outside graph capture, while no execution of the plan is pending.
 * Errors: E_ARG (null plan, other device, queue not 0/1, elems < 0), E_HIP. */
impconv_status impconv_ragged_plan_set_fused(impconv_ragged_plan* plan, int queue, int elems);

/* The plan's schedule as JSON text: {"fused_launch": "queue" or
 * "per-class", "queue_grid": workgroups of the queue launch, "fused_tuned_ms":
 * {"queue": ms, "per-class": ms} (after autotuning), "classes": [...]}, one
 * object per size class, longest first, with its FFT size N, pair count,
 * method ("queue", "fused" or "four-step"), stream lane, values per thread
 * E (fused) or split N1, N2 (four-step), the source of that choice
 * ("default", "timed", "cache", "set") and the autotuner's times per
 * candidate (ms).  Writes at most cap - 1 characters and a terminating NUL to
 * buf (buf may be NULL with cap 0) and the full length to *len.  Errors:
 * E_ARG (null plan or len). */
impconv_status impconv_ragged_plan_schedule(const impconv_ragged_plan* plan, char* buf, size_t cap,
                                            size_t* len);

/* Process-wide schedule cache of the autotuner (host memory, thread-safe).
 * Export writes a JSON array of {"arch", "variant", "dtype", "N", "choice",
 * "ms"} (choice: values per thread E for "fused", column length N2 for
 * "fourstep") to buf as impconv_ragged_plan_schedule does; import merges
 * such an array (all of it or, on a malformed entry, nothing: E_ARG); clear
 * empties the cache. */
impconv_status impconv_schedule_cache_export(char* buf, size_t cap, size_t* len);
impconv_status impconv_schedule_cache_import(const char* json);
impconv_status impconv_schedule_cache_clear(void);

/* ----------------------------------------------------------------------
 * Descriptor-based plans: one create / execute pair for every kind and
 * dimension.  impconv_plan_create validates the descriptor with the same
 * rules (and error codes) as the matching one-shot call, creates the twiddle
 * tables of the current device (with, for complex 1D lengths whose power-of-
 * two size exceeds 8192, that size's column twiddle table) and fixes the
 * workspace size, so that impconv_execute only launches kernels: even its
 * first call may be captured in a hipGraph.
 * A plan is immutable and holds no data-sized memory; it may be executed
 * concurrently with distinct workspaces, on the device it was created on.
 * ---------------------------------------------------------------------- */
typedef struct impconv_desc {
    int kind;         /* impconv_kind */
    int dtype;        /* impconv_dtype */
    int ndim;         /* 1, 2 or 3 (ternary: 1 or 2) */
    int64_t m[3];     /* logical modes per axis; m[0] in 1D */
    int64_t n[3];     /* storage extents per axis (2D/3D; see impconv_conv2d) */
    int64_t batch;    /* independent convolutions */
    int64_t M;        /* dot-product width (Sec. 3.3); ignored for ternary */
    uint32_t flags;   /* as for the one-shot call of this kind */
} impconv_desc;

typedef struct impconv_plan impconv_plan;

/* Errors: E_ARG (null plan/desc, bad ndim or kind), E_SIZE / E_UNSUPPORTED
 * (sizes, as the one-shot calls; ternary with ndim 3 is E_UNSUPPORTED),
 * E_HIP (twiddle table creation).  *plan is NULL on error. */
impconv_status impconv_plan_create(impconv_plan** plan, const impconv_desc* desc);
impconv_status impconv_workspace_bytes(const impconv_plan* plan, size_t* bytes);
/* Runs the plan's convolution: the one-shot call of its kind and dimension
 * with the descriptor's sizes and flags.  e is the third input of a ternary
 * plan and must be NULL for every other kind (E_ARG). */
impconv_status impconv_execute(const impconv_plan* plan, const void* f, const void* g, const void* e,
                               void* h, void* work, size_t work_bytes, void* stream);
impconv_status impconv_plan_destroy(impconv_plan* plan);

/* One-shot ragged batch: impconv_ragged_execute on a plan the library keeps
 * in a process-wide cache (16 most recently used layouts) keyed by device,
 * dtype and the contents of m_host / offset_host.  The first call with a
 * layout creates the plan (synchronous descriptor upload: not under stream
 * capture); later calls only launch kernels.  Evicting a plan waits for
 * that plan's earlier executions (impconv_ragged_plan_destroy).  Errors as
 * impconv_ragged_plan_create and
 * impconv_ragged_execute. */
impconv_status impconv_conv1d_complex_ragged_workspace(int dtype, int64_t npairs, const int64_t* m_host,
                                                       const int64_t* offset_host, size_t* bytes);
impconv_status impconv_conv1d_complex_ragged(int dtype, int64_t npairs, const int64_t* m_host,
                                             const int64_t* offset_host, const void* f, const void* g,
                                             void* h, void* work, size_t work_bytes, uint32_t flags,
                                             void* stream);

#ifdef __cplusplus
}
#endif

#endif /* IMPCONV_H */
