/*
 * hdconv -- hybrid-dealiased linear convolution of two equal-length real arrays
 * on AMD Instinct MI355X (gfx950).
 *
 * Operation (Murasko & Bowman, "Hybrid Dealiasing and Implicit Packing for Real
 * Convolutions", Sec. 1 and Sec. 6: the dealiased binary convolution of two real
 * arrays of equal size): for real f, g of extent L_1 x ... x L_d (d = 1, 2, 3),
 *
 *     h_j = sum_{0 <= k <= j} f_k g_{j-k},     0 <= j < L   (componentwise),
 *
 * i.e. the first L entries (per axis) of the linear convolution, normalised.
 * It is computed with FFTs of length m per axis that carry the zero padding to
 * length M implicitly (hybrid dealiasing, Sec. 2: p = ceil(L/m) explicitly
 * padded blocks, q residues with q m >= M), either by
 *   - implicit packing (Sec. 4 and 5): the real data are read as complex
 *     f~_j = f_{2j} + i f_{2j+1} along the last axis and the product uses the
 *     RCM operator, eqs. (RCM) / (RCM-ndim);                      HDC_HYBRID_RCM
 *   - conjugate symmetries of the real residues (Sec. 3);         HDC_HYBRID_CS
 *   - the same with implicit packing for the self-conjugate residues 0 and q/2
 *     (the combination the discussion in Sec. 6 proposes: every residue is
 *     computed on its own, residues 0 and q/2 at half length); 1D problems whose
 *     residues fit one workgroup; in 2D/3D the first axis's residues 0 and q/2
 *     run as an implicit-packing problem with q = 2 on that axis (q = 1 for an
 *     odd q; the packed last axis planned as for HDC_HYBRID_RCM), the other
 *     residues through conjugate symmetry adding to its result; even m on the
 *     first axis;                                                  HDC_HYBRID_MIX
 * or, as comparators on the same kernels, with materialised zero padding to M:
 *   - implicit packing without hybrid dealiasing (Sec. 5 algorithms);  HDC_EXPLICIT_RCM
 *   - explicit unpacking / product / packing, eqs. (fourierUnpack),
 *     (fourierPack) -- the standard real-to-complex approach;          HDC_EXPLICIT
 *
 * Memory: every data pointer is a DEVICE pointer to a row-major array whose
 * last axis is contiguous; `batch` problems are stored back to back (stride
 * prod(L) reals).  f, g, h (and dh, df, dg) belong to the caller.  FP32 data
 * must be 8-byte aligned and FP64 data 16-byte aligned.  h may alias f, or g
 * when g has f's extents, exactly; other overlaps are rejected.  The caller supplies a device
 * workspace of at least the size reported for the plan.
 *
 * Calls are asynchronous on the given stream (a hipStream_t; 0 = null
 * stream) and perform no implicit synchronisation.  No C++ exception crosses
 * this interface; every call returns an hdc_status and leaves a thread-local
 * message for hdc_last_error().
 */
#ifndef HDCONV_H
#define HDCONV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HDC_OK = 0,
  HDC_ERR_INVALID_ARG = -1, /* bad descriptor, pointer, alignment or overlap */
  HDC_ERR_UNSUPPORTED = -2, /* valid request outside what the kernels implement */
  HDC_ERR_WORKSPACE = -3,   /* workspace missing or smaller than required */
  HDC_ERR_HIP = -4,         /* a HIP runtime call failed (message has the HIP error) */
  HDC_ERR_ALLOC = -5        /* device allocation of plan tables failed */
} hdc_status;

typedef enum { HDC_F32 = 0, HDC_F64 = 1 } hdc_dtype;

typedef enum {
  HDC_HYBRID_RCM = 0,
  HDC_HYBRID_CS = 1,
  HDC_EXPLICIT_RCM = 2,
  HDC_EXPLICIT = 3,
  HDC_HYBRID_MIX = 4
} hdc_variant;

/* hdc_desc.flags (other bits are rejected with HDC_ERR_INVALID_ARG).
 *
 * HDC_SAVE_SPECTRA: hdc_forward keeps the outer-axis transforms of f and g
 *   (the residue columns of the multi-pass 1D form) in the workspace and writes
 *   its product to a separate region, so that hdc_backward, called afterwards
 *   with the same f, g and workspace pointers, transforms only R(dh).  Between
 *   the two calls f, g and the workspace must not change; the workspace must
 *   hold hdc_plan_backward_workspace_size bytes for the backward.  Called with
 *   other pointers, hdc_backward transforms f and g itself (same result, more
 *   work).  In effect for HDC_HYBRID_RCM plans with equal extents that use a
 *   workspace (not the one-workgroup 1D form, which keeps everything on chip)
 *   and whose batch runs in one launch sequence; elsewhere it is accepted and
 *   has no effect.
 *
 * HDC_USE_GRAPH: hdc_forward and hdc_backward run the plan's launch sequence
 *   from a hipGraph: captured (on a stream the plan owns) on the first call
 *   with a given set of data and workspace pointers, replayed on the caller's
 *   stream while the pointers stay the same, captured again when they change
 *   (after the previous replay has finished).  Results are bitwise those of the
 *   launches without the flag; it saves the per-launch host cost of the 3-5
 *   launches of the multi-pass and multi-D forms.  Calls on one plan must not
 *   overlap (they share its graphs).  Calls with hdc_profile_enable on launch
 *   directly.
 *
 * HDC_DETERMINISTIC: the plan's parameters never come from timing:
 *   hdc_autotune on such a descriptor returns the planner's defaults without
 *   timing anything (the same m on every run and device) and ignores the cache
 *   file.
 *
 * Every call is bitwise reproducible for a fixed plan, with or without these
 * flags: each output element has one owner and residue sums run in a fixed
 * order, with no atomics. */
#define HDC_SAVE_SPECTRA 0x2u
#define HDC_USE_GRAPH 0x4u
#define HDC_DETERMINISTIC 0x8u

/*
 * Problem descriptor.
 *   ndim    1..3
 *   L[i]    extent of f and h on axis i (>= 1), and of g unless Lg is set
 *   M[i]    padded length on axis i; 0 selects L[i] + Lg[i] (2 L[i] for equal
 *           lengths); must satisfy M >= L + Lg - 1 so that no wrapped term
 *           reaches j < L (Sec. 2; the paper uses M = 2L)
 *   m[i]    FFT length on axis i in real-sample units (0 = planner's choice).
 *           With implicit packing the last axis runs complex FFTs of length m/2
 *           on the packed data, so m must then be even.  Every FFT length must be
 *           a power of two.
 *   q[i]    residues on axis i (0 = ceil(M/m)); q m >= M is required.
 *           HDC_HYBRID_CS in 1D: when the q/2 + 1 residues of both arrays do
 *           not fit one workgroup (q m above about 8K FP32 / 4K FP64), the
 *           residue transforms run in a multi-pass form (rows of m, a real
 *           length-q transform over the rows) that needs q to be a power of
 *           two (default: the smallest one with q m >= M and q >= p).
 *   variant hdc_variant, dtype hdc_dtype, batch >= 1 problems per call.
 *   Lg[i]   extent of the kernel g on axis i, 1 <= Lg <= L; 0 (or a zeroed
 *           field) means Lg = L.  A shorter kernel is implicitly zero padded
 *           like the data (the unequal-length extension the paper proposes in
 *           its outlook: same m and q for both arrays, p per array); g is a
 *           row-major array of extents Lg, h keeps the extents L, and
 *           h_j = sum_{k <= j, j - k < Lg} f_k g_{j-k}.  Supported by every
 *           variant in every dimension, forward and adjoint (also in uneven
 *           batches); not with nin > 2.
 *   nin     number of input arrays; 0 or 2 for the binary convolution.  For
 *           3 <= nin <= 8 the plan computes the truncated convolution of nin
 *           real arrays of one shape (Sec. 4.1, eqs. (Akn), (Rnk), (RnMk)):
 *           h_j = sum over k^1 + ... + k^nin = j of f^1_{k^1} ... f^nin_{k^nin},
 *           j < L, through hdc_forward_n, with implicit packing: the packed
 *           spectra R^j = R^{j-1} [.] F^j are combined pair by pair in the
 *           line kernels.  Needs HDC_HYBRID_RCM and equal extents; M defaults
 *           to nin L and must satisfy M >= nin (L - 1) + 1.  No adjoint, no
 *           batch items (HDC_ERR_UNSUPPORTED).
 */
typedef struct {
  int32_t ndim;
  int64_t L[3];
  int64_t M[3];
  int32_t m[3];
  int32_t q[3];
  int32_t variant;
  int32_t dtype;
  int64_t batch;
  uint32_t flags;
  int64_t Lg[3];
  int32_t nin;
} hdc_desc;

typedef struct hdc_plan_s* hdc_plan;

/* Validate d, choose the per-axis parameters and build the FP64-generated
 * twiddle tables on the current device (owned by the plan).  *out receives
 * the plan, or NULL on error.  Errors: HDC_ERR_INVALID_ARG (ndim, L, Lg, M < L+Lg-1,
 * m, q m < M, batch), HDC_ERR_UNSUPPORTED (a length the kernels do not cover,
 * among them a padded transform length q m above 2^22 on a strided axis, whose
 * residue table is held single-level), HDC_ERR_ALLOC / HDC_ERR_HIP. */
hdc_status hdc_plan_create(const hdc_desc* d, hdc_plan* out);

/* Bytes of device workspace hdc_forward needs (may be 0). */
hdc_status hdc_plan_workspace_size(hdc_plan p, size_t* bytes);

/* Bytes of device workspace hdc_backward needs: four spectrum regions for the
 * shared-transform adjoint of HDC_HYBRID_RCM (two for the forward, three with
 * HDC_SAVE_SPECTRA); otherwise the forward size, plus f's extents times the
 * batch for a plan with a shorter kernel. */
hdc_status hdc_plan_backward_workspace_size(hdc_plan p, size_t* bytes);

/* Resolved per-axis parameters in the units of each axis' transform
 * (packed complex units on the last axis for the implicit-packing variants):
 * FFT length m, explicit blocks p and residues q (q m >= transform length). */
hdc_status hdc_plan_resolved(hdc_plan p, int32_t m[3], int32_t pp[3], int32_t q[3]);

/* Launch sequence of the plan's kernels, for diagnostics: writes up to n
 * NUL-terminated kernel names separated by ';' into buf. */
hdc_status hdc_plan_describe(hdc_plan p, char* buf, size_t n);

/* h = conv(f, g) for every problem of the batch (the operation above).
 * ws: device workspace of ws_bytes >= hdc_plan_workspace_size.  stream: hipStream_t. */
hdc_status hdc_forward(hdc_plan p, const void* f, const void* g, void* h,
                       void* ws, size_t ws_bytes, void* stream);

/* Adjoint of hdc_forward for an upstream gradient dh = dLoss/dh:
 *   df_k = sum_{0<=i<L-k} g_i dh_{k+i},   dg_k = sum_{0<=i<L-k} f_i dh_{k+i}
 * (componentwise in d dimensions), i.e. df = R(conv(g, R(dh))) and
 * dg = R(conv(f, R(dh))) with R the reversal of every axis; computed by the
 * same residue machinery with the reversals folded into loads and stores.
 * For HDC_HYBRID_RCM with equal extents the two correlations share one
 * transform of R(dh): the line kernel multiplies R(dh)'s spectra with g's and
 * then with f's (with HDC_SAVE_SPECTRA f's and g's outer-axis transforms come
 * from the preceding forward).  df or dg may be NULL to skip it.  With a
 * shorter kernel (Lg < L) df has f's extents and dg has g's (k < Lg); dg is
 * formed in a scratch region of the backward workspace and copied out.  ws
 * must hold hdc_plan_backward_workspace_size bytes. */
hdc_status hdc_backward(hdc_plan p, const void* f, const void* g, const void* dh,
                        void* df, void* dg, void* ws, size_t ws_bytes, void* stream);

hdc_status hdc_plan_destroy(hdc_plan p);

/* h = conv(x[0], ..., x[nin-1]) for a plan with nin input arrays (see
 * hdc_desc.nin): x is a HOST array of nin device pointers, each to a batch of
 * arrays of the plan's shape; h may alias one of them exactly.  ws: device
 * workspace of >= hdc_plan_workspace_size bytes (nin spectrum regions).  A
 * binary plan (nin = 2) runs hdc_forward(x[0], x[1]).  Errors as for
 * hdc_forward; hdc_forward on a plan with nin > 2 reports HDC_ERR_INVALID_ARG. */
hdc_status hdc_forward_n(hdc_plan p, const void* const* x, void* h, void* ws, size_t ws_bytes, void* stream);

/* Cached kernel spectra ("transform once, multiply many"; the conclusion
 * (Sec. 7) notes that a padded, transformed kernel can be precomputed and
 * reused while it does not change, as in CNN inference).  For plans of the
 * implicit-packing hybrid variant (HDC_HYBRID_RCM) of two arrays, in every
 * dimension:
 *   hdc_plan_spectrum_size  bytes of the spectrum buffer: g's implicitly
 *                           padded spectra along the innermost axis -- the
 *                           residue rows of the multi-pass 1D form (after its
 *                           column pass, four-step twiddle and row FFTs), the
 *                           q m values of a one-workgroup 1D line, or q m values
 *                           for every line of a 2D / 3D problem (after the outer
 *                           axes' passes) -- for every batch element;
 *   hdc_transform_kernel    g -> spec (the plan's kernel extents Lg);
 *   hdc_forward_cached      h = conv(f, g) for the g whose spectra are in spec:
 *                           the forward passes and line transforms run for f
 *                           alone.
 * The result equals hdc_forward bit for bit.  spec is a caller-owned device
 * buffer (16-byte aligned), written by hdc_transform_kernel and only read by
 * hdc_forward_cached; ws as for hdc_forward.  Other plans report
 * HDC_ERR_UNSUPPORTED. */
hdc_status hdc_plan_spectrum_size(hdc_plan p, size_t* bytes);
hdc_status hdc_transform_kernel(hdc_plan p, const void* g, void* spec, void* ws, size_t ws_bytes, void* stream);
hdc_status hdc_forward_cached(hdc_plan p, const void* f, const void* spec, void* h, void* ws, size_t ws_bytes,
                              void* stream);

/* Allocation-free forward, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): hdc_forward with the workspace taken from a static device array
 * of HDC_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on,
 * until the process ends.  Allocates nothing (no hipMalloc/hipFree, no
 * allocating library call); the caller passes the inputs and the output as for
 * hdc_forward.  Plans whose workspace exceeds the array are rejected with
 * HDC_ERR_WORKSPACE before any launch.  Every call on one GPU shares that GPU's
 * array, which keeps the last call's contents (nothing needs clearing: every
 * workspace element a kernel reads was written earlier in the same call), so
 * calls that overlap on one GPU -- from several streams or threads -- race and
 * must be serialised by the caller. */
#define HDC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
hdc_status hdc_forward_noalloc(hdc_plan p, const void* f, const void* g, void* h, void* stream);

/* Uneven batch (Sec. 6 treats problems one at a time; batching many problems
 * of differing sizes is this library's addition): n_items descriptors (their
 * batch fields are ignored; one problem each, all of one dtype).  Each item is
 * planned as by hdc_plan_create (identical descriptors share a plan) and owns
 * a 256-byte-aligned region of the batch workspace.  A call records every
 * item's launch sequence and runs launches of the same kernel at the same
 * position of their sequences as ONE grouped launch whose per-item parameters
 * sit in a device table; the sequence is captured once into a hipGraph and
 * replayed.  Groups that share no item are independent: they run on up to four
 * streams (the caller's and three the plan owns, all at the default priority),
 * forked from and joined to the caller's stream with events, so the call is
 * still ordered on the caller's stream as a whole (the environment variable
 * HDC_BATCH_LANES = 1..4, read at creation, caps the number).  The tables are rewritten (an asynchronous copy on the caller's
 * stream) only when the pointer set changes; a graph that also holds per-item
 * launches (explicit padding copies, the conjugate-symmetry passes) is then
 * captured again.  A call with the same pointers as the previous one replays
 * without planning or recording the items again.  Results equal those of
 * hdc_forward/hdc_backward item by item (bitwise: the same kernels run on the
 * same data).
 * Errors: HDC_ERR_INVALID_ARG (NULL/misaligned pointers, item index named in
 * hdc_last_error), HDC_ERR_WORKSPACE, HDC_ERR_HIP; creation fails with the
 * first item's planning error.  Calls on one batch plan must not overlap
 * (they share its tables and workspace layout); calls from several streams
 * are ordered by the plan itself. */
typedef struct hdc_batch_plan_s* hdc_batch_plan;
hdc_status hdc_batch_plan_create(const hdc_desc* items, int64_t n_items, hdc_batch_plan* out);
hdc_status hdc_batch_workspace_size(hdc_batch_plan p, size_t* bytes);
/* f, g, h: HOST arrays of n_items device pointers (item i has the shape of
 * items[i]).  ws: device workspace of >= hdc_batch_workspace_size bytes. */
hdc_status hdc_batch_forward(hdc_batch_plan p, const void* const* f, const void* const* g,
                             void* const* h, void* ws, size_t ws_bytes, void* stream);
/* Adjoint per item as hdc_backward; df[i] or dg[i] may be NULL. */
hdc_status hdc_batch_backward(hdc_batch_plan p, const void* const* f, const void* const* g,
                              const void* const* dh, void* const* df, void* const* dg,
                              void* ws, size_t ws_bytes, void* stream);
hdc_status hdc_batch_plan_destroy(hdc_batch_plan p);

/* Autotuner (Sec. 6 picks m and q by timing candidates; here a coordinate
 * search over power-of-two m per axis): times forward calls of the candidate
 * plans on the current device with scratch buffers of the descriptor's shape
 * (a problem smaller than 2^22 points is timed as a batch of about that many
 * points, at most 4096 problems, so kernel time rather than launch overhead
 * decides and the device is filled as in a large batch; each candidate
 * scores the fastest of five timed calls, and must be at least 3% faster
 * than the current choice to replace it) and writes the
 * fastest m into d->m (real-sample units on every axis; the
 * packed last axis runs FFTs of m/2) and 0 into d->q (the minimal q for that
 * m).  d's own m and q are ignored on entry.  cache_path (may be NULL): text
 * file of lines "<device arch and descriptor>|m0 m1 m2"; a matching line is
 * used without timing, a new choice is appended.  Allocates device memory and
 * synchronises the device; not for use under graph capture. */
hdc_status hdc_autotune(hdc_desc* d, const char* cache_path);

const char* hdc_status_string(hdc_status st);

/* Copies the calling thread's last error message into buf (NUL-terminated,
 * truncated to n) and returns its full length. */
size_t hdc_last_error(char* buf, size_t n);

/* Diagnostics: per-launch timing with HIP events.  While enabled, every
 * hdc_forward / hdc_backward call records one event before its first launch
 * and one after each launch, on the call's stream (no synchronisation).
 * hdc_profile_read waits for the recorded events, writes the average duration
 * in milliseconds of each launch position (in the order hdc_plan_describe
 * lists them) into avg_ms[0..n), sets *n_launches and *n_calls, and clears the
 * record.  At most 4096 events are kept; later calls are not recorded. */
hdc_status hdc_profile_enable(hdc_plan p, int on);
hdc_status hdc_profile_read(hdc_plan p, double* avg_ms, int32_t n, int32_t* n_launches, int32_t* n_calls);

/* Library version string. */
const char* hdc_version(void);

/* Diagnostic (host only, no GPU needed): the value the kernels use for the
 * root of unity zeta_N^k = exp(2 pi i k / N) (Sec. 2, the twiddles of eqs.
 * (forwardr) and (accumulator)), for k = k0 .. k0 + count - 1, in precision
 * dtype, widened to double into re[0..count) and im[0..count) (host arrays the
 * caller owns).  Tables hold each entry computed in extended precision and
 * rounded once; up to 4096 points the value is that entry, above it is the
 * product of two such entries (zeta_N^{k mod 2^b} zeta_N^{2^b floor(k/2^b)},
 * b = ceil(ceil(log2 N)/2)) formed in dtype exactly as the kernels form it.
 * Errors: HDC_ERR_INVALID_ARG (N outside [1, 2^30], k range outside [0, N),
 * unknown dtype, NULL outputs). */
hdc_status hdc_twiddle_values(int64_t N, int32_t dtype, int64_t k0, int64_t count, double* re, double* im);

#ifdef __cplusplus
}
#endif

#endif /* HDCONV_H */
