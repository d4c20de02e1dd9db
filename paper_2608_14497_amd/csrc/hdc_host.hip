// Host planner and C ABI of the hybrid-dealiased real convolution library.
//
// A plan fixes, per axis, the FFT length m, the explicitly padded block count
// p = ceil(L/m) and the residue count q (q m >= M) of hybrid dealiasing
// (Sec. 2), chooses the pass structure, and owns FP64-generated twiddle tables
// rounded once to the working precision.  Pass structures (all HBM traffic is
// coalesced row segments; no global transposes):
//   1D, small   one workgroup per convolution: LINE_1D
//   1D, large   column pass over the p-blocks (complex inner loop, q = n p),
//               residue-row pairs (r, q-r) with the implicit-packing product,
//               inverse column pass with accumulation:  COL -> LINE_ROWS -> COL^-1
//   2D          column pass along axis 1, line pairs (k1, k1*) along the packed
//               axis 2, inverse column pass:           COL -> LINE_2D -> COL^-1
//   3D          two column passes (axes 1, 2), line pairs ((k1,k2),(k1*,k2*)),
//               two inverse column passes
// The explicit comparators pad f and g to M in the workspace, run the same
// passes with transform length M (p = q: nothing implicit) and truncate.
#include <math.h>
#include <stdlib.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hdconv.h"
#include "hdc_kernels.hpp"

using namespace hdc;

namespace {

thread_local std::string g_err;

hdc_status fail(hdc_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

hdc_status ok() {
  g_err.clear();
  return HDC_OK;
}

#define HIP_TRY(expr)                                                                 \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) return fail(HDC_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

bool is_pow2(long long v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(long long v) {
  int r = 0;
  while ((1LL << r) < v) ++r;
  return r;
}
long long next_pow2(long long v) {
  long long r = 1;
  while (r < v) r <<= 1;
  return r;
}
long long cdiv(long long a, long long b) { return (a + b - 1) / b; }
size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }
// register-cached explicit blocks (1, 2, 4) or 0 = generic (re-read per residue)
int pcap_of(int p) { return p <= 1 ? 1 : (p <= 2 ? 2 : (p <= 4 ? 4 : 0)); }
constexpr int kMaxBlocks = 1024;
constexpr uint32_t kKnownFlags = HDC_SAVE_SPECTRA | HDC_USE_GRAPH | HDC_DETERMINISTIC;
constexpr long long kMaxGridY = 65535;

// zeta_N^k = exp(2 pi i k / N) in float64 from an exact integer octant reduction
void zeta64(long long k, long long N, double* c, double* s) {
  k %= N;
  if (k < 0) k += N;
  // angle = 2 pi k / N; reduce with exact integer comparisons
  // quadrant: k8 = 8k vs N
  long double a;
  long long kk = k;
  int quad = 0;
  while (4 * kk >= N) {  // subtract quarter turns exactly when N % 4 == 0, else fall back
    if (N % 4 != 0) break;
    kk -= N / 4;
    ++quad;
  }
  a = 2.0L * 3.14159265358979323846264338327950288L * (long double)kk / (long double)N;
  long double cc = cosl(a), ss = sinl(a);
  if (kk == 0) {
    cc = 1.0L;
    ss = 0.0L;
  }
  for (int i = 0; i < quad; ++i) {  // multiply by i
    long double t = cc;
    cc = -ss;
    ss = t;
  }
  *c = (double)cc;
  *s = (double)ss;
}

struct TwReq {
  long long N;
  int lobits;
  size_t off_lo, off_hi;  // element offsets in the table buffer
  int nlo, nhi;
};

struct TwDev {
  const void* lo = nullptr;
  const void* hi = nullptr;
  int lobits = 0;
  int N = 1;
  int single = 1;
};

template <typename T>
Tw2<T> as_tw(const TwDev& d) {
  Tw2<T> t;
  t.lo = reinterpret_cast<const cx<T>*>(d.lo);
  t.hi = reinterpret_cast<const cx<T>*>(d.hi);
  t.lobits = d.lobits;
  t.N = d.N;
  t.single = d.single;
  return t;
}

}  // namespace

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
enum PathKind { PATH_1D_ONE = 0, PATH_1D_MULTI = 1, PATH_2D = 2, PATH_3D = 3 };

struct hdc_plan_s {
  hdc_desc d;
  int ndim = 1, dtype = 0, variant = 0, mul = MUL_RCM;
  long long batch = 1;
  bool expl = false;           // explicit comparator: materialised padding
  bool cs = false;             // conjugate-symmetry variant (unpacked real data)
  bool mix = false;            // ... with residues 0 and q/2 through implicit packing (HDC_HYBRID_MIX)
  int nres0 = 1;               // CS: residues kept on the real axis (0 .. floor(q/2))
  int Nret = 1;                // CS multi-D: retained first-axis lines
  // mixed variant in 2D/3D: the first axis's residues 0 and q/2 run as an implicit-packing sub-plan with
  // q = 2 (q = 1 for an odd q) on that axis, scaled by 2/q (1/q); the residues 1 .. ceil(q/2) - 1 run here
  // (conjugate symmetry), their Nmid = (ceil(q/2) - 1) m first-axis lines from row mid_row0 on
  hdc_plan_s* sub = nullptr;
  int Nmid = 0, mid_row0 = 0;
  const hdc_plan_s* owner = nullptr;  // sub-plan: the plan whose launch timing records its launches too
  int force_q0 = 0;            // sub-plan: q on the first axis as given (q m < M: a subset of residues)
  double extra_scale = 1.0;    // sub-plan: factor on the inverse transforms' 1/N
  int Lu[3] = {1, 1, 1};       // user extents (reals)
  int Lg[3] = {1, 1, 1};       // user extents of the kernel g (<= Lu)
  int Lge[3] = {1, 1, 1};      // extents of g in the executed problem (explicit: M)
  bool unequal = false;        // some Lg < Lu
  int nin = 2;                 // input arrays (n-ary implicit packing for nin > 2, Sec. 4.1)
  int Mu[3] = {1, 1, 1};       // padded lengths
  int Le[3] = {1, 1, 1};       // extents of the executed problem (explicit: M)
  int path = PATH_1D_ONE;
  // per-axis parameters in transform units (last axis: packed complex units)
  int am[3] = {1, 1, 1}, ap[3] = {1, 1, 1}, aq[3] = {1, 1, 1}, aN[3] = {1, 1, 1};
  int Lh = 1;                  // packed extent of the executed last axis
  // 1D multi-pass: rows of mr complex, column FFT length pc, n shifts, q = n pc
  int mr = 1, pc = 1, nsh = 1, qr = 1;
  // device tables
  void* tables = nullptr;
  int logroot = 1;
  const void* root = nullptr;
  TwDev tw_line, tw_2nf, tw_ax[2], tw_colN, tw_colX;
  // workspace (bytes) and region offsets
  size_t ws_bytes = 0;
  size_t bwd_ws_bytes = 0;     // backward: + scratch of f's extents for dg of a shorter kernel; twin: R0..R3
  bool twin_ok = false;        // the adjoint runs the twin form (R(dh) transformed once for df and dg)
  bool save = false;           // HDC_SAVE_SPECTRA in effect: the forward keeps f's and g's spectra in R0, R1
  // the forward whose spectra R0, R1 hold (the adjoint reuses them only for the same f, g and workspace)
  mutable const void* saved_f = nullptr;
  mutable const void* saved_g = nullptr;
  mutable const void* saved_ws = nullptr;
  size_t off_scr = 0;
  size_t off_fpad = 0, off_gpad = 0, off_hpad = 0, off_F = 0, off_G = 0, off_R2 = 0, off_R3 = 0;
  long long regF = 0;          // complex elements per batch element in F (and G)
  long long chunk = 0;         // batch elements per launch sequence (0 = whole batch)
  std::string describe;
  // HDC_USE_GRAPH: the launch sequence of the last pointer set, captured once (0: forward, 1: backward)
  struct Graphed {
    std::vector<const void*> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;  // recorded after each replay
    bool pending = false;
  };
  mutable Graphed graphs[2];
  mutable hipStream_t gcap = nullptr;  // capture stream
  // per-launch event timing (diagnostics)
  mutable bool prof = false;
  mutable std::vector<hipEvent_t> evpool;
  mutable size_t evused = 0;
  mutable std::vector<std::vector<int>> calls;
};

static const size_t kMaxEvents = 4096;

// launch recorder of the uneven-batch executor (set while recording)
struct RecSink;
thread_local RecSink* g_sink = nullptr;

// record one event on the stream into the current call's list
static void prof_mark(const hdc_plan_s* P, hipStream_t st) {
  if (P->owner) P = P->owner;
  if (!P->prof || P->calls.empty() || g_sink) return;
  if (P->evused >= kMaxEvents) return;
  if (P->evused >= P->evpool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    P->evpool.push_back(e);
  }
  hipEvent_t e = P->evpool[P->evused];
  if (hipEventRecord(e, st) != hipSuccess) return;
  P->calls.back().push_back((int)P->evused);
  ++P->evused;
}
static void prof_begin_call(const hdc_plan_s* P, hipStream_t st) {
  if (!P->prof || P->evused >= kMaxEvents) return;
  P->calls.emplace_back();
  prof_mark(P, st);
}

// Conjugate-symmetry variant (Sec. 3; Sec. 5 for several dimensions): unpacked real data.
static hdc_status resolve_cs(hdc_plan_s* P) {
  const hdc_desc& d = P->d;
  const int nd = d.ndim;
  const bool f64 = d.dtype == HDC_F64;
  P->cs = true;
  P->mul = MUL_ELEM;
  const int line_max_logm = f64 ? kLineMaxLogM64 : kLineMaxLogM32;
  auto axis = [&](int a, int maxlog, bool real_axis, int deflog = 99) -> hdc_status {
    const long long L = P->Lu[a], M = P->Mu[a];
    long long m = d.m[a];
    if (!m) {
      m = next_pow2(L);
      while (ilog2(m) > std::min(maxlog, deflog)) m >>= 1;
      if (m < 2 && real_axis) m = 2;
    }
    if (!is_pow2(m) || ilog2(m) > maxlog)
      return fail(HDC_ERR_UNSUPPORTED, "axis %d: FFT length m = %lld must be a power of two <= %d", a, m, 1 << maxlog);
    const long long p = cdiv(L, m);
    const long long q = d.q[a] ? d.q[a] : cdiv(M, m);
    if (q * m < M) return fail(HDC_ERR_INVALID_ARG, "axis %d: q m = %lld < M = %lld", a, q * m, M);
    if (q < p) return fail(HDC_ERR_INVALID_ARG, "axis %d: q < p", a);
    if (real_axis && q % 2 == 0 && m % 2)
      return fail(HDC_ERR_INVALID_ARG, "axis %d: an even q needs an even m (the q/2 residue is folded)", a);
    if (p > kMaxBlocks) return fail(HDC_ERR_UNSUPPORTED, "axis %d: too many blocks; choose a larger m", a);
    P->am[a] = (int)m;
    P->ap[a] = (int)p;
    P->aq[a] = (int)q;
    P->aN[a] = (int)(q * m);
    return ok();
  };
  for (int a = 0; a < nd; ++a) P->Le[a] = P->Lu[a];
  if (nd == 1) {
    // one workgroup holds the q/2 + 1 residue slots of both arrays when they fit its LDS
    // (q m up to about 8K complex FP32 / 4K FP64); larger problems use the multi-pass form
    bool fits = false;
    // default m: the smallest power of two that takes at most four register-held blocks (one block of a
    // long line spills; measured 2.8-4x slower for L = 1500-3000), shrunk further below if LDS requires
    const int deflog = ilog2(next_pow2(std::max<long long>(cdiv(P->Lu[0], 4), 2)));
    const hdc_status s1 = axis(0, line_max_logm, true, deflog);
    if (s1 != HDC_OK && (d.m[0] || d.q[0])) return s1;  // the caller's m, q are invalid as given
    if (s1 == HDC_OK) {
      bool valid = true;
      if (!d.m[0]) {
        // default m: the largest power of two whose residue slots fit one workgroup's LDS
        while (P->am[0] > 2) {
          const int nres = P->aq[0] / 2 + 1;
          if ((size_t)2 * nres * padded_len(P->am[0]) * (f64 ? 16 : 8) <= 160 * 1024) break;
          const long long m = P->am[0] / 2;
          const long long q = d.q[0] ? d.q[0] : cdiv(P->Mu[0], m);
          P->am[0] = (int)m;
          P->ap[0] = (int)cdiv(P->Lu[0], m);
          P->aq[0] = (int)q;
          P->aN[0] = (int)(q * m);
          // more than four blocks would re-read the input per residue: the multi-pass form is faster
          if (q * m < P->Mu[0] || q < P->ap[0] || P->ap[0] > 4) {
            valid = false;
            break;
          }
        }
      }
      P->nres0 = P->aq[0] / 2 + 1;
      const size_t lds = (size_t)2 * P->nres0 * padded_len(P->am[0]) * (f64 ? 16 : 8);
      fits = valid && lds <= 160 * 1024;
    }
    if (fits) {
      P->path = PATH_1D_ONE;
      return ok();
    }
    // Multi-pass form of the same residue transforms (the complex inner loop of Appendix A
    // on real data): the line viewed as rows of m; a real length-q transform over the rows
    // (implicit zeros beyond the data) keeps the residues r = 0..q/2, the four-step twiddle
    // zeta_{qm}^{r s} and length-m transforms run per retained residue row, the product is
    // elementwise, and the inverse returns through the real row transform.
    const long long L = P->Lu[0], M = P->Mu[0];
    // default rows of 2048 (1024 in FP64): the residue-row kernel's fastest length
    long long m = d.m[0] ? d.m[0] : (f64 ? 1024 : 2048);
    if (!d.m[0]) {
      while (m > 2 && m / 2 >= L) m /= 2;
      // q within 2^kColMaxLogM in FP32: there the column pairs at q = 2048 cost more than the longer
      // rows they save; in FP64 rows of 2048 cost more (1D 2^20, batch 64: 3.4 ms against 2.6 ms per
      // call), so q grows to the pair kernels' limit first
      const int qlog = (f64 && m % 2 == 0) ? kCsPairMaxLogM : kColMaxLogM;
      while (cdiv(M, m) > (1LL << qlog) && ilog2(m) < line_max_logm) m *= 2;
    }
    if (!is_pow2(m) || ilog2(m) > line_max_logm)
      return fail(HDC_ERR_UNSUPPORTED, "1D: FFT length m = %lld must be a power of two <= %d", m, 1 << line_max_logm);
    const long long rows = cdiv(L, m);
    const long long q = d.q[0] ? d.q[0] : next_pow2(std::max<long long>(cdiv(M, m), std::max<long long>(rows, 2)));
    if (!is_pow2(q) || q < 2)
      return fail(HDC_ERR_UNSUPPORTED, "1D multi-pass conjugate symmetry: q = %lld must be a power of two >= 2", q);
    if (q * m < M) return fail(HDC_ERR_INVALID_ARG, "q m = %lld < M = %lld", q * m, M);
    if (q < rows) return fail(HDC_ERR_INVALID_ARG, "q < p");
    // the column-pair kernels take q up to 2^kCsPairMaxLogM (an even m); single columns 2^kColMaxLogM
    const int qmax = (m % 2 == 0) ? kCsPairMaxLogM : kColMaxLogM;
    if (ilog2(q) > qmax)
      return fail(HDC_ERR_UNSUPPORTED, "1D: q = %lld residues exceed %d; choose a larger m", q, 1 << qmax);
    P->am[0] = (int)m;
    P->ap[0] = (int)rows;
    P->aq[0] = (int)q;
    P->aN[0] = (int)(q * m);
    P->mr = (int)m;
    P->pc = (int)q;
    P->nsh = 1;
    P->qr = (int)q;
    P->nres0 = 1;
    P->Nret = (int)(q / 2 + 1);
    P->path = PATH_1D_MULTI;
    return ok();
  }
  hdc_status s = axis(0, kColMaxLogM, true);
  if (s != HDC_OK) return s;
  if (nd == 3) {
    s = axis(1, kColMaxLogM, false);
    if (s != HDC_OK) return s;
  }
  // default line FFT length at most 1024 (512 in FP64): those line kernels keep every value in registers
  s = axis(nd - 1, line_max_logm, false, f64 ? 9 : 10);
  if (s != HDC_OK) return s;
  const size_t lds = (size_t)2 * P->aq[nd - 1] * padded_len(P->am[nd - 1]) * (f64 ? 16 : 8);
  if (lds + kLineStaticLds > 160 * 1024)
    return fail(HDC_ERR_UNSUPPORTED, "last axis: line does not fit LDS (q m too large)");
  P->nres0 = P->aq[0] / 2 + 1;
  {
    const int m0 = P->am[0], q0 = P->aq[0];
    // retained lines: r = 0 -> m/2 + 1; 0 < r < q/2 -> m each; q/2 -> m/2
    int n = m0 / 2 + 1;
    const int nmid = (q0 + 1) / 2 - 1;
    n += nmid * m0;
    if (q0 % 2 == 0 && q0 >= 2) n += m0 / 2;
    P->Nret = n;
  }
  P->Lh = P->Lu[nd - 1];
  P->path = (nd == 2) ? PATH_2D : PATH_3D;
  return ok();
}

static hdc_status resolve(hdc_plan_s* P) {
  const hdc_desc& d = P->d;
  if (d.ndim < 1 || d.ndim > 3) return fail(HDC_ERR_INVALID_ARG, "ndim must be 1, 2 or 3 (got %d)", d.ndim);
  if (d.batch < 1) return fail(HDC_ERR_INVALID_ARG, "batch must be >= 1");
  if (d.dtype != HDC_F32 && d.dtype != HDC_F64) return fail(HDC_ERR_INVALID_ARG, "unknown dtype %d", d.dtype);
  if (d.variant < 0 || d.variant > 4) return fail(HDC_ERR_INVALID_ARG, "unknown variant %d", d.variant);
  if (d.flags & ~kKnownFlags) return fail(HDC_ERR_INVALID_ARG, "unknown flag bits 0x%x", d.flags & ~kKnownFlags);
  P->ndim = d.ndim;
  P->dtype = d.dtype;
  P->variant = d.variant;
  P->batch = d.batch;
  P->nin = d.nin ? d.nin : 2;
  if (P->nin < 2 || P->nin > kMaxNary)
    return fail(HDC_ERR_INVALID_ARG, "nin = %d input arrays: 2..%d supported (0 means 2)", d.nin, kMaxNary);
  if (P->nin > 2 && d.variant != HDC_HYBRID_RCM)
    return fail(HDC_ERR_UNSUPPORTED, "convolutions of %d arrays run the implicit-packing hybrid variant only", P->nin);
  P->expl = (d.variant == HDC_EXPLICIT_RCM || d.variant == HDC_EXPLICIT);
  P->mul = (d.variant == HDC_EXPLICIT) ? MUL_EXPLICIT : MUL_RCM;
  const bool f64 = d.dtype == HDC_F64;
  const int nd = d.ndim;
  for (int a = 0; a < nd; ++a) {
    if (d.L[a] < 1) return fail(HDC_ERR_INVALID_ARG, "L[%d] must be >= 1", a);
    if (d.L[a] > (1LL << 26)) return fail(HDC_ERR_UNSUPPORTED, "L[%d] too large", a);
    // a shorter kernel g (Lg = 0: the same extent as f)
    const long long Lg = d.Lg[a] ? d.Lg[a] : d.L[a];
    if (Lg < 1 || Lg > d.L[a]) return fail(HDC_ERR_INVALID_ARG, "Lg[%d] = %lld must be in 1..L = %lld", a, Lg, (long long)d.L[a]);
    if (P->nin > 2 && Lg != d.L[a])
      return fail(HDC_ERR_UNSUPPORTED, "convolutions of %d arrays need equal extents", P->nin);
    // no wrapped term reaches j < L: the (n-fold) linear convolution has length L + Lg - 1, n (L - 1) + 1
    const long long Mmin = P->nin > 2 ? (long long)P->nin * (d.L[a] - 1) + 1 : d.L[a] + Lg - 1;
    long long M = d.M[a] ? d.M[a] : (P->nin > 2 ? (long long)P->nin * d.L[a] : d.L[a] + Lg);
    // explicit padding runs full-size power-of-two transforms
    if (!d.M[a] && (d.variant == HDC_EXPLICIT_RCM || d.variant == HDC_EXPLICIT)) M = next_pow2(Mmin < 2 ? 2 : Mmin);
    if (M < Mmin)
      return fail(HDC_ERR_INVALID_ARG, "M[%d] = %lld < %s = %lld: wrapped terms would reach j < L (2L-1 for equal lengths)",
                  a, M, P->nin > 2 ? "n(L-1)+1" : "L+Lg-1", Mmin);
    if (d.m[a] < 0 || d.q[a] < 0) return fail(HDC_ERR_INVALID_ARG, "m and q must be >= 0");
    P->Lu[a] = (int)d.L[a];
    P->Lg[a] = (int)Lg;
    P->unequal |= Lg != d.L[a];
    P->Mu[a] = (int)M;
  }
  if (P->expl) {
    if (P->Mu[nd - 1] % 2) return fail(HDC_ERR_INVALID_ARG, "explicit padding needs an even M on the last axis");
    for (int a = 0; a < nd; ++a) P->Le[a] = P->Mu[a];
    for (int a = 0; a < nd; ++a) P->Lge[a] = P->Mu[a];
  } else {
    for (int a = 0; a < nd; ++a) P->Le[a] = P->Lu[a];
    for (int a = 0; a < nd; ++a) P->Lge[a] = P->Lg[a];
  }
  const int last = nd - 1;

  if (d.variant == HDC_HYBRID_MIX) {
    P->mix = true;
    if (d.m[0] && d.m[0] % 2) return fail(HDC_ERR_INVALID_ARG, "the mixed variant packs residues 0 and q/2: m must be even");
    const hdc_status s = resolve_cs(P);
    if (s != HDC_OK) return s;
    if (nd > 1) {
      // residues 1 .. ceil(q/2) - 1 of the first axis: conjugate symmetry; 0 and q/2: the sub-plan
      const int m0 = P->am[0], q0 = P->aq[0];
      P->Nmid = ((q0 + 1) / 2 - 1) * m0;
      P->mid_row0 = m0 / 2 + 1;
      return ok();
    }
    if (P->path != PATH_1D_ONE || P->am[0] < 2)
      return fail(HDC_ERR_UNSUPPORTED, "the mixed variant runs problems whose residues fit one workgroup (q m up to "
                  "about 8K FP32 / 4K FP64) with an even m");
    return ok();
  }
  if (d.variant == HDC_HYBRID_CS) return resolve_cs(P);
  if (d.m[last] && d.m[last] % 2)
    return fail(HDC_ERR_INVALID_ARG, "implicit packing runs length m/2 FFTs on the last axis: m must be even");

  // ---- packed last axis
  P->Lh = (P->Le[last] + 1) / 2;
  const long long Nmin_last = P->expl ? P->Mu[last] / 2 : cdiv(P->Mu[last], 2);
  const int line_max_logm = f64 ? kLineMaxLogM64 : kLineMaxLogM32;

  // ---- outer axes
  for (int a = 0; a < last; ++a) {
    const long long L = P->Le[a], M = P->Mu[a];
    long long m = d.m[a];
    if (!m) {
      m = next_pow2(L);
      while (m > (1 << kColMaxLogM)) m >>= 1;
      if (P->expl) {
        while (M % m) m >>= 1;
      }
    }
    if (!is_pow2(m) || m > (1 << kColMaxLogM))
      return fail(HDC_ERR_UNSUPPORTED, "axis %d: FFT length m = %lld must be a power of two <= %d", a, m,
                  1 << kColMaxLogM);
    long long p = cdiv(L, m);
    long long q = d.q[a] ? d.q[a] : cdiv(M, m);
    const bool forced = a == 0 && P->force_q0;  // a sub-plan computing residues {0, q/2} of a larger q
    if (forced) q = P->force_q0;
    if (!forced && q * m < M) return fail(HDC_ERR_INVALID_ARG, "axis %d: q m = %lld < M = %lld", a, q * m, M);
    if (P->expl && q * m != M)
      return fail(HDC_ERR_INVALID_ARG, "explicit padding: axis %d needs q m == M (m must divide M)", a);
    if (!forced && q < p) return fail(HDC_ERR_INVALID_ARG, "axis %d: q < p", a);
    if (p > kMaxBlocks) return fail(HDC_ERR_UNSUPPORTED, "axis %d: p = %lld blocks; choose a larger m", a, p);
    if (q * m > (1LL << 30)) return fail(HDC_ERR_UNSUPPORTED, "axis %d too long", a);
    P->am[a] = (int)m;
    P->ap[a] = (int)p;
    P->aq[a] = (int)q;
    P->aN[a] = (int)(q * m);
  }

  if (nd == 1) {
    const long long Lh = P->Lh;
    long long m = d.m[0] ? d.m[0] / 2 : 0;
    // one workgroup if the whole packed problem fits the line kernel
    bool one = false;
    long long m1 = m, p1 = 0, q1 = 0;
    if (!m1) {
      m1 = std::max<long long>(1, next_pow2(Lh));
      if (P->expl) {
        m1 = std::max<long long>(1, next_pow2(Nmin_last));
      } else {
        // hybrid default, from timing the autotuner's choices: complex lines of at most 1024 (FP32) or
        // 512 (FP64) when that takes at most four register-held blocks. One long block runs radix-32/64
        // transforms per lane (measured 1.4-2.8x slower in FP32 for L = 3000-8000, 1.7x in FP64 for
        // L = 3000); FP32 problems from 64 packed points take two blocks (6-10% faster for L = 300-1500).
        // Longer problems keep the long line, which sends them to the multi-pass form.
        const long long cap = f64 ? 512 : 1024;
        const long long two = next_pow2(cdiv(Lh, 2));
        if (!f64 && Lh >= 64 && two <= cap) m1 = two;
        if (m1 > cap && cdiv(Lh, cap) <= 4) m1 = cap;
      }
    }
    if (is_pow2(m1) && ilog2(m1) <= line_max_logm) {
      p1 = cdiv(Lh, m1);
      q1 = d.q[0] ? d.q[0] : cdiv(Nmin_last, m1);
      const size_t lds = line_lds_bytes<double>((int)m1, (int)q1, P->nin) / (f64 ? 1 : 2);
      // one workgroup only at line lengths whose kernels keep every value in registers: complex 1024 (FP32;
      // FP64 512), or 2048 (FP64 1024) with a single block; longer lines per lane (radix 32/64) spilled
      // 180-1600 bytes per lane to scratch, so they take the multi-pass form
      const int lg = ilog2(m1);
      const bool in_regs = f64 ? (lg <= 9 || (lg == 10 && p1 == 1)) : (lg <= 10 || (lg == 11 && p1 == 1));
      if (p1 <= kMaxBlocks && q1 >= p1 && lds <= 160 * 1024 && q1 * m1 >= Nmin_last &&
          (!P->expl || q1 * m1 == Nmin_last) && in_regs)
        one = true;
    }
    if (one) {
      P->path = PATH_1D_ONE;
      P->am[0] = (int)m1;
      P->ap[0] = (int)p1;
      P->aq[0] = (int)q1;
      P->aN[0] = (int)(q1 * m1);
    } else {
      // multi-pass: rows of mr, column FFTs of length pc (power of two), q = n pc
      long long mr = m ? m : (f64 ? 1024 : 2048);
      // n arrays: rows short enough that the 2 n row spectra leave room for two workgroups per CU
      if (!m && P->nin > 2)
        while (mr > 64 && line_lds_bytes<double>((int)mr, 1, 2 * P->nin) / (f64 ? 1 : 2) > 80 * 1024) mr >>= 1;
      if (line_lds_bytes<double>((int)mr, 1, 2 * P->nin) / (f64 ? 1 : 2) > 160 * 1024)
        return fail(HDC_ERR_UNSUPPORTED, "1D: rows of %lld for %d arrays do not fit LDS; choose a smaller m", mr, P->nin);
      if (!is_pow2(mr) || ilog2(mr) > line_max_logm)
        return fail(HDC_ERR_UNSUPPORTED, "1D: FFT length m/2 = %lld must be a power of two <= %d", mr,
                    1 << line_max_logm);
      long long pc = next_pow2(cdiv(Lh, mr));
      if (P->expl && (Nmin_last % mr || !is_pow2(Nmin_last / mr)))
        return fail(HDC_ERR_UNSUPPORTED, "explicit padding: M/2 must be a power-of-two multiple of m/2");
      if (P->expl) pc = Nmin_last / mr;
      if (pc > (1 << kColMaxLogM))
        return fail(HDC_ERR_UNSUPPORTED, "1D: L/m = %lld blocks exceed %d; choose a larger m", pc, 1 << kColMaxLogM);
      long long n = cdiv(Nmin_last, pc * mr);
      if (d.q[0]) {
        if (d.q[0] % pc) return fail(HDC_ERR_UNSUPPORTED, "1D multi-pass needs q to be a multiple of p = %lld", pc);
        n = d.q[0] / pc;
        if (n * pc * mr < Nmin_last) return fail(HDC_ERR_INVALID_ARG, "q m < M");
      }
      if (P->expl && n != 1) return fail(HDC_ERR_INVALID_ARG, "explicit padding: q m must equal M");
      if (n > 64) return fail(HDC_ERR_UNSUPPORTED, "1D: padding ratio too large for the inner loop");
      P->path = PATH_1D_MULTI;
      P->mr = (int)mr;
      P->pc = (int)pc;
      P->nsh = (int)n;
      P->qr = (int)(n * pc);
      P->am[0] = (int)mr;
      P->ap[0] = (int)pc;
      P->aq[0] = (int)(n * pc);
      P->aN[0] = (int)(n * pc * mr);
    }
  } else {
    const long long Lh = P->Lh;
    long long m = d.m[last] ? d.m[last] / 2 : 0;
    if (!m) {
      // default at most 1024 in both precisions (measured faster than 512 in FP64 for 2D 1024^2 and
      // 2048^2); longer line transforms leave fewer registers per value
      m = std::max<long long>(1, next_pow2(Lh));
      // one residue (q = 1) on short padded lines, where measured faster (conv/s, batches of ~2^20 points):
      // FP32 2D up to 512 complex points (300^2 +12%, 512^2 +6%; 1024^2 keeps two residues), FP32 3D up to
      // 64 (64^3 +18%; 100^3 was 3-4% slower) and at 129..256 (256^3: 0.98 against 1.05 ms, with the
      // radix-8 lines of 256), FP64 3D up to 512 (64^3 +13%, 100^3 +7%, 256^3 +4%); FP64 2D was even
      const long long qone = (nd == 2) ? (f64 ? 0 : 512) : (f64 ? 512 : 64);
      const bool one256 = !f64 && nd == 3 && next_pow2(Nmin_last) == 256;
      if (P->expl || Nmin_last <= qone || one256) m = std::max<long long>(1, next_pow2(Nmin_last));
      while (ilog2(m) > std::min(line_max_logm, 10)) m >>= 1;
      if (P->expl)
        while (Nmin_last % m) m >>= 1;
    }
    if (!is_pow2(m) || ilog2(m) > line_max_logm)
      return fail(HDC_ERR_UNSUPPORTED, "last axis: FFT length m/2 = %lld must be a power of two <= %d", m,
                  1 << line_max_logm);
    long long p = cdiv(Lh, m);
    long long q = d.q[last] ? d.q[last] : cdiv(Nmin_last, m);
    if (q * m < Nmin_last) return fail(HDC_ERR_INVALID_ARG, "last axis: q m < M");
    if (P->expl && q * m != Nmin_last) return fail(HDC_ERR_INVALID_ARG, "explicit padding: q m must equal M");
    if (q < p) return fail(HDC_ERR_INVALID_ARG, "last axis: q < p");
    if (p > kMaxBlocks) return fail(HDC_ERR_UNSUPPORTED, "last axis: too many blocks; choose a larger m");
    const size_t lds = line_lds_bytes<double>((int)m, (int)q, 2 * P->nin) / (f64 ? 1 : 2);
    if (lds + kLineStaticLds > 160 * 1024)
      return fail(HDC_ERR_UNSUPPORTED, "last axis: line pair does not fit LDS (q m too large)");
    P->am[last] = (int)m;
    P->ap[last] = (int)p;
    P->aq[last] = (int)q;
    P->aN[last] = (int)(q * m);
    P->path = (nd == 2) ? PATH_2D : PATH_3D;
    if (nd == 3 && (long long)P->aN[0] * P->aN[1] > (1LL << 31) - 1)
      return fail(HDC_ERR_UNSUPPORTED, "3D: too many lines");
  }
  return ok();
}

static void sizes_and_describe(hdc_plan_s* P) {
  const size_t w = P->dtype == HDC_F64 ? 8 : 4;
  const size_t cxb = 2 * w;
  const long long B = P->batch;
  size_t off = 0;
  long long padn = 1;
  for (int a = 0; a < P->ndim; ++a) padn *= P->Mu[a];
  if (P->expl) {
    P->off_fpad = off;
    off = align256(off + (size_t)B * padn * w);
    P->off_gpad = off;
    off = align256(off + (size_t)B * padn * w);
    P->off_hpad = off;
    off = align256(off + (size_t)B * padn * w);
  }
  long long reg = 0;
  if (P->cs) {
    const long long nl = P->sub ? P->Nmid : P->Nret;  // first-axis lines held
    if (P->ndim == 1 && P->path == PATH_1D_MULTI) reg = (long long)P->Nret * P->mr;
    if (P->ndim == 2) reg = nl * P->Lu[1];
    else if (P->ndim == 3) reg = nl * P->aN[1] * P->Lu[2];
  } else
  switch (P->path) {
    case PATH_1D_ONE: reg = 0; break;
    case PATH_1D_MULTI: reg = (long long)P->qr * P->mr; break;
    case PATH_2D: reg = (long long)P->aN[0] * P->Lh; break;
    case PATH_3D: reg = (long long)P->aN[0] * P->aN[1] * P->Lh; break;
  }
  P->regF = reg;
  P->off_F = off;
  off = align256(off + (size_t)B * reg * cxb);
  P->off_G = off;
  off = align256(off + (size_t)B * reg * cxb);
  const size_t end2 = off;
  P->off_R2 = off;
  off = align256(off + (size_t)B * reg * cxb);
  const size_t end3 = off;
  P->off_R3 = off;
  off = align256(off + (size_t)B * reg * cxb);
  const size_t end4 = off;
  for (int a = 4; a < P->nin; ++a) off = align256(off + (size_t)B * reg * cxb);  // regions R4.. of n arrays
  const size_t endn = P->nin == 3 ? end3 : off;
  // the twin adjoint: implicit-packing hybrid plans of two arrays with equal extents
  P->twin_ok = !P->cs && !P->expl && !P->unequal && P->nin == 2;
  const bool chunked = P->chunk > 0 && P->chunk < P->batch;
  P->save = P->twin_ok && (P->d.flags & HDC_SAVE_SPECTRA) && P->path != PATH_1D_ONE && !chunked;
  P->ws_bytes = P->nin > 2 ? endn : (P->save ? end3 : end2);
  // the mixed variant's sub-plan runs first over the same workspace (its passes end before the conjugate-
  // symmetry passes start)
  const size_t end_fw = P->sub ? std::max(end2, align256(P->sub->ws_bytes)) : end2;
  if (P->sub) P->ws_bytes = end_fw;
  P->off_scr = end_fw;
  {
    long long nu = 1;
    for (int a = 0; a < P->ndim; ++a) nu *= P->Lu[a];
    if (P->twin_ok) P->bwd_ws_bytes = P->path == PATH_1D_ONE ? 0 : end4;
    else P->bwd_ws_bytes = P->unequal ? align256(end_fw + (size_t)B * nu * (P->dtype == HDC_F64 ? 8 : 4)) : end_fw;
  }

  std::string s;
  if (P->sub) {
    std::string cs = P->Nmid ? (P->ndim == 2 ? "cs_col_fwd;line_plain;cs_col_inv;"
                                             : "cs_col_fwd;col_fwd;line_plain;col_inv;cs_col_inv;")
                             : "";
    P->describe = P->sub->describe + cs;
    return;
  }
  if (P->cs) {
    if (P->ndim == 1) s = P->path == PATH_1D_MULTI ? "cs_col_fwd;line_rows;cs_col_inv;" : (P->mix ? "line_mix;" : "line_cs;");
    else if (P->ndim == 2) s = "cs_col_fwd;line_plain;cs_col_inv;";
    else s = "cs_col_fwd;col_fwd;line_plain;col_inv;cs_col_inv;";
    P->describe = s;
    return;
  }
  if (P->expl) s += "pad;pad;";  // padded copies of f and g: two launches
  // forward passes of the inputs: one launch per two arrays
  std::string fw;
  for (int a = 0; a < P->nin; a += 2) fw += "col_fwd;";
  switch (P->path) {
    case PATH_1D_ONE: s += "line_1d;"; break;
    case PATH_1D_MULTI: s += fw + "line_rows;col_inv;"; break;
    case PATH_2D: s += fw + "line_2d;col_inv;"; break;
    case PATH_3D: s += fw + fw + "line_3d;col_inv;col_inv;"; break;
  }
  if (P->expl) s += "truncate;";
  P->describe = s;
}

// Two-level table of zeta_N^k for one transform length N: lo[j] = zeta_N^j (j < 2^lobits) and
// hi[i] = zeta_N^{i 2^lobits}, each computed in extended precision and rounded once to T.  Up to 4096
// points lo covers every k (single level); above, the kernels form zeta_N^k = lo[k mod 2^lobits] *
// hi[k >> lobits] (one complex product in T).  Appends lo then hi to out.
static int tw_lobits(long long N) {
  int lb = ilog2(N);
  return lb > 12 ? (lb + 1) / 2 : lb;
}
template <typename T>
static void tw_levels(long long N, int lobits, std::vector<cx<T>>& out) {
  const long long nlo = 1LL << lobits;
  const long long nhi = cdiv(N, nlo);
  auto push = [&](double c, double s) {
    cx<T> v;
    v.x = (T)c;
    v.y = (T)s;
    out.push_back(v);
  };
  for (long long j = 0; j < nlo; ++j) {
    double c, s;
    zeta64(j, N, &c, &s);
    push(c, s);
  }
  for (long long i = 0; i < nhi; ++i) {
    double c, s;
    zeta64(i * nlo, N, &c, &s);
    push(c, s);
  }
}

// largest single-level residue table of a strided axis (8 MiB FP32, 16 MiB FP64 per table)
constexpr long long kColTableMax = 1LL << 22;

// twiddle tables: zeta_{2^logroot}^k and two-level tables per transform length
template <typename T>
static hdc_status build_tables(hdc_plan_s* P) {
  int maxlog = 1;
  for (int a = 0; a < P->ndim; ++a) maxlog = std::max(maxlog, ilog2(P->am[a]));
  if (P->path == PATH_1D_MULTI) maxlog = std::max(maxlog, std::max(ilog2(P->pc), ilog2(P->mr)));
  P->logroot = maxlog;

  std::vector<long long> Ns;
  const int last = P->ndim - 1;
  long long Nline = P->aN[last];
  long long Nf = P->aN[last];
  if (P->path == PATH_1D_MULTI) {
    Nline = P->mr;  // rows carry no residue twiddles
    Nf = (long long)P->qr * P->mr;
  }
  Ns.push_back(Nline);                               // 0: line pre/post
  Ns.push_back(2 * Nf);                              // 1: RCM factor / explicit unpack
  Ns.push_back(P->ndim > 1 ? P->aN[0] : 1);          // 2: axis 0
  Ns.push_back(P->ndim > 2 ? P->aN[1] : 1);          // 3: axis 1
  Ns.push_back(P->path == PATH_1D_MULTI ? (long long)P->nsh * P->pc : 1);  // 4: 1D column residues
  Ns.push_back(P->path == PATH_1D_MULTI ? Nf : 1);   // 5: four-step twiddle

  std::vector<cx<T>> host;
  auto push = [&](double c, double s) {
    cx<T> v;
    v.x = (T)c;
    v.y = (T)s;
    host.push_back(v);
  };
  // FFT roots: zeta_{2^L}^k for every L <= kRootMaxLog, table L at element 2^L - 1
  const size_t root_off = 0;
  for (int lg = 0; lg <= kRootMaxLog; ++lg)
    for (long long k = 0; k < (1LL << lg); ++k) {
      double c, s;
      zeta64(k, 1LL << lg, &c, &s);
      push(c, s);
    }
  struct Off { size_t lo, hi; int lobits; long long N; };
  std::vector<Off> offs;
  for (size_t ti = 0; ti < Ns.size(); ++ti) {
    const long long N = Ns[ti];
    Off o;
    // the residue tables of the strided axes (2, 3: axes 0 and 1; 4: the 1D column residues) are
    // single-level: the column kernels read each entry with one load, no product (1D 2^20 x64 FP32:
    // forward column pass 0.416 -> 0.384 ms); the other tables keep two levels above 4096 points
    const bool col_table = ti >= 2 && ti <= 4;
    if (col_table && N > kColTableMax)
      return fail(HDC_ERR_UNSUPPORTED, "padded transform length %lld of a strided axis exceeds 2^22", N);
    o.lobits = col_table ? ilog2(N) : tw_lobits(N);
    o.N = N;
    o.lo = host.size();
    tw_levels<T>(N, o.lobits, host);
    o.hi = o.lo + ((size_t)1 << o.lobits);
    offs.push_back(o);
  }
  const size_t bytes = host.size() * sizeof(cx<T>);
  void* dptr = nullptr;
  hipError_t e = hipMalloc(&dptr, bytes);
  if (e != hipSuccess) return fail(HDC_ERR_ALLOC, "hipMalloc(%zu) for twiddle tables: %s", bytes, hipGetErrorString(e));
  e = hipMemcpy(dptr, host.data(), bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(dptr);
    return fail(HDC_ERR_HIP, "hipMemcpy twiddles: %s", hipGetErrorString(e));
  }
  P->tables = dptr;
  const cx<T>* base = reinterpret_cast<const cx<T>*>(dptr);
  P->root = base + root_off;
  auto mk = [&](const Off& o) {
    TwDev t;
    t.lo = base + o.lo;
    t.hi = base + o.hi;
    t.lobits = o.lobits;
    t.N = (int)o.N;
    t.single = (1LL << o.lobits) >= o.N;
    return t;
  };
  P->tw_line = mk(offs[0]);
  P->tw_2nf = mk(offs[1]);
  P->tw_ax[0] = mk(offs[2]);
  P->tw_ax[1] = mk(offs[3]);
  P->tw_colN = mk(offs[4]);
  P->tw_colX = mk(offs[5]);
  return ok();
}

// ---------------------------------------------------------------------------
// launch records: the executors below either launch directly or, while a
// recorder is installed on this thread, append a record (used to group the
// launches of many problems of an uneven batch)
// ---------------------------------------------------------------------------
enum RecType { REC_LINE = 0, REC_COLF = 1, REC_COLI = 2, REC_CS = 3, REC_PAD = 4 };

template <typename T>
struct Rec {
  int type = 0, logm = 0, pcap = 1, narr = 1, which = 0;
  dim3 grid;
  LineParams<T> line{};
  ColParams<T> col{};
  CsParams<T> cs{};
  SimpleParams pad{};
};

struct RecSink {
  std::vector<Rec<float>> f32;
  std::vector<Rec<double>> f64;
  template <typename T>
  std::vector<Rec<T>>& get() {
    if constexpr (sizeof(T) == 4) return f32;
    else return f64;
  }
};

// ---------------------------------------------------------------------------
// launch dispatch
// ---------------------------------------------------------------------------
template <typename T>
static hipError_t call_line(const LineParams<T>& L, int logm, int pcap, dim3 grid, hipStream_t s,
                            const LineParams<T>* tab = nullptr) {
  if (g_sink && !tab) {
    Rec<T> r;
    r.type = REC_LINE;
    r.logm = logm;
    r.pcap = pcap;
    r.grid = grid;
    r.line = L;
    r.line.njobs = (int)grid.x;
    g_sink->get<T>().push_back(r);
    return hipSuccess;
  }
  switch (logm) {
    case 0: return launch_line_lm<T, 0>(L, pcap, grid, s, tab);
    case 1: return launch_line_lm<T, 1>(L, pcap, grid, s, tab);
    case 2: return launch_line_lm<T, 2>(L, pcap, grid, s, tab);
    case 3: return launch_line_lm<T, 3>(L, pcap, grid, s, tab);
    case 4: return launch_line_lm<T, 4>(L, pcap, grid, s, tab);
    case 5: return launch_line_lm<T, 5>(L, pcap, grid, s, tab);
    case 6: return launch_line_lm<T, 6>(L, pcap, grid, s, tab);
    case 7: return launch_line_lm<T, 7>(L, pcap, grid, s, tab);
    case 8: return launch_line_lm<T, 8>(L, pcap, grid, s, tab);
    case 9: return launch_line_lm<T, 9>(L, pcap, grid, s, tab);
    case 10: return launch_line_lm<T, 10>(L, pcap, grid, s, tab);
    case 11: return launch_line_lm<T, 11>(L, pcap, grid, s, tab);
    case 12:
      if constexpr (sizeof(T) == 4) return launch_line_lm<T, 12>(L, pcap, grid, s, tab);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template <typename T, bool FWD>
static hipError_t call_col(const ColParams<T>& C, int logm, int pcap, int narr, dim3 grid, hipStream_t s,
                           const ColParams<T>* tab = nullptr) {
  if (!C.twN.single) return hipErrorInvalidValue;  // the column kernels read a single-level residue table
  if (g_sink && !tab) {
    Rec<T> r;
    r.type = FWD ? REC_COLF : REC_COLI;
    r.logm = logm;
    r.pcap = pcap;
    r.narr = narr;
    r.grid = grid;
    r.col = C;
    g_sink->get<T>().push_back(r);
    return hipSuccess;
  }
  switch (logm) {
    case 0: return launch_col_lm<T, 0, FWD>(C, pcap, narr, grid, s, tab);
    case 1: return launch_col_lm<T, 1, FWD>(C, pcap, narr, grid, s, tab);
    case 2: return launch_col_lm<T, 2, FWD>(C, pcap, narr, grid, s, tab);
    case 3: return launch_col_lm<T, 3, FWD>(C, pcap, narr, grid, s, tab);
    case 4: return launch_col_lm<T, 4, FWD>(C, pcap, narr, grid, s, tab);
    case 5: return launch_col_lm<T, 5, FWD>(C, pcap, narr, grid, s, tab);
    case 6: return launch_col_lm<T, 6, FWD>(C, pcap, narr, grid, s, tab);
    case 7: return launch_col_lm<T, 7, FWD>(C, pcap, narr, grid, s, tab);
    case 8: return launch_col_lm<T, 8, FWD>(C, pcap, narr, grid, s, tab);
    case 9: return launch_col_lm<T, 9, FWD>(C, pcap, narr, grid, s, tab);
    case 10: return launch_col_lm<T, 10, FWD>(C, pcap, narr, grid, s, tab);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
static hipError_t call_cs(const CsParams<T>& C, int logm, int which, int pcap, dim3 grid, hipStream_t s,
                          bool direct = false) {
  // the column forms (1, 2) read a single-level residue table
  if ((which == 1 || which == 2) && !C.twN.single) return hipErrorInvalidValue;
  if (g_sink && !direct) {
    Rec<T> r;
    r.type = REC_CS;
    r.logm = logm;
    r.pcap = pcap;
    r.which = which;
    r.grid = grid;
    r.cs = C;
    g_sink->get<T>().push_back(r);
    return hipSuccess;
  }
  switch (logm) {
    case 0: return launch_cs_lm<T, 0>(C, which, pcap, grid, s);
    case 1: return launch_cs_lm<T, 1>(C, which, pcap, grid, s);
    case 2: return launch_cs_lm<T, 2>(C, which, pcap, grid, s);
    case 3: return launch_cs_lm<T, 3>(C, which, pcap, grid, s);
    case 4: return launch_cs_lm<T, 4>(C, which, pcap, grid, s);
    case 5: return launch_cs_lm<T, 5>(C, which, pcap, grid, s);
    case 6: return launch_cs_lm<T, 6>(C, which, pcap, grid, s);
    case 7: return launch_cs_lm<T, 7>(C, which, pcap, grid, s);
    case 8: return launch_cs_lm<T, 8>(C, which, pcap, grid, s);
    case 9: return launch_cs_lm<T, 9>(C, which, pcap, grid, s);
    case 10: return launch_cs_lm<T, 10>(C, which, pcap, grid, s);
    case 11: return launch_cs_lm<T, 11>(C, which, pcap, grid, s);
    case 12:
      if constexpr (sizeof(T) == 4) return launch_cs_lm<T, 12>(C, which, pcap, grid, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

#define LAUNCH_TRY(expr)                                                                        \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) return fail(HDC_ERR_HIP, "launch %s: %s", #expr, hipGetErrorString(e_)); \
    prof_mark(P, st);                                                                           \
  } while (0)

// line pairs per workgroup of the multi-D line kernel: as many as keep the
// pairs' spectra within about 40 KB of LDS (several workgroups per CU)
template <typename T>
static int line_ppw(int m, int q, int nspec) {
  const size_t per = line_lds_bytes<T>(m, q, nspec);
  int ppw = 1;
  while (ppw < kLinePairsMax && (size_t)(2 * ppw) * per <= 40 * 1024) ppw *= 2;
  return ppw;
}

static RawGeom geom_1d(int L, long long bstride, int rev) {
  RawGeom g;
  g.batch_stride = bstride;
  g.row_stride = 0;
  g.rows = 1;
  g.mid = 1;
  g.Ld = L;
  g.Lhd = (L + 1) / 2;
  g.rev = rev;
  g.Lhd_c = 0;
  return g;
}

static RawGeom geom_nd(const int* L, int nd, long long bstride, int rev) {
  RawGeom g;
  g.batch_stride = bstride;
  g.rows = L[0];
  g.Ld = L[nd - 1];
  g.Lhd = (L[nd - 1] + 1) / 2;
  g.mid = (nd == 3) ? L[1] : 1;
  g.row_stride = (long long)g.mid * g.Ld;
  g.rev = rev;
  g.Lhd_c = 0;
  return g;
}

// Complex elements of the cached kernel spectra per batch element: the residue rows (1D multi-pass), the
// q m spectrum values of the line (1D one workgroup), or of every innermost line (2D: N0 lines, 3D: N0 N1).
static long long spec_elems(const hdc_plan_s* P) {
  switch (P->path) {
    case PATH_1D_MULTI: return P->regF;
    case PATH_1D_ONE: return P->aN[0];
    case PATH_2D: return (long long)P->aN[0] * P->aN[1];
    default: return (long long)P->aN[0] * P->aN[1] * P->aN[2];
  }
}

// What one run of the pass structure does with the workspace regions R0..R3
// (B x regF complex elements each).
enum ExecMode {
  EXEC_FWD = 0,        // h = conv(f, g); the product lines overwrite R0 in place
  EXEC_FWD_SAVE = 1,   // the same, with the product lines in R2: R0, R1 keep f's and g's outer-axis spectra
  EXEC_TWIN = 2,       // the adjoint: df = R(conv(g, R(dh))) and dg = R(conv(f, R(dh))); f and g transformed here
  EXEC_TWIN_SAVED = 3  // the adjoint with f's and g's outer-axis spectra taken from R0, R1 (EXEC_FWD_SAVE)
};

// Runs the pass structure on (f, g) -> h of the executed extents Le.  In the
// twin modes the arguments are (f, g, dh) -> (df, dg): dh is read reversed, the
// two outputs are written reversed, and the R(dh) spectra are formed once and
// multiplied with g's (pass 0 of the twin line kernel, into R2) and f's (pass 1,
// into R3).
template <typename T>
static hdc_status run_exec(const hdc_plan_s* P, const T* f, const T* g, T* h, char* ws, hipStream_t st, int rf,
                           int rg, int rh, long long B, bool gfull = false, int gmode = 0,
                           void* gspec = nullptr, int mode = EXEC_FWD, const T* dh = nullptr, T* dg = nullptr,
                           const T* const* xs = nullptr) {
  // xs: the P->nin input arrays of an n-ary plan (f, g unused)
  // gfull: g has f's extents even in a plan for a shorter kernel (the adjoint's dg pass).
  // gmode (1D multi-pass only): 1 transforms the kernel g alone and stores its row
  // spectra in gspec; 2 convolves f with the row spectra cached in gspec.
  const int* Lgx = gfull ? P->Le : P->Lge;
  const int nd = P->ndim;
  const int last = nd - 1;
  const bool twin = mode == EXEC_TWIN || mode == EXEC_TWIN_SAVED;
  long long nreal = 1, nreal_g = 1;  // reals per batch element of f (and h), of g
  for (int a = 0; a < nd; ++a) nreal *= P->Le[a];
  for (int a = 0; a < nd; ++a) nreal_g *= Lgx[a];
  const long long regF = P->regF;
  cx<T>* Rg[4];
  Rg[0] = reinterpret_cast<cx<T>*>(ws + P->off_F);
  Rg[1] = reinterpret_cast<cx<T>*>(ws + P->off_G);
  Rg[2] = reinterpret_cast<cx<T>*>(ws + P->off_R2);
  Rg[3] = reinterpret_cast<cx<T>*>(ws + P->off_R3);
  const long long garr = (long long)(Rg[1] - Rg[0]);  // R0 -> R1 offset in complex elements
  // line kernel: first array, second array, product lines (twin: pass-1 first array and products)
  cx<T>* lnF = Rg[0];
  cx<T>* lnG = Rg[1];
  cx<T>* lnH = mode == EXEC_FWD_SAVE ? Rg[2] : nullptr;
  cx<T>* lnF2 = nullptr;
  cx<T>* lnH2 = nullptr;
  if (twin) {
    lnF = Rg[1];   // g's lines: pass 0 gives df
    lnG = Rg[2];   // R(dh)'s lines
    lnF2 = Rg[0];  // f's lines: pass 1 gives dg
    lnH = Rg[2];   // in place over R(dh) (each workgroup has its lines in LDS before it writes)
    lnH2 = Rg[3];
  }
  // regions the inverse passes read, with their raw outputs
  cx<T>* invR[2] = {lnH ? lnH : Rg[0], lnH2};
  T* invOut[2] = {h, dg};
  const int ninv = twin ? 2 : 1;
  const bool fg_fwd = mode != EXEC_TWIN_SAVED;  // the forward passes of f and g run here

  const int nin = xs ? P->nin : 2;
  auto line_common = [&](LineParams<T>& L) {
    L.nin = nin;
    L.ws_arr = garr;
    L.variant = P->mul;
    L.ws_batch = regF;
    L.wsF = lnF;
    L.wsG = lnG;
    L.wsH = lnH;
    L.twin = twin ? 1 : 0;
    L.wsF2 = lnF2;
    L.wsH2 = lnH2;
    L.twN = as_tw<T>(P->tw_line);
    L.tw2Nf = as_tw<T>(P->tw_2nf);
    L.rootpyr = reinterpret_cast<const cx<T>*>(P->root);
  };

  if (P->path == PATH_1D_ONE) {
    LineParams<T> L{};
    L.m = P->am[0];
    L.p = P->ap[0];
    L.q = P->aq[0];
    L.N = P->aN[0];
    L.Lin = P->Lh;
    L.Lin_g = (Lgx[0] + 1) / 2;
    if (!xs && !twin && L.Lin_g < L.Lin) L.p_g = std::min(L.p, (int)cdiv(L.Lin_g, L.m));  // g's blocks with data
    L.Lout = P->Lh;
    L.qrow = 1;
    L.Nf = P->aN[0];
    L.kind = LINE_1D;
    L.scale = (T)(1.0 / (double)P->aN[0]);
    line_common(L);
    L.wsF = L.wsG = L.wsH = L.wsF2 = L.wsH2 = nullptr;
    if (xs) {
      for (int a = 0; a < nin; ++a) L.xin[a] = xs[a];
      L.gf = geom_1d(P->Le[0], nreal, 0);
      L.h = h;
      L.gh = geom_1d(P->Le[0], nreal, 0);
    } else if (!twin) {
      L.f = f;
      L.g = g;
      L.h = h;
      L.gf = geom_1d(P->Le[0], nreal, rf);
      L.gg = geom_1d(Lgx[0], nreal_g, rg);
      L.gh = geom_1d(P->Le[0], nreal, rh);
      L.gmode = gmode;
      L.gspec = reinterpret_cast<cx<T>*>(gspec);
      L.spec_batch = spec_elems(P);
      L.spec_line = 0;
    } else {
      L.f = g;  // pass 0: g with R(dh) -> df
      L.gf = geom_1d(P->Le[0], nreal, 0);
      L.g = dh;
      L.gg = geom_1d(P->Le[0], nreal, 1);
      L.Lin_g = P->Lh;
      L.h = h;
      L.gh = geom_1d(P->Le[0], nreal, 1);
      L.f2 = f;  // pass 1: f with R(dh) -> dg
      L.gf2 = geom_1d(P->Le[0], nreal, 0);
      L.h2 = dg;
      L.gh2 = geom_1d(P->Le[0], nreal, 1);
    }
    LAUNCH_TRY(call_line<T>(L, ilog2(L.m), pcap_of(L.p), dim3(1, (unsigned)B), st));
    return ok();
  }

  if (P->path == PATH_1D_MULTI) {
    const int mr = P->mr, pc = P->pc, n = P->nsh, qr = P->qr;
    const int Nf = qr * mr;
    auto colf = [&](const T* a0, RawGeom g0, const T* a1, RawGeom g1, cx<T>* out, int narr, int arr0) -> hdc_status {
      ColParams<T> C{};
      C.m = pc;
      C.p = 1;
      C.q = n;
      C.N = n * pc;
      C.Lrows = pc;
      C.C = mr;
      C.nslab = 1;
      C.out = out;
      C.out_row = mr;
      C.out_batch = regF;
      C.out_arr = garr;
      C.rawin0 = a0;
      C.rawin1 = a1;
      C.graw0 = g0;
      C.graw1 = g1;
      C.arr0 = arr0;
      C.lin_pitch = mr;
      C.twN = as_tw<T>(P->tw_colN);
      C.rootpyr = reinterpret_cast<const cx<T>*>(P->root);
      LAUNCH_TRY((call_col<T, true>(C, ilog2(pc), 1, narr, dim3(1, (unsigned)B, narr), st)));
      return ok();
    };
    hdc_status s;
    if (xs) {
      const RawGeom gx = geom_1d(P->Le[0], nreal, 0);
      for (int a = 0; a < nin; a += 2)
        if ((s = colf(xs[a], gx, xs[std::min(a + 1, nin - 1)], gx, Rg[0] + a * garr, std::min(2, nin - a), 0)) != HDC_OK)
          return s;
    } else if (twin) {
      if (fg_fwd && (s = colf(f, geom_1d(P->Le[0], nreal, 0), g, geom_1d(P->Le[0], nreal, 0), Rg[0], 2, 0)) != HDC_OK)
        return s;
      const RawGeom gu = geom_1d(P->Le[0], nreal, 1);
      if ((s = colf(dh, gu, dh, gu, Rg[2], 1, 0)) != HDC_OK) return s;
    } else if (gmode == 1) {  // the kernel alone (array 1)
      const RawGeom gg = geom_1d(Lgx[0], nreal_g, rg);
      if ((s = colf(g, gg, g, gg, Rg[0], 1, 1)) != HDC_OK) return s;
    } else if (gmode == 2) {  // f alone
      const RawGeom gf = geom_1d(P->Le[0], nreal, rf);
      if ((s = colf(f, gf, f, gf, Rg[0], 1, 0)) != HDC_OK) return s;
    } else {
      if ((s = colf(f, geom_1d(P->Le[0], nreal, rf), g, geom_1d(Lgx[0], nreal_g, rg), Rg[0], 2, 0)) != HDC_OK)
        return s;
    }

    LineParams<T> L{};
    L.m = mr;
    L.p = 1;
    L.q = 1;
    L.N = mr;
    L.Lin = mr;
    L.Lout = mr;
    L.qrow = qr;
    L.Nf = Nf;
    L.kind = LINE_ROWS;
    L.qres = qr;
    L.scale = (T)(1.0 / (double)Nf);
    L.line_stride = mr;
    line_common(L);
    L.twRow = as_tw<T>(P->tw_colX);
    L.gmode = gmode;
    L.gspec = reinterpret_cast<cx<T>*>(gspec);
    LAUNCH_TRY(call_line<T>(L, ilog2(mr), 1, dim3(qr / 2 + 1, (unsigned)B), st));
    if (gmode == 1) return ok();

    for (int k = 0; k < ninv; ++k) {
      ColParams<T> I{};
      I.m = pc;
      I.p = 1;
      I.q = n;
      I.N = n * pc;
      I.Lrows = pc;
      I.C = mr;
      I.nslab = 1;
      I.in = invR[k];
      I.in_row = mr;
      I.in_batch = regF;
      I.rawout = invOut[k];
      I.graw0 = geom_1d(P->Le[0], nreal, twin ? 1 : rh);
      I.lin_pitch = mr;
      I.twN = as_tw<T>(P->tw_colN);
      I.rootpyr = reinterpret_cast<const cx<T>*>(P->root);
      LAUNCH_TRY((call_col<T, false>(I, ilog2(pc), 1, 1, dim3(1, (unsigned)B, 1), st)));
    }
    return ok();
  }

  // ---- multi-dimensional
  const int Lh = P->Lh;
  const int N0 = P->aN[0];
  const int N1 = nd == 3 ? P->aN[1] : 1;
  const long long Cin0 = (nd == 3) ? (long long)P->Le[1] * Lh : Lh;  // columns of the axis-0 pass
  const long long row0 = (nd == 3) ? (long long)N1 * Lh : Lh;          // workspace row pitch, axis 0
  // axis-0 forward pass of raw arrays a0 (and a1) into region out (and out + garr)
  auto colf0 = [&](const T* a0, RawGeom g0, const T* a1, RawGeom g1, cx<T>* out, int narr) -> hdc_status {
    ColParams<T> C{};
    C.m = P->am[0];
    C.p = P->ap[0];
    C.q = P->aq[0];
    C.N = N0;
    C.Lrows = P->Le[0];
    C.C = (int)Cin0;
    C.nslab = 1;
    C.out = out;
    C.out_row = row0;
    C.out_batch = regF;
    C.out_arr = garr;
    C.rawin0 = a0;
    C.rawin1 = a1;
    C.graw0 = g0;
    C.graw1 = g1;
    C.twN = as_tw<T>(P->tw_ax[0]);
    C.rootpyr = reinterpret_cast<const cx<T>*>(P->root);
    LAUNCH_TRY((call_col<T, true>(C, ilog2(C.m), pcap_of(C.p), narr, dim3(1, (unsigned)B, narr), st)));
    return ok();
  };
  // axis-1 forward pass (3D) in place over region reg (and reg + garr)
  auto colf1 = [&](cx<T>* reg, int narr) -> hdc_status {
    ColParams<T> C{};
    C.m = P->am[1];
    C.p = P->ap[1];
    C.q = P->aq[1];
    C.N = N1;
    C.Lrows = P->Le[1];
    C.C = Lh;
    C.nslab = N0;
    C.in = reg;
    C.in_row = Lh;
    C.in_slab = (long long)N1 * Lh;
    C.in_batch = regF;
    C.in_arr = garr;
    C.out = reg;
    C.out_row = Lh;
    C.out_slab = (long long)N1 * Lh;
    C.out_batch = regF;
    C.out_arr = garr;
    C.twN = as_tw<T>(P->tw_ax[1]);
    C.rootpyr = reinterpret_cast<const cx<T>*>(P->root);
    LAUNCH_TRY((call_col<T, true>(C, ilog2(C.m), pcap_of(C.p), narr, dim3(1, (unsigned)(B * N0), narr), st)));
    return ok();
  };
  hdc_status s;
  if (xs) {
    const RawGeom gx = geom_nd(P->Le, nd, nreal, 0);
    for (int a = 0; a < nin; a += 2)
      if ((s = colf0(xs[a], gx, xs[std::min(a + 1, nin - 1)], gx, Rg[0] + a * garr, std::min(2, nin - a))) != HDC_OK)
        return s;
    for (int a = 0; a < nin && nd == 3; a += 2)
      if ((s = colf1(Rg[0] + a * garr, std::min(2, nin - a))) != HDC_OK) return s;
  } else if (twin) {
    const RawGeom gfw = geom_nd(P->Le, nd, nreal, 0);
    if (fg_fwd) {
      if ((s = colf0(f, gfw, g, gfw, Rg[0], 2)) != HDC_OK) return s;
      if (nd == 3 && (s = colf1(Rg[0], 2)) != HDC_OK) return s;
    }
    const RawGeom gu = geom_nd(P->Le, nd, nreal, 1);
    if ((s = colf0(dh, gu, dh, gu, Rg[2], 1)) != HDC_OK) return s;
    if (nd == 3 && (s = colf1(Rg[2], 1)) != HDC_OK) return s;
  } else {
    RawGeom g1 = geom_nd(Lgx, nd, nreal_g, rg);
    if (Lgx[nd - 1] != P->Le[nd - 1]) g1.Lhd_c = (P->Le[nd - 1] + 1) / 2;  // columns index f's packed layout
    if (gmode == 1) {  // the kernel alone, into R1
      if ((s = colf0(g, g1, g, g1, Rg[1], 1)) != HDC_OK) return s;
      if (nd == 3 && (s = colf1(Rg[1], 1)) != HDC_OK) return s;
    } else if (gmode == 2) {  // f alone, into R0
      const RawGeom g0 = geom_nd(P->Le, nd, nreal, rf);
      if ((s = colf0(f, g0, f, g0, Rg[0], 1)) != HDC_OK) return s;
      if (nd == 3 && (s = colf1(Rg[0], 1)) != HDC_OK) return s;
    } else {
      if ((s = colf0(f, geom_nd(P->Le, nd, nreal, rf), g, g1, Rg[0], 2)) != HDC_OK) return s;
      if (nd == 3 && (s = colf1(Rg[0], 2)) != HDC_OK) return s;
    }
  }
  {
    LineParams<T> L{};
    L.m = P->am[last];
    L.p = P->ap[last];
    L.q = P->aq[last];
    L.N = P->aN[last];
    L.Lin = Lh;
    L.Lout = Lh;
    L.qrow = 1;
    L.Nf = P->aN[last];
    L.kind = nd == 2 ? LINE_2D : LINE_3D;
    L.N1 = N0;
    L.N2 = N1;
    double tot = (double)P->aN[last] * N0 * (nd == 3 ? N1 : 1);
    L.scale = (T)(P->extra_scale / tot);
    L.line_stride = Lh;
    line_common(L);
    L.npairs = line_npairs(L.kind, N0, N1);
    L.ppw = line_ppw<T>(L.m, L.q, 2 * nin);
    const int lhg = (Lgx[last] + 1) / 2;  // g's packed last-axis extent: its blocks with data
    if (!xs && !twin && lhg < Lh) L.p_g = std::min(L.p, (int)cdiv(lhg, L.m));
    L.gmode = gmode;
    L.gspec = reinterpret_cast<cx<T>*>(gspec);
    L.spec_line = (long long)P->aN[last];
    L.spec_batch = spec_elems(P);
    const unsigned jobs = (unsigned)cdiv(L.npairs, L.ppw);
    LAUNCH_TRY(call_line<T>(L, ilog2(L.m), pcap_of(L.p), dim3(jobs, (unsigned)B), st));
    if (gmode == 1) return ok();
  }
  for (int k = 0; k < ninv && nd == 3; ++k) {
    ColParams<T> I{};
    I.m = P->am[1];
    I.p = P->ap[1];
    I.q = P->aq[1];
    I.N = N1;
    I.Lrows = P->Le[1];
    I.C = Lh;
    I.nslab = N0;
    I.in = invR[k];
    I.in_row = Lh;
    I.in_slab = (long long)N1 * Lh;
    I.in_batch = regF;
    I.out = invR[k];
    I.out_row = Lh;
    I.out_slab = (long long)N1 * Lh;
    I.out_batch = regF;
    I.twN = as_tw<T>(P->tw_ax[1]);
    I.rootpyr = reinterpret_cast<const cx<T>*>(P->root);
    LAUNCH_TRY((call_col<T, false>(I, ilog2(I.m), pcap_of(I.p), 1, dim3(1, (unsigned)(B * N0), 1), st)));
  }
  for (int k = 0; k < ninv; ++k) {
    ColParams<T> I{};
    I.m = P->am[0];
    I.p = P->ap[0];
    I.q = P->aq[0];
    I.N = N0;
    I.Lrows = P->Le[0];
    I.C = (int)Cin0;
    I.nslab = 1;
    I.in = invR[k];
    I.in_row = row0;
    I.in_batch = regF;
    I.rawout = invOut[k];
    I.graw0 = geom_nd(P->Le, nd, nreal, twin ? 1 : rh);
    I.twN = as_tw<T>(P->tw_ax[0]);
    I.rootpyr = reinterpret_cast<const cx<T>*>(P->root);
    LAUNCH_TRY((call_col<T, false>(I, ilog2(I.m), pcap_of(I.p), 1, dim3(1, (unsigned)B, 1), st)));
  }
  return ok();
}

// conjugate-symmetry variant (Sec. 3, Sec. 5)
template <typename T>
static hdc_status run_exec_cs(const hdc_plan_s* P, const T* f, const T* g, T* h, char* ws, hipStream_t st, int rf,
                              int rg, int rh, long long B, bool gfull = false) {
  // gfull: g has f's extents even in a plan for a shorter kernel (the adjoint's dg pass)
  const int nd = P->ndim;
  long long nreal = 1;
  for (int a = 0; a < nd; ++a) nreal *= P->Lu[a];
  cx<T>* F = reinterpret_cast<cx<T>*>(ws + P->off_F);
  cx<T>* G = reinterpret_cast<cx<T>*>(ws + P->off_G);
  const long long garr = (long long)(G - F);
  CsParams<T> C{};
  C.m = P->am[0];
  C.p = P->ap[0];
  C.q = P->aq[0];
  C.N = P->aN[0];
  C.nres = P->nres0;
  C.L = P->Lu[0];
  C.in_batch = nreal;
  C.f = f;
  C.g = g;
  C.h = h;
  C.rev_f = rf;
  C.rev_g = rg;
  C.rev_h = rh;
  C.rootpyr = reinterpret_cast<const cx<T>*>(P->root);
  if (P->unequal && !gfull) {
    // the kernel's own extents as (first axis, middle, last); f's last extent splits the column index
    C.g_short = 1;
    C.gL0 = P->Lg[0];
    C.gL1 = nd == 3 ? P->Lg[1] : 1;
    C.gL2 = nd == 1 ? 1 : P->Lg[nd - 1];
    C.fL2 = nd == 1 ? 1 : P->Lu[nd - 1];
    C.g_batch = 1;
    for (int a = 0; a < nd; ++a) C.g_batch *= P->Lg[a];
  }
  if (nd == 1 && P->path == PATH_1D_MULTI) {
    // rows of m: real length-q transform over the rows (one block of q rows, one residue)
    const int m = P->mr, q = P->qr;
    C.m = q;
    C.p = 1;
    C.q = 1;
    C.N = q;
    C.nres = 1;
    C.L = P->ap[0];
    C.C = m;
    C.in_row = m;
    C.ws_row = m;
    C.ws_batch = P->regF;
    C.ws_arr = garr;
    C.ws = F;
    C.lin1d = P->Lu[0];
    C.twN = as_tw<T>(P->tw_colN);
    // two real columns per complex transform when the workspace holds the
    // column pairs 16-byte (FP64: 32-byte) aligned
    const bool pairs = (m % 2 == 0) && (P->regF % 2 == 0) && (garr % 2 == 0) &&
                       (reinterpret_cast<uintptr_t>(F) % (4 * sizeof(T)) == 0);
    LAUNCH_TRY(call_cs<T>(C, ilog2(q), pairs ? 3 : 1, 1, dim3(1, (unsigned)B, 2), st));
    LineParams<T> L{};
    L.m = m;
    L.p = 1;
    L.q = 1;
    L.N = m;
    L.Lin = m;
    L.Lout = m;
    L.qrow = 1;
    L.Nf = q * m;
    L.variant = MUL_ELEM;
    L.kind = LINE_ROWS;  // residue rows, two per workgroup, elementwise product
    L.qres = P->Nret;
    L.scale = (T)(1.0 / ((double)q * m));
    L.line_stride = m;
    L.ws_batch = P->regF;
    L.wsF = F;
    L.wsG = G;
    L.twN = as_tw<T>(P->tw_line);
    L.tw2Nf = as_tw<T>(P->tw_2nf);
    L.twRow = as_tw<T>(P->tw_colX);
    L.rootpyr = reinterpret_cast<const cx<T>*>(P->root);
    LAUNCH_TRY(call_line<T>(L, ilog2(m), 1, dim3((unsigned)cdiv(P->Nret, 2), (unsigned)B), st));
    LAUNCH_TRY(call_cs<T>(C, ilog2(q), pairs ? 4 : 2, 1, dim3(1, (unsigned)B, 1), st));
    return ok();
  }
  if (nd == 1) {
    C.scale = (T)(1.0 / (double)P->aN[0]);
    C.twN = as_tw<T>(P->tw_line);
    LAUNCH_TRY(call_cs<T>(C, ilog2(C.m), P->mix ? 5 : 0, pcap_of(C.p), dim3(1, (unsigned)B), st));
    return ok();
  }
  const int Ld = P->Lu[nd - 1];
  const int N1 = nd == 3 ? P->aN[1] : 1;
  C.C = (nd == 3) ? P->Lu[1] * Ld : Ld;
  C.in_row = C.C;
  C.ws_row = (nd == 3) ? (long long)N1 * Ld : Ld;
  C.ws_batch = P->regF;
  C.ws_arr = garr;
  C.ws = F;
  C.twN = as_tw<T>(P->tw_ax[0]);
  // first-axis lines held: all retained ones, or (mixed variant) those of residues 1 .. ceil(q/2) - 1,
  // stored from line 0 on, with the inverse adding to the sub-plan's h
  const int nl = P->sub ? P->Nmid : P->Nret;
  if (P->sub) {
    C.r_lo = 1;
    C.r_hi = (C.q + 1) / 2;
    C.row0 = P->mid_row0;
    C.accum = 1;
  }
  LAUNCH_TRY(call_cs<T>(C, ilog2(C.m), 1, pcap_of(C.p), dim3(1, (unsigned)B, 2), st));
  if (nd == 3) {
    ColParams<T> X{};
    X.m = P->am[1];
    X.p = P->ap[1];
    X.q = P->aq[1];
    X.N = N1;
    X.Lrows = P->Lu[1];
    X.C = Ld;
    X.nslab = nl;
    X.in = F;
    X.in_row = Ld;
    X.in_slab = (long long)N1 * Ld;
    X.in_batch = P->regF;
    X.in_arr = garr;
    X.out = F;
    X.out_row = Ld;
    X.out_slab = (long long)N1 * Ld;
    X.out_batch = P->regF;
    X.out_arr = garr;
    X.twN = as_tw<T>(P->tw_ax[1]);
    X.rootpyr = reinterpret_cast<const cx<T>*>(P->root);
    LAUNCH_TRY((call_col<T, true>(X, ilog2(X.m), pcap_of(X.p), 2, dim3(1, (unsigned)(B * nl), 2), st)));
  }
  {
    LineParams<T> L{};
    L.m = P->am[nd - 1];
    L.p = P->ap[nd - 1];
    L.q = P->aq[nd - 1];
    L.N = P->aN[nd - 1];
    L.Lin = Ld;
    L.Lout = Ld;
    L.qrow = 1;
    L.Nf = L.N;
    L.variant = MUL_ELEM;
    L.kind = LINE_PLAIN;
    L.scale = (T)(1.0 / ((double)P->aN[0] * N1 * L.N));
    L.line_stride = Ld;
    L.ws_batch = P->regF;
    L.wsF = F;
    L.wsG = G;
    L.twN = as_tw<T>(P->tw_line);
    L.tw2Nf = as_tw<T>(P->tw_2nf);
    L.rootpyr = reinterpret_cast<const cx<T>*>(P->root);
    L.npairs = (long long)nl * N1;
    L.ppw = line_ppw<T>(L.m, L.q, 2);
    const unsigned jobs = (unsigned)cdiv(L.npairs, L.ppw);
    LAUNCH_TRY(call_line<T>(L, ilog2(L.m), pcap_of(L.p), dim3(jobs, (unsigned)B), st));
  }
  if (nd == 3) {
    ColParams<T> X{};
    X.m = P->am[1];
    X.p = P->ap[1];
    X.q = P->aq[1];
    X.N = N1;
    X.Lrows = P->Lu[1];
    X.C = Ld;
    X.nslab = nl;
    X.in = F;
    X.in_row = Ld;
    X.in_slab = (long long)N1 * Ld;
    X.in_batch = P->regF;
    X.out = F;
    X.out_row = Ld;
    X.out_slab = (long long)N1 * Ld;
    X.out_batch = P->regF;
    X.twN = as_tw<T>(P->tw_ax[1]);
    X.rootpyr = reinterpret_cast<const cx<T>*>(P->root);
    LAUNCH_TRY((call_col<T, false>(X, ilog2(X.m), pcap_of(X.p), 1, dim3(1, (unsigned)(B * nl), 1), st)));
  }
  LAUNCH_TRY(call_cs<T>(C, ilog2(C.m), 2, pcap_of(C.p), dim3(1, (unsigned)B, 1), st));
  return ok();
}

template <typename T>
static hdc_status run_conv(const hdc_plan_s* P, const T* f, const T* g, T* h, char* ws, hipStream_t st, int rf,
                           int rg, int rh, bool gfull = false, int mode = EXEC_FWD) {
  if (P->sub) {
    // mixed variant, 2D/3D: residues 0 and q/2 of the first axis write h, the others add to it
    const hdc_status s = run_conv<T>(P->sub, f, g, h, ws, st, rf, rg, rh, gfull);
    if (s != HDC_OK || !P->Nmid) return s;
  }
  if (P->cs) return run_exec_cs<T>(P, f, g, h, ws, st, rf, rg, rh, P->batch, gfull);
  if (!P->expl) {
    // batch chunks reuse the same workspace slots, so a chunk's intermediate
    // spectra can stay resident in the memory-side cache between passes
    long long nreal = 1, nreal_g = 1;
    for (int a = 0; a < P->ndim; ++a) nreal *= P->Le[a];
    for (int a = 0; a < P->ndim; ++a) nreal_g *= gfull ? P->Le[a] : P->Lge[a];
    const long long chunk = (P->chunk > 0 && P->chunk < P->batch) ? P->chunk : P->batch;
    for (long long b0 = 0; b0 < P->batch; b0 += chunk) {
      const long long nb = std::min(chunk, P->batch - b0);
      hdc_status s = run_exec<T>(P, f + b0 * nreal, g + b0 * nreal_g, h + b0 * nreal, ws, st, rf, rg, rh, nb, gfull,
                                 0, nullptr, mode);
      if (s != HDC_OK) return s;
    }
    return ok();
  }
  const int nd = P->ndim;
  long long nu = 1, np = 1, ng = 1;
  for (int a = 0; a < nd; ++a) {
    nu *= P->Lu[a];
    np *= P->Mu[a];
    ng *= gfull ? P->Lu[a] : P->Lg[a];
  }
  T* fp = reinterpret_cast<T*>(ws + P->off_fpad);
  T* gp = reinterpret_cast<T*>(ws + P->off_gpad);
  T* hp = reinterpret_cast<T*>(ws + P->off_hpad);
  auto box = [&](const void* src, void* dst, const int* Ls, const int* Ld, long long sb, long long db,
                 int rev) -> hipError_t {
    SimpleParams S{};
    S.src = src;
    S.dst = dst;
    S.ndim = nd;
    for (int a = 0; a < 3; ++a) {
      S.Ls[a] = 1;
      S.Ld[a] = 1;
    }
    for (int a = 0; a < nd; ++a) {
      S.Ls[3 - nd + a] = Ls[a];
      S.Ld[3 - nd + a] = Ld[a];
    }
    S.src_batch = sb;
    S.dst_batch = db;
    S.batch = (int)P->batch;
    S.rev = rev;
    if (g_sink) {
      Rec<T> r;
      r.type = REC_PAD;
      r.pad = S;
      g_sink->get<T>().push_back(r);
      return hipSuccess;
    }
    return launch_pad<T>(S, st);
  };
  LAUNCH_TRY(box(f, fp, P->Lu, P->Mu, nu, np, rf));
  LAUNCH_TRY(box(g, gp, gfull ? P->Lu : P->Lg, P->Mu, ng, np, rg));
  hdc_status s = run_exec<T>(P, fp, gp, hp, ws, st, 0, 0, 0, P->batch);
  if (s != HDC_OK) return s;
  LAUNCH_TRY(box(hp, h, P->Mu, P->Lu, np, nu, rh));
  return ok();
}

// Adjoint.  Equal extents: df = R(conv(g, R(dh))), dg = R(conv(f, R(dh))).
// A shorter kernel g: df = R(conv(R(dh), g)) keeps g in the kernel slot; dg_k
// (k < Lg) = R(conv(R(dh), f))_k are the last Lg outputs per axis of a
// full-extent convolution, which no wrapped term reaches when M >= L + Lg - 1
// (a wrapped product lands at an index j = k + i - M <= L - Lg - 1); they are
// computed into a scratch region of f's extents and the Lg box is copied out.
// The twin adjoint (hybrid implicit-packing plans, equal extents): f, g and R(dh)
// are transformed once each; R(dh)'s spectra meet g's (-> df) and then f's (-> dg)
// inside one line-kernel launch.  `saved`: f's and g's outer-axis spectra are
// already in R0, R1 (left there by a forward with HDC_SAVE_SPECTRA).
template <typename T>
static hdc_status run_twin(const hdc_plan_s* P, const T* f, const T* g, const T* dh, T* df, T* dg, char* ws,
                           hipStream_t st, bool saved) {
  long long nreal = 1;
  for (int a = 0; a < P->ndim; ++a) nreal *= P->Le[a];
  const long long chunk = (P->chunk > 0 && P->chunk < P->batch) ? P->chunk : P->batch;
  for (long long b0 = 0; b0 < P->batch; b0 += chunk) {
    const long long nb = std::min(chunk, P->batch - b0);
    hdc_status s = run_exec<T>(P, f + b0 * nreal, g + b0 * nreal, df + b0 * nreal, ws, st, 0, 0, 0, nb, false, 0,
                               nullptr, saved ? EXEC_TWIN_SAVED : EXEC_TWIN, dh + b0 * nreal, dg + b0 * nreal);
    if (s != HDC_OK) return s;
  }
  return ok();
}

// the truncated convolution of the plan's nin arrays (Sec. 4.1)
template <typename T>
static hdc_status run_conv_nary(const hdc_plan_s* P, const T* const* xs, T* h, char* ws, hipStream_t st) {
  long long nreal = 1;
  for (int a = 0; a < P->ndim; ++a) nreal *= P->Le[a];
  const long long chunk = (P->chunk > 0 && P->chunk < P->batch) ? P->chunk : P->batch;
  const T* xb[kMaxNary];
  for (long long b0 = 0; b0 < P->batch; b0 += chunk) {
    const long long nb = std::min(chunk, P->batch - b0);
    for (int a = 0; a < P->nin; ++a) xb[a] = xs[a] + b0 * nreal;
    hdc_status s = run_exec<T>(P, nullptr, nullptr, h + b0 * nreal, ws, st, 0, 0, 0, nb, false, 0, nullptr, EXEC_FWD,
                               nullptr, nullptr, xb);
    if (s != HDC_OK) return s;
  }
  return ok();
}

template <typename T>
static hdc_status backward_t(const hdc_plan_s* P, const T* f, const T* g, const T* dh, T* df, T* dg, char* ws,
                             hipStream_t st) {
  hdc_status s;
  if (P->twin_ok && df && dg) {
    const bool saved = P->save && P->saved_ws == ws && P->saved_f == f && P->saved_g == g;
    return run_twin<T>(P, f, g, dh, df, dg, ws, st, saved);
  }
  P->saved_ws = nullptr;  // the single-output adjoint below runs a forward over R0, R1
  if (!P->unequal) {
    if (df && (s = run_conv<T>(P, g, dh, df, ws, st, 0, 1, 1)) != HDC_OK) return s;
    if (dg) return run_conv<T>(P, f, dh, dg, ws, st, 0, 1, 1);
    return ok();
  }
  if (df && (s = run_conv<T>(P, dh, g, df, ws, st, 1, 0, 1)) != HDC_OK) return s;
  if (!dg) return ok();
  T* scr = reinterpret_cast<T*>(ws + P->off_scr);
  if ((s = run_conv<T>(P, dh, f, scr, ws, st, 1, 0, 1, true)) != HDC_OK) return s;
  const int nd = P->ndim;
  SimpleParams S{};
  S.src = scr;
  S.dst = dg;
  S.ndim = nd;
  long long nu = 1, ng = 1;
  for (int a = 0; a < 3; ++a) {
    S.Ls[a] = 1;
    S.Ld[a] = 1;
  }
  for (int a = 0; a < nd; ++a) {
    S.Ls[3 - nd + a] = P->Lu[a];
    S.Ld[3 - nd + a] = P->Lg[a];
    nu *= P->Lu[a];
    ng *= P->Lg[a];
  }
  S.src_batch = nu;
  S.dst_batch = ng;
  S.batch = (int)P->batch;
  S.rev = 0;
  if (g_sink) {  // recorded for an uneven batch
    Rec<T> r;
    r.type = REC_PAD;
    r.pad = S;
    g_sink->get<T>().push_back(r);
    return ok();
  }
  LAUNCH_TRY(launch_pad<T>(S, st));
  return ok();
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
// HDC_USE_GRAPH: run the plan's launch sequence for this pointer set from a captured hipGraph (captured on the
// first call with these pointers, on a private stream; a call with other pointers captures again).  Plans
// without the flag, profiled calls and a capture the runtime refuses launch directly.
template <class Launch>
static hdc_status run_graphed(const hdc_plan_s* P, int which, std::vector<const void*> key, hipStream_t st,
                              Launch&& launch) {
  if (!(P->d.flags & HDC_USE_GRAPH) || P->prof || g_sink) return launch(st);
  hdc_plan_s::Graphed& G = P->graphs[which];
  if (!G.exec || G.key != key) {
    if (G.pending) HIP_TRY(hipEventSynchronize(G.done));  // the last replay has finished with the old graph
    G.pending = false;
    if (G.exec) (void)hipGraphExecDestroy(G.exec);
    if (G.graph) (void)hipGraphDestroy(G.graph);
    G.exec = nullptr;
    G.graph = nullptr;
    G.key.clear();
    if (!P->gcap) HIP_TRY(hipStreamCreateWithFlags(&P->gcap, hipStreamNonBlocking));
    if (!G.done) HIP_TRY(hipEventCreateWithFlags(&G.done, hipEventDisableTiming));
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(P->gcap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipGetLastError();
      return launch(st);
    }
    const hdc_status ls = launch(P->gcap);
    const bool ended = hipStreamEndCapture(P->gcap, &graph) == hipSuccess && graph;
    if (ls != HDC_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return ls;
    }
    if (!ended || hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0) != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      G.exec = nullptr;
      (void)hipGetLastError();
      return launch(st);
    }
    G.graph = graph;
    G.key = std::move(key);
  }
  HIP_TRY(hipGraphLaunch(G.exec, st));
  HIP_TRY(hipEventRecord(G.done, st));
  G.pending = true;
  return ok();
}

extern "C" {

const char* hdc_version(void) { return "hdconv 0.2 (gfx950)"; }

hdc_status hdc_twiddle_values(int64_t N, int32_t dtype, int64_t k0, int64_t count, double* re, double* im) {
  if (N < 1 || N > (1LL << 30)) return fail(HDC_ERR_INVALID_ARG, "N must lie in [1, 2^30]");
  if (dtype != HDC_F32 && dtype != HDC_F64) return fail(HDC_ERR_INVALID_ARG, "unknown dtype");
  if (count < 0 || k0 < 0 || k0 > N || count > N - k0) return fail(HDC_ERR_INVALID_ARG, "k range outside [0, N)");
  if (count && (!re || !im)) return fail(HDC_ERR_INVALID_ARG, "NULL output");
  auto run = [&](auto zero) {
    using T = decltype(zero);
    const int lb = tw_lobits(N);
    std::vector<cx<T>> t;
    tw_levels<T>(N, lb, t);
    const cx<T>* lo = t.data();
    const cx<T>* hi = lo + ((size_t)1 << lb);
    const bool single = (1LL << lb) >= N;
    for (int64_t i = 0; i < count; ++i) {
      const long long k = k0 + i;
      const cx<T> a = lo[k & ((1LL << lb) - 1)];
      const cx<T> b = hi[k >> lb];
      // the kernels' complex product: (fma(a.x, b.x, -(a.y b.y)), fma(a.x, b.y, a.y b.x))
      const T pr = single ? a.x : std::fma(a.x, b.x, -(a.y * b.y));
      const T pi = single ? a.y : std::fma(a.x, b.y, a.y * b.x);
      re[i] = (double)pr;
      im[i] = (double)pi;
    }
  };
  if (dtype == HDC_F32) run(0.0f);
  else run(0.0);
  return ok();
}

// error reporting for entry points in other translation units (the allocation-free forward)
__attribute__((visibility("hidden"))) hdc_status hdc_internal_fail(hdc_status st, const char* msg) {
  return fail(st, "%s", msg);
}

const char* hdc_status_string(hdc_status st) {
  switch (st) {
    case HDC_OK: return "HDC_OK";
    case HDC_ERR_INVALID_ARG: return "HDC_ERR_INVALID_ARG";
    case HDC_ERR_UNSUPPORTED: return "HDC_ERR_UNSUPPORTED";
    case HDC_ERR_WORKSPACE: return "HDC_ERR_WORKSPACE";
    case HDC_ERR_HIP: return "HDC_ERR_HIP";
    case HDC_ERR_ALLOC: return "HDC_ERR_ALLOC";
  }
  return "HDC_ERR_UNKNOWN";
}

size_t hdc_last_error(char* buf, size_t n) {
  if (buf && n) {
    size_t k = std::min(n - 1, g_err.size());
    memcpy(buf, g_err.data(), k);
    buf[k] = 0;
  }
  return g_err.size();
}

// plan creation; force_q0 / extra_scale describe the mixed variant's sub-plan (0 / 1 for every other plan)
static hdc_status plan_create(const hdc_desc* d, int force_q0, double extra_scale, hdc_plan* out) {
  hdc_plan_s* P = new (std::nothrow) hdc_plan_s();
  if (!P) return fail(HDC_ERR_ALLOC, "host allocation failed");
  P->d = *d;
  P->force_q0 = force_q0;
  P->extra_scale = extra_scale;
  hdc_status s = resolve(P);
  if (s != HDC_OK) {
    delete P;
    return s;
  }
  {
    const char* ev = getenv("HDC_CHUNK");
    if (ev) P->chunk = atoll(ev);
  }
  {
    // launches put (batch x slabs) workgroups on the grid's y dimension
    long long ymul = 1;
    if (P->cs && P->ndim > 1) ymul = P->mix ? std::max(P->Nmid, 1) : P->Nret;
    else if (!P->cs && P->ndim == 3) ymul = P->aN[0];
    if (P->batch * ymul > kMaxGridY) {
      if (P->expl || P->cs || ymul > kMaxGridY) {
        delete P;
        return fail(HDC_ERR_UNSUPPORTED, "batch %lld x %lld slabs exceeds %lld workgroup rows; split the batch",
                    (long long)d->batch, ymul, kMaxGridY);
      }
      const long long c = kMaxGridY / ymul;
      P->chunk = (P->chunk > 0) ? std::min(P->chunk, c) : c;
    }
  }
  if (P->mix && P->ndim > 1) {
    // residues 0 and q/2 of the first axis: an implicit-packing plan with the same m on that axis and q = 2
    // (q = 1 when q is odd), whose inverse carries the factor 2/q (1/q) of the full problem's 1/(q m)
    hdc_desc sd = *d;
    sd.variant = HDC_HYBRID_RCM;
    sd.flags = 0;
    sd.nin = 2;
    sd.m[0] = P->am[0];
    sd.q[0] = 0;
    if (P->ndim == 3) {
      sd.m[1] = P->am[1];
      sd.q[1] = P->aq[1];
    }
    sd.m[P->ndim - 1] = 0;  // the packed last axis: the implicit-packing planner's own choice
    sd.q[P->ndim - 1] = 0;
    const int q0 = P->aq[0];
    const int qs = q0 % 2 == 0 ? 2 : 1;
    hdc_plan sub = nullptr;
    s = plan_create(&sd, qs, (double)qs / (double)q0, &sub);
    if (s != HDC_OK) {
      delete P;
      return s;
    }
    P->sub = sub;
    sub->owner = P;
  }
  sizes_and_describe(P);
  s = (P->dtype == HDC_F64) ? build_tables<double>(P) : build_tables<float>(P);
  if (s != HDC_OK) {
    const std::string msg = g_err;  // destroying the plan clears the error text
    hdc_plan_destroy(P);
    return fail(s, "%s", msg.c_str());
  }
  *out = P;
  return ok();
}

hdc_status hdc_plan_create(const hdc_desc* d, hdc_plan* out) {
  if (!out) return fail(HDC_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!d) return fail(HDC_ERR_INVALID_ARG, "descriptor is NULL");
  return plan_create(d, 0, 1.0, out);
}

hdc_status hdc_profile_enable(hdc_plan p, int on) {
  if (!p) return fail(HDC_ERR_INVALID_ARG, "NULL plan");
  p->prof = on != 0;
  return ok();
}

hdc_status hdc_profile_read(hdc_plan p, double* avg_ms, int32_t n, int32_t* n_launches, int32_t* n_calls) {
  if (!p) return fail(HDC_ERR_INVALID_ARG, "NULL plan");
  std::vector<double> sum;
  std::vector<int> cnt;
  int ncalls = 0;
  for (const auto& c : p->calls) {
    if (c.size() < 2) continue;
    ++ncalls;
    for (size_t i = 0; i + 1 < c.size(); ++i) {
      HIP_TRY(hipEventSynchronize(p->evpool[c[i + 1]]));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, p->evpool[c[i]], p->evpool[c[i + 1]]));
      if (sum.size() <= i) {
        sum.resize(i + 1, 0.0);
        cnt.resize(i + 1, 0);
      }
      sum[i] += ms;
      cnt[i] += 1;
    }
  }
  for (int i = 0; i < n && avg_ms; ++i) avg_ms[i] = (i < (int)sum.size() && cnt[i]) ? sum[i] / cnt[i] : 0.0;
  if (n_launches) *n_launches = (int32_t)sum.size();
  if (n_calls) *n_calls = ncalls;
  p->calls.clear();
  p->evused = 0;
  return ok();
}

hdc_status hdc_plan_destroy(hdc_plan p) {
  if (!p) return ok();
  if (p->sub) hdc_plan_destroy(p->sub);
  for (auto& G : p->graphs) {
    if (G.pending) (void)hipEventSynchronize(G.done);
    if (G.exec) (void)hipGraphExecDestroy(G.exec);
    if (G.graph) (void)hipGraphDestroy(G.graph);
    if (G.done) (void)hipEventDestroy(G.done);
  }
  if (p->gcap) (void)hipStreamDestroy(p->gcap);
  for (hipEvent_t e : p->evpool) (void)hipEventDestroy(e);
  if (p->tables) (void)hipFree(p->tables);
  delete p;
  return ok();
}

hdc_status hdc_plan_workspace_size(hdc_plan p, size_t* bytes) {
  if (!p || !bytes) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
  *bytes = p->ws_bytes;
  return ok();
}

hdc_status hdc_plan_backward_workspace_size(hdc_plan p, size_t* bytes) {
  if (!p || !bytes) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
  *bytes = p->bwd_ws_bytes;
  return ok();
}

hdc_status hdc_plan_resolved(hdc_plan p, int32_t m[3], int32_t pp[3], int32_t q[3]) {
  if (!p) return fail(HDC_ERR_INVALID_ARG, "NULL plan");
  for (int a = 0; a < 3; ++a) {
    if (m) m[a] = a < p->ndim ? p->am[a] : 0;
    if (pp) pp[a] = a < p->ndim ? p->ap[a] : 0;
    if (q) q[a] = a < p->ndim ? p->aq[a] : 0;
  }
  return ok();
}

hdc_status hdc_plan_describe(hdc_plan p, char* buf, size_t n) {
  if (!p || !buf || !n) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
  size_t k = std::min(n - 1, p->describe.size());
  memcpy(buf, p->describe.data(), k);
  buf[k] = 0;
  return ok();
}

static hdc_status check_io(const hdc_plan_s* P, const void* const* ins, int nin, void* const* outs, int nout,
                           void* ws, size_t ws_bytes, size_t need = (size_t)-1) {
  if (need == (size_t)-1) need = P->ws_bytes;
  const size_t w = P->dtype == HDC_F64 ? 8 : 4;
  const size_t align = 2 * w;
  long long n = P->batch, ng = P->batch;
  for (int a = 0; a < P->ndim; ++a) n *= P->Lu[a];
  for (int a = 0; a < P->ndim; ++a) ng *= P->Lg[a];
  const size_t bytes = (size_t)n * w;
  // input 1 is always g, which may be a shorter kernel
  auto in_bytes = [&](int i) -> size_t { return i == 1 ? (size_t)ng * w : bytes; };
  // the adjoint's second output is dg, of g's extents
  auto out_bytes = [&](int o) -> size_t { return (nout == 2 && o == 1) ? (size_t)ng * w : bytes; };
  for (int i = 0; i < nin; ++i) {
    if (!ins[i]) return fail(HDC_ERR_INVALID_ARG, "input pointer %d is NULL", i);
    if ((uintptr_t)ins[i] % align) return fail(HDC_ERR_INVALID_ARG, "input %d not %zu-byte aligned", i, align);
  }
  for (int o = 0; o < nout; ++o) {
    if (!outs[o]) continue;
    if ((uintptr_t)outs[o] % align) return fail(HDC_ERR_INVALID_ARG, "output %d not %zu-byte aligned", o, align);
    const uintptr_t a0 = (uintptr_t)outs[o], a1 = a0 + out_bytes(o);
    for (int i = 0; i < nin; ++i) {
      const uintptr_t b0 = (uintptr_t)ins[i], b1 = b0 + in_bytes(i);
      if ((a0 != b0 || in_bytes(i) != out_bytes(o)) && a0 < b1 && b0 < a1)
        return fail(HDC_ERR_INVALID_ARG, "output %d overlaps input %d (only an exact alias of an input of the "
                    "output's extents is allowed)", o, i);
    }
  }
  if (need) {
    if (!ws) return fail(HDC_ERR_WORKSPACE, "workspace of %zu bytes required", need);
    if (ws_bytes < need)
      return fail(HDC_ERR_WORKSPACE, "workspace %zu bytes < required %zu", ws_bytes, need);
    if ((uintptr_t)ws % 256) return fail(HDC_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  }
  return ok();
}

hdc_status hdc_forward(hdc_plan p, const void* f, const void* g, void* h, void* ws, size_t ws_bytes, void* stream) {
  if (!p) return fail(HDC_ERR_INVALID_ARG, "NULL plan");
  if (p->nin != 2) return fail(HDC_ERR_INVALID_ARG, "this plan convolves %d arrays: use hdc_forward_n", p->nin);
  const void* ins[2] = {f, g};
  void* outs[1] = {h};
  if (!h) return fail(HDC_ERR_INVALID_ARG, "output pointer is NULL");
  hdc_status s = check_io(p, ins, 2, outs, 1, ws, ws_bytes);
  if (s != HDC_OK) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  prof_begin_call(p, st);
  const int mode = p->save ? EXEC_FWD_SAVE : EXEC_FWD;
  p->saved_ws = nullptr;
  auto launch = [&](hipStream_t ls) -> hdc_status {
    return (p->dtype == HDC_F64)
               ? run_conv<double>(p, (const double*)f, (const double*)g, (double*)h, (char*)ws, ls, 0, 0, 0, false, mode)
               : run_conv<float>(p, (const float*)f, (const float*)g, (float*)h, (char*)ws, ls, 0, 0, 0, false, mode);
  };
  s = run_graphed(p, 0, {f, g, h, ws}, st, launch);
  if (s == HDC_OK && p->save) {
    p->saved_f = f;
    p->saved_g = g;
    p->saved_ws = ws;
  }
  return s;
}

hdc_status hdc_forward_n(hdc_plan p, const void* const* x, void* h, void* ws, size_t ws_bytes, void* stream) {
  if (!p) return fail(HDC_ERR_INVALID_ARG, "NULL plan");
  if (!x) return fail(HDC_ERR_INVALID_ARG, "NULL input array list");
  if (p->nin == 2) return hdc_forward(p, x[0], x[1], h, ws, ws_bytes, stream);
  if (!h) return fail(HDC_ERR_INVALID_ARG, "output pointer is NULL");
  const size_t w = p->dtype == HDC_F64 ? 8 : 4;
  long long n = p->batch;
  for (int a = 0; a < p->ndim; ++a) n *= p->Lu[a];
  const uintptr_t h0 = (uintptr_t)h, h1 = h0 + (size_t)n * w;
  if (h0 % (2 * w)) return fail(HDC_ERR_INVALID_ARG, "output not %zu-byte aligned", 2 * w);
  for (int a = 0; a < p->nin; ++a) {
    if (!x[a]) return fail(HDC_ERR_INVALID_ARG, "input pointer %d is NULL", a);
    if ((uintptr_t)x[a] % (2 * w)) return fail(HDC_ERR_INVALID_ARG, "input %d not %zu-byte aligned", a, 2 * w);
    const uintptr_t b0 = (uintptr_t)x[a], b1 = b0 + (size_t)n * w;
    if (b0 != h0 && b0 < h1 && h0 < b1)
      return fail(HDC_ERR_INVALID_ARG, "output overlaps input %d (only an exact alias is allowed)", a);
  }
  if (p->ws_bytes) {
    if (!ws) return fail(HDC_ERR_WORKSPACE, "workspace of %zu bytes required", p->ws_bytes);
    if (ws_bytes < p->ws_bytes) return fail(HDC_ERR_WORKSPACE, "workspace %zu bytes < required %zu", ws_bytes, p->ws_bytes);
    if ((uintptr_t)ws % 256) return fail(HDC_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  prof_begin_call(p, st);
  p->saved_ws = nullptr;
  if (p->dtype == HDC_F64)
    return run_conv_nary<double>(p, reinterpret_cast<const double* const*>(x), (double*)h, (char*)ws, st);
  return run_conv_nary<float>(p, reinterpret_cast<const float* const*>(x), (float*)h, (char*)ws, st);
}

}  // extern "C"

// ---- cached kernel spectra ("transform once, multiply many"; the implicit-packing hybrid variant)
static bool cacheable(const hdc_plan_s* P) { return !P->cs && !P->expl && P->nin == 2; }


// gmode 1: g -> spec (the kernel's row spectra); gmode 2: f, spec -> h
template <typename T>
static hdc_status run_cached(const hdc_plan_s* P, const T* f, const T* g, T* h, char* ws, hipStream_t st, int gmode,
                             char* spec) {
  long long nreal = 1, nreal_g = 1;
  for (int a = 0; a < P->ndim; ++a) nreal *= P->Le[a];
  for (int a = 0; a < P->ndim; ++a) nreal_g *= P->Lge[a];
  const size_t specb = (size_t)spec_elems(P) * sizeof(cx<T>);
  const long long chunk = (P->chunk > 0 && P->chunk < P->batch) ? P->chunk : P->batch;
  for (long long b0 = 0; b0 < P->batch; b0 += chunk) {
    const long long nb = std::min(chunk, P->batch - b0);
    hdc_status s = run_exec<T>(P, f ? f + b0 * nreal : nullptr, g ? g + b0 * nreal_g : nullptr,
                               h ? h + b0 * nreal : nullptr, ws, st, 0, 0, 0, nb, false, gmode, spec + b0 * specb);
    if (s != HDC_OK) return s;
  }
  return ok();
}

static hdc_status check_cached(const hdc_plan_s* P, const void* x, const void* spec, void* ws, size_t ws_bytes) {
  if (!cacheable(P))
    return fail(HDC_ERR_UNSUPPORTED, "cached kernel spectra need an implicit-packing hybrid plan of two arrays "
                "(this plan: %s)", P->describe.c_str());
  const size_t align = P->dtype == HDC_F64 ? 16 : 8;
  if (!x || !spec) return fail(HDC_ERR_INVALID_ARG, "NULL data or spectrum pointer");
  if ((uintptr_t)x % align || (uintptr_t)spec % 16)
    return fail(HDC_ERR_INVALID_ARG, "data must be %zu-byte and the spectrum 16-byte aligned", align);
  if (P->ws_bytes) {
    if (!ws || ws_bytes < P->ws_bytes) return fail(HDC_ERR_WORKSPACE, "workspace of %zu bytes required", P->ws_bytes);
    if ((uintptr_t)ws % 256) return fail(HDC_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  }
  return ok();
}


extern "C" {

hdc_status hdc_plan_spectrum_size(hdc_plan p, size_t* bytes) {
  if (!p || !bytes) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
  if (!cacheable(p))
    return fail(HDC_ERR_UNSUPPORTED, "cached kernel spectra need an implicit-packing hybrid plan of two arrays "
                "(this plan: %s)", p->describe.c_str());
  *bytes = (size_t)p->batch * (size_t)spec_elems(p) * (p->dtype == HDC_F64 ? 16 : 8);
  return ok();
}

hdc_status hdc_transform_kernel(hdc_plan p, const void* g, void* spec, void* ws, size_t ws_bytes, void* stream) {
  if (!p) return fail(HDC_ERR_INVALID_ARG, "NULL plan");
  hdc_status s = check_cached(p, g, spec, ws, ws_bytes);
  if (s != HDC_OK) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  prof_begin_call(p, st);
  p->saved_ws = nullptr;
  if (p->dtype == HDC_F64)
    return run_cached<double>(p, nullptr, (const double*)g, nullptr, (char*)ws, st, 1, (char*)spec);
  return run_cached<float>(p, nullptr, (const float*)g, nullptr, (char*)ws, st, 1, (char*)spec);
}

hdc_status hdc_forward_cached(hdc_plan p, const void* f, const void* spec, void* h, void* ws, size_t ws_bytes,
                              void* stream) {
  if (!p) return fail(HDC_ERR_INVALID_ARG, "NULL plan");
  hdc_status s = check_cached(p, f, spec, ws, ws_bytes);
  if (s != HDC_OK) return s;
  const void* ins[1] = {f};
  void* outs[1] = {h};
  if ((s = check_io(p, ins, 1, outs, 1, ws, ws_bytes)) != HDC_OK) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  prof_begin_call(p, st);
  p->saved_ws = nullptr;
  char* sp = const_cast<char*>(reinterpret_cast<const char*>(spec));  // read only in this mode
  if (p->dtype == HDC_F64) return run_cached<double>(p, (const double*)f, nullptr, (double*)h, (char*)ws, st, 2, sp);
  return run_cached<float>(p, (const float*)f, nullptr, (float*)h, (char*)ws, st, 2, sp);
}

hdc_status hdc_backward(hdc_plan p, const void* f, const void* g, const void* dh, void* df, void* dg, void* ws,
                        size_t ws_bytes, void* stream) {
  if (!p) return fail(HDC_ERR_INVALID_ARG, "NULL plan");
  if (p->nin != 2) return fail(HDC_ERR_UNSUPPORTED, "the adjoint is built for the convolution of two arrays");
  const void* ins[3] = {f, g, dh};
  void* outs[2] = {df, dg};
  hdc_status s = check_io(p, ins, 3, outs, 2, ws, ws_bytes, p->bwd_ws_bytes);
  if (s != HDC_OK) return s;
  if ((df && (df == f || df == g || df == dh)) || (dg && (dg == f || dg == g || dg == dh)))
    return fail(HDC_ERR_INVALID_ARG, "gradients may not alias the inputs");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  prof_begin_call(p, st);
  // the saved-spectra form launches fewer passes: part of the graph's key
  const void* saved = (p->twin_ok && p->save && p->saved_ws == ws && p->saved_f == f && p->saved_g == g)
                          ? ws : nullptr;
  auto launch = [&](hipStream_t ls) -> hdc_status {
    if (p->dtype == HDC_F64)
      return backward_t<double>(p, (const double*)f, (const double*)g, (const double*)dh, (double*)df, (double*)dg,
                                (char*)ws, ls);
    return backward_t<float>(p, (const float*)f, (const float*)g, (const float*)dh, (float*)df, (float*)dg,
                             (char*)ws, ls);
  };
  return run_graphed(p, 1, {f, g, dh, df, dg, ws, saved}, st, launch);
}

// ---------------------------------------------------------------------------
// uneven batches: every item has its own plan and workspace region; the
// launches of all items are recorded, then records of the same kernel
// instantiation at the same position in their item's sequence run as one
// grouped launch whose per-item parameters live in a device table.  The
// grouped sequence is captured once in a hipGraph and replayed; only the
// tables are refreshed (when the caller's pointers change).
// ---------------------------------------------------------------------------
}  // extern "C"

struct BGroup {
  int type = 0, logm = 0, pcap = 1, narr = 1, which = 0, level = 0, kind = 0;
  int lane = 0;                // stream lane the group runs on (its items' launches never cross lanes)
  std::vector<int> item, rec;  // members: item index, record index in that item's list
  size_t tab_off = 0, elem = 0;
  int maxjobs = 1, maxnslab = 1, maxC = 1, maxq = 1, maxppw = 1;
  long long maxpitch = 0;
};

constexpr int kMaxLanes = 4;

struct BatchExec {
  bool built = false;
  bool groupable = true;       // no per-item (pad / conjugate-symmetry) launches
  std::vector<int> sig;        // launch structure the groups were built for
  std::vector<BGroup> groups;  // in execution order
  void* dtab = nullptr;
  void* staging = nullptr;
  size_t tab_bytes = 0, tab_cap = 0;
  hipEvent_t copy_ev = nullptr;  // staging buffer consumed
  hipEvent_t done_ev = nullptr;  // last launch sequence finished reading the tables
  bool copy_pending = false, done_pending = false;
  std::vector<const void*> last_ptrs;
  // the launch records of the last call (their pointers are last_ptrs): a call with the same pointers
  // reuses them instead of planning and recording every item again
  std::vector<std::vector<Rec<float>>> recs32;
  std::vector<std::vector<Rec<double>>> recs64;
  template <typename T>
  std::vector<std::vector<Rec<T>>>& recs() {
    if constexpr (sizeof(T) == 4) return recs32;
    else return recs64;
  }
  // independent chains of groups run on up to kMaxLanes streams (lane 0: the caller's stream); forked from
  // and joined to the caller's stream by events, so a captured graph holds them as parallel branches
  int nlanes = 1;
  hipStream_t side[kMaxLanes - 1] = {};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[kMaxLanes - 1] = {};
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
  }
};

struct hdc_batch_plan_s {
  std::vector<hdc_plan> plans;  // one per item (identical descriptors share a plan object)
  std::vector<int> owner;       // plans[i] owned (destroy) flags
  std::vector<size_t> ws_off;   // per-item workspace region
  size_t ws_bytes = 0;
  int dtype = 0;
  BatchExec ex[2];              // forward, backward
  hipStream_t cap = nullptr;    // capture stream
  bool use_graph = true;
  int max_lanes = kMaxLanes;    // streams the independent chains of groups may use (1: one stream)
  std::vector<double> cost;     // per item: reals of f (balances the lanes)
};

template <typename T>
static hdc_status batch_record(hdc_batch_plan_s* B, int bwd, const void* const* f, const void* const* g,
                               const void* const* dh, void* const* o1, void* const* o2, char* ws,
                               std::vector<std::vector<Rec<T>>>& recs) {
  const size_t n = B->plans.size();
  recs.assign(n, {});
  RecSink sink;
  g_sink = &sink;
  hdc_status st = HDC_OK;
  for (size_t i = 0; i < n && st == HDC_OK; ++i) {
    sink.get<T>().clear();
    const hdc_plan_s* P = B->plans[i];
    char* w = ws + B->ws_off[i];
    if (!bwd) {
      st = run_conv<T>(P, (const T*)f[i], (const T*)g[i], (T*)o1[i], w, nullptr, 0, 0, 0);
    } else {
      // the same launch sequence as hdc_backward (shared transform of R(dh), or per-output passes and
      // the copy-out of a shorter kernel's gradient); never with saved spectra
      const void* keep = P->saved_ws;
      P->saved_ws = nullptr;
      st = backward_t<T>(P, (const T*)f[i], (const T*)g[i], (const T*)dh[i], (T*)o1[i], (T*)o2[i], w, nullptr);
      P->saved_ws = keep;
    }
    recs[i] = sink.get<T>();
  }
  g_sink = nullptr;
  return st;
}

template <typename T>
static std::vector<int> batch_signature(const std::vector<std::vector<Rec<T>>>& recs) {
  std::vector<int> sig;
  for (const auto& v : recs) {
    sig.push_back(-1);
    for (const auto& r : v)
      sig.insert(sig.end(), {r.type, r.logm, r.pcap, r.narr, r.which, (int)r.line.kind, r.col.q > 2,
                             (r.type == REC_COLF || r.type == REC_COLI) && col_general(r.col, r.type == REC_COLF)});
  }
  return sig;
}

// Groups that share an item depend on each other (an item's launches run in order); groups with no item in
// common do not.  The connected components of that relation are independent chains, spread over up to
// max_lanes stream lanes, largest first onto the least loaded lane.  A component costing more than an even
// share of the batch (the items of one problem family easily share every group and form one) cannot be
// balanced whole: it is dealt to the lanes in classes of items with the same launch sequence (the same
// groups), largest first onto the least loaded lane, so a group splits only where classes part; a class
// costing more than a share is dealt item by item.  Groups are then formed per lane.  Returns the lane of
// every item.
static std::vector<int> batch_item_lanes(const BatchExec& E, int nitems, const std::vector<double>& cost,
                                         int max_lanes, int* nlanes) {
  const int ng = (int)E.groups.size();
  std::vector<int> parent(ng);
  for (int i = 0; i < ng; ++i) parent[i] = i;
  std::function<int(int)> find = [&](int x) { return parent[x] == x ? x : parent[x] = find(parent[x]); };
  std::vector<int> first(nitems, -1);  // first group of each item
  std::vector<std::vector<int>> seq(nitems);  // the groups of each item: its launch sequence
  for (int gi = 0; gi < ng; ++gi)
    for (int it : E.groups[gi].item) {
      seq[it].push_back(gi);
      if (first[it] < 0) first[it] = gi;
      else parent[find(gi)] = find(first[it]);
    }
  auto cost_of = [&](int it) { return it < (int)cost.size() ? cost[it] : 1.0; };
  std::map<int, double> comp_cost;
  std::map<int, std::vector<int>> comp_items;
  double total = 0.0;
  for (int it = 0; it < nitems; ++it)
    if (first[it] >= 0) {
      const int c = find(first[it]);
      comp_cost[c] += cost_of(it);
      comp_items[c].push_back(it);
      total += cost_of(it);
    }
  std::vector<std::pair<double, int>> order;
  for (const auto& kv : comp_cost) order.push_back({-kv.second, kv.first});
  std::sort(order.begin(), order.end());
  const int nl = std::max(1, std::min({max_lanes, kMaxLanes, nitems}));
  const double share = total / nl;
  std::vector<double> load(nl, 0.0);
  std::vector<int> lane(nitems, 0);
  auto least = [&]() { return (int)(std::min_element(load.begin(), load.end()) - load.begin()); };
  int used = 0;
  for (const auto& o : order) {
    std::vector<int>& items = comp_items[o.second];
    if (-o.first > share && nl > 1) {
      std::map<std::vector<int>, std::vector<int>> cls;  // launch sequence -> items
      for (int it : items) cls[seq[it]].push_back(it);
      std::vector<std::pair<double, const std::vector<int>*>> corder;
      for (const auto& kv : cls) {
        double c = 0.0;
        for (int it : kv.second) c += cost_of(it);
        corder.push_back({-c, &kv.second});
      }
      std::stable_sort(corder.begin(), corder.end(),
                       [](const auto& x, const auto& y) { return x.first < y.first; });
      for (const auto& co : corder) {
        if (-co.first > share) {  // one class alone exceeds a share: item by item
          std::vector<int> its = *co.second;
          std::stable_sort(its.begin(), its.end(), [&](int a, int b) { return cost_of(a) > cost_of(b); });
          for (int it : its) {
            const int l = least();
            lane[it] = l;
            load[l] += cost_of(it);
            used = std::max(used, l + 1);
          }
        } else {
          const int l = least();
          for (int it : *co.second) lane[it] = l;
          load[l] -= co.first;
          used = std::max(used, l + 1);
        }
      }
    } else {
      const int l = least();
      for (int it : items) lane[it] = l;
      load[l] -= o.first;
      used = std::max(used, l + 1);
    }
  }
  *nlanes = std::max(1, used);
  return lane;
}

// item_lane (optional): the lane of every item; groups then never mix lanes and carry theirs
template <typename T>
static void batch_build_groups(BatchExec& E, const std::vector<std::vector<Rec<T>>>& recs,
                               const std::vector<int>* item_lane = nullptr) {
  E.groups.clear();
  E.groupable = true;
  std::map<std::vector<int>, int> index;
  int maxlevel = 0;
  for (const auto& r : recs) maxlevel = std::max(maxlevel, (int)r.size());
  for (int lv = 0; lv < maxlevel; ++lv) {
    for (size_t i = 0; i < recs.size(); ++i) {
      if (lv >= (int)recs[i].size()) continue;
      const Rec<T>& r = recs[i][lv];
      if (r.type == REC_CS || r.type == REC_PAD) E.groupable = false;
      std::vector<int> key = {lv, r.type, r.logm, r.pcap, r.narr, r.which};
      if (r.type == REC_LINE) key.push_back(r.line.kind);
      if (r.type == REC_COLI) key.push_back(r.col.q > 2);
      if (r.type == REC_COLF || r.type == REC_COLI) key.push_back(col_general(r.col, r.type == REC_COLF));
      if (r.type == REC_CS || r.type == REC_PAD) key.push_back((int)i);  // never grouped
      const int ln = item_lane ? (*item_lane)[i] : 0;
      key.push_back(ln);
      auto it = index.find(key);
      int gi;
      if (it == index.end()) {
        gi = (int)E.groups.size();
        index[key] = gi;
        BGroup gr;
        gr.type = r.type;
        gr.logm = r.logm;
        gr.pcap = r.pcap;
        gr.narr = r.narr;
        gr.which = r.which;
        gr.level = lv;
        gr.lane = ln;
        E.groups.push_back(gr);
      } else {
        gi = it->second;
      }
      BGroup& gr = E.groups[gi];
      gr.item.push_back((int)i);
      gr.rec.push_back(lv);
      if (r.type == REC_LINE) {
        gr.maxjobs = std::max(gr.maxjobs, (int)r.grid.x);
        gr.maxq = std::max(gr.maxq, r.line.q);
        gr.maxppw = std::max(gr.maxppw, r.line.ppw);
      } else if (r.type == REC_COLF || r.type == REC_COLI) {
        gr.maxnslab = std::max(gr.maxnslab, r.col.nslab);
        gr.maxC = std::max(gr.maxC, r.col.C);
        gr.maxpitch = std::max(gr.maxpitch, col_pitch(r.col, r.type == REC_COLF));
      }
    }
  }
  size_t off = 0;
  for (auto& gr : E.groups) {
    gr.elem = gr.type == REC_LINE ? sizeof(LineParams<T>) : sizeof(ColParams<T>);
    off = align256(off);
    gr.tab_off = off;
    if (gr.type == REC_LINE || gr.type == REC_COLF || gr.type == REC_COLI) off += gr.elem * gr.item.size();
  }
  E.tab_bytes = std::max<size_t>(off, 256);
}

template <typename T>
static hdc_status batch_launch(BatchExec& E, const std::vector<std::vector<Rec<T>>>& recs, hipStream_t st0) {
  const char* dtab = static_cast<const char*>(E.dtab);
  if (E.nlanes > 1) {
    // fork: the side lanes start after everything queued on the caller's stream (the table copy included);
    // their streams and events exist already (created outside any capture)
    HIP_TRY(hipEventRecord(E.fork_ev, st0));
    for (int l = 1; l < E.nlanes; ++l) HIP_TRY(hipStreamWaitEvent(E.side[l - 1], E.fork_ev, 0));
  }
  for (const auto& gr : E.groups) {
    hipStream_t st = gr.lane ? E.side[gr.lane - 1] : st0;
    const Rec<T>& r0 = recs[gr.item[0]][gr.rec[0]];
    const long long nm = (long long)gr.item.size();
    hipError_t e = hipSuccess;
    if (gr.type == REC_LINE) {
      LineParams<T> P0 = r0.line;
      P0.q = gr.maxq;  // sizes the dynamic LDS for the largest member
      P0.ppw = gr.maxppw;
      const LineParams<T>* tab = reinterpret_cast<const LineParams<T>*>(dtab + gr.tab_off);
      for (long long k0 = 0; k0 < nm && e == hipSuccess; k0 += kMaxGridY) {
        const unsigned n = (unsigned)std::min(kMaxGridY, nm - k0);
        e = call_line<T>(P0, gr.logm, gr.pcap, dim3((unsigned)gr.maxjobs, n), st, tab + k0);
      }
    } else if (gr.type == REC_COLF || gr.type == REC_COLI) {
      ColParams<T> P0 = r0.col;
      P0.nslab = gr.maxnslab;
      P0.C = gr.maxC;
      P0.pitch_hint = gr.maxpitch;
      const ColParams<T>* tab = reinterpret_cast<const ColParams<T>*>(dtab + gr.tab_off);
      const long long per = std::max(1LL, kMaxGridY / gr.maxnslab);
      for (long long k0 = 0; k0 < nm && e == hipSuccess; k0 += per) {
        const unsigned n = (unsigned)std::min(per, nm - k0);
        const dim3 grid(1, n * (unsigned)gr.maxnslab, gr.type == REC_COLF ? (unsigned)gr.narr : 1u);
        e = gr.type == REC_COLF ? call_col<T, true>(P0, gr.logm, gr.pcap, gr.narr, grid, st, tab + k0)
                                : call_col<T, false>(P0, gr.logm, gr.pcap, 1, grid, st, tab + k0);
      }
    } else {
      // per-item launches (explicit padding, conjugate-symmetry first axis)
      for (long long k = 0; k < nm && e == hipSuccess; ++k) {
        const Rec<T>& r = recs[gr.item[k]][gr.rec[k]];
        if (r.type == REC_PAD) e = launch_pad<T>(r.pad, st);
        else e = call_cs<T>(r.cs, r.logm, r.which, r.pcap, r.grid, st, true);
      }
    }
    if (e != hipSuccess) return fail(HDC_ERR_HIP, "batch launch: %s", hipGetErrorString(e));
  }
  // join: the caller's stream waits for every lane
  for (int l = 1; l < E.nlanes; ++l) {
    HIP_TRY(hipEventRecord(E.join_ev[l - 1], E.side[l - 1]));
    HIP_TRY(hipStreamWaitEvent(st0, E.join_ev[l - 1], 0));
  }
  return ok();
}

template <typename T>
static hdc_status batch_run(hdc_batch_plan_s* B, int bwd, const void* const* f, const void* const* g,
                            const void* const* dh, void* const* o1, void* const* o2, void* ws, size_t ws_bytes,
                            hipStream_t st) {
  const size_t n = B->plans.size();
  if (B->ws_bytes) {
    if (!ws) return fail(HDC_ERR_WORKSPACE, "batch workspace of %zu bytes required", B->ws_bytes);
    if (ws_bytes < B->ws_bytes)
      return fail(HDC_ERR_WORKSPACE, "batch workspace %zu bytes < required %zu", ws_bytes, B->ws_bytes);
  }
  BatchExec& E = B->ex[bwd];
  std::vector<const void*> ptrs;
  ptrs.reserve(n * 5 + 1);
  for (size_t i = 0; i < n; ++i) {
    ptrs.push_back(f[i]);
    ptrs.push_back(g[i]);
    ptrs.push_back(bwd ? dh[i] : nullptr);
    ptrs.push_back(o1[i]);
    ptrs.push_back(bwd ? o2[i] : nullptr);
  }
  ptrs.push_back(ws);
  if (E.built && ptrs == E.last_ptrs && !E.recs<T>().empty()) {
    // the same pointers as the last call: they were validated and recorded then, and the tables hold them
    if (B->use_graph && E.gexec) {
      HIP_TRY(hipGraphLaunch(E.gexec, st));
    } else {
      hdc_status s = batch_launch<T>(E, E.recs<T>(), st);
      if (s != HDC_OK) return s;
    }
    HIP_TRY(hipEventRecord(E.done_ev, st));
    E.done_pending = true;
    return ok();
  }
  for (size_t i = 0; i < n; ++i) {
    const hdc_plan_s* P = B->plans[i];
    const void* ins[3] = {f[i], g[i], bwd ? dh[i] : nullptr};
    void* outs[2] = {o1[i], bwd ? o2[i] : nullptr};
    if (!bwd && !o1[i]) return fail(HDC_ERR_INVALID_ARG, "item %zu: output pointer is NULL", i);
    hdc_status s = check_io(P, ins, bwd ? 3 : 2, outs, bwd ? 2 : 1, ws ? (char*)ws + B->ws_off[i] : nullptr,
                            bwd ? P->bwd_ws_bytes : P->ws_bytes);
    if (s != HDC_OK) return fail(s, "item %zu: %s", i, std::string(g_err).c_str());
    if (bwd) {
      for (int o = 0; o < 2; ++o)
        for (int k = 0; k < 3; ++k)
          if (outs[o] && outs[o] == ins[k]) return fail(HDC_ERR_INVALID_ARG, "item %zu: gradients may not alias the inputs", i);
    }
  }
  std::vector<std::vector<Rec<T>>>& recs = E.recs<T>();
  hdc_status s = batch_record<T>(B, bwd, f, g, dh, o1, o2, (char*)ws, recs);
  if (s != HDC_OK) {
    recs.clear();
    return s;
  }
  std::vector<int> sig = batch_signature<T>(recs);
  if (!E.built || sig != E.sig) {
    // (re)build the groups; earlier launches must be done with the old tables
    if (E.done_pending) HIP_TRY(hipEventSynchronize(E.done_ev));
    if (E.copy_pending) HIP_TRY(hipEventSynchronize(E.copy_ev));
    E.done_pending = E.copy_pending = false;
    E.drop_graph();
    batch_build_groups<T>(E, recs);  // across all items: the components
    int nl = 1;
    const std::vector<int> lanes = batch_item_lanes(E, (int)n, B->cost, B->max_lanes, &nl);
    batch_build_groups<T>(E, recs, &lanes);  // per lane
    E.nlanes = nl;
    for (int l = 1; l < E.nlanes; ++l) {
      if (!E.side[l - 1]) HIP_TRY(hipStreamCreateWithFlags(&E.side[l - 1], hipStreamNonBlocking));
      if (!E.join_ev[l - 1]) HIP_TRY(hipEventCreateWithFlags(&E.join_ev[l - 1], hipEventDisableTiming));
    }
    if (E.nlanes > 1 && !E.fork_ev) HIP_TRY(hipEventCreateWithFlags(&E.fork_ev, hipEventDisableTiming));
    E.sig = sig;
    E.last_ptrs.clear();
    if (E.tab_bytes > E.tab_cap) {
      if (E.dtab) HIP_TRY(hipFree(E.dtab));
      if (E.staging) HIP_TRY(hipHostFree(E.staging));
      E.dtab = E.staging = nullptr;
      E.tab_cap = 0;
      HIP_TRY(hipMalloc(&E.dtab, E.tab_bytes));
      HIP_TRY(hipHostMalloc(&E.staging, E.tab_bytes, hipHostMallocDefault));
      E.tab_cap = E.tab_bytes;
    }
    if (!E.copy_ev) HIP_TRY(hipEventCreateWithFlags(&E.copy_ev, hipEventDisableTiming));
    if (!E.done_ev) HIP_TRY(hipEventCreateWithFlags(&E.done_ev, hipEventDisableTiming));
    E.built = true;
  }
  // refresh the parameter tables when the caller's pointers changed; a graph that holds per-item launches
  // (padding copies, conjugate-symmetry passes) has their pointers in its nodes and is captured again
  if (ptrs != E.last_ptrs && !E.groupable && E.gexec) {
    if (E.done_pending) HIP_TRY(hipEventSynchronize(E.done_ev));  // the last replay has finished
    E.done_pending = false;
    E.drop_graph();
  }
  if (ptrs != E.last_ptrs) {
    if (E.copy_pending) HIP_TRY(hipEventSynchronize(E.copy_ev));
    char* stg = static_cast<char*>(E.staging);
    for (const auto& gr : E.groups) {
      if (gr.type != REC_LINE && gr.type != REC_COLF && gr.type != REC_COLI) continue;
      for (size_t k = 0; k < gr.item.size(); ++k) {
        const Rec<T>& r = recs[gr.item[k]][gr.rec[k]];
        const void* src = gr.type == REC_LINE ? (const void*)&r.line : (const void*)&r.col;
        memcpy(stg + gr.tab_off + k * gr.elem, src, gr.elem);
      }
    }
    // the previous sequence (possibly on another stream) still reads the tables
    if (E.done_pending) HIP_TRY(hipStreamWaitEvent(st, E.done_ev, 0));
    HIP_TRY(hipMemcpyAsync(E.dtab, E.staging, E.tab_bytes, hipMemcpyHostToDevice, st));
    HIP_TRY(hipEventRecord(E.copy_ev, st));
    E.copy_pending = true;
    E.last_ptrs = ptrs;
  }
  if (B->use_graph && !E.gexec) {
    // capture once on a private stream; a failed capture falls back to eager launches
    if (!B->cap) HIP_TRY(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    bool good = hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (good) {
      const hdc_status ls = batch_launch<T>(E, recs, B->cap);
      good = hipStreamEndCapture(B->cap, &graph) == hipSuccess && ls == HDC_OK && graph;
    }
    if (good) good = hipGraphInstantiate(&E.gexec, graph, nullptr, nullptr, 0) == hipSuccess;
    if (good) {
      E.graph = graph;
    } else {
      if (graph) (void)hipGraphDestroy(graph);
      E.gexec = nullptr;
      B->use_graph = false;
      (void)hipGetLastError();
    }
  }
  if (B->use_graph && E.gexec) {
    HIP_TRY(hipGraphLaunch(E.gexec, st));
  } else {
    s = batch_launch<T>(E, recs, st);
    if (s != HDC_OK) return s;
  }
  HIP_TRY(hipEventRecord(E.done_ev, st));
  E.done_pending = true;
  return ok();
}

extern "C" {

hdc_status hdc_batch_plan_create(const hdc_desc* items, int64_t n_items, hdc_batch_plan* out) {
  if (!out) return fail(HDC_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!items || n_items < 1) return fail(HDC_ERR_INVALID_ARG, "need at least one item");
  hdc_batch_plan_s* B = new (std::nothrow) hdc_batch_plan_s();
  if (!B) return fail(HDC_ERR_ALLOC, "host allocation failed");
  B->dtype = items[0].dtype;
  std::map<std::vector<long long>, hdc_plan> cache;
  size_t off = 0;
  for (int64_t i = 0; i < n_items; ++i) {
    hdc_desc d = items[i];
    d.batch = 1;
    if (d.nin && d.nin != 2) {
      hdc_batch_plan_destroy(B);
      return fail(HDC_ERR_UNSUPPORTED, "item %lld: batch items convolve two arrays", (long long)i);
    }
    if (d.dtype != B->dtype) {
      hdc_batch_plan_destroy(B);
      return fail(HDC_ERR_INVALID_ARG, "all items of a batch must share one dtype");
    }
    // items with the same descriptor share one plan (every field that shapes a plan is in the key)
    std::vector<long long> key = {d.ndim, d.L[0], d.L[1], d.L[2], d.M[0], d.M[1], d.M[2], d.m[0], d.m[1],
                                  d.m[2], d.q[0], d.q[1], d.q[2], d.variant, d.dtype,
                                  d.Lg[0] ? d.Lg[0] : d.L[0], d.Lg[1] ? d.Lg[1] : d.L[1],
                                  d.Lg[2] ? d.Lg[2] : d.L[2], (long long)d.flags};
    auto it = cache.find(key);
    hdc_plan p = nullptr;
    if (it == cache.end()) {
      hdc_status s = hdc_plan_create(&d, &p);
      if (s != HDC_OK) {
        std::string msg = g_err;
        hdc_batch_plan_destroy(B);
        return fail(s, "item %lld: %s", (long long)i, msg.c_str());
      }
      cache[key] = p;
      B->owner.push_back(1);
    } else {
      p = it->second;
      B->owner.push_back(0);
    }
    B->plans.push_back(p);
    double nr = 1.0;
    for (int a = 0; a < d.ndim; ++a) nr *= (double)d.L[a];
    B->cost.push_back(nr);
    B->ws_off.push_back(off);
    off = align256(off + std::max(p->ws_bytes, p->bwd_ws_bytes));
  }
  B->ws_bytes = off;
  if (getenv("HDC_BATCH_NO_GRAPH")) B->use_graph = false;
  if (const char* ev = getenv("HDC_BATCH_LANES")) B->max_lanes = std::max(1, std::min(kMaxLanes, atoi(ev)));
  *out = B;
  return ok();
}

hdc_status hdc_batch_workspace_size(hdc_batch_plan p, size_t* bytes) {
  if (!p || !bytes) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
  *bytes = p->ws_bytes;
  return ok();
}

hdc_status hdc_batch_forward(hdc_batch_plan p, const void* const* f, const void* const* g, void* const* h, void* ws,
                             size_t ws_bytes, void* stream) {
  if (!p || !f || !g || !h) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (p->dtype == HDC_F64) return batch_run<double>(p, 0, f, g, nullptr, h, nullptr, ws, ws_bytes, st);
  return batch_run<float>(p, 0, f, g, nullptr, h, nullptr, ws, ws_bytes, st);
}

hdc_status hdc_batch_backward(hdc_batch_plan p, const void* const* f, const void* const* g, const void* const* dh,
                              void* const* df, void* const* dg, void* ws, size_t ws_bytes, void* stream) {
  if (!p || !f || !g || !dh || !df || !dg) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (p->dtype == HDC_F64) return batch_run<double>(p, 1, f, g, dh, df, dg, ws, ws_bytes, st);
  return batch_run<float>(p, 1, f, g, dh, df, dg, ws, ws_bytes, st);
}

hdc_status hdc_batch_plan_destroy(hdc_batch_plan p) {
  if (!p) return ok();
  for (auto& E : p->ex) {
    if (E.done_pending) (void)hipEventSynchronize(E.done_ev);
    if (E.copy_pending) (void)hipEventSynchronize(E.copy_ev);
    E.drop_graph();
    if (E.dtab) (void)hipFree(E.dtab);
    if (E.staging) (void)hipHostFree(E.staging);
    if (E.copy_ev) (void)hipEventDestroy(E.copy_ev);
    if (E.done_ev) (void)hipEventDestroy(E.done_ev);
    if (E.fork_ev) (void)hipEventDestroy(E.fork_ev);
    for (int l = 0; l < kMaxLanes - 1; ++l) {
      if (E.join_ev[l]) (void)hipEventDestroy(E.join_ev[l]);
      if (E.side[l]) (void)hipStreamDestroy(E.side[l]);
    }
  }
  if (p->cap) (void)hipStreamDestroy(p->cap);
  for (size_t k = 0; k < p->plans.size(); ++k)
    if (p->owner[k]) hdc_plan_destroy(p->plans[k]);
  delete p;
  return ok();
}

}  // extern "C"

// time one descriptor: average milliseconds of a forward call (or < 0 if it does not plan)
static double autotune_time(const hdc_desc& d, void* f, void* g, void* h, hipStream_t st,
                            hipEvent_t e0, hipEvent_t e1) {
  hdc_plan p = nullptr;
  if (hdc_plan_create(&d, &p) != HDC_OK) return -1.0;
  size_t wsb = p->ws_bytes;
  void* ws = nullptr;
  double ms = -1.0;
  if (!wsb || hipMalloc(&ws, wsb) == hipSuccess) {
    // n-ary plans: the inputs alternate between the two scratch arrays
    const void* xs[kMaxNary];
    for (int a = 0; a < kMaxNary; ++a) xs[a] = (a & 1) ? g : f;
    auto fwd = [&]() { return hdc_forward_n(p, xs, h, ws, wsb, st); };
    bool good = fwd() == HDC_OK;
    // each repetition timed on its own; the minimum is the least disturbed by other work on the device
    const int reps = 5;
    float best = -1.f;
    for (int r = 0; r < reps && good; ++r) {
      good = hipEventRecord(e0, st) == hipSuccess && fwd() == HDC_OK &&
             hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
      float t = 0.f;
      if (good && hipEventElapsedTime(&t, e0, e1) == hipSuccess && (best < 0.f || t < best)) best = t;
    }
    if (good && best >= 0.f) ms = best;
    (void)hipStreamSynchronize(st);
  }
  if (ws) (void)hipFree(ws);
  hdc_plan_destroy(p);
  return ms;
}

static std::string autotune_key(const hdc_desc& d) {
  hipDeviceProp_t prop{};
  int dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipGetDeviceProperties(&prop, dev);
  char buf[512];
  snprintf(buf, sizeof(buf), "%s nd=%d L=%lld,%lld,%lld M=%lld,%lld,%lld v=%d t=%d b=%lld Lg=%lld,%lld,%lld n=%d",
           prop.gcnArchName, d.ndim, (long long)d.L[0], (long long)d.L[1], (long long)d.L[2], (long long)d.M[0],
           (long long)d.M[1], (long long)d.M[2], d.variant, d.dtype, (long long)d.batch, (long long)d.Lg[0],
           (long long)d.Lg[1], (long long)d.Lg[2], d.nin ? d.nin : 2);
  for (char* c = buf; *c; ++c)
    if (*c == '|') *c = '_';
  return buf;
}

extern "C" {

hdc_status hdc_autotune(hdc_desc* d, const char* cache_path) {
  if (!d) return fail(HDC_ERR_INVALID_ARG, "NULL descriptor");
  hdc_desc base = *d;
  for (int a = 0; a < 3; ++a) {
    base.m[a] = 0;
    base.q[a] = 0;
  }
  {
    hdc_plan p = nullptr;
    hdc_status s = hdc_plan_create(&base, &p);
    if (s != HDC_OK) return s;
    hdc_plan_destroy(p);
  }
  if (base.flags & HDC_DETERMINISTIC) {
    // no timing: the planner's defaults, the same on every run and device
    hdc_plan p = nullptr;
    hdc_status s = hdc_plan_create(&base, &p);
    if (s != HDC_OK) return s;
    for (int a = 0; a < 3; ++a) base.m[a] = 0;
    for (int a = 0; a < base.ndim; ++a) {
      const bool packed = !p->cs && a == base.ndim - 1;  // the packed last axis reports complex units
      base.m[a] = packed ? 2 * p->am[a] : p->am[a];
      if (!p->cs && base.ndim == 1 && p->path == PATH_1D_MULTI) base.m[a] = 2 * p->mr;
    }
    hdc_plan_destroy(p);
    *d = base;
    return ok();
  }
  const std::string key = autotune_key(base);
  if (cache_path) {
    // text lines "<key>|m0 m1 m2"; the last matching line wins
    FILE* fp = fopen(cache_path, "r");
    if (fp) {
      char line[1024];
      bool found = false;
      long long mm[3] = {0, 0, 0};
      while (fgets(line, sizeof(line), fp)) {
        char* bar = strchr(line, '|');
        if (!bar) continue;
        *bar = 0;
        long long t[3];
        if (key == line && sscanf(bar + 1, "%lld %lld %lld", &t[0], &t[1], &t[2]) == 3) {
          found = true;
          for (int a = 0; a < 3; ++a) mm[a] = t[a];
        }
      }
      fclose(fp);
      if (found) {
        hdc_desc c = base;
        for (int a = 0; a < 3; ++a) c.m[a] = mm[a];
        hdc_plan p = nullptr;
        if (hdc_plan_create(&c, &p) == HDC_OK) {
          hdc_plan_destroy(p);
          *d = c;
          return ok();
        }
      }
    }
  }
  // scratch problem of the descriptor's shape (contents do not change the timing); small problems are timed
  // as a batch of at least 2^22 points so that kernel time, not launch overhead, decides
  const size_t w = base.dtype == HDC_F64 ? 8 : 4;
  long long npts = 1;
  for (int a = 0; a < base.ndim; ++a) npts *= base.L[a];
  hdc_desc tb = base;
  tb.batch = std::max<long long>(base.batch, std::min<long long>(cdiv(1LL << 22, npts), 4096));
  {
    hdc_plan p = nullptr;
    if (hdc_plan_create(&tb, &p) == HDC_OK) hdc_plan_destroy(p);
    else tb.batch = base.batch;  // e.g. too many workgroup rows for one launch
  }
  const long long n = tb.batch * npts;
  const size_t bytes = (size_t)n * w;
  void *f = nullptr, *g = nullptr, *h = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hdc_status rs = HDC_OK;
  auto cleanup = [&]() {
    if (f) (void)hipFree(f);
    if (g) (void)hipFree(g);
    if (h) (void)hipFree(h);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
  };
  if (hipMalloc(&f, bytes) != hipSuccess || hipMalloc(&g, bytes) != hipSuccess || hipMalloc(&h, bytes) != hipSuccess ||
      hipMemset(f, 0, bytes) != hipSuccess || hipMemset(g, 0, bytes) != hipSuccess ||
      hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return fail(HDC_ERR_HIP, "autotune: scratch allocation failed");
  }
  // coordinate search over power-of-two m per axis, starting from the defaults
  hdc_desc best = tb;
  double tbest = autotune_time(best, f, g, h, st, e0, e1);
  if (tbest < 0) {
    cleanup();
    return fail(HDC_ERR_HIP, "autotune: the default plan failed to run");
  }
  for (int a = 0; a < base.ndim; ++a) {
    const long long L = base.L[a];
    const long long lo = std::min<long long>(16, next_pow2(L));
    for (long long m = lo; m <= 8192; m <<= 1) {
      if (m > 4 * next_pow2(L)) break;
      hdc_desc c = best;
      c.m[a] = m;
      hdc_plan p = nullptr;
      if (hdc_plan_create(&c, &p) != HDC_OK) continue;
      // more than 4 input blocks on an axis leaves the register-blocked kernels for the
      // generic form that re-reads its input for every residue (work ~ p q per element):
      // never faster, and slow enough to dominate the search, so it is not timed
      bool generic = false;
      if (p->path != PATH_1D_MULTI)
        for (int x = 0; x < p->ndim; ++x) generic |= p->ap[x] > 4;
      hdc_plan_destroy(p);
      if (generic) continue;
      const double t = autotune_time(c, f, g, h, st, e0, e1);
      if (t >= 0 && t < 0.97 * tbest) {  // a clear win, not timing noise
        tbest = t;
        best = c;
      }
    }
  }
  cleanup();
  best.batch = base.batch;
  // report the m in use on every axis (0 entries become the resolved default)
  {
    hdc_plan p = nullptr;
    rs = hdc_plan_create(&best, &p);
    if (rs != HDC_OK) return rs;
    for (int a = 0; a < best.ndim; ++a) {
      if (best.m[a]) continue;
      const bool packed = best.variant != HDC_HYBRID_CS && best.variant != HDC_HYBRID_MIX && a == best.ndim - 1;
      long long m = p->am[a];
      if (p->path == PATH_1D_MULTI && best.ndim == 1) m = p->mr;
      best.m[a] = packed ? 2 * m : m;
    }
    hdc_plan_destroy(p);
  }
  for (int a = 0; a < 3; ++a) best.q[a] = 0;
  if (cache_path) {
    FILE* fp = fopen(cache_path, "a");
    if (fp) {
      fprintf(fp, "%s|%lld %lld %lld\n", key.c_str(), (long long)best.m[0], (long long)best.m[1],
              (long long)best.m[2]);
      fclose(fp);
    }
  }
  *d = best;
  return ok();
}

}  // extern "C"
