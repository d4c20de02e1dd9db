// Kernel parameter blocks and launchers shared by the host planner and the
// HIP translation units.  Host code sees only these declarations.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hdc_device.hpp"

namespace hdc {

// Line kinds handled by the line kernel.
enum LineKind : int {
  LINE_1D = 0,     // one whole 1D convolution per workgroup, raw real input/output
  LINE_2D = 1,     // innermost-axis line pairs (k1, k1*) of a 2D problem (workspace in place)
  LINE_3D = 2,     // innermost-axis line pairs ((k1,k2), (k1*,k2*)) of a 3D problem
  LINE_ROWS = 3,   // residue rows (r, q-r) of a multi-pass 1D problem (workspace in place)
  LINE_PLAIN = 4,  // one complex line per workgroup (sub-convolutions of the conjugate-symmetry variant)
};

enum MulVariant : int {
  MUL_RCM = 0,       // implicit packing operator, eqs. (RCM), (RCM-ndim)
  MUL_EXPLICIT = 1,  // explicit unpack (fourierUnpack), product, pack (fourierPack)
  MUL_ELEM = 2,      // elementwise product (complex sub-convolutions, Sec. 2 and Sec. 5)
};

template <typename T>
struct LineParams {
  int m, p, q, N;      // hybrid along the line: FFT length m, p input blocks, q residues, N = q m
  int p_g;             // blocks of the second array (a shorter kernel g; 0: p)
  int Lin;             // valid input elements per line (complex units)
  int Lin_g;           // kind 0: valid elements of g (a kernel shorter than f; else Lin)
  int Lout;            // output elements written per line
  int qrow;            // RCM index of element l: kappa = qrow * l + rline (kinds 0-2: qrow = 1)
  int Nf;              // transform length of the packed axis (the (1 + zeta_Nf^kappa) factor)
  int variant;         // MulVariant
  int kind;            // LineKind
  int N1, N2;          // outer transform lengths (kinds 1, 2)
  int qres;            // kind 3: residue rows of the 1D problem
  T scale;             // 1 / prod(transform lengths), folded into the product
  long long line_stride;  // complex elements between lines in the workspace
  long long ws_batch;     // complex elements per batch element in the workspace
  cx<T>* wsF;
  cx<T>* wsG;
  const T* f;  // kind 0: raw real input/output
  const T* g;
  T* h;
  RawGeom gf, gg, gh;
  Tw2<T> twN;    // zeta_N for the line's pre/post-processing
  Tw2<T> tw2Nf;  // zeta_{2 Nf}
  Tw2<T> twRow;  // kind 3: zeta_Nf, the four-step twiddle of row k (N = 1: none)
  const cx<T>* rootpyr;  // FFT root tables of every power-of-two length (root_of)
  int njobs;             // grouped launches: valid blockIdx.x range of this problem
  int gmode;             // 0 plain; 1 transform the kernel's lines (rows) only and store their spectra
                         // in gspec; 2 take the kernel's spectra from gspec (cached kernel)
  cx<T>* gspec;          // gmode 1/2: kernel spectra; kind 3 laid out like wsG, kinds 0-2 one block of
                         // q m values per line ([r][l]) at gspec + b spec_batch + line spec_line
  long long spec_batch, spec_line;
  int ppw;               // kinds 1, 2, 4: line pairs per workgroup
  long long npairs;      // kinds 1, 2, 4: canonical line pairs (kind 4: lines)
  // Output region of the product lines (kinds 1-3; null: in place over wsF).
  cx<T>* wsH;
  // Twin mode (the adjoint): the second array (g / wsG) is transformed once and
  // multiplied by two first arrays in turn -- pass 0 takes f / wsF and stores to
  // h / wsH, pass 1 takes f2 / wsF2 and stores to h2 / wsH2.
  int twin;
  const T* f2;
  T* h2;
  RawGeom gf2, gh2;
  cx<T>* wsF2;
  cx<T>* wsH2;
  // n-ary mode (nin > 2 arrays, Sec. 4.1): array a is xin[a] (kind 0, f's geometry) or
  // the workspace region wsF + a * ws_arr (kinds 1-3); the product is R^nin in array 0's slots
  int nin;
  long long ws_arr;
  const T* xin[8];
};

constexpr int kMaxNary = 8;

constexpr int kLinePairsMax = 8;
// static LDS of the multi-D line kernel (the pair table), beside its dynamic LDS
constexpr size_t kLineStaticLds = 2 * kLinePairsMax * sizeof(long long);

// Canonical pair number pp -> lines (A, C) with C the conjugate partner k* of A
// (Sec. 5: k*_i = (N_i - k_i) mod N_i on every outer axis).  Kind 1 (2D): A = k1
// for k1 <= N1/2.  Kind 2 (3D): rows 1 <= k1 <= (N1-1)/2 with every k2, then the
// self-conjugate rows k1 = 0 (and N1/2 for even N1) with k2 <= N2/2.  Kind 4:
// one line per pair (A = C).
template <typename T>
__device__ __forceinline__ void line_pair(const LineParams<T>& P, long long pp, long long& A, long long& C) {
  if (P.kind == LINE_PLAIN) {
    A = C = pp;
    return;
  }
  if (P.kind == LINE_2D) {
    A = pp;
    C = (P.N1 - pp) % P.N1;
    return;
  }
  const long long N1 = P.N1, N2 = P.N2;
  const long long nfull = (N1 - 1) / 2;
  long long k1, k2;
  if (pp < nfull * N2) {
    k1 = 1 + pp / N2;
    k2 = pp - (k1 - 1) * N2;
  } else {
    const long long x = pp - nfull * N2;
    const long long npr = N2 / 2 + 1;
    const long long row = x / npr;
    k2 = x - row * npr;
    k1 = row ? N1 / 2 : 0;
  }
  A = k1 * N2 + k2;
  C = ((N1 - k1) % N1) * N2 + (N2 - k2) % N2;
}

// number of canonical pairs of line_pair for kinds 1, 2
inline long long line_npairs(int kind, long long N1, long long N2) {
  if (kind == LINE_2D) return N1 / 2 + 1;
  return ((N1 - 1) / 2) * N2 + (1 + (N1 % 2 == 0)) * (N2 / 2 + 1);
}

template <typename T>
struct ColParams {
  int m, p, q, N;   // along the column axis: FFT length m, input blocks p, residues q, N = q m
  int Lrows;        // forward: valid input rows; inverse: output rows written
  int C;            // columns (complex elements per row)
  int nslab;        // independent slabs per batch element (grid.y = batch * nslab)
  long long in_row, in_slab, in_batch, in_arr;      // workspace input strides (complex elements)
  long long out_row, out_slab, out_batch, out_arr;  // workspace output strides
  const cx<T>* in;
  cx<T>* out;
  const T* rawin0;  // forward pass on raw real input (f, g); null -> workspace input
  const T* rawin1;
  T* rawout;        // inverse pass to raw real output (h); null -> workspace output
  RawGeom graw0, graw1;
  int lin_pitch;    // > 0: raw element of (row, col) is the linear packed index row*lin_pitch + col
  Tw2<T> twN;       // residue twiddles zeta_N^k, single-level
  const cx<T>* rootpyr;
  long long pitch_hint;  // grouped launches: largest row pitch of the group (0: from this block)
  int arr0;              // forward: array of blockIdx.z = 0 (1: the kernel g alone)
};

// Column kernels read raw real data through the fast strided (packed complex)
// form unless a raw array has odd length or is read reversed.
template <typename T>
inline bool col_general(const ColParams<T>& P, bool fwd) {
  if (fwd) return P.rawin0 && (!raw_packed(P.graw0) || !raw_packed(P.graw1));
  return P.rawout && !raw_packed(P.graw0);
}
// largest row pitch (complex elements) a lane offset spans
template <typename T>
inline long long col_pitch(const ColParams<T>& P, bool fwd) {
  if (P.pitch_hint > 0) return P.pitch_hint;
  const bool raw = fwd ? P.rawin0 != nullptr : P.rawout != nullptr;
  const long long rs = raw ? (P.lin_pitch ? P.lin_pitch : (P.graw0.row_stride >> 1)) : (fwd ? P.in_row : P.out_row);
  const long long qs = (long long)P.q * (fwd ? P.out_row : P.in_row);
  return rs > qs ? rs : qs;
}
// Grouped launches: several problems that share a kernel instantiation run in
// one launch; blockIdx.y selects the problem (times the largest slab count for
// column kernels) and its parameters come from a device table.

template <typename T>
struct CsParams {
  int m, p, q, N;         // the real-transformed axis: FFT length m, blocks p, residues q, N = q m
  int nres;               // residues kept: 0 .. floor(q/2)
  int L;                  // extent of that axis (1D: the problem length)
  int C;                  // first-axis kernels: real columns (inner extent product)
  long long in_row;       // reals between rows of f, g, h (first-axis kernels)
  long long in_batch;     // reals per batch element of f, g, h
  long long ws_row;       // complex elements between retained lines in the workspace
  long long ws_batch;     // complex elements per batch element in the workspace
  long long ws_arr;       // offset of the g region from the f region (complex elements)
  const T* f;
  const T* g;
  T* h;
  cx<T>* ws;
  int rev_f, rev_g, rev_h;  // reversed access (adjoint)
  T scale;                  // 1D: 1 / (q m)
  Tw2<T> twN;
  const cx<T>* rootpyr;
  long long lin1d;          // first-axis kernels on a 1D problem of this length viewed as rows of C (0: off)
  // a shorter kernel g (g_short, read forwards): extents along (first axis, middle, last) and reals per batch
  // element; the first-axis kernels address it with f's column index c = x1 fL2 + x2 (fL2: f's last extent)
  int g_short;
  int gL0, gL1, gL2, fL2;
  long long g_batch;
  // multi-D first-axis kernels: residues r_lo .. r_hi - 1 only (r_hi = 0: all), their lines stored from
  // workspace line cs_rowbase(r) - row0; accum: the inverse adds to h instead of writing it
  int r_lo, r_hi, row0, accum;
};

struct SimpleParams {
  // pad / truncate / copy helpers for the explicit comparators
  const void* src;
  void* dst;
  int ndim;
  int Ls[3];   // source extents (reals)
  int Ld[3];   // destination extents (reals)
  long long src_batch, dst_batch;
  int batch;
  int rev;     // read the common box reversed on every axis
};

// launchers; return hipSuccess or an error.  Line kernels: one object file per
// (type, log2 m, kind group, block cap); kind groups: 0 one raw 1D problem,
// 1 multi-D line pairs / plain lines, 2 1D residue rows.
template <typename T, int LOGM, int KG, int PMAX>
hipError_t launch_line_kp(const LineParams<T>& P, dim3 grid, hipStream_t s, const LineParams<T>* tab);

template <typename T, int LOGM, int KG>
inline hipError_t launch_line_k(const LineParams<T>& P, int pcap, dim3 grid, hipStream_t s,
                                const LineParams<T>* tab) {
  switch (pcap) {
    case 0: return launch_line_kp<T, LOGM, KG, 0>(P, grid, s, tab);
    case 1: return launch_line_kp<T, LOGM, KG, 1>(P, grid, s, tab);
    case 2: return launch_line_kp<T, LOGM, KG, 2>(P, grid, s, tab);
    case 4: return launch_line_kp<T, LOGM, KG, 4>(P, grid, s, tab);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int LOGM>
inline hipError_t launch_line_lm(const LineParams<T>& P, int pcap, dim3 grid, hipStream_t s,
                                 const LineParams<T>* tab = nullptr) {
  switch (P.kind) {
    case LINE_1D: return launch_line_k<T, LOGM, 0>(P, pcap, grid, s, tab);
    case LINE_2D:
    case LINE_3D:
    case LINE_PLAIN: return launch_line_k<T, LOGM, 1>(P, pcap, grid, s, tab);
    case LINE_ROWS:
      if (pcap != 1) return hipErrorInvalidValue;
      return launch_line_kp<T, LOGM, 2, 1>(P, grid, s, tab);
    default: return hipErrorInvalidValue;
  }
}
template <typename T, int LOGM, bool FWD>
hipError_t launch_col_lm(const ColParams<T>& P, int pcap, int narr, dim3 grid, hipStream_t s,
                         const ColParams<T>* tab = nullptr);
template <typename T>
hipError_t launch_pad(const SimpleParams& P, hipStream_t s);
// which: 0 = whole 1D problem, 1 = first-axis forward, 2 = first-axis inverse,
// 3 / 4 = forward / inverse over column pairs of the multi-pass 1D form,
// 5 = whole 1D problem with residues 0 and q/2 packed (the mixed variant)
template <typename T, int LOGM>
hipError_t launch_cs_lm(const CsParams<T>& P, int which, int pcap, dim3 grid, hipStream_t s);

constexpr int kLineMaxLogM32 = 12;
constexpr int kLineMaxLogM64 = 11;
constexpr int kColMaxLogM = 10;
// column-pair transforms of the multi-pass 1D conjugate-symmetry form
constexpr int kCsPairMaxLogM = 11;

// geometry helpers shared by the planner and the kernels
// radix of the in-register first stage: m / 64 so that a team is one wavefront,
// at least 4 (short lines: several teams per wavefront)
constexpr int line_logr(int logm) { return logm <= 2 ? logm : (logm - 6 < 2 ? 2 : logm - 6); }
// the same for a line kernel of geometry kg; multi-D line pairs of 256 take radix 8 in teams of half a
// wavefront (three stages instead of four: 3D 256^3 conjugate-symmetry lines 0.545 against 0.657 ms; radix 8
// measured slower at 128 and for the one-workgroup 1D lines)
constexpr int line_logr(int logm, int kg) { return (kg == 1 && logm == 8) ? 3 : line_logr(logm); }
constexpr int line_waves = 4;
constexpr int col_logr(int logm, int pmax) { return logm <= (pmax >= 4 ? 3 : 4) ? logm : (pmax >= 4 ? 3 : 4); }

// Column tile of a workgroup.  Workgroups are dealt to the 8 XCDs (each with
// its own L2) round-robin by linear id.  When a tile's row segment is narrower
// than a 128-byte cache line, G neighbouring tiles share every line; giving
// them to blocks b, b + 8, ... (one XCD, dispatched back to back) lets their
// pieces of each line meet in one L2 instead of being fetched, and written
// back, once per XCD.  nbx is the problem's own tile count (grouped launches
// size the grid for their largest problem; blocks beyond nbx keep their index
// and exit).  A permutation of [0, nbx) when nbx is a multiple of 8 G and the
// grid width a multiple of 8 (then blockIdx.x % 8 is the XCD for every
// blockIdx.y, z); identity otherwise.
template <int G>
__device__ __forceinline__ int xcd_tile(int bx, int nbx) {
  if constexpr (G <= 1) {
    return bx;
  } else {
    if (nbx % (8 * G) || bx >= nbx || (gridDim.x & 7)) return bx;
    const int x = bx & 7, k = bx >> 3;
    return ((k / G) * 8 + x) * G + (k % G);
  }
}
// tiles per 128-byte line for row segments of `bytes` bytes
constexpr int tiles_per_line(int bytes) { return bytes >= 128 ? 1 : 128 / bytes; }

template <typename T>
inline size_t line_lds_bytes(int m, int q, int nspec) {
  return (size_t)nspec * q * padded_len(m) * sizeof(cx<T>);
}

}  // namespace hdc
