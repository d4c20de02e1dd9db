// Column kernels: the implicitly padded transform along a strided axis.
//
// A workgroup owns W adjacent columns (W complex elements = 128 bytes of a row,
// so every global access is a coalesced row segment) and the whole axis of
// those columns, so no global transpose is ever needed.  Thread (w, j) keeps
// the input rows t m + s, s = j + i TS (i < R), t < p of column w in registers
// and walks the residues one at a time (Sec. 2.1):
//   forward  X_r[s] = zeta_N^{r s} sum_{t<p} zeta_q^{r t} x[t m + s]   (eq. (forwardr))
//            length-m FFT over s, output row k = q l + r (natural order);
//   inverse  length-m inverse FFT of rows q l + r, post-twiddle zeta_N^{-r s},
//            h[t m + s] += zeta_q^{-r t} w_r[s] with TwoSum compensation
//            (eqs. (accumulator), (accumulation)); rows j < L are written.
// The same kernels perform the length-p stage of the multi-pass 1D form with
// (m, p, q) -> (p, 1, n) (the complex inner loop: q = n p, r = u n + v); the
// four-step twiddle between the two stages is applied by the row kernel.
#include <type_traits>

#include "hdc_kernels.hpp"

namespace hdc {

template <typename T, int LOGM, int PMAX, bool INV = false>
struct ColCfg {
  static constexpr int M = 1 << LOGM;
  static constexpr int PE = PMAX > 0 ? PMAX : 4;
  // radix 16; 8 with four register blocks, in FP64 (complex values take twice
  // the registers) and in the inverse over two or more blocks (two sets of
  // compensated accumulators of 16 values spill); 4 in the FP64 inverse over
  // four blocks (four compensated FP64 sets of 8 values fill the register file)
  static constexpr int LOGR0 = col_logr(LOGM, PE);
  static constexpr int LOGR1 = (LOGR0 > 3 && (sizeof(T) == 8 || (INV && PE >= 2))) ? 3 : LOGR0;
  static constexpr int LOGR = (LOGR1 > 2 && sizeof(T) == 8 && INV && PE >= 4) ? 2 : LOGR1;
  // batched twiddle loads, unless two sets of compensated accumulators leave no registers
  static constexpr bool BATCH = !(INV && PE >= 2);
  static constexpr int R = 1 << LOGR;
  static constexpr int TS = M / R;
  // columns per workgroup: whole 128-byte row segments (16 FP32 / 8 FP64 complex) while the tile stays
  // within 512 threads; FP64 columns of 512 on 4 columns wrote about 1.19x their bytes
  static constexpr int WB = (sizeof(T) == 4) ? ((M * PE < 1024) ? 16 : 8) : ((M * PE < 1024) ? 8 : 4);
  static constexpr int W0 = (WB * TS >= 64) ? WB : 64 / TS;
  // at most 512 threads, so that a lane may hold 256 VGPRs (1024 threads leave 128, and the
  // register blocks of m = 1024 spill there)
  static constexpr int W = (W0 * TS > 512 && TS <= 512) ? 512 / TS : W0;
  static constexpr int NTHR = W * TS;
  // register budget: at least WPE waves per SIMD (512 / WPE VGPRs per lane)
  static constexpr int WPE = 2;
};

// Column element (row, c) addressing.  Fast form (GEN = false): a complex
// array with element (row, c) at base[row * rs + c] -- the workspace, or real
// input/output read as packed complex (even length, not reversed), where the
// 1D form's rows are consecutive pieces of one line (rs = row length).  Each
// access is a uniform row base (scalar registers) plus the lane's 32-bit byte
// offset (j rs + c) * sizeof(cx); valid elements: row < rows, c < climit and
// row * rs + c < linmax.  General form (GEN = true): real arrays of any parity,
// read or written reversed (the adjoint), through raw_load / raw_store.
template <typename T>
struct ColView {
  char* base;
  long long rs;
  int linmax;  // 1D form: elements of the line (0: rows form)
  int climit;
  int rowmax;  // rows present (a kernel g shorter than f has fewer)
  uint32_t loff;
  __device__ __forceinline__ bool valid(int row, int c) const {
    return (c < climit) & (row < rowmax) & ((linmax == 0) | (row * (int)rs + c < linmax));
  }
  // element (rowblock + lane row j, c) where rowblock is uniform
  __device__ __forceinline__ cx<T>* at(int rowblock) const {
    return reinterpret_cast<cx<T>*>(base + (long long)rowblock * rs * (long long)sizeof(cx<T>) + loff);
  }
};

template <typename T, int LOGM, int PMAX, bool TAB, bool GEN>
__global__ __launch_bounds__((ColCfg<T, LOGM, PMAX>::NTHR))
__attribute__((amdgpu_waves_per_eu(ColCfg<T, LOGM, PMAX>::WPE))) void k_col_fwd(ColParams<T> P0, const ColParams<T>* __restrict__ tab) {
  // grouped launch (TAB): blockIdx.y = problem * (largest slab count) + slab, parameters from the table
  const ColParams<T> P = TAB ? tab[blockIdx.y / P0.nslab] : P0;
  using C = ColCfg<T, LOGM, PMAX>;
  constexpr int M = C::M, R = C::R, TS = C::TS, W = C::W, LOGR = C::LOGR;
  extern __shared__ char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  const int w = tid % W;
  const int j = tid / W;
  // grouped launches rotate the tiles by the problem index so that the first
  // tiles of many small problems do not all land on the same XCDs
  const int tile = TAB ? (int)((blockIdx.x + gridDim.x - blockIdx.y % gridDim.x) % gridDim.x)
                       : xcd_tile<tiles_per_line(W * (int)sizeof(cx<T>))>((int)blockIdx.x, (P.C + W - 1) / W);
  const int c = tile * W + w;
  const int slab = blockIdx.y % P0.nslab;
  const int b = TAB ? 0 : blockIdx.y / P0.nslab;
  if (TAB && (slab >= P.nslab || tile * W >= P.C)) return;
  const int arr = blockIdx.z + P.arr0;
  const int p = P.p, q = P.q;
  const bool cval = c < P.C;
  const cx<T>* root = root_of<T, LOGM>(P.rootpyr);

  // ---- input
  ColView<T> vw{};
  const T* raw = nullptr;
  RawGeom rg{};
  if constexpr (!GEN) {
    if (P.rawin0) {
      rg = arr ? P.graw1 : P.graw0;
      vw.base = (char*)((arr ? P.rawin1 : P.rawin0) + (long long)b * rg.batch_stride);
      vw.rs = P.lin_pitch ? P.lin_pitch : (rg.row_stride >> 1);
      vw.linmax = P.lin_pitch ? rg.Lhd : 0;
      vw.climit = P.lin_pitch ? P.C : rg.mid * rg.Lhd;
      vw.rowmax = P.lin_pitch ? 0x7fffffff : rg.rows;
    } else {
      vw.base = (char*)(P.in + (long long)b * P.in_batch + (long long)arr * P.in_arr + (long long)slab * P.in_slab);
      vw.rs = P.in_row;
      vw.linmax = 0;
      vw.climit = P.C;
      vw.rowmax = 0x7fffffff;
    }
    vw.loff = (uint32_t)((long long)j * vw.rs + c) * (uint32_t)sizeof(cx<T>);
  } else {
    rg = arr ? P.graw1 : P.graw0;
    raw = (arr ? P.rawin1 : P.rawin0) + (long long)b * rg.batch_stride;
  }
  auto load = [&](int row) -> cx<T> {  // element (row, c), zero outside the data
    if (!cval || row >= P.Lrows) return mk<T>(0, 0);
    if constexpr (!GEN) {
      if (!vw.valid(row, c)) return mk<T>(0, 0);
      return *reinterpret_cast<const cx<T>*>(vw.base + ((long long)row * vw.rs + c) * (long long)sizeof(cx<T>));
    } else {
      return P.lin_pitch ? raw_load(raw, rg, 0, row * P.lin_pitch + c) : raw_load(raw, rg, row, c);
    }
  };

  constexpr int PX = PMAX > 0 ? PMAX : 1;
  // blocks holding data: a shorter raw array (the kernel g) has fewer rows than the problem, and its blocks
  // beyond them are skipped rather than masked (Sec. 7: p per array)
  int pa = p;
  if (P.rawin0 && !P.lin_pitch) pa = min(p, (rg.rows + M - 1) / M);
  cx<T> x[PX][R];
  if constexpr (PMAX > 0) {
#pragma unroll
    for (int t = 0; t < PMAX; ++t)
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int row = t * M + j + i * TS;
        if constexpr (!GEN) {
          // branch-free: a masked lane reads element 0 of the array and drops it
          const bool ok = cval && t < pa && row < P.Lrows && vw.valid(row, c);
          const cx<T> val = *(ok ? vw.at(t * M + i * TS) : reinterpret_cast<const cx<T>*>(vw.base));
          x[t][i] = ok ? val : mk<T>(0, 0);
        } else {
          x[t][i] = (t < pa) ? load(row) : mk<T>(0, 0);
        }
      }
  }
  char* obase = reinterpret_cast<char*>(P.out + (long long)b * P.out_batch + (long long)arr * P.out_arr +
                                        (long long)slab * P.out_slab);
  const uint32_t ooff = (uint32_t)((long long)(q * j) * P.out_row + c) * (uint32_t)sizeof(cx<T>);
  const long long ostep = (long long)q * TS * P.out_row;

  for (int r = 0; r < q; ++r) {
    cx<T> v[R];
    if constexpr (PMAX > 0) {
      // sum_t zeta_q^{r t} x[t m + s]; blocks t >= p were loaded as zeros
      cx<T> wq[PX];
#pragma unroll
      for (int t = 1; t < PX; ++t) wq[t] = tw1(P.twN, ((r * t) % q) * M);
#pragma unroll
      for (int i = 0; i < R; ++i) {
        cx<T> acc = x[0][i];
#pragma unroll
        for (int t = 1; t < PX; ++t)
          if (t < pa) acc = acc + cmul(x[t][i], wq[t]);
        v[i] = acc;
      }
    } else {
      // many explicit blocks: re-read the column for every residue
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int s = j + i * TS;
        cx<T> acc = load(s);
        for (int t = 1; t < pa; ++t) acc = acc + cmul(load(t * M + s), tw1(P.twN, ((r * t) % q) * M));
        v[i] = acc;
      }
    }
    residue_twiddle<T, R, TS, +1, true, 1>(v, j, r, P.twN);
    team_fft<T, LOGM, LOGR, +1, W, BlockSync>(v, j, lds + w, root, BlockSync());
    if (cval) {
      char* ob = obase + (long long)r * P.out_row * (long long)sizeof(cx<T>) + ooff;
#pragma unroll
      for (int i = 0; i < R; ++i)
        *reinterpret_cast<cx<T>*>(ob + (long long)i * ostep * (long long)sizeof(cx<T>)) = v[i];
    }
  }
}

// Inverse column pass.  COMP selects TwoSum-compensated accumulation over the
// residues; with at most two terms per output (q <= 2) a compensated sum equals
// the plain rounded sum exactly, so the plain form is used there.
template <typename T, int LOGM, int PMAX, bool COMP, bool TAB, bool GEN>
__global__ __launch_bounds__((ColCfg<T, LOGM, PMAX, true>::NTHR))
__attribute__((amdgpu_waves_per_eu(ColCfg<T, LOGM, PMAX, true>::WPE))) void k_col_inv(ColParams<T> P0, const ColParams<T>* __restrict__ tab) {
  // grouped launch (TAB): blockIdx.y = problem * (largest slab count) + slab, parameters from the table
  const ColParams<T> P = TAB ? tab[blockIdx.y / P0.nslab] : P0;
  using C = ColCfg<T, LOGM, PMAX, true>;
  using Acc = typename std::conditional<COMP, CAcc<T>, PAcc<T>>::type;
  constexpr int M = C::M, R = C::R, TS = C::TS, W = C::W, LOGR = C::LOGR;
  extern __shared__ char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  const int w = tid % W;
  const int j = tid / W;
  // grouped launches rotate the tiles by the problem index so that the first
  // tiles of many small problems do not all land on the same XCDs
  const int tile = TAB ? (int)((blockIdx.x + gridDim.x - blockIdx.y % gridDim.x) % gridDim.x)
                       : xcd_tile<tiles_per_line(W * (int)sizeof(cx<T>))>((int)blockIdx.x, (P.C + W - 1) / W);
  const int c = tile * W + w;
  const bool cval = c < P.C;
  const int slab = blockIdx.y % P0.nslab;
  const int b = TAB ? 0 : blockIdx.y / P0.nslab;
  if (TAB && (slab >= P.nslab || tile * W >= P.C)) return;
  const int p = P.p, q = P.q;
  const cx<T>* root = root_of<T, LOGM>(P.rootpyr);

  // ---- output
  ColView<T> vw{};
  T* rawo = nullptr;
  RawGeom og{};
  if constexpr (!GEN) {
    if (P.rawout) {
      og = P.graw0;
      vw.base = (char*)(P.rawout + (long long)b * og.batch_stride);
      vw.rs = P.lin_pitch ? P.lin_pitch : (og.row_stride >> 1);
      vw.linmax = P.lin_pitch ? og.Lhd : 0;
      vw.climit = P.lin_pitch ? P.C : og.mid * og.Lhd;
    } else {
      vw.base = (char*)(P.out + (long long)b * P.out_batch + (long long)slab * P.out_slab);
      vw.rs = P.out_row;
      vw.linmax = 0;
      vw.climit = P.C;
    }
    vw.rowmax = 0x7fffffff;  // output rows are limited by Lrows
    vw.loff = (uint32_t)((long long)j * vw.rs + c) * (uint32_t)sizeof(cx<T>);
  } else {
    og = P.graw0;
    rawo = P.rawout + (long long)b * og.batch_stride;
  }

  constexpr int PC = PMAX > 0 ? PMAX : 4;  // blocks accumulated per sweep over the residues
  const char* ibase = reinterpret_cast<const char*>(P.in + (long long)b * P.in_batch + (long long)slab * P.in_slab);
  const uint32_t ioff = (uint32_t)((long long)(q * j) * P.in_row + c) * (uint32_t)sizeof(cx<T>);
  const long long istep = (long long)q * TS * P.in_row;

  for (int t0 = 0; t0 < p; t0 += PC) {
    Acc acc[PC][R];
#pragma unroll
    for (int t = 0; t < PC; ++t)
#pragma unroll
      for (int i = 0; i < R; ++i) acc[t][i].zero();
    for (int r = 0; r < q; ++r) {
      // keep this residue's loads from being hoisted over the previous FFT (register pressure)
      __builtin_amdgcn_sched_barrier(0);
      cx<T> v[R];
      const char* ib = ibase + (long long)r * P.in_row * (long long)sizeof(cx<T>) + ioff;
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const cx<T> val = *(cval ? reinterpret_cast<const cx<T>*>(ib + (long long)i * istep * (long long)sizeof(cx<T>))
                                 : reinterpret_cast<const cx<T>*>(ibase));
        v[i] = cval ? val : mk<T>(0, 0);
      }
      team_fft<T, LOGM, LOGR, -1, W, BlockSync, 1>(v, j, lds + w, root, BlockSync());
      if constexpr (!C::BATCH) {
        // register-limited form, element by element and branch-free
        // (zeta^0 = 1 exactly: residue 0 and block 0 pass through unchanged)
        cx<T> wt[PC];
#pragma unroll
        for (int tt = 0; tt < PC; ++tt) wt[tt] = tw1(P.twN, ((r * (t0 + tt)) % q) * M);
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const cx<T> y = cmulc(v[i], tw1(P.twN, r * (j + i * TS)));
#pragma unroll
          for (int tt = 0; tt < PC; ++tt) acc[tt][i].add(cmulc(y, wt[tt]));
        }
        continue;
      }
      residue_twiddle<T, R, TS, -1, true, 1>(v, j, r, P.twN);
      // h[t m + s] += zeta_q^{-r t} w_r[s]; accumulators of blocks t >= p are never stored
      if (t0 == 0) {
#pragma unroll
        for (int i = 0; i < R; ++i) acc[0][i].add(v[i]);
      } else {
        const cx<T> wt = tw1(P.twN, ((r * t0) % q) * M);
#pragma unroll
        for (int i = 0; i < R; ++i) acc[0][i].add(cmulc(v[i], wt));
      }
#pragma unroll
      for (int tt = 1; tt < PC; ++tt) {
        const cx<T> wt = tw1(P.twN, ((r * (t0 + tt)) % q) * M);
#pragma unroll
        for (int i = 0; i < R; ++i) acc[tt][i].add(cmulc(v[i], wt));
      }
    }
    if (!cval) continue;
#pragma unroll
    for (int tt = 0; tt < PC; ++tt)
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int row = (t0 + tt) * M + j + i * TS;
        if (t0 + tt >= p || row >= P.Lrows) continue;
        if constexpr (!GEN) {
          if (vw.valid(row, c)) *vw.at((t0 + tt) * M + i * TS) = acc[tt][i].get();
        } else {
          if (P.lin_pitch) raw_store(rawo, og, 0, row * P.lin_pitch + c, acc[tt][i].get());
          else raw_store(rawo, og, row, c, acc[tt][i].get());
        }
      }
  }
}

template <typename T, int LOGM, int PMAX, bool FWD, bool GEN>
static hipError_t launch_col_g(const ColParams<T>& P, int narr, dim3 grid, hipStream_t s, const ColParams<T>* tab) {
  using C = ColCfg<T, LOGM, PMAX, !FWD>;
  const size_t lds = (C::M > C::R) ? (size_t)padded_len(C::M) * C::W * sizeof(cx<T>) : 0;
  grid.x = (P.C + C::W - 1) / C::W;
  grid.z = FWD ? narr : 1;
  using KFn = void (*)(ColParams<T>, const ColParams<T>*);
  const bool comp = P.q > 2;
  KFn fn;
  if (tab)
    fn = FWD ? k_col_fwd<T, LOGM, PMAX, true, GEN>
             : (comp ? k_col_inv<T, LOGM, PMAX, true, true, GEN> : k_col_inv<T, LOGM, PMAX, false, true, GEN>);
  else
    fn = FWD ? k_col_fwd<T, LOGM, PMAX, false, GEN>
             : (comp ? k_col_inv<T, LOGM, PMAX, true, false, GEN> : k_col_inv<T, LOGM, PMAX, false, false, GEN>);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fn, grid, dim3(C::NTHR), lds, s, P, tab);
  return hipGetLastError();
}

// Both forms address the workspace with 32-bit lane byte offsets from uniform
// row bases: (TS - 1) * (row pitch) + C complex elements must stay below 2^32
// bytes (far beyond any problem that fits in device memory with its workspace).
template <typename T, int LOGM, int PMAX, bool FWD>
static hipError_t launch_col_t(const ColParams<T>& P, int narr, dim3 grid, hipStream_t s, const ColParams<T>* tab) {
  using C = ColCfg<T, LOGM, PMAX, !FWD>;
  const bool gen = col_general(P, FWD);
  if (((long long)(C::TS - 1) * col_pitch(P, FWD) + P.C) * (long long)sizeof(cx<T>) >= (1LL << 32))
    return hipErrorInvalidValue;
  return gen ? launch_col_g<T, LOGM, PMAX, FWD, true>(P, narr, grid, s, tab)
             : launch_col_g<T, LOGM, PMAX, FWD, false>(P, narr, grid, s, tab);
}

template <typename T, int LOGM, bool FWD>
hipError_t launch_col_lm(const ColParams<T>& P, int pcap, int narr, dim3 grid, hipStream_t s,
                         const ColParams<T>* tab) {
  switch (pcap) {
    case 0: return launch_col_t<T, LOGM, 0, FWD>(P, narr, grid, s, tab);
    case 1: return launch_col_t<T, LOGM, 1, FWD>(P, narr, grid, s, tab);
    case 2: return launch_col_t<T, LOGM, 2, FWD>(P, narr, grid, s, tab);
    case 4: return launch_col_t<T, LOGM, 4, FWD>(P, narr, grid, s, tab);
    default: return hipErrorInvalidValue;
  }
}

#if defined(HDC_T) && defined(HDC_LOGM)
template hipError_t launch_col_lm<HDC_T, HDC_LOGM, true>(const ColParams<HDC_T>&, int, int, dim3, hipStream_t,
                                                         const ColParams<HDC_T>*);
template hipError_t launch_col_lm<HDC_T, HDC_LOGM, false>(const ColParams<HDC_T>&, int, int, dim3, hipStream_t,
                                                          const ColParams<HDC_T>*);
#endif

#if defined(HDC_MISC)
// ---------------------------------------------------------------------------
// box copy for the explicit comparators: dst (extents Ld) <- src (extents Ls),
// zero outside the common box; rev reads the box reversed on every axis
// ---------------------------------------------------------------------------
// One workgroup copies a chunk of kBoxChunk consecutive elements of one
// destination row (x0, x1); the row and chunk come from blockIdx.x (uniform
// integer arithmetic), lanes walk x2 contiguously (reversed reads stay
// contiguous, descending).
constexpr int kBoxChunk = 2048;

template <typename T>
__global__ __launch_bounds__(256) void k_boxcopy(SimpleParams P, int rev, int nch) {
  const int b = blockIdx.y;
  const long long row = blockIdx.x / nch;
  const int x2s = (int)(blockIdx.x - row * nch) * kBoxChunk;
  const int x1 = (int)(row % P.Ld[1]);
  const int x0 = (int)(row / P.Ld[1]);
  const T* src = reinterpret_cast<const T*>(P.src) + (long long)b * P.src_batch;
  T* dst = reinterpret_cast<T*>(P.dst) + (long long)b * P.dst_batch + row * P.Ld[2];
  const int E0 = P.Ls[0] < P.Ld[0] ? P.Ls[0] : P.Ld[0];
  const int E1 = P.Ls[1] < P.Ld[1] ? P.Ls[1] : P.Ld[1];
  const int E2 = P.Ls[2] < P.Ld[2] ? P.Ls[2] : P.Ld[2];
  const bool inrow = x0 < E0 && x1 < E1;
  const int y0 = rev ? E0 - 1 - x0 : x0;
  const int y1 = rev ? E1 - 1 - x1 : x1;
  const T* srow = src + (inrow ? ((long long)y0 * P.Ls[1] + y1) * P.Ls[2] : 0);
  const int x2e = (x2s + kBoxChunk < P.Ld[2]) ? x2s + kBoxChunk : P.Ld[2];
#pragma unroll 8
  for (int x2 = x2s + (int)threadIdx.x; x2 < x2e; x2 += 256) {
    const bool ok = inrow && x2 < E2;
    const int y2 = rev ? E2 - 1 - x2 : x2;
    const T v = *(ok ? srow + y2 : src);  // a masked lane reads element 0 of the source
    dst[x2] = ok ? v : (T)0;
  }
}

template <typename T>
hipError_t launch_pad(const SimpleParams& P, hipStream_t s) {
  const long long rows = (long long)P.Ld[0] * P.Ld[1];
  const int nch = (P.Ld[2] + kBoxChunk - 1) / kBoxChunk;
  const long long blocks = rows * nch;
  if (blocks < 1 || blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_boxcopy<T>, dim3((unsigned)blocks, P.batch), dim3(256), 0, s, P, P.rev, nch);
  return hipGetLastError();
}
template hipError_t launch_pad<float>(const SimpleParams&, hipStream_t);
template hipError_t launch_pad<double>(const SimpleParams&, hipStream_t);
#endif

}  // namespace hdc
