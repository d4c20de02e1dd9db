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
// (m, p, q) -> (p, 1, n) and the extra twiddle zeta_Nx^{k c} between the two
// stages (the complex inner loop: q = n p, r = u n + v).
#include <type_traits>

#include "hdc_kernels.hpp"

namespace hdc {

template <typename T, int LOGM, int PMAX>
struct ColCfg {
  static constexpr int M = 1 << LOGM;
  static constexpr int PE = PMAX > 0 ? PMAX : 4;
  static constexpr int LOGR = col_logr(LOGM, PE);
  static constexpr int R = 1 << LOGR;
  static constexpr int TS = M / R;
  static constexpr int WB = (sizeof(T) == 4) ? ((M * PE <= 1024) ? 16 : 8) : ((M * PE <= 512) ? 8 : 4);
  static constexpr int W = (WB * TS >= 64) ? WB : 64 / TS;
  static constexpr int NTHR = W * TS;
  // register budget: at least WPE waves per SIMD (512 / WPE VGPRs per lane)
  static constexpr int WPE = 2;
};

// Column element (row, c) addressing: rows advance by a uniform stride, so each
// access is a uniform (scalar) row base plus the thread's own offset.
template <typename T>
struct ColIn {
  const cx<T>* ws;   // workspace input (complex), or null
  const cx<T>* pk;   // raw input read as packed complex (fast path), or null
  const T* raw;      // raw input, general path (odd extents, reversed)
  RawGeom g;
  long long rs;      // complex elements per row (workspace or packed raw)
  int lin_pitch;
  int Lrows, C;
  int cval;
  __device__ __forceinline__ cx<T> at(int row, int c) const {
    if (!cval || row >= Lrows) return mk<T>(0, 0);
    if (ws) return ws[(long long)row * rs + c];
    if (pk) {
      if (lin_pitch) {
        const int lin = row * lin_pitch + c;
        return lin < g.Lhd ? pk[lin] : mk<T>(0, 0);
      }
      return c < g.mid * g.Lhd ? pk[(long long)row * rs + c] : mk<T>(0, 0);
    }
    return lin_pitch ? raw_load(raw, g, 0, row * lin_pitch + c) : raw_load(raw, g, row, c);
  }
};

template <typename T, int LOGM, int PMAX, bool TAB>
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
  const int c = blockIdx.x * W + w;
  const int slab = blockIdx.y % P0.nslab;
  const int b = TAB ? 0 : blockIdx.y / P0.nslab;
  if (TAB && (slab >= P.nslab || (int)blockIdx.x * W >= P.C)) return;
  const int arr = blockIdx.z;
  const int p = P.p, q = P.q;
  const cx<T>* root = root_of<T, LOGM>(P.rootpyr);

  ColIn<T> in;
  in.Lrows = P.Lrows;
  in.C = P.C;
  in.cval = c < P.C;
  in.lin_pitch = P.lin_pitch;
  in.ws = nullptr;
  in.pk = nullptr;
  in.raw = nullptr;
  if (P.rawin0) {
    in.g = arr ? P.graw1 : P.graw0;
    const T* base = (arr ? P.rawin1 : P.rawin0) + (long long)b * in.g.batch_stride;
    if (raw_packed(in.g)) {
      in.pk = reinterpret_cast<const cx<T>*>(base);
      in.rs = in.g.row_stride >> 1;
    } else {
      in.raw = base;
    }
  } else {
    in.ws = P.in + (long long)b * P.in_batch + (long long)arr * P.in_arr + (long long)slab * P.in_slab;
    in.rs = P.in_row;
  }

  constexpr int PX = PMAX > 0 ? PMAX : 1;
  cx<T> x[PX][R];
  if constexpr (PMAX > 0) {
    const bool cval = c < P.C;
    if (in.ws || (in.pk && !in.lin_pitch)) {
      // uniform row bases: element (row, c) at base[row * rs] + (j * rs + c)
      const cx<T>* base = in.ws ? in.ws : in.pk;
      const int climit = in.ws ? P.C : in.g.mid * in.g.Lhd;
      const cx<T>* pt = base + (long long)j * in.rs + c;
      const bool ok = cval && c < climit;
#pragma unroll
      for (int t = 0; t < PMAX; ++t)
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const int row = t * M + j + i * TS;
          x[t][i] = (ok && t < p && row < P.Lrows) ? pt[(long long)(t * M + i * TS) * in.rs] : mk<T>(0, 0);
        }
    } else if (in.pk) {
      // 1D: packed linear index row * lin_pitch + c
      const cx<T>* pt = in.pk + j * in.lin_pitch + c;
#pragma unroll
      for (int t = 0; t < PMAX; ++t)
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const int row = t * M + j + i * TS;
          const int lin = row * in.lin_pitch + c;
          x[t][i] = (cval && t < p && row < P.Lrows && lin < in.g.Lhd) ? pt[(t * M + i * TS) * in.lin_pitch]
                                                                         : mk<T>(0, 0);
        }
    } else {
#pragma unroll
      for (int t = 0; t < PMAX; ++t)
#pragma unroll
        for (int i = 0; i < R; ++i) x[t][i] = (t < p) ? in.at(t * M + j + i * TS, c) : mk<T>(0, 0);
    }
  }
  cx<T>* outp = P.out + (long long)b * P.out_batch + (long long)arr * P.out_arr + (long long)slab * P.out_slab +
                (long long)(q * j) * P.out_row + c;
  const long long ostep = (long long)q * TS * P.out_row;

  for (int r = 0; r < q; ++r) {
    cx<T> v[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int s = j + i * TS;
      cx<T> acc;
      if constexpr (PMAX > 0) {
        acc = x[0][i];
#pragma unroll
        for (int t = 1; t < PMAX; ++t)
          if (t < p) acc = acc + cmul(x[t][i], tw_get(P.twN, ((r * t) % q) * M));
      } else {
        // many explicit blocks: re-read the column for every residue
        acc = in.at(s, c);
        for (int t = 1; t < p; ++t) acc = acc + cmul(in.at(t * M + s, c), tw_get(P.twN, ((r * t) % q) * M));
      }
      v[i] = r ? cmul(acc, tw_get(P.twN, r * s)) : acc;
    }
    team_fft<T, LOGM, LOGR, +1, W, BlockSync>(v, j, lds + w, root, BlockSync());
    if (P.nx) {
      // four-step twiddle zeta_Nx^{k c} between the length-p and the length-m stages
#pragma unroll
      for (int i = 0; i < R; ++i) v[i] = cmul(v[i], tw_get(P.twX, (q * (j + i * TS) + r) * c));
    }
    if (c < P.C) {
      cx<T>* op = outp + (long long)r * P.out_row;
#pragma unroll
      for (int i = 0; i < R; ++i) op[i * ostep] = v[i];
    }
  }
}

// Inverse column pass.  COMP selects TwoSum-compensated accumulation over the
// residues; with at most two terms per output (q <= 2) a compensated sum equals
// the plain rounded sum exactly, so the plain form is used there.
template <typename T, int LOGM, int PMAX, bool COMP, bool TAB>
__global__ __launch_bounds__((ColCfg<T, LOGM, PMAX>::NTHR))
__attribute__((amdgpu_waves_per_eu(ColCfg<T, LOGM, PMAX>::WPE))) void k_col_inv(ColParams<T> P0, const ColParams<T>* __restrict__ tab) {
  // grouped launch (TAB): blockIdx.y = problem * (largest slab count) + slab, parameters from the table
  const ColParams<T> P = TAB ? tab[blockIdx.y / P0.nslab] : P0;
  using C = ColCfg<T, LOGM, PMAX>;
  using Acc = typename std::conditional<COMP, CAcc<T>, PAcc<T>>::type;
  constexpr int M = C::M, R = C::R, TS = C::TS, W = C::W, LOGR = C::LOGR;
  extern __shared__ char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  const int w = tid % W;
  const int j = tid / W;
  const int c = blockIdx.x * W + w;
  const bool cval = c < P.C;
  const int slab = blockIdx.y % P0.nslab;
  const int b = TAB ? 0 : blockIdx.y / P0.nslab;
  if (TAB && (slab >= P.nslab || (int)blockIdx.x * W >= P.C)) return;
  const int p = P.p, q = P.q;
  const cx<T>* root = root_of<T, LOGM>(P.rootpyr);

  constexpr int PC = PMAX > 0 ? PMAX : 4;  // blocks accumulated per sweep over the residues
  const cx<T>* inp = P.in + (long long)b * P.in_batch + (long long)slab * P.in_slab + (long long)(q * j) * P.in_row + c;
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
      const cx<T>* ip = inp + (long long)r * P.in_row;
#pragma unroll
      for (int i = 0; i < R; ++i) v[i] = cval ? ip[i * istep] : mk<T>(0, 0);
      if (P.nx) {
#pragma unroll
        for (int i = 0; i < R; ++i) v[i] = cmulc(v[i], tw_get(P.twX, (q * (j + i * TS) + r) * c));
      }
      team_fft<T, LOGM, LOGR, -1, W, BlockSync>(v, j, lds + w, root, BlockSync());
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int s = j + i * TS;
        const cx<T> y = r ? cmulc(v[i], tw_get(P.twN, r * s)) : v[i];
        acc[0][i].add((r && t0) ? cmulc(y, tw_get(P.twN, ((r * t0) % q) * M)) : y);
#pragma unroll
        for (int tt = 1; tt < PC; ++tt) {
          const int t = t0 + tt;
          if (t < p) acc[tt][i].add(r ? cmulc(y, tw_get(P.twN, ((r * t) % q) * M)) : y);
        }
      }
    }
    if (!cval) continue;
    if (P.rawout == nullptr) {
      cx<T>* outp = P.out + (long long)b * P.out_batch + (long long)slab * P.out_slab + (long long)j * P.out_row + c;
#pragma unroll
      for (int tt = 0; tt < PC; ++tt)
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const int row = (t0 + tt) * M + j + i * TS;
          if (t0 + tt < p && row < P.Lrows) outp[(long long)((t0 + tt) * M + i * TS) * P.out_row] = acc[tt][i].get();
        }
      continue;
    }
    const RawGeom& g = P.graw0;
    T* rbase = P.rawout + (long long)b * g.batch_stride;
    if (raw_packed(g)) {
      cx<T>* pk = reinterpret_cast<cx<T>*>(rbase);
      if (P.lin_pitch) {
#pragma unroll
        for (int tt = 0; tt < PC; ++tt)
#pragma unroll
          for (int i = 0; i < R; ++i) {
            const int row = (t0 + tt) * M + j + i * TS;
            const int lin = row * P.lin_pitch + c;
            if (t0 + tt < p && row < P.Lrows && lin < g.Lhd) pk[lin] = acc[tt][i].get();
          }
      } else {
        const long long prs = g.row_stride >> 1;
        cx<T>* pt = pk + (long long)j * prs + c;
#pragma unroll
        for (int tt = 0; tt < PC; ++tt)
#pragma unroll
          for (int i = 0; i < R; ++i) {
            const int row = (t0 + tt) * M + j + i * TS;
            if (t0 + tt < p && row < P.Lrows && c < g.mid * g.Lhd)
              pt[(long long)((t0 + tt) * M + i * TS) * prs] = acc[tt][i].get();
          }
      }
    } else {
#pragma unroll
      for (int tt = 0; tt < PC; ++tt)
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const int row = (t0 + tt) * M + j + i * TS;
          if (t0 + tt >= p || row >= P.Lrows) continue;
          if (P.lin_pitch) raw_store(rbase, g, 0, row * P.lin_pitch + c, acc[tt][i].get());
          else raw_store(rbase, g, row, c, acc[tt][i].get());
        }
    }
  }
}

template <typename T, int LOGM, int PMAX, bool FWD>
static hipError_t launch_col_t(const ColParams<T>& P, int narr, dim3 grid, hipStream_t s, const ColParams<T>* tab) {
  using C = ColCfg<T, LOGM, PMAX>;
  const size_t lds = (C::M > C::R) ? (size_t)padded_len(C::M) * C::W * sizeof(cx<T>) : 0;
  grid.x = (P.C + C::W - 1) / C::W;
  grid.z = FWD ? narr : 1;
  using KFn = void (*)(ColParams<T>, const ColParams<T>*);
  const bool comp = P.q > 2;
  KFn fn;
  if (tab)
    fn = FWD ? k_col_fwd<T, LOGM, PMAX, true> : (comp ? k_col_inv<T, LOGM, PMAX, true, true> : k_col_inv<T, LOGM, PMAX, false, true>);
  else
    fn = FWD ? k_col_fwd<T, LOGM, PMAX, false>
             : (comp ? k_col_inv<T, LOGM, PMAX, true, false> : k_col_inv<T, LOGM, PMAX, false, false>);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fn, grid, dim3(C::NTHR), lds, s, P, tab);
  return hipGetLastError();
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
template <typename T>
__global__ void k_boxcopy(SimpleParams P, int rev) {
  const long long total = (long long)P.Ld[0] * P.Ld[1] * P.Ld[2];
  const int b = blockIdx.y;
  const T* src = reinterpret_cast<const T*>(P.src) + (long long)b * P.src_batch;
  T* dst = reinterpret_cast<T*>(P.dst) + (long long)b * P.dst_batch;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int x2 = (int)(idx % P.Ld[2]);
    const long long r1 = idx / P.Ld[2];
    const int x1 = (int)(r1 % P.Ld[1]);
    const int x0 = (int)(r1 / P.Ld[1]);
    const int E0 = P.Ls[0] < P.Ld[0] ? P.Ls[0] : P.Ld[0];
    const int E1 = P.Ls[1] < P.Ld[1] ? P.Ls[1] : P.Ld[1];
    const int E2 = P.Ls[2] < P.Ld[2] ? P.Ls[2] : P.Ld[2];
    T v = (T)0;
    if (x0 < E0 && x1 < E1 && x2 < E2) {
      const int y0 = rev ? E0 - 1 - x0 : x0;
      const int y1 = rev ? E1 - 1 - x1 : x1;
      const int y2 = rev ? E2 - 1 - x2 : x2;
      v = src[((long long)y0 * P.Ls[1] + y1) * P.Ls[2] + y2];
    }
    dst[idx] = v;
  }
}

template <typename T>
hipError_t launch_pad(const SimpleParams& P, hipStream_t s) {
  const long long total = (long long)P.Ld[0] * P.Ld[1] * P.Ld[2];
  long long blocks = (total + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_boxcopy<T>, dim3((unsigned)blocks, P.batch), dim3(256), 0, s, P, P.rev);
  return hipGetLastError();
}
template hipError_t launch_pad<float>(const SimpleParams&, hipStream_t);
template hipError_t launch_pad<double>(const SimpleParams&, hipStream_t);
#endif

}  // namespace hdc
