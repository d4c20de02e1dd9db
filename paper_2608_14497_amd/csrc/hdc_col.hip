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
};

template <typename T, int LOGM, int PMAX>
__global__ __launch_bounds__((ColCfg<T, LOGM, PMAX>::NTHR)) void k_col_fwd(ColParams<T> P) {
  using C = ColCfg<T, LOGM, PMAX>;
  constexpr int M = C::M, R = C::R, TS = C::TS, W = C::W, LOGR = C::LOGR;
  extern __shared__ char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  const int w = tid % W;
  const int j = tid / W;
  const int c = blockIdx.x * W + w;
  const bool cval = c < P.C;
  const int slab = blockIdx.y % P.nslab;
  const int b = blockIdx.y / P.nslab;
  const int arr = blockIdx.z;
  const int p = P.p, q = P.q;

  const RawGeom& g = arr ? P.graw1 : P.graw0;
  const T* rbase = P.rawin0 ? (arr ? P.rawin1 : P.rawin0) + (long long)b * g.batch_stride : nullptr;
  const cx<T>* inp = P.in + (long long)b * P.in_batch + (long long)arr * P.in_arr + (long long)slab * P.in_slab;
  auto load = [&](int row) -> cx<T> {
    if (!cval || row >= P.Lrows) return mk<T>(0, 0);
    if (rbase) return P.lin_pitch ? raw_load(rbase, g, 0, row * P.lin_pitch + c) : raw_load(rbase, g, row, c);
    return inp[(long long)row * P.in_row + c];
  };
  constexpr int PX = PMAX > 0 ? PMAX : 1;
  cx<T> x[PX][R];
  if constexpr (PMAX > 0) {
#pragma unroll
    for (int t = 0; t < PMAX; ++t)
#pragma unroll
      for (int i = 0; i < R; ++i) x[t][i] = (t < p) ? load(t * M + j + i * TS) : mk<T>(0, 0);
  }
  cx<T>* outp = P.out + (long long)b * P.out_batch + (long long)arr * P.out_arr + (long long)slab * P.out_slab;

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
        acc = load(s);
        for (int t = 1; t < p; ++t) acc = acc + cmul(load(t * M + s), tw_get(P.twN, ((r * t) % q) * M));
      }
      v[i] = r ? cmul(acc, tw_get(P.twN, r * s)) : acc;
    }
    team_fft<T, LOGM, LOGR, +1, BlockSync>(v, j, lds + w, W, P.root, P.logroot, BlockSync());
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int l = j + i * TS;
      const int k = q * l + r;
      cx<T> y = v[i];
      if (P.nx) y = cmul(y, tw_get(P.twX, k * c));
      if (cval) outp[(long long)k * P.out_row + c] = y;
    }
  }
}

template <typename T, int LOGM, int PMAX>
__global__ __launch_bounds__((ColCfg<T, LOGM, PMAX>::NTHR)) void k_col_inv(ColParams<T> P) {
  using C = ColCfg<T, LOGM, PMAX>;
  constexpr int M = C::M, R = C::R, TS = C::TS, W = C::W, LOGR = C::LOGR;
  extern __shared__ char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  const int w = tid % W;
  const int j = tid / W;
  const int c = blockIdx.x * W + w;
  const bool cval = c < P.C;
  const int slab = blockIdx.y % P.nslab;
  const int b = blockIdx.y / P.nslab;
  const int p = P.p, q = P.q;

  constexpr int PC = PMAX > 0 ? PMAX : 4;  // blocks accumulated per sweep over the residues
  const cx<T>* inp = P.in + (long long)b * P.in_batch + (long long)slab * P.in_slab;
  for (int t0 = 0; t0 < p; t0 += PC) {
    CAcc<T> acc[PC][R];
#pragma unroll
    for (int t = 0; t < PC; ++t)
#pragma unroll
      for (int i = 0; i < R; ++i) acc[t][i].zero();
    for (int r = 0; r < q; ++r) {
      cx<T> v[R];
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int l = j + i * TS;
        const int k = q * l + r;
        cx<T> y = cval ? inp[(long long)k * P.in_row + c] : mk<T>(0, 0);
        if (P.nx) y = cmulc(y, tw_get(P.twX, k * c));
        v[i] = y;
      }
      team_fft<T, LOGM, LOGR, -1, BlockSync>(v, j, lds + w, W, P.root, P.logroot, BlockSync());
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int s = j + i * TS;
        const cx<T> y = r ? cmulc(v[i], tw_get(P.twN, r * s)) : v[i];
#pragma unroll
        for (int tt = 0; tt < PC; ++tt) {
          const int t = t0 + tt;
          if (t < p) acc[tt][i].add((r && t) ? cmulc(y, tw_get(P.twN, ((r * t) % q) * M)) : y);
        }
      }
    }
    if (P.rawout) {
      const RawGeom& g = P.graw0;
      T* base = P.rawout + (long long)b * g.batch_stride;
#pragma unroll
      for (int tt = 0; tt < PC; ++tt)
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const int row = (t0 + tt) * M + j + i * TS;
          if (cval && t0 + tt < p && row < P.Lrows) {
            const cx<T> val = acc[tt][i].get();
            if (P.lin_pitch) raw_store(base, g, 0, row * P.lin_pitch + c, val);
            else raw_store(base, g, row, c, val);
          }
        }
    } else {
      cx<T>* outp = P.out + (long long)b * P.out_batch + (long long)slab * P.out_slab;
#pragma unroll
      for (int tt = 0; tt < PC; ++tt)
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const int row = (t0 + tt) * M + j + i * TS;
          if (cval && t0 + tt < p && row < P.Lrows) outp[(long long)row * P.out_row + c] = acc[tt][i].get();
        }
    }
  }
}

template <typename T, int LOGM, int PMAX, bool FWD>
static hipError_t launch_col_t(const ColParams<T>& P, int narr, dim3 grid, hipStream_t s) {
  using C = ColCfg<T, LOGM, PMAX>;
  const size_t lds = (C::M > C::R) ? (size_t)padded_len(C::M) * C::W * sizeof(cx<T>) : 0;
  grid.x = (P.C + C::W - 1) / C::W;
  grid.z = FWD ? narr : 1;
  auto fn = FWD ? k_col_fwd<T, LOGM, PMAX> : k_col_inv<T, LOGM, PMAX>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fn, grid, dim3(C::NTHR), lds, s, P);
  return hipGetLastError();
}

template <typename T, int LOGM, bool FWD>
hipError_t launch_col_lm(const ColParams<T>& P, int pcap, int narr, dim3 grid, hipStream_t s) {
  switch (pcap) {
    case 0: return launch_col_t<T, LOGM, 0, FWD>(P, narr, grid, s);
    case 1: return launch_col_t<T, LOGM, 1, FWD>(P, narr, grid, s);
    case 2: return launch_col_t<T, LOGM, 2, FWD>(P, narr, grid, s);
    case 4: return launch_col_t<T, LOGM, 4, FWD>(P, narr, grid, s);
    default: return hipErrorInvalidValue;
  }
}

#if defined(HDC_T) && defined(HDC_LOGM)
template hipError_t launch_col_lm<HDC_T, HDC_LOGM, true>(const ColParams<HDC_T>&, int, int, dim3, hipStream_t);
template hipError_t launch_col_lm<HDC_T, HDC_LOGM, false>(const ColParams<HDC_T>&, int, int, dim3, hipStream_t);
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
