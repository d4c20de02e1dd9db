// Real hybrid dealiasing via conjugate symmetries (Sec. 3) -- the hybridCS variant.
//
// For real input only the residues r = 0 .. floor(q/2) are needed
// (eq. (real-accumulation)):
//   f = (1/qm) (h_0 + 2 sum_{r=1}^{ceil(q/2)-1} Re h_r + h_{q/2}),
//   r = 0        transform of the real sum_t f_{tm+s}; its contribution is real (Sec. 3.1.1);
//   0 < r < q/2  complex residue transform of real data (Sec. 3.1.2);
//   r = q/2      (q even) only the even spectral indices are formed, from the folded
//                data sum_t (-1)^t (f_{tm+b} + i f_{tm+e+b}) and a length-m/2 FFT;
//                the inverse gives h_{q/2} through 2 Re w_b, 2 Im w_b (eqs. (forwardq2),
//                (wb), (accumulateq2)).
// Products are elementwise per residue.
//
// k_line_cs    one whole 1D convolution per workgroup (LDS slots per residue).
// k_col_cs_fwd the first axis of a 2D/3D problem: real columns -> retained
//              residue lines (r = 0: l <= m/2; 0 < r < q/2: all m; q/2: m/2 lines).
// k_col_cs_inv the inverse with real accumulation of the residue contributions.
// The remaining axes are complex sub-convolutions (Sec. 5) run by the complex
// column kernel and the plain line kernel.
#include <type_traits>

#include "hdc_kernels.hpp"

namespace hdc {

// real TwoSum accumulator
template <typename T>
struct RAcc {
  T s, c;
  __device__ __forceinline__ void zero() {
    s = (T)0;
    c = (T)0;
  }
  __device__ __forceinline__ void add(T x) { two_sum_add(s, c, x); }
  __device__ __forceinline__ T get() const { return s + c; }
};

// first retained line of residue r in the compact layout
__device__ __forceinline__ int cs_rowbase(int r, int m) { return r == 0 ? 0 : (m / 2 + 1) + (r - 1) * m; }

// ============================================================================ 1D
// MIX: residues 0 and q/2 through implicit packing instead (the combination of
// both variants that the discussion of Sec. 6 proposes): the real sums
// y_s = sum_t x_{tm+s} and y'_s = sum_t (-1)^t x_{tm+s} are packed into
// y~_j = y_{2j} + i y_{2j+1} (eq. (complexPacking)), transformed at length m/2
// (residue q/2 after the twist zeta_m^j), multiplied by the RCM operator of
// length m/2 (eq. (RCM); for q/2 with the frequency l moved to l + 1/2: partner
// m/2 - 1 - l, factor 1 + zeta_m^{2l+1}), inverted and unpacked.  The middle
// residues are unchanged, and every residue is computed on its own.
template <typename T, int LOGM, int PMAX, bool MIX = false>
__global__ __launch_bounds__(line_waves * 64) __attribute__((amdgpu_waves_per_eu(2))) void k_line_cs(
    CsParams<T> P) {
  constexpr int M = 1 << LOGM;
  constexpr int LOGR = line_logr(LOGM);
  constexpr int R = 1 << LOGR;
  constexpr int TS = M / R;
  constexpr int NTHR = line_waves * 64;
  constexpr int NTEAMS = NTHR / TS;
  constexpr int LOGE = LOGM > 0 ? LOGM - 1 : 0;
  constexpr int LOGRE = LOGR > 0 ? LOGR - 1 : 0;
  constexpr int RE = 1 << LOGRE;
  constexpr int E = M / 2;
  extern __shared__ char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  const int team = tid / TS;
  const int j = tid - team * TS;
  const int b = blockIdx.y;
  const int q = P.q, p = P.p, nres = P.nres, N = P.N;
  const int SL = padded_len(M);
  const bool qeven = (q % 2) == 0;
  auto slot = [&](int arr, int r) -> cx<T>* { return lds + (arr * nres + r) * SL; };

  // ---------------------------------------------------------------- forward
  {
    const int nchunk = NTEAMS >= 2 ? NTEAMS / 2 : 1;
    for (int u = team; u < 2 * nchunk; u += NTEAMS) {
      const int arr = u & 1;
      const int chunk = u >> 1;
      if (chunk >= nres) continue;
      const bool gs = arr && P.g_short;  // a shorter kernel g (read forwards)
      const T* base = (arr ? P.g : P.f) + (long long)b * (gs ? P.g_batch : P.in_batch);
      const int rev = arr ? P.rev_g : P.rev_f;
      const int La = gs ? P.gL0 : P.L;
      const int pa = gs ? min(p, (La + M - 1) / M) : p;  // blocks holding data (fewer for a shorter kernel)
      auto ld = [&](int pos) -> T {
        if (pos >= La) return (T)0;
        return base[rev ? La - 1 - pos : pos];
      };
      constexpr int PX = PMAX > 0 ? PMAX : 1;
      T x[PX][R];
      if constexpr (PMAX > 0) {
#pragma unroll
        for (int t = 0; t < PMAX; ++t)
#pragma unroll
          for (int i = 0; i < R; ++i) x[t][i] = (t < pa) ? ld(t * M + j + i * TS) : (T)0;
      }
      auto xt = [&](int t, int i) -> T {
        if constexpr (PMAX > 0) return x[t][i];
        else return ld(t * M + j + i * TS);
      };
      for (int r = chunk; r < nres; r += nchunk) {
        cx<T>* sl = slot(arr, r);
        if (MIX && (r == 0 || (qeven && 2 * r == q))) {
          // packed real sum of the blocks (signs (-1)^t for q/2), length-m/2 transform
          const bool half = r != 0;
          cx<T> v[RE];
#pragma unroll
          for (int i = 0; i < RE; ++i) {
            const int jj = j + i * TS;
            T a0 = (T)0, a1 = (T)0;
            for (int t = 0; t < pa; ++t) {
              const T sg = (half && (t & 1)) ? (T)-1 : (T)1;
              a0 += sg * ld(t * M + 2 * jj);
              a1 += sg * ld(t * M + 2 * jj + 1);
            }
            v[i] = mk(a0, a1);
            if (half) v[i] = cmul(v[i], tw_get(P.twN, jj * q));  // zeta_m^{jj} = zeta_N^{jj q}
          }
          team_fft<T, LOGE, LOGRE, +1, 1, WaveSync>(v, j, sl, root_of<T, LOGE>(P.rootpyr), WaveSync());
#pragma unroll
          for (int i = 0; i < RE; ++i) sl[pidx_strided<TS>(j, i)] = v[i];
        } else if (qeven && 2 * r == q) {
          // folded data, length-e transform of the even indices
          cx<T> v[RE];
#pragma unroll
          for (int i = 0; i < RE; ++i) {
            cx<T> acc = mk<T>(0, 0);
            for (int t = 0; t < (PMAX > 0 ? PMAX : p); ++t) {
              if (t >= pa) break;
              const T sg = (t & 1) ? (T)-1 : (T)1;
              acc = acc + mk<T>(sg * xt(t, i), sg * xt(t, i + RE));
            }
            const int bb = j + i * TS;
            v[i] = cmul(acc, tw_get(P.twN, bb * (q / 2)));  // zeta_{2m}^b = zeta_N^{b q/2}
          }
          team_fft<T, LOGE, LOGRE, +1, 1, WaveSync>(v, j, sl, root_of<T, LOGE>(P.rootpyr), WaveSync());
#pragma unroll
          for (int i = 0; i < RE; ++i) sl[pidx_strided<TS>(j, i)] = v[i];
        } else {
          cx<T> v[R];
#pragma unroll
          for (int i = 0; i < R; ++i) {
            cx<T> acc = mk<T>(xt(0, i), (T)0);
            for (int t = 1; t < (PMAX > 0 ? PMAX : p); ++t) {
              if (t >= pa) break;
              const cx<T> z = tw_get(P.twN, ((r * t) % q) * M);
              acc = acc + scale(z, xt(t, i));
            }
            const int s = j + i * TS;
            v[i] = r ? cmul(acc, tw_get(P.twN, r * s)) : acc;
          }
          team_fft<T, LOGM, LOGR, +1, 1, WaveSync>(v, j, sl, root_of<T, LOGM>(P.rootpyr), WaveSync());
#pragma unroll
          for (int i = 0; i < R; ++i) sl[pidx_strided<TS>(j, i)] = v[i];
        }
      }
    }
  }
  __syncthreads();
  // ---------------------------------------------------------------- product
  for (int idx = tid; idx < nres * M; idx += NTHR) {
    const int r = idx >> LOGM;
    const int l = idx & (M - 1);
    if (MIX && (r == 0 || (qeven && 2 * r == q))) {
      // RCM at length m/2 over unordered pairs (l, l'); one owner per pair
      if (l >= E) continue;
      const bool half = r != 0;
      const int lp = half ? E - 1 - l : (E - l) & (E - 1);
      if (lp < l) continue;
      cx<T>* pa = slot(0, r) + pidx(l);
      cx<T>* pc = slot(0, r) + pidx(lp);
      const cx<T> fa = *pa, fc = *pc;
      const cx<T> ga = slot(1, r)[pidx(l)], gc = slot(1, r)[pidx(lp)];
      const cx<T> z = tw_get(P.twN, (half ? 2 * l + 1 : 2 * l) * q);  // zeta_m^{2l (+1)}
      const cx<T> a1 = fa - conj(fc), a2 = ga - conj(gc);
      const cx<T> alpha = scale(cmul(cmul(a1, a2), mk<T>(z.x + (T)1, z.y)), (T)0.25);
      *pa = scale(cmul(fa, ga) - alpha, P.scale);
      if (lp != l) *pc = scale(cmul(fc, gc) - conj(alpha), P.scale);
      continue;
    }
    if (qeven && 2 * r == q && l >= E) continue;
    cx<T>* pf = slot(0, r) + pidx(l);
    const cx<T> gv = slot(1, r)[pidx(l)];
    *pf = scale(cmul(*pf, gv), P.scale);
  }
  __syncthreads();
  // ---------------------------------------------------------------- inverse per residue
  for (int r = team; r < nres; r += NTEAMS) {
    cx<T>* sl = slot(0, r);
    if (MIX && (r == 0 || (qeven && 2 * r == q))) {
      // inverse length-m/2 transform (and the twist back for q/2); unpacked in the accumulation
      cx<T> v[RE];
#pragma unroll
      for (int i = 0; i < RE; ++i) v[i] = sl[pidx_strided<TS>(j, i)];
      WaveSync()();
      team_fft<T, LOGE, LOGRE, -1, 1, WaveSync>(v, j, sl, root_of<T, LOGE>(P.rootpyr), WaveSync());
#pragma unroll
      for (int i = 0; i < RE; ++i)
        sl[pidx_strided<TS>(j, i)] = r ? cmulc(v[i], tw_get(P.twN, (j + i * TS) * q)) : v[i];
    } else if (qeven && 2 * r == q) {
      cx<T> v[RE];
#pragma unroll
      for (int i = 0; i < RE; ++i) v[i] = sl[pidx_strided<TS>(j, i)];
      WaveSync()();
      team_fft<T, LOGE, LOGRE, -1, 1, WaveSync>(v, j, sl, root_of<T, LOGE>(P.rootpyr), WaveSync());
#pragma unroll
      for (int i = 0; i < RE; ++i) sl[pidx_strided<TS>(j, i)] = cmulc(v[i], tw_get(P.twN, (j + i * TS) * (q / 2)));
    } else {
      cx<T> v[R];
#pragma unroll
      for (int i = 0; i < R; ++i) v[i] = sl[pidx_strided<TS>(j, i)];
      WaveSync()();
      team_fft<T, LOGM, LOGR, -1, 1, WaveSync>(v, j, sl, root_of<T, LOGM>(P.rootpyr), WaveSync());
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int s = j + i * TS;
        sl[pidx_strided<TS>(j, i)] = r ? cmulc(v[i], tw_get(P.twN, r * s)) : v[i];
      }
    }
  }
  __syncthreads();
  // ---------------------------------------------------------------- real accumulation
  {
    T* hb = P.h + (long long)b * P.in_batch;
    const int nmid = (q + 1) / 2;  // residues 1 .. ceil(q/2) - 1 are doubled
    for (int o = tid; o < P.L; o += NTHR) {
      const int t = o >> LOGM;
      const int s = o & (M - 1);
      RAcc<T> acc;
      acc.zero();
      if constexpr (MIX) {
        // h_0 = 2 x the unpacked inverse of the packed residue-0 product
        const cx<T> y0 = slot(0, 0)[pidx(s >> 1)];
        acc.add((T)2 * ((s & 1) ? y0.y : y0.x));
      } else {
        acc.add(slot(0, 0)[pidx(s)].x);
      }
      int rt = 0;
      for (int r = 1; r < nmid; ++r) {
        rt += t;
        while (rt >= q) rt -= q;
        cx<T> y = slot(0, r)[pidx(s)];
        if (rt) y = cmulc(y, tw_get(P.twN, rt * M));
        acc.add((T)2 * y.x);
      }
      if (qeven) {
        T val;
        if constexpr (MIX) {
          const cx<T> wv = slot(0, q / 2)[pidx(s >> 1)];
          val = (T)2 * ((s & 1) ? wv.y : wv.x);
        } else {
          const int a = s >= E;
          const cx<T> wv = slot(0, q / 2)[pidx(s - a * E)];
          val = (T)2 * (a ? wv.y : wv.x);
        }
        acc.add((t & 1) ? -val : val);
      }
      hb[P.rev_h ? P.L - 1 - o : o] = acc.get();
    }
  }
}

// ============================================================================ first axis (2D / 3D)
template <typename T, int LOGM, int PMAX, bool INV = false>
struct CsColCfg {
  static constexpr int M = 1 << LOGM;
  static constexpr int PE = PMAX > 0 ? PMAX : 4;
  // radix 16 (8 in FP64, and in the inverse over two or more blocks, whose accumulators
  // spill at 16 values; 4 in the FP64 inverse over four blocks); at most 512 threads so
  // that a lane may use 256 VGPRs
  static constexpr int LOGR1 =
      ((sizeof(T) == 8 || (INV && PE >= 2)) && col_logr(LOGM, PE) > 3) ? 3 : col_logr(LOGM, PE);
  static constexpr int LOGR = (LOGR1 > 2 && sizeof(T) == 8 && INV && PE >= 4) ? 2 : LOGR1;
  static constexpr int R = 1 << LOGR;
  static constexpr int TS = M / R;
  static constexpr int WB = (sizeof(T) == 4) ? ((M * PE <= 1024) ? 32 : 16) : ((M * PE <= 512) ? 16 : 8);
  static constexpr int W0 = (WB * TS >= 64) ? WB : 64 / TS;
  static constexpr int W = (W0 * TS > 512) ? (512 / TS > 0 ? 512 / TS : 1) : W0;
  static constexpr int NTHR = W * TS;
  static constexpr int LOGE = LOGM > 0 ? LOGM - 1 : 0;
  static constexpr int LOGRE = LOGR > 0 ? LOGR - 1 : 0;
  static constexpr int RE = 1 << LOGRE;
};

template <typename T, int LOGM, int PMAX>
__global__ __launch_bounds__((CsColCfg<T, LOGM, PMAX>::NTHR)) __attribute__((amdgpu_waves_per_eu(2)))
void k_col_cs_fwd(CsParams<T> P) {
  using C = CsColCfg<T, LOGM, PMAX>;
  constexpr int M = C::M, R = C::R, TS = C::TS, W = C::W, LOGR = C::LOGR, RE = C::RE;
  extern __shared__ char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  const int w = tid % W;
  const int j = tid / W;
  // real columns: W * sizeof(T) bytes of each row
  const int c = xcd_tile<tiles_per_line(W * (int)sizeof(T))>((int)blockIdx.x, (P.C + W - 1) / W) * W + w;
  const bool cval = c < P.C;
  const int b = blockIdx.y;
  const int arr = blockIdx.z;
  const int p = P.p, q = P.q, nres = P.nres;
  const bool qeven = (q % 2) == 0;
  const bool gs = arr && P.g_short;  // a shorter kernel g (read forwards), addressed with f's column index
  const T* base = (arr ? P.g : P.f) + (long long)b * (gs ? P.g_batch : P.in_batch);
  const int rev = arr ? P.rev_g : P.rev_f;
  auto ld = [&](int row) -> T {
    if (!cval || row >= P.L) return (T)0;
    if (gs) {
      if (P.lin1d) {
        const long long lin = (long long)row * P.in_row + c;
        return lin < P.gL0 ? base[lin] : (T)0;
      }
      const int x1 = c / P.fL2, x2 = c - (c / P.fL2) * P.fL2;
      if (row >= P.gL0 || x1 >= P.gL1 || x2 >= P.gL2) return (T)0;
      return base[((long long)row * P.gL1 + x1) * P.gL2 + x2];
    }
    if (P.lin1d) {
      // 1D problem viewed as rows of C: element (row, c) is x[row C + c], zero beyond the length
      const long long lin = (long long)row * P.in_row + c;
      if (lin >= P.lin1d) return (T)0;
      return base[rev ? P.lin1d - 1 - lin : lin];
    }
    return rev ? base[(long long)(P.L - 1 - row) * P.in_row + (P.C - 1 - c)] : base[(long long)row * P.in_row + c];
  };
  constexpr int PX = PMAX > 0 ? PMAX : 1;
  T x[PX][R];
  if constexpr (PMAX > 0) {
#pragma unroll
    for (int t = 0; t < PMAX; ++t)
#pragma unroll
      for (int i = 0; i < R; ++i) x[t][i] = (t < p) ? ld(t * M + j + i * TS) : (T)0;
  }
  auto xt = [&](int t, int i) -> T {
    if constexpr (PMAX > 0) return x[t][i];
    else return ld(t * M + j + i * TS);
  };
  cx<T>* out = P.ws + (long long)b * P.ws_batch + (long long)arr * P.ws_arr + c;
  const int r_hi = P.r_hi ? P.r_hi : nres;
  for (int r = P.r_lo; r < r_hi; ++r) {
    const int rb = cs_rowbase(r, M) - P.row0;
    if (qeven && 2 * r == q) {
      cx<T> v[RE];
#pragma unroll
      for (int i = 0; i < RE; ++i) {
        cx<T> acc = mk<T>(0, 0);
        for (int t = 0; t < (PMAX > 0 ? PMAX : p); ++t) {
          if (t >= p) break;
          const T sg = (t & 1) ? (T)-1 : (T)1;
          acc = acc + mk<T>(sg * xt(t, i), sg * xt(t, i + RE));
        }
        v[i] = cmul(acc, tw1(P.twN, (j + i * TS) * (q / 2)));
      }
      team_fft<T, C::LOGE, C::LOGRE, +1, W, BlockSync>(v, j, lds + w, root_of<T, C::LOGE>(P.rootpyr), BlockSync());
      if (cval) {
#pragma unroll
        for (int i = 0; i < RE; ++i) out[(long long)(rb + j + i * TS) * P.ws_row] = v[i];
      }
    } else {
      cx<T> v[R];
#pragma unroll
      for (int i = 0; i < R; ++i) {
        cx<T> acc = mk<T>(xt(0, i), (T)0);
        for (int t = 1; t < (PMAX > 0 ? PMAX : p); ++t) {
          if (t >= p) break;
          acc = acc + scale(tw1(P.twN, ((r * t) % q) * M), xt(t, i));
        }
        const int s = j + i * TS;
        v[i] = r ? cmul(acc, tw1(P.twN, r * s)) : acc;
      }
      team_fft<T, LOGM, LOGR, +1, W, BlockSync>(v, j, lds + w, root_of<T, LOGM>(P.rootpyr), BlockSync());
      if (cval) {
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const int l = j + i * TS;
          if (r == 0 && l > M / 2) continue;  // Hermitian half of the r = 0 residue
          out[(long long)(rb + l) * P.ws_row] = v[i];
        }
      }
    }
  }
}

template <typename T, int LOGM, int PMAX>
__global__ __launch_bounds__((CsColCfg<T, LOGM, PMAX, true>::NTHR)) __attribute__((amdgpu_waves_per_eu(2)))
void k_col_cs_inv(CsParams<T> P) {
  using C = CsColCfg<T, LOGM, PMAX, true>;
  constexpr int M = C::M, R = C::R, TS = C::TS, W = C::W, LOGR = C::LOGR, RE = C::RE;
  constexpr int E = M / 2;
  extern __shared__ char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  const int w = tid % W;
  const int j = tid / W;
  // real columns: W * sizeof(T) bytes of each row
  const int c = xcd_tile<tiles_per_line(W * (int)sizeof(T))>((int)blockIdx.x, (P.C + W - 1) / W) * W + w;
  const bool cval = c < P.C;
  const int b = blockIdx.y;
  const int p = P.p, q = P.q, nres = P.nres;
  const bool qeven = (q % 2) == 0;
  const int nmid = (q + 1) / 2;
  const cx<T>* in = P.ws + (long long)b * P.ws_batch + c;
  T* hb = P.h + (long long)b * P.in_batch;
  constexpr int PC = PMAX > 0 ? PMAX : 4;
  for (int t0 = 0; t0 < p; t0 += PC) {
    RAcc<T> acc[PC][R];
#pragma unroll
    for (int t = 0; t < PC; ++t)
#pragma unroll
      for (int i = 0; i < R; ++i) acc[t][i].zero();
    const int r_hi = P.r_hi ? P.r_hi : nres;
    for (int r = P.r_lo; r < r_hi; ++r) {
      const int rb = cs_rowbase(r, M) - P.row0;
      if (qeven && 2 * r == q) {
        cx<T> v[RE];
#pragma unroll
        for (int i = 0; i < RE; ++i) v[i] = cval ? in[(long long)(rb + j + i * TS) * P.ws_row] : mk<T>(0, 0);
        team_fft<T, C::LOGE, C::LOGRE, -1, W, BlockSync>(v, j, lds + w, root_of<T, C::LOGE>(P.rootpyr),
                                                          BlockSync());
#pragma unroll
        for (int i = 0; i < RE; ++i) {
          const cx<T> wv = cmulc(v[i], tw1(P.twN, (j + i * TS) * (q / 2)));
#pragma unroll
          for (int tt = 0; tt < PC; ++tt) {
            if (t0 + tt >= p) continue;
            const T sg = ((t0 + tt) & 1) ? (T)-2 : (T)2;
            acc[tt][i].add(sg * wv.x);       // s = b
            acc[tt][i + RE].add(sg * wv.y);  // s = e + b
          }
        }
      } else {
        cx<T> v[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
          // Hermitian extension of residue 0 (branch-free; masked lanes read line 0)
          const int l = j + i * TS;
          const bool ext = r == 0 && l > E;
          const cx<T> y = in[cval ? (long long)(ext ? M - l : rb + l) * P.ws_row : 0];
          v[i] = cval ? (ext ? conj(y) : y) : mk<T>(0, 0);
        }
        team_fft<T, LOGM, LOGR, -1, W, BlockSync>(v, j, lds + w, root_of<T, LOGM>(P.rootpyr), BlockSync());
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const int s = j + i * TS;
          if (r == 0) {
#pragma unroll
            for (int tt = 0; tt < PC; ++tt)
              if (t0 + tt < p) acc[tt][i].add(v[i].x);
          } else if (r < nmid) {
            const cx<T> y = cmulc(v[i], tw1(P.twN, r * s));
#pragma unroll
            for (int tt = 0; tt < PC; ++tt) {
              const int t = t0 + tt;
              if (t >= p) continue;
              const cx<T> z = t ? cmulc(y, tw1(P.twN, ((r * t) % q) * M)) : y;
              acc[tt][i].add((T)2 * z.x);
            }
          }
        }
      }
    }
    if (!cval) continue;
#pragma unroll
    for (int tt = 0; tt < PC; ++tt)
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int row = (t0 + tt) * M + j + i * TS;
        if (t0 + tt >= p || row >= P.L) continue;
        const T val = acc[tt][i].get();
        if (P.lin1d) {
          const long long lin = (long long)row * P.in_row + c;
          if (lin < P.lin1d) hb[P.rev_h ? P.lin1d - 1 - lin : lin] = val;
        } else {
          T* o = hb + (P.rev_h ? (long long)(P.L - 1 - row) * P.in_row + (P.C - 1 - c) : (long long)row * P.in_row + c);
          *o = P.accum ? *o + val : val;  // accum: residues 0 and q/2 are already in h
        }
      }
  }
}


// ============================================================================ 1D multi-pass, column pairs
// The multi-pass 1D form of the conjugate-symmetry variant keeps one residue
// (r = 0) of a real length-q transform over the rows of the 1D data viewed as
// rows of C reals (lin1d).  Two adjacent real columns a, b travel as one
// complex column z = x_a + i x_b: with Z = FFT(z),
//   X_a[l] = (Z[l] + conj Z[q - l]) / 2,   X_b[l] = (Z[l] - conj Z[q - l]) / (2 i),
// so one complex FFT serves two columns and loads and stores are twice as
// wide.  The inverse rebuilds Z = X_a + i X_b from the retained half with the
// Hermitian extension X[q - l] = conj X[l], and one complex inverse FFT yields
// both real columns (real and imaginary parts).  The imaginary parts of X[0]
// and X[q/2] are dropped: they add nothing to the real part of a single
// column's inverse and would leak into the partner column here.
template <typename T, int LOGM>
struct CsPairCfg {
  static constexpr int M = 1 << LOGM;
  static constexpr int LOGR = LOGM < (sizeof(T) == 4 ? 4 : 3) ? LOGM : (sizeof(T) == 4 ? 4 : 3);
  static constexpr int R = 1 << LOGR;
  static constexpr int TS = M / R;
  static constexpr int W0 = (8 * TS <= 512) ? 8 : (512 / TS > 0 ? 512 / TS : 1);  // column pairs per workgroup
  static constexpr int W = (W0 * TS >= 64) ? W0 : 64 / TS;
  static constexpr int NTHR = W * TS;
  static constexpr int WPE = NTHR >= 512 ? 4 : 2;
};

template <typename T>
struct alignas(4 * sizeof(T)) cx2 {
  cx<T> a, b;
};

template <typename T, int LOGM>
__global__ __launch_bounds__((CsPairCfg<T, LOGM>::NTHR))
__attribute__((amdgpu_waves_per_eu(CsPairCfg<T, LOGM>::WPE))) void k_cs_pair_fwd(CsParams<T> P) {
  using C = CsPairCfg<T, LOGM>;
  constexpr int M = C::M, R = C::R, TS = C::TS, W = C::W, LOGR = C::LOGR;
  extern __shared__ char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  const int w = tid % W;
  const int j = tid / W;
  const long long cp =
      (long long)xcd_tile<tiles_per_line(W * 2 * (int)sizeof(T))>((int)blockIdx.x, (P.C / 2 + W - 1) / W) * W + w;
  const bool pval = cp < P.C / 2;
  const int b = blockIdx.y;
  const int arr = blockIdx.z;
  const bool gs = arr && P.g_short;  // a shorter kernel g (read forwards)
  const T* base = (arr ? P.g : P.f) + (long long)b * (gs ? P.g_batch : P.in_batch);
  const int rev = arr ? P.rev_g : P.rev_f;
  const long long n = gs ? P.gL0 : P.lin1d;
  // packed loads when read forwards from an even length at an aligned address (uniform)
  const bool fast = !rev && !(n & 1) && !(reinterpret_cast<uintptr_t>(base) & (2 * sizeof(T) - 1));
  cx<T> v[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int row = j + i * TS;
    const long long lin = (long long)row * P.in_row + 2 * cp;
    const bool in0 = pval && row < P.L && lin < n;
    if (fast) {
      // n even and lin even: column b is present whenever column a is; masked lanes read element 0
      const cx<T> t = *reinterpret_cast<const cx<T>*>(base + (in0 ? lin : 0));
      v[i] = in0 ? t : mk<T>(0, 0);
    } else {
      const bool in1 = pval && row < P.L && lin + 1 < n;
      const T xa = in0 ? base[rev ? n - 1 - lin : lin] : (T)0;
      const T xb = in1 ? base[rev ? n - 2 - lin : lin + 1] : (T)0;
      v[i] = mk<T>(xa, xb);
    }
  }
  team_fft<T, LOGM, LOGR, +1, W, BlockSync>(v, j, lds + w, root_of<T, LOGM>(P.rootpyr), BlockSync());
  // Z in natural order to LDS; each retained index l <= q/2 pairs with q - l
#pragma unroll
  for (int i = 0; i < R; ++i) lds[pidx(j + i * TS) * W + w] = v[i];
  __syncthreads();
  if (!pval) return;
  cx<T>* out = P.ws + (long long)b * P.ws_batch + (long long)arr * P.ws_arr + 2 * cp;
  const T half = (T)0.5;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int l = j + i * TS;
    if (l > M / 2) continue;
    const cx<T> zl = lds[pidx(l) * W + w];
    const cx<T> zm = lds[pidx((M - l) & (M - 1)) * W + w];
    cx2<T> o;
    o.a = mk<T>(half * (zl.x + zm.x), half * (zl.y - zm.y));
    o.b = mk<T>(half * (zl.y + zm.y), half * (zm.x - zl.x));
    *reinterpret_cast<cx2<T>*>(out + (long long)l * P.ws_row) = o;
  }
}

template <typename T, int LOGM>
__global__ __launch_bounds__((CsPairCfg<T, LOGM>::NTHR))
__attribute__((amdgpu_waves_per_eu(CsPairCfg<T, LOGM>::WPE))) void k_cs_pair_inv(CsParams<T> P) {
  using C = CsPairCfg<T, LOGM>;
  constexpr int M = C::M, R = C::R, TS = C::TS, W = C::W, LOGR = C::LOGR;
  constexpr int E = M / 2;
  extern __shared__ char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  const int w = tid % W;
  const int j = tid / W;
  const long long cp =
      (long long)xcd_tile<tiles_per_line(W * 2 * (int)sizeof(T))>((int)blockIdx.x, (P.C / 2 + W - 1) / W) * W + w;
  const bool pval = cp < P.C / 2;
  const int b = blockIdx.y;
  // masked lanes read pair 0 of row 0
  const cx<T>* in = P.ws + (long long)b * P.ws_batch + 2 * (pval ? cp : 0);
  cx<T> v[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int l = j + i * TS;
    const bool ext = l > E;
    const int row = ext ? M - l : l;
    cx2<T> ab = *reinterpret_cast<const cx2<T>*>(in + (long long)(pval ? row : 0) * P.ws_row);
    if (row == 0 || row == E) {
      ab.a.y = (T)0;
      ab.b.y = (T)0;
    }
    // Z = X_a + i X_b, or conj X_a + i conj X_b on the extended half
    const T sy = ext ? (T)-1 : (T)1;
    const cx<T> z = mk<T>(ab.a.x - sy * ab.b.y, sy * ab.a.y + ab.b.x);
    v[i] = pval ? z : mk<T>(0, 0);
  }
  team_fft<T, LOGM, LOGR, -1, W, BlockSync>(v, j, lds + w, root_of<T, LOGM>(P.rootpyr), BlockSync());
  if (!pval) return;
  T* hb = P.h + (long long)b * P.in_batch;
  const long long n = P.lin1d;
  const bool fast = !P.rev_h && !(n & 1) && !(reinterpret_cast<uintptr_t>(hb) & (2 * sizeof(T) - 1));
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int row = j + i * TS;
    if (row >= P.L) continue;
    const long long lin = (long long)row * P.in_row + 2 * cp;
    if (fast) {
      if (lin < n) *reinterpret_cast<cx<T>*>(hb + lin) = v[i];
    } else {
      if (lin < n) hb[P.rev_h ? n - 1 - lin : lin] = v[i].x;
      if (lin + 1 < n) hb[P.rev_h ? n - 2 - lin : lin + 1] = v[i].y;
    }
  }
}

// ---------------------------------------------------------------------------- launchers
template <typename T, int LOGM, int PMAX, int WHICH>
static hipError_t launch_cs_t(const CsParams<T>& P, dim3 grid, hipStream_t s) {
  if constexpr (WHICH == 0 || WHICH == 5) {
    const size_t lds = (size_t)2 * P.nres * padded_len(1 << LOGM) * sizeof(cx<T>);
    auto fn = k_line_cs<T, LOGM, PMAX, WHICH == 5>;
    if (lds > 65536) {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(fn, grid, dim3(line_waves * 64), lds, s, P);
  } else if constexpr (WHICH == 3 || WHICH == 4) {
    using C = CsPairCfg<T, LOGM>;
    const size_t lds = (size_t)padded_len(C::M) * C::W * sizeof(cx<T>);
    grid.x = (unsigned)((P.C / 2 + C::W - 1) / C::W);
    auto fn = (WHICH == 3) ? k_cs_pair_fwd<T, LOGM> : k_cs_pair_inv<T, LOGM>;
    if (lds > 65536) {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(fn, grid, dim3(C::NTHR), lds, s, P);
  } else {
    using C = CsColCfg<T, LOGM, PMAX, WHICH == 2>;
    const size_t lds = (C::M > C::R) ? (size_t)padded_len(C::M) * C::W * sizeof(cx<T>) : 0;
    grid.x = (P.C + C::W - 1) / C::W;
    auto fn = (WHICH == 1) ? k_col_cs_fwd<T, LOGM, PMAX> : k_col_cs_inv<T, LOGM, PMAX>;
    if (lds > 65536) {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(fn, grid, dim3(C::NTHR), lds, s, P);
  }
  return hipGetLastError();
}

template <typename T, int LOGM>
hipError_t launch_cs_lm(const CsParams<T>& P, int which, int pcap, dim3 grid, hipStream_t s) {
#define HDC_CS_P(W)                                             \
  switch (pcap) {                                               \
    case 0: return launch_cs_t<T, LOGM, 0, W>(P, grid, s);      \
    case 1: return launch_cs_t<T, LOGM, 1, W>(P, grid, s);      \
    case 2: return launch_cs_t<T, LOGM, 2, W>(P, grid, s);      \
    case 4: return launch_cs_t<T, LOGM, 4, W>(P, grid, s);      \
    default: return hipErrorInvalidValue;                       \
  }
  if (which == 0) {
    HDC_CS_P(0)
  } else if (which == 5) {
    if constexpr (LOGM >= 1) {
      HDC_CS_P(5)
    }
    return hipErrorInvalidValue;
  } else if (which == 1) {
    if constexpr (LOGM <= kColMaxLogM) {
      HDC_CS_P(1)
    }
    return hipErrorInvalidValue;
  } else if (which == 2) {
    if constexpr (LOGM <= kColMaxLogM) {
      HDC_CS_P(2)
    }
    return hipErrorInvalidValue;
  } else if (which == 3 || which == 4) {
    // column pairs of the multi-pass 1D form (one residue, no blocks)
    if constexpr (LOGM <= kCsPairMaxLogM) {
      if (which == 3) return launch_cs_t<T, LOGM, 1, 3>(P, grid, s);
      return launch_cs_t<T, LOGM, 1, 4>(P, grid, s);
    }
    return hipErrorInvalidValue;
  }
  return hipErrorInvalidValue;
#undef HDC_CS_P
}

#if defined(HDC_T) && defined(HDC_LOGM)
template hipError_t launch_cs_lm<HDC_T, HDC_LOGM>(const CsParams<HDC_T>&, int, int, dim3, hipStream_t);
#endif

}  // namespace hdc
