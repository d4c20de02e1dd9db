// Device primitives for the hybrid-dealiased real convolution on gfx950.
//
// Conventions (Murasko & Bowman, Sec. 2): zeta_N = exp(+2 pi i / N); the
// forward DFT is X_k = sum_j zeta_N^{kj} x_j, the inverse carries zeta^{-}.
// DIR = +1 selects the forward sign, DIR = -1 the inverse (unnormalised).
//
// Complex values are stored interleaved (re, im).  Twiddle factors come from
// tables the host generates in float64 from exact integer angle reductions and
// rounds once to the working precision; no recurrences are used on device.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hdc {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T a, T b) {
  cx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return mk(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return mk(fma(a.x, b.x, a.y * b.y), fma(a.y, b.x, -a.x * b.y));
}
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return mk(a.x, -a.y); }
template <typename T>
__device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return mk(a.x * s, a.y * s); }
// multiply by i^(+1) or i^(-1)
template <int DIR, typename T>
__device__ __forceinline__ cx<T> mul_i(cx<T> a) {
  if constexpr (DIR > 0) return mk(-a.y, a.x);
  else return mk(a.y, -a.x);
}
// twiddle multiply with sign: DIR > 0 -> a * w, DIR < 0 -> a * conj(w)
template <int DIR, typename T>
__device__ __forceinline__ cx<T> twmul(cx<T> a, cx<T> w) {
  if constexpr (DIR > 0) return cmul(a, w);
  else return cmulc(a, w);
}

// ---------------------------------------------------------------------------
// compile-time cos/sin of 2 pi k / n (Taylor series after octant reduction);
// only used for the constant twiddles inside the in-register radix-2^k DFTs.
// ---------------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double taylor_sin(double x) {
  double t = x, s = x;
  for (int n = 1; n < 14; ++n) {
    t *= -x * x / ((2.0 * n) * (2.0 * n + 1.0));
    s += t;
  }
  return s;
}
constexpr double taylor_cos(double x) {
  double t = 1.0, s = 1.0;
  for (int n = 1; n < 14; ++n) {
    t *= -x * x / ((2.0 * n - 1.0) * (2.0 * n));
    s += t;
  }
  return s;
}
// (cos, sin) of 2 pi k / n for 0 <= k < n, exact symmetry reductions
constexpr double ccos_frac(int k, int n) {
  k %= n;
  if (k < 0) k += n;
  // reduce to the first quadrant with exact integer arithmetic
  if (4 * k > 3 * n) return ccos_frac(n - k, n);          // cos(2pi - a) = cos a
  if (2 * k > n) return -ccos_frac(k - n / 2, n);         // only used for even n here
  if (4 * k > n) return -taylor_sin(2.0 * kPi * (4 * k - n) / (4.0 * n));  // cos(pi/2 + a) = -sin a
  return taylor_cos(2.0 * kPi * k / n);
}
constexpr double csin_frac(int k, int n) { return ccos_frac(k - n / 4, n); }  // sin a = cos(a - pi/2), n % 4 == 0

// multiply by zeta_N^{DIR*K}, with exact forms at multiples of N/8
template <int N, int K, int DIR, typename T>
__device__ __forceinline__ cx<T> mulc(cx<T> a) {
  constexpr int k = ((K % N) + N) % N;
  if constexpr (k == 0) {
    return a;
  } else if constexpr (4 * k == N) {
    return mul_i<DIR>(a);
  } else if constexpr (2 * k == N) {
    return mk(-a.x, -a.y);
  } else if constexpr (4 * k == 3 * N) {
    return mul_i<-DIR>(a);
  } else if constexpr (8 * k == N || 8 * k == 3 * N || 8 * k == 5 * N || 8 * k == 7 * N) {
    constexpr T h = (T)0.70710678118654752440084436210484903928;
    // zeta_8^j = ((+-1) + (+-i)) / sqrt 2
    constexpr int j = 8 * k / N;
    constexpr T cr = (j == 1 || j == 7) ? h : -h;
    constexpr T ci0 = (j == 1 || j == 3) ? h : -h;
    constexpr T ci = DIR > 0 ? ci0 : -ci0;
    return mk(cr * a.x - ci * a.y, cr * a.y + ci * a.x);
  } else {
    constexpr T cr = (T)ccos_frac(k, N);
    constexpr T ci0 = (T)csin_frac(k, N);
    constexpr T ci = DIR > 0 ? ci0 : -ci0;
    return mk(fma(cr, a.x, -ci * a.y), fma(cr, a.y, ci * a.x));
  }
}

// In-register DFT of length N (power of two <= 16) on a[0], a[S], ..., a[(N-1)S]
// by recursive decimation in time; natural order in and out.
template <int N, int DIR, typename T, int K>
struct RegCombine {
  template <int S>
  __device__ __forceinline__ static void run(cx<T>* a, const cx<T>* e, const cx<T>* o) {
    cx<T> t = mulc<N, K, DIR>(o[K]);
    a[K * S] = e[K] + t;
    a[(K + N / 2) * S] = e[K] - t;
    RegCombine<N, DIR, T, K + 1>::template run<S>(a, e, o);
  }
};
template <int N, int DIR, typename T>
struct RegCombine<N, DIR, T, N / 2> {
  template <int S>
  __device__ __forceinline__ static void run(cx<T>*, const cx<T>*, const cx<T>*) {}
};

template <int N, int DIR, typename T, int S>
__device__ __forceinline__ void reg_dft(cx<T>* a);

template <int N, int DIR, typename T, int S>
struct RegDFTS {
  __device__ __forceinline__ static void run(cx<T>* a) {
    cx<T> e[N / 2], o[N / 2];
#pragma unroll
    for (int n = 0; n < N / 2; ++n) {
      e[n] = a[(2 * n) * S];
      o[n] = a[(2 * n + 1) * S];
    }
    RegDFTS<N / 2, DIR, T, 1>::run(e);
    RegDFTS<N / 2, DIR, T, 1>::run(o);
    RegCombine<N, DIR, T, 0>::template run<S>(a, e, o);
  }
};
template <int DIR, typename T, int S>
struct RegDFTS<1, DIR, T, S> {
  __device__ __forceinline__ static void run(cx<T>*) {}
};
template <int DIR, typename T, int S>
struct RegDFTS<2, DIR, T, S> {
  __device__ __forceinline__ static void run(cx<T>* a) {
    cx<T> u = a[0], v = a[S];
    a[0] = u + v;
    a[S] = u - v;
  }
};
template <int DIR, typename T, int S>
struct RegDFTS<4, DIR, T, S> {
  __device__ __forceinline__ static void run(cx<T>* a) {
    cx<T> a0 = a[0], a1 = a[S], a2 = a[2 * S], a3 = a[3 * S];
    cx<T> s02 = a0 + a2, d02 = a0 - a2, s13 = a1 + a3, d13 = mul_i<DIR>(a1 - a3);
    a[0] = s02 + s13;
    a[2 * S] = s02 - s13;
    a[S] = d02 + d13;
    a[3 * S] = d02 - d13;
  }
};

template <int N, int DIR, typename T, int S>
__device__ __forceinline__ void reg_dft(cx<T>* a) {
  RegDFTS<N, DIR, T, S>::run(a);
}

// ---------------------------------------------------------------------------
// twiddle tables
// ---------------------------------------------------------------------------
template <int V>
struct IntTag {
  static constexpr int value = V;
};

// zeta_N^k for 0 <= k < N from two tables: lo[j] = zeta_N^j (j < 2^lobits) and
// hi[i] = zeta_N^{i 2^lobits}; hi[0] = 1 exactly, so small N needs one table.
template <typename T>
struct Tw2 {
  const cx<T>* lo;
  const cx<T>* hi;
  int lobits;
  int N;
  int single;  // lo covers every k < N (hi is the trivial table {1})
};

// Branch-free: a single-level table has hi = {1} and k >> lobits = 0, so both
// loads are always valid; keeping the lookup free of branches lets unrolled
// loops issue all their table loads before the first use.
template <typename T>
__device__ __forceinline__ cx<T> tw_get(const Tw2<T>& t, int k) {
  const cx<T> a = t.lo[k & ((1 << t.lobits) - 1)];
  const cx<T> b = t.hi[k >> t.lobits];
  const cx<T> ab = cmul(a, b);
  return t.single ? a : ab;
}
// Single-level lookup (every k < N is an entry of lo).  The residue tables of
// the strided axes are built single-level (up to 2^22 points), so the column
// kernels read each twiddle with one load and no product.
template <typename T>
__device__ __forceinline__ cx<T> tw1(const Tw2<T>& t, int k) {
  return t.lo[k];
}
// zeta_N^{k} for any integer k (reduced mod N)
template <typename T>
__device__ __forceinline__ cx<T> tw_mod(const Tw2<T>& t, long long k) {
  long long r = k % (long long)t.N;
  if (r < 0) r += t.N;
  return tw_get(t, (int)r);
}

// The same lookup with the table's form fixed at compile time: a single-level
// table returns its entry, a two-level one the product of its two entries.
// tw_dispatch branches once on the form (uniform across a launch) and runs f
// with the specialised lookup, so a loop of lookups into a single-level table
// issues neither the hi[0] load nor the product that tw_get forms and drops.
// Worth it where the branch does not raise the kernel's register count (the
// multi-D line kernels); elsewhere the kernels keep tw_get (TwSel).
template <typename T, bool SINGLE>
struct TwLook {
  static constexpr bool single = SINGLE;
  const cx<T>* lo;
  const cx<T>* hi;
  int lobits;
  __device__ __forceinline__ cx<T> operator()(int k) const {
    if constexpr (SINGLE) return lo[k];
    else return cmul(lo[k & ((1 << lobits) - 1)], hi[k >> lobits]);
  }
};
template <typename T>
struct TwSel {
  const Tw2<T>& t;
  __device__ __forceinline__ cx<T> operator()(int k) const { return tw_get(t, k); }
};
template <typename T, typename F>
__device__ __forceinline__ void tw_dispatch(const Tw2<T>& t, F&& f) {
  if (t.single) f(TwLook<T, true>{t.lo, t.hi, t.lobits});
  else f(TwLook<T, false>{t.lo, t.hi, t.lobits});
}

// Residue twiddle v[i] *= zeta_N^{DIR r s}, s = j + i TS (eqs. (forwardr) and
// (accumulator)), for a uniform residue r: one branch on r around the loop and
// the table loads issued together.  FORM: 0 = either table form (tw_get),
// 1 = a table known to be single-level (tw1), 2 = one branch on the form.
template <typename T, int R, int TS, int DIR, bool BATCH = true, int FORM = 0>
__device__ __forceinline__ void residue_twiddle(cx<T> (&v)[R], int j, int r, const Tw2<T>& tw) {
  if (r == 0) return;
  constexpr int GM = !BATCH ? 1 : (sizeof(T) == 4 ? 8 : 4);
  constexpr int G = R < GM ? R : GM;  // loads issued per batch
  // S: 0 = either form (both loads, product, select), 1 = single-level, 2 = two-level
  auto body = [&](auto stag) {
    constexpr int S = decltype(stag)::value;
    const int mask = (1 << tw.lobits) - 1;
#pragma unroll
    for (int i0 = 0; i0 < R; i0 += G) {
      cx<T> a[G], b[G];
#pragma unroll
      for (int i = 0; i < G; ++i) {
        const int k = r * (j + (i0 + i) * TS);
        if constexpr (S == 1) {
          a[i] = tw.lo[k];
        } else {
          a[i] = tw.lo[k & mask];
          b[i] = tw.hi[k >> tw.lobits];
        }
      }
      if constexpr (G > 1) __builtin_amdgcn_sched_barrier(0);  // issue the batch before its first use
#pragma unroll
      for (int i = 0; i < G; ++i) {
        cx<T> w;
        if constexpr (S == 1) {
          w = a[i];
        } else if constexpr (S == 2) {
          w = cmul(a[i], b[i]);
        } else {
          const cx<T> ab = cmul(a[i], b[i]);
          w = tw.single ? a[i] : ab;
        }
        v[i0 + i] = DIR > 0 ? cmul(v[i0 + i], w) : cmulc(v[i0 + i], w);
      }
    }
  };
  if constexpr (FORM == 2) {
    if (tw.single) body(IntTag<1>{});
    else body(IntTag<2>{});
  } else {
    body(IntTag<FORM>{});
  }
}

// value of lane `lane` of the wavefront, in every lane (uniform result)
__device__ __forceinline__ float lane_bcast(float x, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}
__device__ __forceinline__ double lane_bcast(double x, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}

// Four-step twiddle of one row of the multi-pass 1D form (Sec. 4, the complex
// inner loop): element c = j + i TS of row k is multiplied by zeta_Nf^{+-k c}.
// zeta^{k c} = zeta^{k j} zeta^{k TS i}: the first factor is one lookup per lane,
// the second one lookup per i shared by the wavefront (lane i computes it and
// every lane reads it), so each element costs two complex products.
template <typename T, int R, int TS, int DIR>
__device__ __forceinline__ void four_step_row(cx<T> (&v)[R], int j, int k, const Tw2<T>& tw) {
  const cx<T> a = tw_get(tw, k * j);
  if constexpr (TS % 64 == 0 && R <= 64) {  // a team is whole wavefronts: k is wave-uniform
    const int lane = __lane_id();
    const cx<T> bl = tw_get(tw, k * TS * (lane < R ? lane : 0));
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const cx<T> b = mk<T>(lane_bcast(bl.x, i), lane_bcast(bl.y, i));
      const cx<T> t = cmul(a, b);
      v[i] = DIR > 0 ? cmul(v[i], t) : cmulc(v[i], t);
    }
  } else {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const cx<T> t = cmul(a, tw_get(tw, k * TS * i));
      v[i] = DIR > 0 ? cmul(v[i], t) : cmulc(v[i], t);
    }
  }
}

// ---------------------------------------------------------------------------
// LDS padding: one spare slot every 16 elements breaks power-of-two strides
// ---------------------------------------------------------------------------
__device__ __forceinline__ int pidx(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int padded_len(int n) { return n + (n >> 4) + 1; }

// synchronisation for a team that lives inside one wavefront
struct WaveSync {
  __device__ __forceinline__ void operator()() const {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
};
// synchronisation for a team spread over a workgroup
struct BlockSync {
  __device__ __forceinline__ void operator()() const { __syncthreads(); }
};

constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n / 2); }

// v[ip NB] *= zeta_{NN}^{DIR ip (k0 + CC)} for 1 <= ip < RHO, given w[ip] = zeta_{NN}^{ip k0}:
// the factor zeta_{NN}^{ip CC} is a compile-time constant (exact at multiples of NN/8)
template <typename T, int NN, int RHO, int NB, int DIR, int CC, int IP>
struct TwShared {
  __device__ __forceinline__ static void apply(cx<T>* v, const cx<T>* w) {
    if constexpr (IP < RHO) {
      const cx<T> t = (CC == 0) ? w[IP] : mulc<NN, IP * CC, +1>(w[IP]);
      v[IP * NB] = twmul<DIR>(v[IP * NB], t);
      TwShared<T, NN, RHO, NB, DIR, CC, IP + 1>::apply(v, w);
    }
  }
};

// twiddles and the radix-RHO DFT of butterflies C .. NB-1 of one stage with shared twiddles
template <typename T, int NN, int RHO, int NB, int DIR, int TS, int NS, int C>
struct SharedStage {
  __device__ __forceinline__ static void run(cx<T>* v, const cx<T>* w) {
    if constexpr (C < NB) {
      TwShared<T, NN, RHO, NB, DIR, (C * TS) & (NS - 1), 1>::apply(v + C, w);
      reg_dft<RHO, DIR, T, NB>(v + C);
      SharedStage<T, NN, RHO, NB, DIR, TS, NS, C + 1>::run(v, w);
    }
  }
};

// ---------------------------------------------------------------------------
// Team FFT (Stockham autosort, radix <= 16 in registers, LDS between stages).
//
// A team of TS = N/R threads computes one length-N DFT.  Team thread j holds
// v[i] = x[j + i*TS] (i < R) on entry and v[i] = X[j + i*TS] on exit.  The
// exchange buffer holds N complex values at lds[pidx(idx)*ES].  Every stage of
// radix rho performs R/rho butterflies per thread; butterfly b = j + c*TS uses
// inputs x[b + i'*N/rho] (register c + i'*R/rho), applies zeta_{Ns rho}^{i' (b mod Ns)},
// a radix-rho DFT, and writes to (b / Ns) Ns rho + (b mod Ns) + i' Ns.  The last
// stage leaves its outputs in registers in natural order.
// root: the table zeta_N^k, k < N, of exactly this length (see root_of).
// ---------------------------------------------------------------------------
template <typename T, int LOGN, int LOGR, int DIR, int ES, typename Sync, int LOGNS = 0, int BATCH = 1>
struct TeamFFT {
  static constexpr int N = 1 << LOGN;
  static constexpr int R = 1 << LOGR;
  static constexpr int TS = N / R;
  static constexpr int LOGRHO_MAX = LOGR < 4 ? LOGR : 4;
  static constexpr int REM = LOGN - LOGNS;
  static constexpr int LOGRHO = REM < LOGRHO_MAX ? REM : LOGRHO_MAX;
  static constexpr int RHO = 1 << LOGRHO;
  static constexpr int NS = 1 << LOGNS;
  static constexpr bool LAST = (LOGNS + LOGRHO == LOGN);
  // pidx(base + ip*NS) = pidx(base) + ip*OFFW when the padding term does not depend on ip
  static constexpr bool WIMM = (NS % 16 == 0) || (NS * RHO <= 16) || (NS == 1 && 16 % RHO == 0);
  static constexpr int OFFW = (NS % 16 == 0) ? NS + NS / 16 : NS;
  static constexpr bool RIMM = (TS % 16 == 0);
  static constexpr int OFFR = TS + TS / 16;

  __device__ __forceinline__ static void run(cx<T> (&v)[R], int j, cx<T>* lds, const cx<T>* __restrict__ root,
                                             Sync sync) {
    if constexpr (REM <= 0) {
      return;
    } else {
      constexpr int NB = R / RHO;  // butterflies per thread
      // Stage twiddles zeta_{NS RHO}^{i' k}, k = (j + c TS) mod NS, shared across the lane's butterflies
      // (TS and NS are powers of two): NS <= TS gives every c the same k; NS > TS gives
      // k = j + (c TS mod NS), whose extra factor zeta_{NS RHO}^{i' (c TS mod NS)} is a compile-time
      // constant.  One table row of RHO - 1 loads per stage instead of one per butterfly.
      constexpr bool SHARED = (BATCH != 0) && (NS > 1) && (NB > 1);
      if constexpr (SHARED) {
        constexpr int sh = LOGN - (LOGNS + LOGRHO);
        const int step = (j & (NS - 1)) << sh;
        cx<T> ws[RHO];
#pragma unroll
        for (int ip = 1; ip < RHO; ++ip) ws[ip] = root[ip * step];
        SharedStage<T, NS * RHO, RHO, NB, DIR, TS, NS, 0>::run(v, ws);
      }
#pragma unroll
      for (int c = 0; c < (SHARED ? 0 : NB); ++c) {
        const int b = j + c * TS;
        const int k = b & (NS - 1);
        if constexpr (NS > 1) {
          // zeta_{NS*RHO}^{i' k} = zeta_N^{i' k N/(NS RHO)}; all loads are issued
          // before the first product (the scheduler would otherwise pair each
          // load with its use and wait for every one in turn)
          constexpr int sh = LOGN - (LOGNS + LOGRHO);
          const int step = k << sh;
          // batch size: BATCH 0 -> one at a time, 1 -> all when the lane holds at
          // most 16 FP32 / 8 FP64 values, 2 -> always (FP64 in groups of 8)
          constexpr int GB = BATCH == 0 ? 1
                             : BATCH == 1 ? (R * sizeof(T) <= 64 ? RHO : 1)
                                          : (sizeof(T) == 4 ? RHO : 8);
#pragma unroll
          for (int ip0 = 1; ip0 < RHO; ip0 += GB) {
            cx<T> w[GB];
#pragma unroll
            for (int g = 0; g < GB; ++g)
              if (ip0 + g < RHO) w[g] = root[(ip0 + g) * step];
            if constexpr (GB > 1) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int g = 0; g < GB; ++g)
              if (ip0 + g < RHO) v[c + (ip0 + g) * NB] = twmul<DIR>(v[c + (ip0 + g) * NB], w[g]);
          }
        }
        reg_dft<RHO, DIR, T, NB>(&v[c]);
      }
      if constexpr (!LAST) {
#pragma unroll
        for (int c = 0; c < NB; ++c) {
          const int b = j + c * TS;
          const int k = b & (NS - 1);
          const int base = (b >> LOGNS) * (NS * RHO) + k;
          if constexpr (WIMM) {
            cx<T>* pb = lds + pidx(base) * ES;
#pragma unroll
            for (int ip = 0; ip < RHO; ++ip) pb[ip * OFFW * ES] = v[c + ip * NB];
          } else {
#pragma unroll
            for (int ip = 0; ip < RHO; ++ip) lds[pidx(base + ip * NS) * ES] = v[c + ip * NB];
          }
        }
        sync();
        if constexpr (RIMM) {
          const cx<T>* pr = lds + pidx(j) * ES;
#pragma unroll
          for (int i = 0; i < R; ++i) v[i] = pr[i * OFFR * ES];
        } else {
#pragma unroll
          for (int i = 0; i < R; ++i) v[i] = lds[pidx(j + i * TS) * ES];
        }
        sync();
        TeamFFT<T, LOGN, LOGR, DIR, ES, Sync, LOGNS + LOGRHO, BATCH>::run(v, j, lds, root, sync);
      }
    }
  }
};

// number of team synchronisations one TeamFFT<.., LOGN, LOGR, ..> performs (two per LDS exchange)
template <int LOGN, int LOGR, int LOGNS = 0>
constexpr int team_fft_syncs() {
  constexpr int LRM = LOGR < 4 ? LOGR : 4;
  constexpr int REM = LOGN - LOGNS;
  if constexpr (REM <= 0) {
    return 0;
  } else {
    constexpr int LR = REM < LRM ? REM : LRM;
    if constexpr (LOGNS + LR == LOGN) return 0;
    else return 2 + team_fft_syncs<LOGN, LOGR, LOGNS + LR>();
  }
}

// lds points at element 0 of the exchange buffer (already offset by the team's column)
template <typename T, int LOGN, int LOGR, int DIR, int ES, typename Sync, int BATCH = 1>
__device__ __forceinline__ void team_fft(cx<T> (&v)[1 << LOGR], int j, cx<T>* lds, const cx<T>* __restrict__ root,
                                         Sync sync) {
  TeamFFT<T, LOGN, LOGR, DIR, ES, Sync, 0, BATCH>::run(v, j, lds, root, sync);
}

// Root tables of every power-of-two length are stored back to back: the table
// zeta_{2^L}^k (k < 2^L) starts at element 2^L - 1.
template <typename T, int LOGN>
__device__ __forceinline__ const cx<T>* root_of(const cx<T>* pyramid) {
  return pyramid + ((1 << LOGN) - 1);
}
constexpr int kRootMaxLog = 12;

// slot-padded element access: pidx(j + i*TS) for a compile-time stride TS
template <int TS>
__device__ __forceinline__ int pidx_strided(int j, int i) {
  if constexpr (TS % 16 == 0) return pidx(j) + i * (TS + TS / 16);
  else return pidx(j + i * TS);
}

// ---------------------------------------------------------------------------
// compensated (TwoSum) complex accumulator
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void two_sum_add(T& s, T& c, T x) {
  T t = s + x;
  T bp = t - s;
  T ap = t - bp;
  c += (s - ap) + (x - bp);
  s = t;
}
template <typename T>
struct PAcc {
  cx<T> s;
  __device__ __forceinline__ void zero() { s = mk<T>(0, 0); }
  __device__ __forceinline__ void add(cx<T> x) { s = s + x; }
  __device__ __forceinline__ cx<T> get() const { return s; }
};

template <typename T>
struct CAcc {
  cx<T> s, c;
  __device__ __forceinline__ void zero() {
    s = mk<T>(0, 0);
    c = mk<T>(0, 0);
  }
  __device__ __forceinline__ void add(cx<T> x) {
    two_sum_add(s.x, c.x, x.x);
    two_sum_add(s.y, c.y, x.y);
  }
  __device__ __forceinline__ cx<T> get() const { return mk(s.x + c.x, s.y + c.y); }
};

// ---------------------------------------------------------------------------
// raw real arrays viewed as complex-packed data (Sec. 4, eq. (complexPacking))
// ---------------------------------------------------------------------------
// Packed element (row, c) of a real array whose rows hold `mid` sub-rows of Ld
// reals each (c = jm * Lhd + jd, Lhd = ceil(Ld/2)): reals 2*jd and 2*jd+1 of
// sub-row jm.  `rev` reads the array reversed along every axis (used by the
// adjoint).  Elements outside the array read as zero.
struct RawGeom {
  long long batch_stride;  // reals per batch element
  long long row_stride;    // reals per row (outermost axis step)
  int rows;                // rows present (extent of the outermost axis)
  int mid;                 // middle extent (1 for 1D/2D)
  int Ld;                  // last-axis real extent
  int Lhd;                 // ceil(Ld/2)
  int rev;                 // nonzero: reversed on every axis
  int Lhd_c;               // packed extent that splits a column index c = jm * Lhd_c + jd (0: Lhd): a
                           // kernel g whose last axis is shorter than f's, addressed with f's column indices
};

// Packed complex access is possible when the array is read forwards, its last
// axis has an even length and column indices split like its own layout:
// packed element (row, c) is then complex element row * (row_stride / 2) + c.
// The test is uniform per launch.
__host__ __device__ __forceinline__ bool raw_packed(const RawGeom& g) {
  return !g.rev && !(g.Ld & 1) && (g.Lhd_c == 0 || g.mid == 1);
}

template <typename T>
__device__ __forceinline__ cx<T> raw_load(const T* __restrict__ base, const RawGeom& g, int row, int c) {
  cx<T> r = mk<T>(0, 0);
  if (row < 0 || row >= g.rows) return r;
  int jm, jd;
  if (g.Lhd_c == 0) {
    jm = c / g.Lhd;
    jd = c - jm * g.Lhd;
  } else {  // a shorter kernel addressed with f's column indices (uniform branch)
    jm = c / g.Lhd_c;
    jd = c - jm * g.Lhd_c;
    if (jd >= g.Lhd) return r;
  }
  if (jm >= g.mid) return r;
  int e0 = 2 * jd;
  if (!g.rev) {
    const T* p = base + (long long)row * g.row_stride + (long long)jm * g.Ld + e0;
    if (e0 + 1 < g.Ld) {
      if ((g.Ld & 1) == 0) {
        r = *reinterpret_cast<const cx<T>*>(p);
      } else {
        r.x = p[0];
        r.y = p[1];
      }
    } else if (e0 < g.Ld) {
      r.x = p[0];
    }
  } else {
    const T* p = base + (long long)(g.rows - 1 - row) * g.row_stride + (long long)(g.mid - 1 - jm) * g.Ld;
    int a = g.Ld - 1 - e0;
    if (a >= 0) r.x = p[a];
    if (a - 1 >= 0) r.y = p[a - 1];
  }
  return r;
}

template <typename T>
__device__ __forceinline__ void raw_store(T* __restrict__ base, const RawGeom& g, int row, int c, cx<T> v) {
  if (row < 0 || row >= g.rows) return;
  int jm = c / g.Lhd;
  int jd = c - jm * g.Lhd;
  if (jm >= g.mid) return;
  int e0 = 2 * jd;
  if (!g.rev) {
    T* p = base + (long long)row * g.row_stride + (long long)jm * g.Ld + e0;
    if (e0 + 1 < g.Ld) {
      if ((g.Ld & 1) == 0) {
        *reinterpret_cast<cx<T>*>(p) = v;
      } else {
        p[0] = v.x;
        p[1] = v.y;
      }
    } else if (e0 < g.Ld) {
      p[0] = v.x;
    }
  } else {
    T* p = base + (long long)(g.rows - 1 - row) * g.row_stride + (long long)(g.mid - 1 - jm) * g.Ld;
    int a = g.Ld - 1 - e0;
    if (a >= 0) p[a] = v.x;
    if (a - 1 >= 0) p[a - 1] = v.y;
  }
}

}  // namespace hdc
