// Line kernel: implicitly padded transforms along the contiguous (packed)
// axis, the implicit-packing product with the conjugate partner line, and the
// inverse with accumulation over residues -- all inside one workgroup's LDS.
//
// One workgroup owns one line pair {A, C}: A and its conjugate partner C
// (Sec. 5: slices k and k*; in 1D a single self-conjugate line; for the
// multi-pass 1D form the residue rows r and q - r of Sec. 4, eqs. (Hr),
// (Hr-conj)).  Phases, separated by workgroup barriers:
//   F  forward: for each residue r, pre-process
//        X_r[s] = zeta_N^{r s} sum_{t<p} zeta_q^{r t} x[t m + s]     (Sec. 2, eq. (forwardr))
//      and run a length-m FFT; spectra land in LDS slots [array][line][r][l].
//   M  product over unordered pairs (k on A, k* on C), in place:
//        alpha = 1/4 (F_A - conj F_C)(G_A - conj G_C)(1 + zeta_Nf^kappa),
//        H_A = F_A G_A - alpha,  H_C = F_C G_C - conj(alpha)          (eqs. (RCM), (RCM-ndim))
//      or, for the explicit comparator, unpack -> product -> pack    (eqs. (fourierUnpack), (fourierPack)).
//   I  inverse length-m FFT per (line, residue), post-twiddle zeta_N^{-r s}  (eq. (accumulator))
//   R  h[t m + s] = sum_r zeta_q^{-r t} w_r[s] with compensated (TwoSum) summation  (eq. (accumulation))
//
// Teams of TS = m/R lanes (TS <= 64, one wavefront or less) each run one FFT
// at a time with wavefront-level synchronisation; the workgroup has 4 waves.
#include "hdc_kernels.hpp"

namespace hdc {

// kind groups compiled separately: one raw 1D problem, multi-D line pairs, 1D residue rows
enum KindGroup : int { KG_1D = 0, KG_ND = 1, KG_ROWS = 2 };

// register budget: two waves per SIMD, four for FP32 residue rows of 1024
// (measured faster there despite a few spills)
template <typename T, int LOGM, int KG, bool NARY = false>
constexpr int line_wpe() { return (KG == KG_ROWS && sizeof(T) == 4 && LOGM == 10 && !NARY) ? 4 : 2; }

// Product of one unordered pair of spectrum entries: A at index kappa and its
// conjugate partner C (eqs. (RCM), (RCM-ndim)):
//   alpha = 1/4 (F_A - conj F_C)(G_A - conj G_C)(1 + zeta_Nf^kappa),
//   H_A = F_A G_A - alpha,  H_C = F_C G_C - conj(alpha);   z = zeta_Nf^kappa.
template <typename T>
__device__ __forceinline__ void rcm_product(cx<T> fa, cx<T> ga, cx<T> fc, cx<T> gc, cx<T> z, cx<T>& ha,
                                            cx<T>& hc) {
  const cx<T> zp1 = mk<T>(z.x + (T)1, z.y);
  const cx<T> a1 = fa - conj(fc);
  const cx<T> a2 = ga - conj(gc);
  const cx<T> alpha = scale(cmul(cmul(a1, a2), zp1), (T)0.25);
  ha = cmul(fa, ga) - alpha;
  hc = cmul(fc, gc) - conj(alpha);
}

// The explicit comparator's product: unpack both members of the pair into
// the real transform's spectrum (eq. (fourierUnpack)), multiply, pack again
// (eq. (fourierPack)); tw2Nf looks up zeta_{2 Nf}.
template <typename T, typename Look>
__device__ __forceinline__ void explicit_product(cx<T> fa, cx<T> ga, cx<T> fc, cx<T> gc, const Look& tw2Nf,
                                                 int kap, int Nf, cx<T>& ha, cx<T>& hc) {
  const T half = (T)0.5;
  const cx<T> sF = fa + conj(fc), dF = fa - conj(fc);
  const cx<T> sG = ga + conj(gc), dG = ga - conj(gc);
  const cx<T> sFc = fc + conj(fa), dFc = fc - conj(fa);
  const cx<T> sGc = gc + conj(ga), dGc = gc - conj(ga);
  if (kap != 0) {
    const cx<T> wA = tw2Nf(kap);
    const cx<T> wC = tw2Nf(Nf - kap);
    const cx<T> UA = scale(sF - mul_i<+1>(cmul(dF, wA)), half);
    const cx<T> VA = scale(sG - mul_i<+1>(cmul(dG, wA)), half);
    const cx<T> UC = scale(sFc - mul_i<+1>(cmul(dFc, wC)), half);
    const cx<T> VC = scale(sGc - mul_i<+1>(cmul(dGc, wC)), half);
    const cx<T> PA = cmul(UA, VA), PC = cmul(UC, VC);
    ha = scale((PA + conj(PC)) + mul_i<+1>(cmulc(PA - conj(PC), wA)), half);
    hc = scale((PC + conj(PA)) + mul_i<+1>(cmulc(PC - conj(PA), wC)), half);
  } else {
    // kappa = 0 pairs with the Nyquist index Nf of the real transform
    const cx<T> UA0 = scale(sF - mul_i<+1>(dF), half), UAN = scale(sF + mul_i<+1>(dF), half);
    const cx<T> VA0 = scale(sG - mul_i<+1>(dG), half), VAN = scale(sG + mul_i<+1>(dG), half);
    const cx<T> UC0 = scale(sFc - mul_i<+1>(dFc), half), UCN = scale(sFc + mul_i<+1>(dFc), half);
    const cx<T> VC0 = scale(sGc - mul_i<+1>(dGc), half), VCN = scale(sGc + mul_i<+1>(dGc), half);
    const cx<T> PA0 = cmul(UA0, VA0), PAN = cmul(UAN, VAN);
    const cx<T> PC0 = cmul(UC0, VC0), PCN = cmul(UCN, VCN);
    ha = scale((PA0 + conj(PCN)) + mul_i<+1>(PA0 - conj(PCN)), half);
    hc = scale((PC0 + conj(PAN)) + mul_i<+1>(PC0 - conj(PAN)), half);
  }
}

template <typename T, int LOGM, int PMAX, int KG, bool TAB, bool TWIN, bool NARY = false>
__global__ __launch_bounds__(line_waves * 64)
__attribute__((amdgpu_waves_per_eu(line_wpe<T, LOGM, KG, NARY>()))) void k_line(LineParams<T> P0,
                                                                      const LineParams<T>* __restrict__ tab) {
  // grouped launch (TAB): blockIdx.y is one problem of the group, parameters from the table
  const LineParams<T> P = TAB ? tab[blockIdx.y] : P0;
  if (TAB && (int)blockIdx.x >= P.njobs) return;
  constexpr int M = 1 << LOGM;
  constexpr int LOGR = line_logr(LOGM, KG);
  constexpr int R = 1 << LOGR;
  constexpr int TS = M / R;
  constexpr int NTHR = line_waves * 64;
  constexpr int NTEAMS = NTHR / TS;
  extern __shared__ char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);

  const int tid = threadIdx.x;
  const int team = tid / TS;
  const int j = tid - team * TS;
  const int b = TAB ? 0 : blockIdx.y;
  const int q = P.q;
  const int p = P.p;
  const int SL = padded_len(M);
  const cx<T>* root = root_of<T, LOGM>(P.rootpyr);
  // loops of table lookups: specialised on the table's form for the multi-D
  // line pairs only (there it lowers the register count; elsewhere it raises it)
  auto with_tw = [&](const Tw2<T>& t, auto&& f) {
    if constexpr (KG == KG_ND) tw_dispatch(t, f);
    else f(TwSel<T>{t});
  };

  // ---- which line pairs this workgroup owns: one for the 1D kinds, up to
  // kLinePairsMax canonical pairs {k, k*} for the multi-D kinds (small m)
  __shared__ long long s_line[2 * kLinePairsMax];
  int npw = 1;
  int NLS = 1;  // line slots per array and pair
  // residue rows: RCM pairs rows r and q - r; an elementwise product (the
  // conjugate-symmetry form, rows 0..qres-1 independent) takes rows 2x, 2x + 1
  const bool elem = (KG == KG_ROWS) && P.variant == MUL_ELEM;
  const int rA = (KG == KG_ROWS) ? (elem ? 2 * (int)blockIdx.x : (int)blockIdx.x) : 0;
  const int rC = (KG == KG_ROWS) ? (elem ? (rA + 1 < P.qres ? rA + 1 : rA) : (P.qres - rA) % P.qres) : 0;
  if constexpr (KG == KG_ROWS) {
    NLS = (rA == rC) ? 1 : 2;
  } else if constexpr (KG == KG_ND) {
    const long long first = (long long)blockIdx.x * P.ppw;
    npw = (int)((P.npairs - first) < P.ppw ? (P.npairs - first) : P.ppw);
    NLS = P.kind == LINE_PLAIN ? 1 : 2;
    if (tid < npw) {
      long long A, Cl;
      line_pair(P, first + tid, A, Cl);
      s_line[2 * tid] = A;
      s_line[2 * tid + 1] = Cl;
    }
    __syncthreads();
  }
  auto line_of = [&](int pp, int li) -> long long {
    if constexpr (KG == KG_ND) return s_line[2 * pp + li];
    else return li ? rC : rA;
  };
  auto nl_of = [&](int pp) -> int {
    if constexpr (KG == KG_1D) return 1;
    else if constexpr (KG == KG_ROWS) return NLS;
    else return s_line[2 * pp] == s_line[2 * pp + 1] ? 1 : 2;
  };

  const int NARR = NARY ? P.nin : 2;  // arrays (their slots per pair and line)
  auto slot = [&](int pp, int arr, int li, int r) -> cx<T>* {
    return lds + (((pp * NARR + arr) * NLS + li) * q + r) * SL;
  };
  // workspace line of array arr (pass 1 of the twin mode reads its first array from wsF2)
  auto line_ptr = [&](int pp, int arr, int li, int pass) -> cx<T>* {
    cx<T>* base = NARY ? P.wsF + arr * P.ws_arr : (arr ? P.wsG : (pass ? P.wsF2 : P.wsF));
    return base + (long long)b * P.ws_batch + line_of(pp, li) * P.line_stride;
  };
  auto out_ptr = [&](int pp, int li, int pass) -> cx<T>* {
    cx<T>* base = pass ? P.wsH2 : (P.wsH ? P.wsH : P.wsF);
    return base + (long long)b * P.ws_batch + line_of(pp, li) * P.line_stride;
  };

  // ---------------------------------------------------------------- phase F
  // pass 1 (twin mode) transforms only the first array; the second keeps its spectra in LDS
  auto phase_F = [&](int pass) {
    const int narr = pass ? 1 : NARR;
    const int ntask = npw * narr * NLS;  // (pair, array, line)
    const int nchunk = NTEAMS >= ntask ? NTEAMS / ntask : 1;
    const int nunits = ntask * nchunk;
    for (int u = team; u < nunits; u += NTEAMS) {
      const int task = u % ntask;
      const int chunk = u / ntask;
      const int pp = task / (narr * NLS);
      const int arr = (task / NLS) % narr;
      const int li = task % NLS;
      if (li >= nl_of(pp)) continue;  // self-conjugate pair: one line
      const T* rbase = NARY ? P.xin[arr] : (arr ? P.g : (pass ? P.f2 : P.f));
      const RawGeom rg = NARY ? P.gf : (arr ? P.gg : (pass ? P.gf2 : P.gf));
      rbase += (long long)b * rg.batch_stride;
      // packed complex view: the workspace line, or the raw array when read forwards with even length
      const cx<T>* lp = (KG != KG_1D) ? line_ptr(pp, arr, li, pass)
                                      : (raw_packed(rg) ? reinterpret_cast<const cx<T>*>(rbase) : nullptr);
      auto load = [&](int pos) -> cx<T> {
        if constexpr (KG == KG_ROWS) return lp[pos];  // rows are full (Lin = m)
        // branch-free for the complex views: a masked lane reads element 0
        const bool in = pos < ((KG == KG_1D && arr && !NARY) ? P.Lin_g : P.Lin);
        if constexpr (KG == KG_ND) {
          const cx<T> v = lp[in ? pos : 0];
          return in ? v : mk<T>(0, 0);
        }
        if (lp) {
          const cx<T> v = lp[in ? pos : 0];
          return in ? v : mk<T>(0, 0);
        }
        return in ? raw_load(rbase, rg, 0, pos) : mk<T>(0, 0);
      };
      if constexpr (KG == KG_ROWS) {
        // a residue row: no pre-processing (p = q = 1); load, transform, keep in LDS.
        // Only the first residue chunk has work (q = 1); the other teams of this
        // task must not touch the slot.
        if (chunk != 0) continue;
        cx<T>* sl = slot(0, arr, li, 0);
        cx<T>* gsp = P.gspec + (long long)b * P.ws_batch + line_of(0, li) * P.line_stride;
        if (arr == 1 && P.gmode == 2) {
          // cached kernel: the row's spectrum in natural order
#pragma unroll
          for (int i = 0; i < R; ++i) sl[pidx_strided<TS>(j, i)] = gsp[j + i * TS];
          continue;
        }
        if (arr == 0 && P.gmode == 1) continue;  // transforming the kernel alone
        cx<T> v[R];
#pragma unroll
        for (int i = 0; i < R; ++i) v[i] = lp[j + i * TS];
        if (P.twRow.N > 1) four_step_row<T, R, TS, +1>(v, j, (int)line_of(0, li), P.twRow);
        team_fft<T, LOGM, LOGR, +1, 1, WaveSync, 2>(v, j, sl, root, WaveSync());
        if (P.gmode == 1) {
#pragma unroll
          for (int i = 0; i < R; ++i) gsp[j + i * TS] = v[i];
          continue;
        }
#pragma unroll
        for (int i = 0; i < R; ++i) sl[pidx_strided<TS>(j, i)] = v[i];
        continue;
      }
      // cached kernel spectra (kinds 0-2): the kernel's line spectra, [r][l] per line
      const int gmode = (NARY || TWIN) ? 0 : P.gmode;
      const long long goff = (long long)b * P.spec_batch + line_of(pp, li) * P.spec_line;
      if (arr == 1 && gmode == 2) {
        const cx<T>* gsl = P.gspec + goff;
        for (int r = chunk; r < q; r += nchunk) {
          cx<T>* sl = slot(pp, 1, li, r);
#pragma unroll
          for (int i = 0; i < R; ++i) sl[pidx_strided<TS>(j, i)] = gsl[r * M + j + i * TS];
        }
        continue;
      }
      if (arr == 0 && gmode == 1) continue;  // transforming the kernel alone
      constexpr int PX = PMAX > 0 ? PMAX : 1;
      // blocks holding data: the kernel g may have fewer (p per array, Sec. 7); the rest are skipped
      const int pa = (arr && !NARY && P.p_g) ? P.p_g : p;
      cx<T> x[PX][R];
      if constexpr (PMAX > 0) {
#pragma unroll
        for (int t = 0; t < PMAX; ++t)
#pragma unroll
          for (int i = 0; i < R; ++i) x[t][i] = (t < pa) ? load(t * M + j + i * TS) : mk<T>(0, 0);
      }
      for (int r = chunk; r < q; r += nchunk) {
        cx<T> v[R];
        if constexpr (PMAX > 0) {
          // sum_t zeta_q^{r t} x[t m + s]; blocks t >= p were loaded as zeros
          cx<T> wq[PX];
#pragma unroll
          for (int t = 1; t < PX; ++t) wq[t] = tw_get(P.twN, ((r * t) % q) * M);
#pragma unroll
          for (int i = 0; i < R; ++i) {
            cx<T> acc = x[0][i];
#pragma unroll
            for (int t = 1; t < PX; ++t)
              if (t < pa) acc = acc + cmul(x[t][i], wq[t]);
            v[i] = acc;
          }
        } else {
          // many explicit blocks: re-read the input for every residue
          with_tw(P.twN, [&](auto twN) {
#pragma unroll
            for (int i = 0; i < R; ++i) {
              const int s = j + i * TS;
              cx<T> acc = load(s);
              for (int t = 1; t < pa; ++t) acc = acc + cmul(load(t * M + s), twN(((r * t) % q) * M));
              v[i] = acc;
            }
          });
        }
        residue_twiddle<T, R, TS, +1, true, KG == KG_ND ? 2 : 0>(v, j, r, P.twN);
        if constexpr (KG == KG_ND)  // plain lines of a large 1D problem: four-step twiddle of row k
          if (P.twRow.N > 1) four_step_row<T, R, TS, +1>(v, j, (int)line_of(pp, li), P.twRow);
        cx<T>* sl = slot(pp, arr, li, r);
        team_fft<T, LOGM, LOGR, +1, 1, WaveSync>(v, j, sl, root, WaveSync());
        if (gmode == 1) {  // the kernel's spectrum, stored for later calls
          cx<T>* gsl = P.gspec + goff + r * M;
#pragma unroll
          for (int i = 0; i < R; ++i) gsl[j + i * TS] = v[i];
          continue;
        }
#pragma unroll
        for (int i = 0; i < R; ++i) sl[pidx_strided<TS>(j, i)] = v[i];
      }
    }
  };

  // ---------------------------------------------------------------- phase M
  // unordered pairs: element (r, l) of line A and its conjugate partner (rs, ls)
  // of line C; k = q l + r is the index along the packed axis.  For residue rows
  // (kind 3) the line is itself residue rA of the 1D problem (q = 1 here).
  // The product overwrites the first array's slots; the second array's stay.
  auto phase_M = [&]() {
    const int Nf = P.Nf;
    const T sc = P.scale;
    const cx<T> zrow = (KG == KG_ROWS) ? tw_get(P.tw2Nf, 2 * rA) : mk<T>(1, 0);
    const int QM = q * M;
    if (KG != KG_1D && P.variant == MUL_ELEM) {
      // plain complex convolution: H = F G at every element of every line
      for (int pl = 0; pl < npw * NLS; ++pl) {
        const int pp = pl / NLS;
        const int li = pl - pp * NLS;
        if (li >= nl_of(pp)) continue;
        for (int idx = tid; idx < QM; idx += NTHR) {
          cx<T>* pF = slot(pp, 0, li, idx >> LOGM) + pidx(idx & (M - 1));
          const cx<T> gv = slot(pp, 1, li, idx >> LOGM)[pidx(idx & (M - 1))];
          *pF = scale(cmul(*pF, gv), sc);
        }
      }
      return;
    }
    with_tw(P.tw2Nf, [&](auto tw2Nf) {
      for (int pp = 0; pp < npw; ++pp) {
        const int nl = nl_of(pp);
        for (int idx = tid; idx < QM; idx += NTHR) {
          const int r = idx >> LOGM;
          const int l = idx & (M - 1);
          int rs, ls, kap;
          if (KG == KG_ROWS) {
            rs = 0;
            ls = rA ? (M - 1 - l) : ((M - l) & (M - 1));
            kap = P.qrow * l + rA;
          } else {
            rs = r ? q - r : 0;
            ls = r ? (M - 1 - l) : ((M - l) & (M - 1));
            kap = l * q + r;
          }
          if (nl == 1 && (ls * q + rs) < (l * q + r)) continue;
          cx<T>* pFA = slot(pp, 0, 0, r) + pidx(l);
          cx<T>* pGA = slot(pp, 1, 0, r) + pidx(l);
          cx<T>* pFC = slot(pp, 0, nl - 1, rs) + pidx(ls);
          cx<T>* pGC = slot(pp, 1, nl - 1, rs) + pidx(ls);
          if constexpr (NARY) {
            // R^1 = F^1; R^j = R^{j-1} [.] F^j at the pair (A, C) by eqs. (Akn), (Rnk), (RnMk),
            // in registers; R^nin overwrites array 0
            const cx<T> z = (KG == KG_ROWS) ? cmul(root[l], zrow) : tw2Nf(2 * kap);
            cx<T> ra = *pFA, rc = *pFC;
            for (int a = 1; a < NARR; ++a) {
              const cx<T> xa = slot(pp, a, 0, r)[pidx(l)];
              const cx<T> xc = slot(pp, a, nl - 1, rs)[pidx(ls)];
              rcm_product(ra, xa, rc, xc, z, ra, rc);
            }
            *pFA = scale(ra, sc);
            if (pFC != pFA) *pFC = scale(rc, sc);
            continue;
          }
          const cx<T> fa = *pFA, ga = *pGA, fc = *pFC, gc = *pGC;
          cx<T> ha, hc;
          if (P.variant == MUL_RCM) {
            // for residue rows kappa = qres l + rA, so zeta_Nf^kappa = zeta_m^l zeta_Nf^rA
            // (one FFT-root lookup per element)
            const cx<T> z = (KG == KG_ROWS) ? cmul(root[l], zrow) : tw2Nf(2 * kap);
            rcm_product(fa, ga, fc, gc, z, ha, hc);
          } else {
            explicit_product(fa, ga, fc, gc, tw2Nf, kap, Nf, ha, hc);
          }
          *pFA = scale(ha, sc);
          if (pFC != pFA) *pFC = scale(hc, sc);
        }
      }
    });
  };

  // ---------------------------------------------------------------- phases I, R
  auto phase_IR = [&](int pass) {
    auto store = [&](int pp, int li, int o, cx<T> val) {
      if constexpr (KG == KG_1D) {
        T* hb = (pass ? P.h2 : P.h);
        const RawGeom gh = pass ? P.gh2 : P.gh;
        hb += (long long)b * gh.batch_stride;
        if (raw_packed(gh)) reinterpret_cast<cx<T>*>(hb)[o] = val;
        else raw_store(hb, gh, 0, o, val);
      } else {
        out_ptr(pp, li, pass)[o] = val;
      }
    };
    if constexpr (KG == KG_ROWS && LOGR >= 5 && TS == 64 && NTEAMS == 4) {
      // residue rows: at most two lines for four wavefronts, so teams of two
      // wavefronts run the inverse with half the elements per lane.  For a
      // self-conjugate row the second team has no line: it scribbles on the free
      // G slot and discards the result, or -- when the G slot still holds spectra
      // the next pass needs (pass 0 of the twin mode) -- only joins the barriers.
      constexpr int LOGR2 = LOGR - 1, R2 = R / 2, TS2 = 2 * TS;
      const int li = tid / TS2;
      const int j2 = tid - li * TS2;
      const bool act = li < NLS;
      if (TWIN && !act && pass == 0) {
        __syncthreads();
        constexpr int NSYNC = team_fft_syncs<LOGM, LOGR2>();
#pragma unroll
        for (int k = 0; k < NSYNC; ++k) __syncthreads();
        return;
      }
      cx<T>* sl = act ? slot(0, 0, li, 0) : slot(0, 1, 0, 0);
      cx<T> v[R2];
#pragma unroll
      for (int i = 0; i < R2; ++i) v[i] = sl[pidx(j2 + i * TS2)];
      __syncthreads();
      team_fft<T, LOGM, LOGR2, -1, 1, BlockSync, 2>(v, j2, sl, root, BlockSync());
      if (act) {
        if (P.twRow.N > 1) four_step_row<T, R2, TS2, -1>(v, j2, (int)line_of(0, li), P.twRow);
#pragma unroll
        for (int i = 0; i < R2; ++i) store(0, li, j2 + i * TS2, v[i]);
      }
      return;
    }
    if (q == 1) {
      // one residue (then p = 1): the inverse FFT output is the result
      for (int u = team; u < npw * NLS; u += NTEAMS) {
        const int pp = u / NLS;
        const int li = u - pp * NLS;
        if (li >= nl_of(pp)) continue;
        cx<T>* sl = slot(pp, 0, li, 0);
        cx<T> v[R];
#pragma unroll
        for (int i = 0; i < R; ++i) v[i] = sl[pidx_strided<TS>(j, i)];
        WaveSync()();
        team_fft<T, LOGM, LOGR, -1, 1, WaveSync>(v, j, sl, root, WaveSync());
        if constexpr (KG == KG_ROWS || KG == KG_ND)
          if (P.twRow.N > 1) four_step_row<T, R, TS, -1>(v, j, (int)line_of(pp, li), P.twRow);
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const int s = j + i * TS;
          if (KG == KG_ROWS || s < P.Lout) store(pp, li, s, v[i]);
        }
      }
      return;
    }
    if constexpr (PMAX > 0 && PMAX <= 2 && LOGM <= 9) {
      if (npw * NLS >= NTEAMS) {
        // enough lines for every team: one team per line runs the inverse of
        // every residue and accumulates h[t m + s] = sum_r zeta_q^{-r t} w_r[s] in
        // registers (residues in fixed order; compensated when q > 2 -- with two
        // terms the compensated sum equals the rounded sum exactly)
        auto lines = [&](auto tag) {
          using Acc = decltype(tag);
          for (int u = team; u < npw * NLS; u += NTEAMS) {
            const int pp = u / NLS;
            const int li = u - pp * NLS;
            if (li >= nl_of(pp)) continue;
            Acc acc[PMAX][R];
#pragma unroll
            for (int t = 0; t < PMAX; ++t)
#pragma unroll
              for (int i = 0; i < R; ++i) acc[t][i].zero();
            for (int r = 0; r < q; ++r) {
              cx<T>* sl = slot(pp, 0, li, r);
              cx<T> v[R];
#pragma unroll
              for (int i = 0; i < R; ++i) v[i] = sl[pidx_strided<TS>(j, i)];
              WaveSync()();
              team_fft<T, LOGM, LOGR, -1, 1, WaveSync>(v, j, sl, root, WaveSync());
              residue_twiddle<T, R, TS, -1, true, KG == KG_ND ? 2 : 0>(v, j, r, P.twN);
#pragma unroll
              for (int i = 0; i < R; ++i) acc[0][i].add(v[i]);
#pragma unroll
              for (int t = 1; t < PMAX; ++t) {
                const cx<T> wt = tw_get(P.twN, ((r * t) % q) * M);
#pragma unroll
                for (int i = 0; i < R; ++i) acc[t][i].add(cmulc(v[i], wt));
              }
            }
#pragma unroll
            for (int t = 0; t < PMAX; ++t)
#pragma unroll
              for (int i = 0; i < R; ++i) {
                const int o = t * M + j + i * TS;
                if (t < p && o < P.Lout) store(pp, li, o, acc[t][i].get());
              }
          }
        };
        if (q > 2) lines(CAcc<T>{});
        else lines(PAcc<T>{});
        return;
      }
    }
    {
      const int ntask = npw * NLS * q;
      for (int u = team; u < ntask; u += NTEAMS) {
        const int pp = u / (NLS * q);
        const int rem = u - pp * (NLS * q);
        const int li = rem / q;
        const int r = rem - li * q;
        if (li >= nl_of(pp)) continue;
        cx<T>* sl = slot(pp, 0, li, r);
        cx<T> v[R];
#pragma unroll
        for (int i = 0; i < R; ++i) v[i] = sl[pidx_strided<TS>(j, i)];
        WaveSync()();
        team_fft<T, LOGM, LOGR, -1, 1, WaveSync>(v, j, sl, root, WaveSync());
        residue_twiddle<T, R, TS, -1, true, KG == KG_ND ? 2 : 0>(v, j, r, P.twN);
#pragma unroll
        for (int i = 0; i < R; ++i) sl[pidx_strided<TS>(j, i)] = v[i];
      }
    }
    __syncthreads();
    {
      // h[t m + s] = sum_r zeta_q^{-r t} w_r[s], residues in fixed order, compensated when q > 2 (with two
      // terms the compensated sum equals the rounded sum exactly)
      const int Lout = P.Lout;
      auto accumulate = [&](auto twN, auto tag) {
        using Acc = decltype(tag);
        for (int pl = 0; pl < npw * NLS; ++pl) {
          const int pp = pl / NLS;
          const int li = pl - pp * NLS;
          if (li >= nl_of(pp)) continue;
          for (int o = tid; o < Lout; o += NTHR) {
            const int t = o >> LOGM;
            const int s = o & (M - 1);
            Acc acc;
            acc.zero();
            int rt = 0;  // (r t) mod q
            for (int r = 0; r < q; ++r) {
              cx<T> y = slot(pp, 0, li, r)[pidx(s)];
              if (rt) y = cmulc(y, twN(rt * M));
              acc.add(y);
              rt += t;
              if (rt >= q) rt -= q;
            }
            store(pp, li, o, acc.get());
          }
        }
      };
      with_tw(P.twN, [&](auto twN) {
        if (q > 2) accumulate(twN, CAcc<T>{});
        else accumulate(twN, PAcc<T>{});
      });
    }
  };

  // ---------------------------------------------------------------- passes
  // One pass: F, M, I/R.  The twin mode (the adjoint) runs a second pass whose
  // first array is new and whose second array keeps its spectra from pass 0.
  phase_F(0);
  if (P.gmode == 1) return;  // the kernel's spectra are stored
  __syncthreads();
  phase_M();
  __syncthreads();
  phase_IR(0);
  if constexpr (TWIN) {
    __syncthreads();  // pass 0 has finished reading its product slots
    phase_F(1);
    __syncthreads();
    phase_M();
    __syncthreads();
    phase_IR(1);
  }
}

template <typename T, int LOGM, int PMAX, int KG>
static hipError_t launch_line_t(const LineParams<T>& P, dim3 grid, hipStream_t s, const LineParams<T>* tab) {
  const bool nary = P.nin > 2;
  if (nary && (P.nin > kMaxNary || tab || P.twin || P.variant != MUL_RCM || P.kind == LINE_PLAIN))
    return hipErrorInvalidValue;
  const int narr = nary ? P.nin : 2;
  const int nspec = (KG == KG_1D || P.kind == LINE_PLAIN) ? narr : 2 * narr;
  const int ppw = (KG == KG_ND && P.ppw > 1) ? P.ppw : 1;
  if (ppw > kLinePairsMax) return hipErrorInvalidValue;
  const size_t lds = (size_t)ppw * line_lds_bytes<T>(1 << LOGM, P.q, nspec);
  auto fn = nary ? k_line<T, LOGM, PMAX, KG, false, false, true>
            : P.twin ? (tab ? k_line<T, LOGM, PMAX, KG, true, true> : k_line<T, LOGM, PMAX, KG, false, true>)
                     : (tab ? k_line<T, LOGM, PMAX, KG, true, false> : k_line<T, LOGM, PMAX, KG, false, false>);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fn, grid, dim3(line_waves * 64), lds, s, P, tab);
  return hipGetLastError();
}

// one object per (type, log2 m, kind group[, block cap]): see hdc_kernels.hpp (launch_line_lm)
template <typename T, int LOGM, int KG, int PMAX>
hipError_t launch_line_kp(const LineParams<T>& P, dim3 grid, hipStream_t s, const LineParams<T>* tab) {
  return launch_line_t<T, LOGM, PMAX, KG>(P, grid, s, tab);
}

#if defined(HDC_T) && defined(HDC_LOGM) && defined(HDC_KG)
#if HDC_KG == 2
template hipError_t launch_line_kp<HDC_T, HDC_LOGM, 2, 1>(const LineParams<HDC_T>&, dim3, hipStream_t,
                                                          const LineParams<HDC_T>*);
#elif defined(HDC_PMAX)
template hipError_t launch_line_kp<HDC_T, HDC_LOGM, HDC_KG, HDC_PMAX>(const LineParams<HDC_T>&, dim3, hipStream_t,
                                                                      const LineParams<HDC_T>*);
#else
template hipError_t launch_line_kp<HDC_T, HDC_LOGM, HDC_KG, 0>(const LineParams<HDC_T>&, dim3, hipStream_t,
                                                               const LineParams<HDC_T>*);
template hipError_t launch_line_kp<HDC_T, HDC_LOGM, HDC_KG, 1>(const LineParams<HDC_T>&, dim3, hipStream_t,
                                                               const LineParams<HDC_T>*);
template hipError_t launch_line_kp<HDC_T, HDC_LOGM, HDC_KG, 2>(const LineParams<HDC_T>&, dim3, hipStream_t,
                                                               const LineParams<HDC_T>*);
template hipError_t launch_line_kp<HDC_T, HDC_LOGM, HDC_KG, 4>(const LineParams<HDC_T>&, dim3, hipStream_t,
                                                               const LineParams<HDC_T>*);
#endif
#endif

}  // namespace hdc
