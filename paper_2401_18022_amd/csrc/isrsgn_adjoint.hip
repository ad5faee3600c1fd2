// Adjoint of the ISRS GN throughput (arXiv:2401.18022, eq. loss and C = 2 B_ch (-L)) with
// respect to every launch power: the chain through the SNR reduction, the pair integrals
// (PSD products and the power term of eq. pk inside eq. psi_fin) and the power profile
// (closed form or RK4 ODE, differentiated exactly as discretised).
#include "isrsgn_device.h"

namespace isrsgn {
namespace {

// ---------------------------------------------------------------------------- upstream weights
// Per channel i with P_i > 0: N_i = P_NLI,i + P_ASE,i, S0 = P_i / N_i, SNR = S0 (or combined
// with the transceiver SNR), T_i = 2 R_i log2(1 + SNR).  lam_i = dT/dtile(i,.) =
// dT/dN_i * 16/27 gamma_i^2 R_i; gP_i starts as the direct dT/dP_i; gLL_i = dT/d ln rho(L, f_i)
// through the ASE term.
__global__ void k_grad_prep(PlanView pv, const double* __restrict__ P, const double* __restrict__ nf, double snr_trx,
                            Work w, int g_begin, int g_end, int n_spans) {
  const int g = g_begin + blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= g_end) return;
  const double p = P[g], R = pv.R[g], f = pv.f[g], gm = pv.gamma[g];
  double lamN = 0.0, direct = 0.0, pase = 0.0;
  if (p > 0.0) {
    pase = nf[g] * kH * f * R * exp(-w.ellL[g]) * n_spans;  // one amplifier per span
    const double N = w.pnli[g] + pase, s0 = p / N;
    double snr = s0, dsnr = 1.0;
    if (snr_trx > 0.0) {
      snr = 1.0 / (1.0 / s0 + 1.0 / snr_trx);
      dsnr = (snr / s0) * (snr / s0);
    }
    const double u = 2.0 * R / ((1.0 + snr) * 0.69314718055994530942) * dsnr;  // dT/dS0
    lamN = -u * s0 / N;
    direct = u / N;
  }
  w.lam[g] = lamN * (16.0 / 27.0) * gm * gm * R;
  w.gP[g] = direct;
  w.gLL[g] = -lamN * pase;
}

__global__ void k_fill(double* x, int64_t n) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
    x[q] = 0.0;
}

__global__ void k_zero_counter2(unsigned int* c) { c[0] = c[1] = 0u; }

// ---------------------------------------------------------------------------- adjoint pair integrals
// For every node of tile (i,k) with upstream weight lam_i:
//   d/dG_c:   lam w |S|^2 times the other two PSDs, for c in {c1, c2, k}       (LDS histogram)
//   d/dE_m:   Q_m = lam w G1 G2 Gk Re(conj(S) term_m)  where term_m is the m-th summand of S
// and dT/d ln rho(m, c) = Q_m times the interpolation weights of f1, f2, f3 (+) and f_i (-),
// each with the factor 1/2 of eq. (pk) absorbed (linear profile: E_m = ln rho(f3), weight 2).
//
// Scatter: after a node batch has S (pass 1), the batch recomputes its terms in chunks of MC
// steps (pass 2) and stages Q in LDS; then the lanes are re-mapped to (step, node group):
// each lane walks its group's nodes in row order, keeping running sums while the f1 (f2)
// segment stays the same and flushing them when it changes -- along a row f1 and f2 move
// monotonically, so runs are long.  Flushes to the tile's hot channels (k-1, k, k+1, i-1, i,
// i+1) land in per-tile LDS rows; the rest go to HBM with FP64 atomics.  The f3 and f_i
// contributions only touch channels k-1, k, k+1 and i: they accumulate in the LDS rows too.
// Staging and metadata are private to a wave, so the re-map needs wave-level ordering only.
//
// Per-node metadata, struct of arrays, group g of MC nodes starting at g (MC + 1) so that the
// groups a wave reads at once sit in distinct LDS banks:
//   key: s1 | s2 << 16 (-1: node off the support); (t1, t2, w3a, w3c) as one 16-byte record
//   (w3b = wgt - w3a - w3c); f1, f2: 1 when the node's f1 (f2) segment is the upper of its
//   group's two.
constexpr int kMetaStride = 72;  // >= 64 + 64 / MC for MC in {8, 16}
// Workgroup of the adjoint: kWaves wave64 sharing the tile's channel, row, step and accumulator
// arrays in LDS; the staging and metadata are per wave.  Four waves hold up to 256 VGPRs (2 waves
// per SIMD, register-bound); the FP32 form with the stored S also comes with sixteen waves,
// held to 128 VGPRs (4 waves per SIMD; the node set-up spills) and one block per CU, used where
// its LDS fits.
constexpr int kAdjWavesMax = 16;
// Row stride of the per-wave staging [step][node], in elements.  FP32: 68, so that a re-map
// lane's run of node values starts on a 16-byte boundary (4 values per read); FP64: 65 (odd).
// The node-lane writes of one step are consecutive either way.
__host__ __device__ constexpr int stage_row(int prec) { return prec == 0 ? 68 : 65; }

template <int kPrec>
struct AdjCfg {
  using real = float;
  static constexpr int MC = 16;
};
template <>
struct AdjCfg<1> {
  using real = double;
  static constexpr int MC = 8;
};

__host__ __device__ inline size_t adjoint_lds_bytes(int nmax, int gs, int M, int prec, int waves) {
  const int mc = prec == 0 ? 16 : 8;
  const size_t rb = prec == 0 ? 4 : 8;
  // doubles: channels (3 nmax), rows (4 gs), the dT/dG histogram (nmax), the hot-channel and
  // f-term rows (7 M), block_sum's scratch, the low-rank f term (kRank floats), one to start the
  // column tables on a 16-byte boundary and the FP64 form's f-term column (M, rounded up to even);
  // then the f3 columns, staging and metadata
  return sizeof(double) * (3 * (size_t)nmax + 4 * (size_t)gs + (size_t)nmax + 7 * (size_t)M + kAdjWavesMax +
                           kRank / 2 + 1 + (size_t)((M + 1) & ~1)) +
         sizeof(Col4) * (size_t)M + waves * (size_t)mc * stage_row(prec) * rb + waves * 7 * kMetaStride * 4 + 16;
}

constexpr int kRow32 = stage_row(0);

// Four consecutive staged values of one re-map lane: one 16-byte LDS read in the FP32 form
// (a lane's run starts on a 16-byte boundary with the 68-element rows).
template <int kPrec, class real>
__device__ inline void load_q4(const real* p, real* q) {
  if constexpr (kPrec == 0) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    q[0] = v.x;
    q[1] = v.y;
    q[2] = v.z;
    q[3] = v.w;
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) q[j] = p[j];
  }
}

// Pass 2 of the FP32 form projects each step term on S: with S = |S| e^(2 pi j th),
//   Re(conj(S) term_m) = |S| amp_m cos 2 pi (phr z_m - th)                  (midpoint forms)
//                      = |S| p_m [s(z_(m+1/2)) - s(z_(m-1/2))] / (2 pi phr)  (edge form),
// s(z) = sin 2 pi (phr z - th): one hardware sine or cosine per step instead of both.
// NodePhase: cqs = cq |S| (the node's factor), th in FP32, and -th in FP64 for the reduction.
struct NodePhase {
  float cqs, th;
  double nth;
};

// arg(x + j y) / (2 pi) in revolutions, FP32: octant reduction to t = min/max in [0, 1], then
// atan(t) / (2 pi) as t P(t^2) with P of degree 7 (coefficients and their bound, 2.7e-8
// revolutions, from fit_atan_rev.py).  x = y = 0 gives 0.
__device__ inline float atan_rev32(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
  const float t = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
  const float u = t * t;
  float p = -0.000645301945f;
  p = fmaf(p, u, 0.00347958924f);
  p = fmaf(p, u, -0.00889871176f);
  p = fmaf(p, u, 0.0153460251f);
  p = fmaf(p, u, -0.0221362691f);
  p = fmaf(p, u, 0.0317459442f);
  p = fmaf(p, u, -0.0530461222f);
  p = fmaf(p, u, 0.159154832f);
  float r = p * t;
  r = ay > ax ? 0.25f - r : r;
  r = x < 0.0f ? 0.5f - r : r;
  return y < 0.0f ? -r : r;
}

// s(z) at a step edge, the FP64 phase reduced to [0, 1) revolutions.
__device__ inline float edge_sine32(double phr, double z, double nth) {
  return __builtin_amdgcn_sinf((float)__builtin_amdgcn_fract(fma(phr, z, nth)));
}

template <bool kLinear, int kTier, class Src>
__device__ inline float term32_proj(const Term32& q, int m, ConstStep* __restrict__ st,
                                    const Col4* __restrict__ col, const Src& src, const NodePhase& ph) {
  const StepRec sv = step_at(st, m);
  const float2 cab = col_pair(q, col, m);
  // small form: |phr z_m| < 1/4 and |th| <= 1/2, within the hardware cosine's direct range
  const float fr = kTier == kTierSmall ? fmaf(q.phrf, sv.zmf, -ph.th)
                                       : (float)__builtin_amdgcn_fract(fma(q.phr, sv.zm, ph.nth));
  return amp32<kLinear, kTier>(q, m, sv, cab, src) * __builtin_amdgcn_cosf(fr);
}

// Pass 2 for one chunk of MC steps: out[mm * row] = cq Re(conj(S) term_{m0+mm}), each step in the
// form of the wave's range it falls in (zero past the last step).
template <bool kLinear, int kTier, class Src>
__device__ inline void stage_range32(const Term32& t, int m0, int ma, int mb, const NodePhase& ph,
                                     ConstStep* __restrict__ st, const Col4* __restrict__ col, const Src& src,
                                     float* out) {
#pragma unroll 2
  for (int m = ma; m < mb; ++m) out[(m - m0) * kRow32] = ph.cqs * term32_proj<kLinear, kTier>(t, m, st, col, src, ph);
}

template <bool kLinear, int MC, class Src>
__device__ inline void stage_chunk32(const Term32& t, bool valid, const Split32& sp, int m0, int M, const NodePhase& ph,
                                     ConstStep* __restrict__ st, const Col4* __restrict__ col, const Src& src,
                                     float* out) {
  if (!valid) {  // one branch per chunk, not per step
#pragma unroll
    for (int mm = 0; mm < MC; ++mm) out[mm * kRow32] = 0.0f;
    return;
  }
  const int m1 = min(m0 + MC, M);
  if (sp.small) {
    stage_range32<kLinear, kTierSmall>(t, m0, m0, m1, ph, st, col, src, out);
  } else {
    const int pe = max(m0, min(sp.m_lo, m1)), xe = max(pe, min(sp.m_hi, m1));
    if (pe > m0) stage_range32<kLinear, kTierPoly>(t, m0, m0, pe, ph, st, col, src, out);
    if (xe > pe) stage_range32<kLinear, kTierMixed>(t, m0, pe, xe, ph, st, col, src, out);
    if (m1 > xe) {  // edge form
      const float c = ph.cqs * 0.5f * t.inv_piphr;
      float s0 = edge_sine32(t.phr, xe > 0 ? st[xe - 1].zu : 0.0, ph.nth);
#pragma unroll 2
      for (int m = xe; m < m1; ++m) {
        const float s1 = edge_sine32(t.phr, st[m].zu, ph.nth);
        const float p = __builtin_amdgcn_exp2f(log2p32<kLinear>(t, m, col_pair(t, col, m), src));
        out[(m - m0) * kRow32] = c * (p * (s1 - s0));
        s0 = s1;
      }
    }
  }
  for (int m = m1; m < m0 + MC; ++m) out[(m - m0) * kRow32] = 0.0f;
}

struct AdjArgs {
  PlanView pv;
  FibreParams fp;
  const double* P;
  Work w;
  int nmax;
  unsigned int t_begin, t_end;  // tiles [t_begin, t_end) of the concatenated tile list
};

// kStored: S of every node comes from w.s_store, written by the forward tile kernel for the
// same row batch, instead of a recomputing sweep over the steps.
// kRc: raised-cosine spectra (node shapes in the G products; a separate instantiation)
// kLr: FP32 form with the ODE profile, where each plan has a low-rank table or not (lr_rank): the
// kLr instantiation takes the tiles of plans that have one and evaluates the exponent from it,
// the other takes the remaining tiles with table gathers.  (One kernel holding both step loops
// needs more than 256 VGPRs and runs one wave per SIMD.)
// kWaves: waves per workgroup (4, or 16 with at least 4 waves per SIMD).
template <int kPrec, bool kLinear, bool kStored, bool kRc, bool kLr, int kWaves>
__global__ void __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(kWaves / 4)))
k_adjoint(AdjArgs A) {
  constexpr bool kSplit = kPrec == 0 && !kLinear;
  constexpr int kAdjWaves = kWaves, kAdjBlock = 64 * kAdjWaves;
  using real = typename AdjCfg<kPrec>::real;
  constexpr int MC = AdjCfg<kPrec>::MC;
  constexpr int NG = 64 / MC;  // node groups per wave in the re-mapped phase
  extern __shared__ __align__(16) char smem_raw[];
  const int nmax = A.nmax, GS = A.fp.grid_s, GV = A.fp.grid_v, M = A.fp.n_steps, tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  double* d = reinterpret_cast<double*>(smem_raw);
  const ChanLds ch{d, d + nmax, d + 2 * nmax};
  d += 3 * nmax;
  const RowLds rw{d, d + GS, d + 2 * GS, d + 3 * GS};
  d += 4 * GS;
  double* gGl = d;
  d += nmax;
  double* tacc = d;  // [7][M]: the tile's hot channels k-1, k, k+1, i-1, i, i+1; row 6: the f term
  d += 7 * M;
  double* red = d;  // [kAdjWavesMax]: block_sum
  d += kAdjWavesMax;
  float* lr_bf = reinterpret_cast<float*>(d);  // [kRank]: the tile's f term of the low-rank exponent
  d += kRank / 2;
  d += (d - reinterpret_cast<double*>(smem_raw)) & 1;  // 16-byte boundary for the column tables
  double* lf64 = d;  // [M]: the FP64 form's f-term column
  d += (M + 1) & ~1;
  Col4* col = reinterpret_cast<Col4*>(d);
  constexpr int kRow = stage_row(kPrec);
  real* stage = reinterpret_cast<real*>(col + M);  // [waves][MC][kRow]
  int* meta0 = reinterpret_cast<int*>(stage + kAdjWaves * MC * kRow);
  int* mkey = meta0 + wv * kMetaStride;  // this wave's metadata
  // (t1, t2, w3a, w3c): one 16-byte read per node in the re-map loops
  float4* mtw = reinterpret_cast<float4*>(meta0 + kAdjWaves * kMetaStride) + wv * kMetaStride;
  float2* mff = reinterpret_cast<float2*>(reinterpret_cast<float4*>(meta0 + kAdjWaves * kMetaStride) +
                                          kAdjWaves * kMetaStride) + wv * kMetaStride;  // (f1, f2)
  unsigned int* tile_slot = reinterpret_cast<unsigned int*>(meta0 + 7 * kAdjWaves * kMetaStride);
  const PlanView& pv = A.pv;
  unsigned int* counter = A.w.counter + (kLr ? 3 : 2);
  if (kSplit && !kLr) {  // the gather form: nothing to do when every plan of the range has a table
    int b0, b1, x0, x1, x2;
    decode_tile(pv, A.t_begin, &b0, &x0, &x1, &x2);
    decode_tile(pv, A.t_end - 1, &b1, &x0, &x1, &x2);
    bool any = false;
    for (int b = b0; b <= b1; ++b) any = any || A.w.lr_rank[b] < 0;
    if (!any) return;
  }
  int cur_b = -1;
  for (;;) {
    if (tid == 0) *tile_slot = A.t_begin + atomicAdd(counter, 1u);
    __syncthreads();
    const unsigned int t = *tile_slot;
    if (t >= A.t_end) break;
    int b, i, j, k;
    decode_tile(pv, t, &b, &i, &j, &k);
    const int o = pv.off[b], n = pv.off[b + 1] - o;
    // the tile's upstream weight: the COI's lambda times the weight of its point in the tile row
    const double lam = A.w.lam[o + i] * pv.wpt[(size_t)(o + i) * pv.nli + j];
    const double fnli = pv.fpt[(size_t)(o + i) * pv.nli + j];
    int sf;
    double tf;
    nli_segment(pv.f + o, n, i, fnli, &sf, &tf);
    sf = __builtin_amdgcn_readfirstlane(sf);  // tile-uniform: scalar registers
    tf = uniform_f64(tf);
    // COI outside the throughput (an empty channel): nothing flows back; and the split form's
    // tiles of the other instantiation
    if (lam == 0.0 || (kSplit && (__builtin_amdgcn_readfirstlane(A.w.lr_rank[b]) >= 0) != kLr)) {
      __syncthreads();
      continue;
    }
    if (b != cur_b) {
      load_channels(ch, pv, A.P, o, n, A.fp.rolloff);
      cur_b = b;
    }
    // (kLr reads no columns, but skipping the load moves the register allocation to more spills)
    if (kPrec == 0) load_cols<kLinear>(col, A.w.lt32 + (size_t)M * o, n, M, sf, tf, k);
    if (kLr) lowrank_f_term(A.w.lr_b + (size_t)kRank * o, sf, (float)tf, lr_bf);  // (the f term only)
    // the plan's step records: wave-uniform reads through scalar loads
    ConstStep* stc = (ConstStep*)(A.w.step_rec + (size_t)4 * M * b);
    if (kPrec == 1 && !kLinear) load_fcol64(lf64, A.w.ell64 + (size_t)M * o, n, M, sf, tf);
    for (int c = tid; c < n; c += kAdjBlock) gGl[c] = 0.0;
    for (int q = tid; q < 7 * M; q += kAdjBlock) tacc[q] = 0.0;
    __syncthreads();
    const TileGeo g = uniform_geo(tile_geo(ch, n, fnli, k, A.fp.f_ref));
    const double* zm = A.w.zm + (size_t)b * M;
    const double* dz = A.w.dz + (size_t)b * M;
    const float* hdz = A.w.hdz32 + (size_t)b * M;
    double* gL = A.w.gL + (size_t)M * o;  // [c][m]
    // Most f1/f2 runs sit next to the interferer or the COI (rows near the axes): their sums go
    // to per-tile LDS rows and reach HBM once per tile; other channels go straight to HBM.
    const int hot[6] = {k - 1, k, k + 1, i - 1, i, i + 1};
    double gk_acc = 0.0;
    for (int part = kQ1; part <= kQ4; ++part) {
      if (!layout_rows(rw, g, part, GS, GV, A.fp.s_decades)) continue;
      __syncthreads();
      const int64_t nodes = (int64_t)GS * GV;
      for (int64_t base = 0; base < nodes; base += kAdjBlock) {
        const int64_t q = base + tid;
        Node nd;
        // (the FP32 form's segment weights as the forward kernel forms them)
        const bool valid =
            q < nodes && make_node<kPrec == 0>(ch, rw, g, n, k, part, (int)(q / GV), (int)(q % GV), A.fp, &nd);
        // raised-cosine shapes at f1, f2, f3 relative to the flat PSDs (1: rectangle)
        double sh1 = 1.0, sh2 = 1.0, sh3 = 1.0;
        if (kRc && valid)
          node_shapes(ch, rw, g, k, part, (int)(q / GV), (int)(q % GV), nd.c1, nd.c2, A.fp.rolloff, &sh1, &sh2, &sh3);
        // per-node values used after pass 1 (taken now: the node's other fields die here)
        const real cq = valid ? (real)(lam * nd.w * nd.gprod * (sh1 * sh2 * sh3)) : (real)0;
        const double lw = valid ? lam * nd.w : 0.0;
        const int c1 = valid ? nd.c1 : 0, c2 = valid ? nd.c2 : 0;
        const float wgt = kLinear ? 2.0f : 1.0f;
        int gkey, g1lo, g1hi, g2lo, g2hi;
        bool one_run, two_valued;
        {
          const int jm = lane + lane / MC;
          int key = -1;
          float w3a = 0.0f, w3c = 0.0f;
          if (valid) {
            const float t3 = (float)nd.t3;
            if (n > 1) {
              const bool lower = nd.s3 < k;  // segment (k-1, k) or (k, k+1)
              w3a = lower ? wgt * (1.0f - t3) : 0.0f;
              w3c = lower ? 0.0f : wgt * t3;
            }
            key = kLinear ? -1 : (nd.s1 | (nd.s2 << 16));
          }
          mkey[jm] = key;
          mtw[jm] = valid ? make_float4((float)nd.t1, (float)nd.t2, w3a, w3c) : make_float4(0.0f, 0.0f, w3a, w3c);
          // Most groups of MC nodes lie in one f1 segment and one f2 segment (one run each); nearly
          // all the others in two of each.  Waves whose groups all do take branch-free re-maps.
          const int s1v = key >= 0 ? (key & 0xffff) : -1, s2v = key >= 0 ? (key >> 16) : -1;
          int lo1 = key >= 0 ? s1v : 0x7fffffff, hi1 = s1v, lo2 = key >= 0 ? s2v : 0x7fffffff, hi2 = s2v;
#pragma unroll
          for (int sh = 1; sh < MC; sh <<= 1) {
            lo1 = min(lo1, __shfl_xor(lo1, sh));
            hi1 = max(hi1, __shfl_xor(hi1, sh));
            lo2 = min(lo2, __shfl_xor(lo2, sh));
            hi2 = max(hi2, __shfl_xor(hi2, sh));
          }
          g1lo = lo1;
          g1hi = hi1;  // -1: no node of the group on the support
          g2lo = lo2;
          g2hi = hi2;
          gkey = hi1 >= 0 ? (hi1 | (hi2 << 16)) : -1;  // the group's key when it has one run
          one_run = hi1 < 0 || (lo1 == hi1 && lo2 == hi2);
          two_valued = key < 0 || ((s1v == lo1 || s1v == hi1) && (s2v == lo2 || s2v == hi2));
          mff[jm] = make_float2(key >= 0 && s1v == hi1 && hi1 != lo1 ? 1.0f : 0.0f,
                                key >= 0 && s2v == hi2 && hi2 != lo2 ? 1.0f : 0.0f);
        }
        const bool wave_one_run = __all(one_run);
        const bool wave_two_valued = !wave_one_run && __all(two_valued);
        // pass 1: S
        real sr = 0, si = 0;
        Term32 t32{};
        Term64 t64;
        if (valid && kPrec == 0) t32 = term32_setup(nd, k, n);
        Split32 sp{};
        if (kPrec == 0) sp = wave_split(valid, t32, stc, M);
        // the exponent of the FP32 form: the f1 + f2 profile terms by table gathers, or the whole
        // exponent from the low-rank table (its step factors through scalar loads)
        const Gather32 gsrc{make_tab32(A.w.lt32 + (size_t)M * o, n, M), n};
        LowRank32 lsrc;
        if constexpr (kLr) {
          lsrc.a = const_f32(A.w.lr_a + (size_t)M * kRank * b);
          int sa, sb;
          col_segments(k, n, &sa, &sb);
          // the f3 segment's row straight from global memory: staging it in LDS like the forward
          // does moves this kernel's register allocation to more spills and runs slower
          lsrc.setup<true>(t32, A.w.lr_b + (size_t)kRank * o, A.w.lr_b + (size_t)kRank * (o + (t32.up3 ? sb : sa)),
                           lr_bf);
        }
        if (valid) {
          if (kStored) {
            const int64_t slot = ((int64_t)(t - A.t_begin) * 3 + part) * nodes + q;
            if constexpr (kPrec == 0) {
              const float2 sv = static_cast<const float2*>(A.w.s_store)[slot];
              sr = sv.x;
              si = sv.y;
            } else {
              const double2 sv = static_cast<const double2*>(A.w.s_store)[slot];
              sr = sv.x;
              si = sv.y;
            }
            if (kPrec == 1) t64 = term64_setup(nd);
          } else if (kPrec == 0) {
            float a32, b32;
            if constexpr (kLr) accumulate32<kLinear, 4>(t32, sp, stc, col, lsrc, M, &a32, &b32);
            else accumulate32<kLinear, 4>(t32, sp, stc, col, gsrc, M, &a32, &b32);
            sr = a32;
            si = b32;
          } else {
            t64 = term64_setup(nd);
            const double* tab = A.w.ell64 + (size_t)M * o;
            for (int m = 0; m < M; ++m) {
              const double2 a = term64<kLinear>(t64, m, zm, dz, tab, n, lf64);
              sr += a.x;
              si += a.y;
            }
          }
          const double s2 = (double)sr * sr + (double)si * si;
          const double base2 = lw * s2, p1 = ch.psd[c1], p2 = ch.psd[c2];
          if constexpr (kRc) {  // dG(f)/dP_c = shape / R_c: the shape of the differentiated factor
            const double g1 = p1 * sh1, g2 = p2 * sh2, g3 = g.gk * sh3;
            atomicAdd(&gGl[c1], base2 * sh1 * g2 * g3);
            atomicAdd(&gGl[c2], base2 * sh2 * g1 * g3);
            gk_acc += base2 * g1 * g2 * sh3;
          } else {
            atomicAdd(&gGl[c1], base2 * p2 * g.gk);
            atomicAdd(&gGl[c2], base2 * p1 * g.gk);
            gk_acc += base2 * p1 * p2;
          }
        }
        real* my_stage = stage + (size_t)wv * MC * kRow;
        NodePhase ph{0.0f, 0.0f, 0.0};
        if (kPrec == 0 && valid) {
          ph.cqs = (float)((double)cq * sqrt((double)sr * sr + (double)si * si));
          ph.th = atan_rev32((float)si, (float)sr);
          ph.nth = -(double)ph.th;
        }
        // pass 2 in chunks of MC steps
        for (int m0 = 0; m0 < M; m0 += MC) {
          if (kPrec == 0) {
            float* out = reinterpret_cast<float*>(my_stage) + lane;
            if constexpr (kLr)
              stage_chunk32<kLinear, MC>(t32, valid, sp, m0, M, ph, stc, col, lsrc, out);
            else
              stage_chunk32<kLinear, MC>(t32, valid, sp, m0, M, ph, stc, col, gsrc, out);
          } else {
            for (int mm = 0; mm < MC; ++mm) {
              const int m = m0 + mm;
              real qv = 0;
              if (valid && m < M) {
                const double2 a = term64<kLinear>(t64, m, zm, dz, A.w.ell64 + (size_t)M * o, n, lf64);
                qv = (real)(cq * (sr * a.x + si * a.y));
              }
              my_stage[mm * kRow + lane] = qv;
            }
          }
          __syncwarp();
          // re-mapped phase: lane -> (step m0 + mm, node group gr)
          {
            const int mm = lane % MC, gr = lane / MC, m = m0 + mm;
            const bool live = m < M;
            const int jb = gr * (MC + 1);
            const real* qrow = my_stage + mm * kRow + gr * MC;
            int cur1 = -1, cur2 = -1;
            // run sums in the form's precision (at most MC nodes each), flushed to FP64:
            // a = sum q, ah = sum q t; the segment's lower channel gets a - ah, the upper ah
            real a1 = 0, a1h = 0, a2 = 0, a2h = 0, qs = 0, x3a = 0, x3c = 0;
            auto put = [=](int c, double v) {
              // the hot rows: k-1, k, k+1 (rows 0-2), then i-1, i, i+1 (rows 3-5); the first wins
              const unsigned dk = (unsigned)(c - k + 1), di = (unsigned)(c - i + 1);
              const int hs = dk < 3u ? (int)dk : (di < 3u ? 3 + (int)di : -1);
              // distinct scopes keep the LDS and global adds apart (no flat atomic)
              if (hs >= 0) __hip_atomic_fetch_add(&tacc[hs * M + m], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
              else __hip_atomic_fetch_add(&gL[(size_t)c * M + m], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            };
            auto flush = [=](int cur, real a, real ah) {
              if (!live || cur < 0) return;
              put(cur, (double)(a - ah));
              if (n > 1) put(cur + 1, (double)ah);
            };
            if (wave_one_run) {
              auto node = [&](int it, real qv) {
                const float4 tw = mtw[jb + it];
                qs += qv;
                x3a += qv * (real)tw.z;
                x3c += qv * (real)tw.w;
                if (!kLinear) {
                  a1h += qv * (real)tw.x;
                  a2h += qv * (real)tw.y;
                }
              };
              if constexpr (kPrec == 0) {
#pragma unroll 2
                for (int i4 = 0; i4 < MC; i4 += 4) {
                  real q4[4];
                  load_q4<kPrec>(qrow + i4, q4);
#pragma unroll
                  for (int j = 0; j < 4; ++j) node(i4 + j, q4[j]);
                }
              } else {  // (the FP64 form's registers allow no more than the plain loop)
#pragma unroll 4
                for (int it = 0; it < MC; ++it) node(it, qrow[it]);
              }
              if (!kLinear && gkey >= 0) {
                flush(gkey & 0xffff, qs, a1h);
                flush(gkey >> 16, qs, a2h);
              }
            } else if (kPrec == 0 && !kLinear && wave_two_valued) {
              // two runs at most per segment key: the upper run's sums are selected by the
              // node's 0/1 flag, the lower run's are the rest
              real b1 = 0, b1h = 0, b2 = 0, b2h = 0;
#pragma unroll 2
              for (int i4 = 0; i4 < MC; i4 += 4) {
                real q4[4];
                load_q4<kPrec>(qrow + i4, q4);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                  const real qv = q4[j];
                  const float4 tw = mtw[jb + i4 + j];
                  const float2 ff = mff[jb + i4 + j];
                  qs += qv;
                  x3a += qv * (real)tw.z;
                  x3c += qv * (real)tw.w;
                  const real u1 = qv * (real)tw.x, u2 = qv * (real)tw.y;
                  a1h += u1;
                  a2h += u2;
                  b1 += qv * (real)ff.x;
                  b1h += u1 * (real)ff.x;
                  b2 += qv * (real)ff.y;
                  b2h += u2 * (real)ff.y;
                }
              }
              if (g1hi >= 0) {
                flush(g1lo, qs - b1, a1h - b1h);
                if (g1hi != g1lo) flush(g1hi, b1, b1h);
                flush(g2lo, qs - b2, a2h - b2h);
                if (g2hi != g2lo) flush(g2hi, b2, b2h);
              }
            } else {
#pragma unroll 4
              for (int it = 0; it < MC; ++it) {
                const real qv = qrow[it];
                qs += qv;
                const float4 tw = mtw[jb + it];
                x3a += qv * (real)tw.z;
                x3c += qv * (real)tw.w;
                if (!kLinear) {
                  const int key = mkey[jb + it];
                  if (key >= 0) {
                    const int s1 = key & 0xffff, s2 = key >> 16;
                    if (s1 != cur1) {
                      flush(cur1, a1, a1h);
                      cur1 = s1;
                      a1 = a1h = (real)0;
                    }
                    if (s2 != cur2) {
                      flush(cur2, a2, a2h);
                      cur2 = s2;
                      a2 = a2h = (real)0;
                    }
                    a1 += qv;
                    a1h += qv * (real)tw.x;
                    a2 += qv;
                    a2h += qv * (real)tw.y;
                  }
                }
              }
              if (!kLinear) {
                flush(cur1, a1, a1h);
                flush(cur2, a2, a2h);
              }
            }
            if (live) {
              atomicAdd(&tacc[0 * M + m], (double)x3a);
              atomicAdd(&tacc[1 * M + m], (double)((real)wgt * qs - x3a - x3c));
              atomicAdd(&tacc[2 * M + m], (double)x3c);
              if (!kLinear) atomicAdd(&tacc[6 * M + m], -(double)qs);  // the f term (row 6)
            }
          }
          __syncwarp();  // the next chunk overwrites this wave's staging
        }
      }
      __syncthreads();
    }
    // tile end: flush the per-tile accumulators
    gk_acc = block_sum(gk_acc, red);
    if (tid == 0) gGl[k] += gk_acc;
    // the f term to the NLI frequency's segment (sf, sf + 1), both among the COI's hot rows
    for (int m = tid; m < M && !kLinear; m += kAdjBlock) {
      const double v = tacc[6 * M + m];
      if (tf == 0.0) {
        tacc[(sf - i + 4) * M + m] += v;
      } else {
        tacc[(sf - i + 4) * M + m] += (1.0 - tf) * v;
        tacc[(sf - i + 5) * M + m] += tf * v;
      }
    }
    __syncthreads();
    for (int c = tid; c < n; c += kAdjBlock)
      if (gGl[c] != 0.0) atomicAdd(&A.w.gG[o + c], gGl[c]);
    for (int q = tid; q < 6 * M; q += kAdjBlock) {
      const int c = hot[q / M], m = q % M;
      const double v = tacc[q];
      if (v != 0.0 && c >= 0 && c < n) atomicAdd(&gL[(size_t)c * M + m], v);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------- profile adjoint
// Closed form: ln rho(z_m, f_c) = -alpha z_m - a_m (f_c - f_ref) - ln N_m with
// a_m = P_tot C_r L_eff(z_m), N_m = sum_j (P_j/P_tot) E_j(a_m), E_j(a) = exp(-a d_j) M_j(a) (M_j the
// spectrum's transform: sinhc(a R_j/2) for the rectangle).
// With A1_m = sum_c dT/dln rho(m,c) and A2_m = sum_c dT/dln rho(m,c) (f_c - f_ref):
//   dT/dP_j += sum_m [ -A2_m C L_m - A1_m ((E_j(a_m)/N_m - 1)/P_tot + C L_m D_m / N_m) ],
//   D_m = sum_j (P_j/P_tot) E_j'(a_m).  Row m == M is the span end.
__device__ inline double Ej(double a, double dj, double Rj, double beta) {
  return exp(-a * dj) * spectrum_m(a, Rj, beta);
}
__device__ inline double Ejd(double a, double dj, double Rj, double beta) {
  return exp(-a * dj) * (-dj * spectrum_m(a, Rj, beta) + spectrum_md(a, Rj, beta));
}

__global__ void k_cf_adj_rows(PlanView pv, FibreParams fp, const double* __restrict__ P, Work w, double* coef) {
  __shared__ double red[16];
  const int m = blockIdx.x, b = blockIdx.y, o = pv.off[b], n = pv.off[b + 1] - o, M = fp.n_steps;
  const double z = m < M ? w.zm[b * M + m] : fp.span;
  const double alpha = pv.alpha[o], cr = pv.cr[o];
  double pt = 0.0, A1 = 0.0, A2 = 0.0;
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    pt += P[o + c];
    const double gl = m < M ? w.gL[(size_t)M * o + (size_t)c * M + m] : w.gLL[o + c];
    A1 += gl;
    A2 += gl * (pv.f[o + c] - fp.f_ref);
  }
  pt = block_sum(pt, red);
  A1 = block_sum(A1, red);
  A2 = block_sum(A2, red);
  double a = 0.0, N = 1.0, D = 0.0, CL = 0.0;
  if (pt > 0.0) {
    CL = cr * (alpha > 0 ? -expm1(-alpha * z) / alpha : z);
    a = pt * CL;
    double sN = 0.0, sD = 0.0;
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
      const double dj = pv.f[o + c] - fp.f_ref, Rj = pv.R[o + c], wj = P[o + c] / pt;
      sN += wj * Ej(a, dj, Rj, fp.rolloff);
      sD += wj * Ejd(a, dj, Rj, fp.rolloff);
    }
    N = block_sum(sN, red);
    D = block_sum(sD, red);
  }
  if (threadIdx.x == 0) {
    double* cf = coef + ((size_t)b * (M + 1) + m) * 8;
    cf[0] = a; cf[1] = N; cf[2] = D; cf[3] = A1; cf[4] = A2; cf[5] = CL; cf[6] = pt;
  }
}

__global__ void k_cf_adj_channels(PlanView pv, FibreParams fp, Work w, const double* coef) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= pv.n_total) return;
  const int b = plan_of_channel(pv, g), M = fp.n_steps;
  const double dj = pv.f[g] - fp.f_ref, Rj = pv.R[g];
  double acc = 0.0;
  for (int m = 0; m <= M; ++m) {
    const double* cf = coef + ((size_t)b * (M + 1) + m) * 8;
    const double a = cf[0], N = cf[1], D = cf[2], A1 = cf[3], A2 = cf[4], CL = cf[5], pt = cf[6];
    if (!(pt > 0.0)) continue;
    acc += -A2 * CL - A1 * ((Ej(a, dj, Rj, fp.rolloff) / N - 1.0) / pt + CL * D / N);
  }
  w.gP[g] += acc;
}

// RK4 ODE adjoint, one block of 1024 threads per plan.  The forward stored ell at the start of
// every sub-step; going backwards, each sub-step recomputes its stages and applies the exact
// transpose of RK4, with the vector-Jacobian product of f_k(ell) = -alpha_k + sum_j g_kj P_j e^ell_j:
//   (J^T v)_j = P_j e^ell_j s_j,  dT/dP_j += e^ell_j s_j,  s_j = sum_k g_kj v_k,
// where k ranges over j's loss window (k gains from j) and gain window (k feeds j); s_j comes from
// prefix sums of C_r,k v_k, C_r,k v_k (f_k - f_mid), C_r,k v_k (f_k - f_mid)^2.
__device__ inline double ode_rhs_a(const OdeChan& ch, int c, double ell, bool active, int photon, OdeShared& sh) {
  double p = active ? ch.p0 * exp(ell) : 0.0;
  double a = p, bb = ch.ft * p, cc = active ? p / ch.f : 0.0;
  block_scan3(a, bb, cc, sh);
  __syncthreads();
  if (active) { sh.sA[c] = a; sh.sB[c] = bb; sh.sC[c] = cc; }
  __syncthreads();
  double r = 0.0;
  if (active) {
    double gA, gB, gC, lA, lB, lC;
    window_above(sh, ch, c, &gA, &gB, &gC);
    window_below(sh, ch, c, &lA, &lB, &lC);
    const double gain = ch.cr * (gB - ch.ft * gA);
    const double loss = photon ? ch.cr * ch.f * (ch.f * lC - lA) : ch.cr * (ch.ft * lA - lB);
    r = -ch.alpha + gain - loss;
  }
  __syncthreads();
  return r;
}

// Returns e^ell s (so that J^T v = P0 * result and dT/dP0 += result).
__device__ inline double ode_vjp(const OdeChan& ch, int c, double ell, double v, bool active, int photon,
                                 double fmid, OdeShared& sh) {
  const double wv = active ? ch.cr * v : 0.0;
  double a = wv, bb = wv * ch.ft, cc = wv * ch.ft * ch.ft;
  block_scan3(a, bb, cc, sh);
  __syncthreads();
  if (active) { sh.sA[c] = a; sh.sB[c] = bb; sh.sC[c] = cc; }
  __syncthreads();
  double r = 0.0;
  if (active) {
    double gA, gB, gC, lA, lB, lC;
    window_below(sh, ch, c, &lA, &lB, &lC);  // k gains from c
    window_above(sh, ch, c, &gA, &gB, &gC);  // k feeds c
    double s = ch.ft * lA - lB;
    if (photon) s -= (gC + (fmid - ch.ft) * gB - ch.ft * fmid * gA) / ch.f;
    else s -= gB - ch.ft * gA;
    r = exp(ell) * s;
  }
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(1024) k_ode_adjoint(PlanView pv, FibreParams fp, const double* __restrict__ P,
                                                      Work w) {
  __shared__ OdeShared sh;
  const int b = blockIdx.x, o = pv.off[b], n = pv.off[b + 1] - o, M = fp.n_steps, c = threadIdx.x;
  const bool active = c < n;
  const double fmid = 0.5 * (pv.f[o] + pv.f[o + n - 1]);
  OdeChan ch{};
  if (active) ch = ode_chan(pv, fp, P, o, n, c, fmid);
  const int sub = fp.ode_sub, ph = fp.photon_ratio;
  const double* st = w.states + w.state_off[b];
  double yb = active ? w.gLL[o + c] : 0.0, pb = 0.0;
  int step = M * 2 * sub;
  for (int m = M - 1; m >= 0; --m) {
    const double h = w.dz[b * M + m] / (2.0 * sub);
    for (int half = 1; half >= 0; --half) {
      if (half == 0 && active) yb += w.gL[(size_t)M * o + (size_t)c * M + m];  // ell recorded at z_m
      for (int q = 0; q < sub; ++q) {
        --step;
        const double y = active ? st[(size_t)step * n + c] : 0.0;
        const double k1 = ode_rhs_a(ch, c, y, active, ph, sh);
        const double u2 = y + 0.5 * h * k1;
        const double k2 = ode_rhs_a(ch, c, u2, active, ph, sh);
        const double u3 = y + 0.5 * h * k2;
        const double k3 = ode_rhs_a(ch, c, u3, active, ph, sh);
        const double u4 = y + h * k3;
        double kb4 = yb * (h / 6.0), kb3 = yb * (h / 3.0), kb2 = yb * (h / 3.0), kb1 = yb * (h / 6.0);
        double ybn = yb;
        double e = ode_vjp(ch, c, u4, kb4, active, ph, fmid, sh);
        ybn += ch.p0 * e; kb3 += h * ch.p0 * e; pb += e;
        e = ode_vjp(ch, c, u3, kb3, active, ph, fmid, sh);
        ybn += ch.p0 * e; kb2 += 0.5 * h * ch.p0 * e; pb += e;
        e = ode_vjp(ch, c, u2, kb2, active, ph, fmid, sh);
        ybn += ch.p0 * e; kb1 += 0.5 * h * ch.p0 * e; pb += e;
        e = ode_vjp(ch, c, y, kb1, active, ph, fmid, sh);
        ybn += ch.p0 * e; pb += e;
        yb = ybn;
      }
    }
  }
  if (active) w.gP[o + c] += pb;
}

__global__ void k_grad_final(PlanView pv, Work w, double* dthr) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= pv.n_total) return;
  dthr[g] = w.gP[g] + w.gG[g] / pv.R[g];
}

}  // namespace

size_t adjoint_lds(int nmax, int gs, int M, int prec) { return adjoint_lds_bytes(nmax, gs, M, prec, 4); }

namespace {
using AdjKernel = void (*)(AdjArgs);
// (the low-rank instantiation exists for the FP32 form with the ODE profile only)
// [low-rank][wide]: the sixteen-wave form exists for the FP32 form with the stored S only (the
// narrow kernel stands in elsewhere); the low-rank one for the FP32 form with the ODE profile
#define ISRSGN_ADJ_LW(P, L, S, RC)                                                                 \
  {{k_adjoint<P, L, S, RC, false, 4>, k_adjoint<P, L, S, RC, false, (P == 0 && S) ? 16 : 4>},       \
   {k_adjoint<P, L, S, RC, P == 0 && !L, 4>, k_adjoint<P, L, S, RC, P == 0 && !L, (P == 0 && S) ? 16 : 4>}}
#define ISRSGN_ADJ(P, RC)                                                                          \
  {{ISRSGN_ADJ_LW(P, false, false, RC), ISRSGN_ADJ_LW(P, false, true, RC)},                        \
   {ISRSGN_ADJ_LW(P, true, false, RC), ISRSGN_ADJ_LW(P, true, true, RC)}}
// [precision][raised cosine][linear profile][stored S][low-rank][wide]
const AdjKernel kAdjKernels[2][2][2][2][2][2] = {{ISRSGN_ADJ(0, false), ISRSGN_ADJ(0, true)},
                                                 {ISRSGN_ADJ(1, false), ISRSGN_ADJ(1, true)}};

// FP32 form with the ODE profile: the tiles are split between the low-rank and gather forms
bool adjoint_split(const FibreParams& fp) { return fp.precision == 0 && fp.profile != 0; }

// Waves per workgroup: sixteen for the FP32 form with the stored S when that layout's LDS fits
// (unless fp.adj_wide is off), else four
int adjoint_waves(const FibreParams& fp, int nmax, bool stored, size_t lds_max) {
  const bool wide = fp.adj_wide && fp.precision == 0 && stored &&
                    adjoint_lds_bytes(nmax, fp.grid_s, fp.n_steps, 0, 16) <= lds_max;
  return wide ? 16 : 4;
}

const void* adjoint_kernel(const FibreParams& fp, bool stored, bool lr, int waves) {
  return reinterpret_cast<const void*>(kAdjKernels[fp.precision ? 1 : 0][fp.rolloff > 0.0 ? 1 : 0][fp.profile == 0 ? 1 : 0]
                                                  [stored ? 1 : 0][lr && adjoint_split(fp) ? 1 : 0][waves == 16 ? 1 : 0]);
}
}  // namespace

int adjoint_blocks_per_cu(const FibreParams& fp, int nmax, bool stored, size_t lds_max) {
  int nb = 0;
  const int waves = adjoint_waves(fp, nmax, stored, lds_max);
  const size_t shm = adjoint_lds_bytes(nmax, fp.grid_s, fp.n_steps, fp.precision, waves);
  // the split form's two instantiations launch with the same grid: the fewer blocks of the two
  for (int lr = 0; lr <= (adjoint_split(fp) ? 1 : 0); ++lr) {
    const void* k = adjoint_kernel(fp, stored, lr != 0, waves);
    // above 64 KiB the kernel must opt in before the occupancy query counts its blocks
    if (shm > 65536) (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k, 64 * waves, shm) != hipSuccess || b < 1) b = 1;
    nb = lr == 0 ? b : std::min(nb, b);
  }
  return nb;
}

hipError_t launch_grad_init(const PlanView& pv, const FibreParams& fp, const Work& w, hipStream_t s) {
  const int64_t ngl = (int64_t)fp.n_steps * pv.n_total;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((ngl + 255) / 256 < 4096 ? (ngl + 255) / 256 : 4096)), dim3(256), 0, s,
                     w.gL, ngl);
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((pv.n_total + 255) / 256)), dim3(256), 0, s, w.gG, (int64_t)pv.n_total);
  return hipGetLastError();
}

hipError_t launch_grad_rows(const PlanView& pv, const FibreParams& fp, const double* P, const double* nf,
                            double snr_trx, const Work& w, int g_begin, int g_end, hipStream_t s) {
  if (g_end <= g_begin) return hipSuccess;
  hipLaunchKernelGGL(k_grad_prep, dim3((unsigned)((g_end - g_begin + 255) / 256)), dim3(256), 0, s, pv, P, nf,
                     snr_trx, w, g_begin, g_end, fp.n_spans);
  return hipGetLastError();
}

hipError_t launch_adjoint_tiles(const PlanView& pv, const FibreParams& fp, const double* P, const Work& w, int nmax,
                                int grid, unsigned int t_begin, unsigned int t_end, bool stored, size_t lds_max,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_zero_counter2, dim3(1), dim3(1), 0, s, w.counter + 2);
  AdjArgs a{pv, fp, P, w, nmax, t_begin, t_end};
  const int waves = adjoint_waves(fp, nmax, stored, lds_max);
  const size_t shm = adjoint_lds_bytes(nmax, fp.grid_s, fp.n_steps, fp.precision, waves);
  // split form: the low-rank instantiation (its own tile counter), then the gather one, which
  // returns at once when every plan of the range has a low-rank table
  for (int lr = adjoint_split(fp) && fp.lowrank > 0 ? 1 : 0; lr >= 0; --lr) {
    const void* k = adjoint_kernel(fp, stored, lr != 0, waves);
    if (shm > 65536) (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    void* args[] = {&a};
    const hipError_t e = hipLaunchKernel(k, dim3(grid), dim3(64 * waves), args, shm, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t launch_grad_finish(const PlanView& pv, const FibreParams& fp, const double* P, const Work& w,
                              double* coef, double* dthr, hipStream_t s) {
  const int M = fp.n_steps;
  if (fp.profile == 0) {
    hipLaunchKernelGGL(k_cf_adj_rows, dim3(M + 1, pv.n_batch), dim3(256), 0, s, pv, fp, P, w, coef);
    hipLaunchKernelGGL(k_cf_adj_channels, dim3((pv.n_total + 255) / 256), dim3(256), 0, s, pv, fp, w,
                       (const double*)coef);
  } else {
    hipLaunchKernelGGL(k_ode_adjoint, dim3(pv.n_batch), dim3(1024), 0, s, pv, fp, P, w);
  }
  hipLaunchKernelGGL(k_grad_final, dim3((pv.n_total + 255) / 256), dim3(256), 0, s, pv, w, dthr);
  return hipGetLastError();
}


}  // namespace isrsgn
