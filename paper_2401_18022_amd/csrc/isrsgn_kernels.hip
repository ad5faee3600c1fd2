// HIP kernels of libisrsgn.so for gfx950 (MI355X): setup, distance steps, power
// profile, COI x interferer pair integrals, and the NLI / SNR / throughput reduction.
//
// Model: arXiv:2401.18022 -- eq. (new_gn_model) with the step sum of eq. (slow_vary),
// the power term of eq. (pk), the phase mismatch of eq. (phi), hyperbolic coordinates
// of eqs. (q1)-(q4), assembly eqs. (gain_fin)/(psi_fin), cost eq. (loss).
#include "isrsgn_device.h"

namespace isrsgn {
namespace {

// ---------------------------------------------------------------------------- setup (Sec. II)

__device__ inline double gamma_at(const FibreParams& fp, double f) {  // eq. (gamma)
  return fp.gamma_const > 0 ? fp.gamma_const : 2.0 * kPi * fp.n2 * f / (kC * tab_at(fp.n_tab, fp.tab_f, fp.tab_aeff, f));
}

__global__ void k_channel_setup(PlanView pv, FibreParams fp) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= pv.n_total) return;
  double f = pv.f[c];
  double a = tab_at(fp.n_tab, fp.tab_f, fp.tab_alpha, f);
  double ae = tab_at(fp.n_tab, fp.tab_f, fp.tab_aeff, f);
  pv.alpha[c] = a;
  pv.aeff[c] = ae;
  const double gc = fp.gamma_const > 0 ? fp.gamma_const : 2.0 * kPi * fp.n2 * f / (kC * ae);  // eq. (gamma)
  pv.gamma[c] = gc;
  pv.cr[c] = fp.cr * fp.aeff_ref / ae;  // Raman gain scaled by A_eff at the channel frequency
  // the within-channel NLI rule: nli midpoints of equal parts of the support (1 + beta) R, weights
  // proportional to the receiver response (the spectrum's shape) and normalised to R, each point's
  // tiles weighted by gamma(f_j)^2: w_j = q_j gamma(f_j)^2 / (gamma_c^2 R_c); one point: f_c, weight 1
  const int J = fp.nli;
  const double R = pv.R[c], d = (1.0 + fp.rolloff) * R / J;
  double sum = 0.0;
  for (int j = 0; j < J; ++j) sum += fp.rolloff > 0.0 ? rc_shape(f + (j + 0.5 - 0.5 * J) * d - f, R, fp.rolloff) : 1.0;
  for (int j = 0; j < J; ++j) {
    const double fj = f + (j + 0.5 - 0.5 * J) * d;
    const double q = (fp.rolloff > 0.0 ? rc_shape(fj - f, R, fp.rolloff) : 1.0) / sum;
    const double gr = gc > 0.0 ? gamma_at(fp, fj) / gc : 1.0;
    pv.fpt[(size_t)c * J + j] = fj;
    pv.wpt[(size_t)c * J + j] = q * gr * gr;
  }
}

// ---------------------------------------------------------------------------- distance steps
// Equal power decrement per step under the mean loss of the occupied channels, midpoints
// as evaluation points (eqs. slow_vary0-slow_vary).  One block per plan.
__global__ void k_steps(PlanView pv, FibreParams fp, const double* __restrict__ P, Work w) {
  __shared__ double red[16];
  const int b = blockIdx.x, o = pv.off[b], n = pv.off[b + 1] - o, M = fp.n_steps;
  double sa = 0.0, cnt = 0.0, sall = 0.0;
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    double a = pv.alpha[o + c];
    sall += a;
    if (P[o + c] > 0.0) { sa += a; cnt += 1.0; }
  }
  sa = block_sum(sa, red);
  cnt = block_sum(cnt, red);
  sall = block_sum(sall, red);
  const double ab = cnt > 0 ? sa / cnt : sall / n;
  if (threadIdx.x == 0) w.abar[b] = ab;
  const double L = fp.span, q = -expm1(-ab * L);
  auto edge = [&](int j) -> double {
    if (j >= M) return L;
    if (ab * L < 1e-12) return L * j / M;
    return -log1p(-q * j / (double)M) / ab;
  };
  for (int m = threadIdx.x; m < M; m += blockDim.x) {
    double z0 = edge(m), z1 = edge(m + 1);
    w.zm[b * M + m] = 0.5 * (z0 + z1);
    w.dz[b * M + m] = z1 - z0;
    w.hdz32[b * M + m] = (float)(0.5 * (z1 - z0));
    reinterpret_cast<StepRec*>(w.step_rec)[b * M + m] =
        step_record(0.5 * (z0 + z1), z1 - z0, (float)(0.5 * (z1 - z0)));
  }
}

// ---------------------------------------------------------------------------- power profile
// Closed form (linear Raman slope, uniform loss):
//   ln rho(z,F) = -alpha z - a (F - f_ref) - ln sum_j (P_j/P_tot) exp(-a (f_j - f_ref)) M_j(a)
// with M_j the transform of channel j's spectrum (sinhc(a R_j/2) for the rectangle)
//   a = P_tot C_r L_eff(z).  Grid (M + 1, n_batch): row M is the span end.
__global__ void k_profile_closed_form(PlanView pv, FibreParams fp, const double* __restrict__ P, Work w) {
  __shared__ double red[16];
  const int m = blockIdx.x, b = blockIdx.y, o = pv.off[b], n = pv.off[b + 1] - o, M = fp.n_steps;
  const double z = m < M ? w.zm[b * M + m] : fp.span;
  const double alpha = pv.alpha[o], cr = pv.cr[o];
  double pt = 0.0;
  for (int c = threadIdx.x; c < n; c += blockDim.x) pt += P[o + c];
  pt = block_sum(pt, red);
  double a = 0.0, lnn = 0.0;
  if (pt > 0.0) {
    const double leff = alpha > 0 ? -expm1(-alpha * z) / alpha : z;
    a = pt * cr * leff;
    double s = 0.0;
    for (int c = threadIdx.x; c < n; c += blockDim.x)
      s += P[o + c] / pt * exp(-a * (pv.f[o + c] - fp.f_ref)) * spectrum_m(a, pv.R[o + c], fp.rolloff);
    s = block_sum(s, red);
    lnn = log(s);
  }
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    double l = -alpha * z - a * (pv.f[o + c] - fp.f_ref) - lnn;
    if (m < M) w.ell64[(size_t)M * o + (size_t)m * n + c] = l;
    else w.ellL[o + c] = l;
  }
}


// Raman power-evolution ODEs for ell_k = ln(P_k(z)/P_k(0)) (App. A):
//   d ell_k/dz = -alpha_k + gain_k - loss_k
//   gain_k = C_r,k sum_{0 < f_j - f_k <= cut} (f_j - f_k) P_j
//   loss_k = C_r,k sum_{0 < f_k - f_j <= cut} (f_k - f_j) P_j (f_k/f_j if photon ratio)
// with P_j = P_j(0) exp(ell_j).  The window sums come from block prefix sums of P_j,
// (f_j - f_mid) P_j and P_j / f_j, so each right-hand side costs O(N).  Classical RK4 with
// 2*ode_sub equal sub-steps per distance step; one block of 1024 threads per plan, thread c
// owning channel c.
__device__ inline double ode_rhs(const OdeChan& ch, int c, double ell, bool active, int photon, OdeShared& sh) {
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

__global__ void __launch_bounds__(1024) k_profile_ode(PlanView pv, FibreParams fp, const double* __restrict__ P,
                                                      Work w, int keep_states) {
  __shared__ OdeShared sh;
  const int b = blockIdx.x, o = pv.off[b], n = pv.off[b + 1] - o, M = fp.n_steps, c = threadIdx.x;
  const bool active = c < n;
  const double fmid = 0.5 * (pv.f[o] + pv.f[o + n - 1]);
  OdeChan ch{};
  if (active) ch = ode_chan(pv, fp, P, o, n, c, fmid);
  double ell = 0.0;
  double* st = keep_states ? w.states + w.state_off[b] : nullptr;
  const int sub = fp.ode_sub;
  int step = 0;
  for (int m = 0; m < M; ++m) {
    const double h = w.dz[b * M + m] / (2.0 * sub);
    for (int half = 0; half < 2; ++half) {
      for (int q = 0; q < sub; ++q) {
        if (st && active) st[(size_t)step * n + c] = ell;
        double k1 = ode_rhs(ch, c, ell, active, fp.photon_ratio, sh);
        double k2 = ode_rhs(ch, c, ell + 0.5 * h * k1, active, fp.photon_ratio, sh);
        double k3 = ode_rhs(ch, c, ell + 0.5 * h * k2, active, fp.photon_ratio, sh);
        double k4 = ode_rhs(ch, c, ell + h * k3, active, fp.photon_ratio, sh);
        ell = ell + (k1 + 2.0 * k2 + 2.0 * k3 + k4) * (h / 6.0);
        ++step;
      }
      if (half == 0 && active) w.ell64[(size_t)M * o + (size_t)m * n + c] = ell;
    }
  }
  if (st && active) st[(size_t)step * n + c] = ell;
  if (active) w.ellL[o + c] = ell;
}

// FP32 table for the FP32 integrand: ell * log2(e)/2 and its forward difference.
__global__ void k_table32(PlanView pv, FibreParams fp, Work w) {
  const int M = fp.n_steps;
  const int64_t total = (int64_t)M * pv.n_total;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    const int g = (int)(q % pv.n_total);  // not the layout index; recover (b, m, c) below
    (void)g;
    // layout: plan b block at M*off[b], [m][c] with n = N_b
    int b = 0;
    {
      int lo = 0, hi = pv.n_batch;
      while (hi - lo > 1) { int mid = (lo + hi) >> 1; if ((int64_t)M * pv.off[mid] <= q) lo = mid; else hi = mid; }
      b = lo;
    }
    const int o = pv.off[b], n = pv.off[b + 1] - o;
    const int64_t loc = q - (int64_t)M * o;
    const int c = (int)(loc % n);
    const double v = w.ell64[q];
    const double nx = c + 1 < n ? w.ell64[q + 1] : v;
    w.lt32[q] = make_float2((float)(v * kHalfLog2e), (float)((nx - v) * kHalfLog2e));
  }
}

// ---------------------------------------------------------------------------- low-rank table
// The scaled ODE profile table L(m, c) = ln rho(z_m, f_c) log2(e) / 2 of a plan is close to a
// matrix of small rank: along z every channel follows a few smooth loss and Raman-transfer
// shapes.  Gram-Schmidt with column pivoting in FP64 (next direction: the residual column of
// largest norm, normalised) gives L ~ sum_r a_r(m) b_r(c) with orthonormal a_r, and stops once
// max |residual| <= kLowRankTol -- below the half-ulp of the FP32 table itself (2.4e-7 for
// |L| in [4, 8)).  The FP32 factors are then checked at every table point with the FP32 sum
// the tile kernels form.  A plan that needs more than kRank terms (or the cap ISRSGN_LOWRANK=N)
// or fails the check gets rank -1, and the tile kernels read the table for it.  Linear
// interpolation in f commutes with the factorisation, so the bound also holds between channel
// centres.  One block per plan.
constexpr double kLowRankTol = 2.5e-7;
constexpr double kLowRankCheck = 1.0e-6;

__device__ inline void block_max_arg(double* v, int* arg, double* rv, int* ri) {
  // largest v over the block (ties: smallest arg), result on every thread
  double x = *v;
  int k = *arg;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double y = __shfl_xor(x, o, 64);
    const int j = __shfl_xor(k, o, 64);
    if (y > x || (y == x && j < k)) { x = y; k = j; }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) { rv[wid] = x; ri[wid] = k; }
  __syncthreads();
  x = rv[0];
  k = ri[0];
  for (int q = 1; q < nw; ++q)
    if (rv[q] > x || (rv[q] == x && ri[q] < k)) { x = rv[q]; k = ri[q]; }
  __syncthreads();
  *v = x;
  *arg = k;
}

__global__ void __launch_bounds__(1024) k_lowrank(PlanView pv, FibreParams fp, Work w) {
  extern __shared__ double lq[];  // [M] current direction a_r
  __shared__ double rv[16];
  __shared__ int ri[16];
  const int b = blockIdx.x, o = pv.off[b], n = pv.off[b + 1] - o, M = fp.n_steps, tid = threadIdx.x;
  const int nth = blockDim.x;
  if (!fp.lowrank) {
    if (tid == 0) w.lr_rank[b] = -1;
    return;
  }
  const double* L = w.ell64 + (size_t)M * o;
  double* R = w.lr_res + (size_t)M * o;  // residual, [m][c] like the table
  double* B = w.lr_b64 + (size_t)kRank * o;
  float* Aout = w.lr_a + (size_t)M * kRank * b;
  for (int64_t q = tid; q < (int64_t)M * n; q += nth) R[q] = L[q] * kHalfLog2e;
  for (int64_t q = tid; q < (int64_t)M * kRank; q += nth) Aout[q] = 0.0f;
  for (int64_t q = tid; q < (int64_t)n * kRank; q += nth) B[q] = 0.0;
  __syncthreads();
  int rank = -1;
  const int most = fp.lowrank;  // terms allowed (kRank unless capped)
  for (int r = 0; r <= most; ++r) {
    double amax = 0.0, best = -1.0;
    int bc = 0;
    for (int c = tid; c < n; c += nth) {
      double ss = 0.0;
      for (int m = 0; m < M; ++m) {
        const double v = R[(size_t)m * n + c];
        ss = fma(v, v, ss);
        amax = fmax(amax, fabs(v));
      }
      if (ss > best) { best = ss; bc = c; }
    }
    int dummy = 0;
    block_max_arg(&amax, &dummy, rv, ri);
    if (amax <= kLowRankTol) {
      rank = r;
      break;
    }
    if (r == most) break;
    block_max_arg(&best, &bc, rv, ri);
    const double inv = 1.0 / sqrt(best);
    for (int m = tid; m < M; m += nth) lq[m] = R[(size_t)m * n + bc] * inv;
    __syncthreads();
    for (int c = tid; c < n; c += nth) {
      double cf = 0.0;
      for (int m = 0; m < M; ++m) cf = fma(lq[m], R[(size_t)m * n + c], cf);
      for (int m = 0; m < M; ++m) R[(size_t)m * n + c] = fma(-lq[m], cf, R[(size_t)m * n + c]);
      B[(size_t)c * kRank + r] = cf;
    }
    for (int m = tid; m < M; m += nth) Aout[(size_t)m * kRank + r] = (float)lq[m];
    __syncthreads();
  }
  float2* Bout = w.lr_b + (size_t)kRank * o;
  if (rank >= 0) {
    for (int64_t q = tid; q < (int64_t)n * kRank; q += nth) {
      const int c = (int)(q / kRank), r = (int)(q % kRank);
      const double v = B[q], nx = c + 1 < n ? B[q + kRank] : v;
      Bout[q] = make_float2((float)v, (float)(nx - v));
    }
    __syncthreads();
    // the FP32 sum of the tile kernels at every table point
    double worst = 0.0;
    for (int64_t q = tid; q < (int64_t)M * n; q += nth) {
      const int m = (int)(q / n), c = (int)(q % n);
      float e = 0.0f;
      for (int r = kRank - 1; r >= 0; --r) e = fmaf(Aout[(size_t)m * kRank + r], Bout[(size_t)c * kRank + r].x, e);
      worst = fmax(worst, fabs((double)e - L[q] * kHalfLog2e));
    }
    int dummy = 0;
    block_max_arg(&worst, &dummy, rv, ri);
    if (!(worst <= kLowRankCheck)) rank = -1;
  }
  if (tid == 0) w.lr_rank[b] = rank;
}

// ---------------------------------------------------------------------------- pair integrals
struct TileArgs {
  PlanView pv;
  FibreParams fp;
  const double* P;
  Work w;
  int nmax;               // largest plan
  unsigned int t_begin;   // tiles [t_begin, t_end) of the concatenated tile list
  unsigned int t_end;
};

// lowrank: room for the tile's terms of the low-rank exponent (FP32 form with the ODE profile only)
__host__ __device__ inline size_t tile_lds_bytes(int nmax, int gs, int M, bool lowrank) {
  return sizeof(double) * (3 * (size_t)nmax + 4 * (size_t)gs + 4) + (sizeof(StepRec) + sizeof(Col4)) * (size_t)M +
         (lowrank ? sizeof(float) * kLrTileFloats : 0) + 16;
}

__host__ __device__ inline bool tile_lowrank(const FibreParams& fp) { return fp.precision == 0 && fp.profile != 0; }

__device__ inline double shape_product(const ChanLds& ch, const RowLds& rw, const TileGeo& g, int k, int part,
                                       int64_t q, int GV, const Node& nd, double beta) {
  double s1, s2, s3;
  node_shapes(ch, rw, g, k, part, (int)(q / GV), (int)(q % GV), nd.c1, nd.c2, beta, &s1, &s2, &s3);
  return s1 * s2 * s3;
}

// Forward pair-integral kernel.  Persistent: each workgroup takes tiles (b, i, k) from a
// work counter; per tile it lays out the rows of each part in LDS, then strides the
// part's grid_s x grid_v nodes across its 256 lanes (a wave covers consecutive nodes of a
// row), accumulates node values w G1 G2 G3 |S|^2 in FP64 and reduces over the workgroup in
// a fixed order, so results are bitwise reproducible.
// kRc: raised-cosine spectra (the node's shapes multiply its value after the step sum; a separate
// instantiation, so the rectangular kernels carry none of that code)
template <int kPrec, bool kLinear, int kUnroll, int kWaves, bool kRc = false>
__global__ void __launch_bounds__(kTileBlock) __attribute__((amdgpu_waves_per_eu(kWaves > 0 ? kWaves : 1, 8)))
k_tiles(TileArgs A) {
  extern __shared__ __align__(16) char smem_raw[];
  const int nmax = A.nmax, GS = A.fp.grid_s, GV = A.fp.grid_v, M = A.fp.n_steps, tid = threadIdx.x;
  double* d = reinterpret_cast<double*>(smem_raw);
  const ChanLds ch{d, d + nmax, d + 2 * nmax};
  d += 3 * nmax;
  const RowLds rw{d, d + GS, d + 2 * GS, d + 3 * GS};
  d += 4 * GS;
  double* red = d;
  d += 4;
  StepRec* steps = reinterpret_cast<StepRec*>(d);
  Col4* col = reinterpret_cast<Col4*>(steps + M);
  float* lr_t = reinterpret_cast<float*>(col + M);  // the tile's low-rank terms (lowrank_tile_terms)
  unsigned int* tile_slot = reinterpret_cast<unsigned int*>(lr_t + (kPrec == 0 && !kLinear ? kLrTileFloats : 0));
  const PlanView& pv = A.pv;
  int cur_b = -1, cur_lr = -1;
  for (;;) {
    if (tid == 0) *tile_slot = A.t_begin + atomicAdd(A.w.counter, 1u);
    __syncthreads();
    const unsigned int t = *tile_slot;
    if (t >= A.t_end) break;
    int b, i, j, k;
    decode_tile(pv, t, &b, &i, &j, &k);
    const int o = pv.off[b], n = pv.off[b + 1] - o;
    const double* zm = A.w.zm + (size_t)b * M;
    const double* dz = A.w.dz + (size_t)b * M;
    const double fnli = pv.fpt[(size_t)(o + i) * pv.nli + j];  // the NLI frequency of this tile
    int sf;
    double tf;
    nli_segment(pv.f + o, n, i, fnli, &sf, &tf);
    sf = __builtin_amdgcn_readfirstlane(sf);  // tile-uniform: scalar registers
    tf = uniform_f64(tf);
    if (b != cur_b) {
      load_channels(ch, pv, A.P, o, n, A.fp.rolloff);
      if (kPrec == 0) load_steps(steps, zm, dz, A.w.hdz32 + (size_t)b * M, M);
      if (kPrec == 0 && !kLinear) cur_lr = __builtin_amdgcn_readfirstlane(A.w.lr_rank[b]);
      cur_b = b;
    }
    // (the low-rank exponent has every profile term: no table columns)
    if (kPrec == 0 && (kLinear || cur_lr < 0)) load_cols<kLinear>(col, A.w.lt32 + (size_t)M * o, n, M, sf, tf, k);
    // FP64 form: the f-term column in the step-table slot (unused by that form)
    double* lf64 = reinterpret_cast<double*>(steps);
    if (kPrec == 1 && !kLinear) load_fcol64(lf64, A.w.ell64 + (size_t)M * o, n, M, sf, tf);
    if (kPrec == 0 && !kLinear && cur_lr >= 0) {
      int sa, sb;
      col_segments(k, n, &sa, &sb);
      lowrank_tile_terms(A.w.lr_b + (size_t)kRank * o, sf, (float)tf, sa, sb, lr_t);
    }
    __syncthreads();
    const TileGeo g = uniform_geo(tile_geo(ch, n, fnli, k, A.fp.f_ref));
    double acc = 0.0;
    unsigned int evaluated = 0;
    for (int part = kQ1; part <= kQ4; ++part) {
      if (!layout_rows(rw, g, part, GS, GV, A.fp.s_decades)) continue;
      __syncthreads();
      const int64_t nodes = (int64_t)GS * GV;
      // whole waves stay in the loop (the FP32 form plans its step ranges across the wave)
      for (int64_t base = 0; base < nodes; base += kTileBlock) {
        const int64_t q = base + tid;
        Node nd;
        const bool valid =
            q < nodes && make_node<kPrec == 0>(ch, rw, g, n, k, part, (int)(q / GV), (int)(q % GV), A.fp, &nd);
        double s2v;
        if (kPrec == 0) {
          Term32 tq{};
          if (valid) tq = term32_setup(nd, k, n);
          const Split32 sp = wave_split(valid, tq, steps, M);
          if (!valid) continue;
          float sr, si;
          if (!kLinear && cur_lr >= 0) {
            LowRank32 src;
            src.a = const_f32(A.w.lr_a + (size_t)M * kRank * b);
            src.setup(tq, A.w.lr_b + (size_t)kRank * o, reinterpret_cast<const float2*>(lr_t + kRank) + (tq.up3 ? kRank : 0),
                      lr_t);
            accumulate32<kLinear, kUnroll>(tq, sp, steps, col, src, M, &sr, &si);
          } else {
            const Gather32 src{make_tab32(A.w.lt32 + (size_t)M * o, n, M), n};
            accumulate32<kLinear, kUnroll>(tq, sp, steps, col, src, M, &sr, &si);
          }
          s2v = (double)sr * sr + (double)si * si;
          if (A.w.s_store)
            static_cast<float2*>(A.w.s_store)[((int64_t)(t - A.t_begin) * 3 + part) * nodes + q] = make_float2(sr, si);
          if constexpr (kRc) s2v *= shape_product(ch, rw, g, k, part, q, GV, nd, A.fp.rolloff);
        } else {
          if (!valid) continue;
          const Term64 tq = term64_setup(nd);
          const double* tab = A.w.ell64 + (size_t)M * o;
          double sr = 0.0, si = 0.0;
#pragma unroll kUnroll
          for (int m = 0; m < M; ++m) {
            const double2 a = term64<kLinear>(tq, m, zm, dz, tab, n, lf64);
            sr += a.x;
            si += a.y;
          }
          s2v = sr * sr + si * si;
          if (A.w.s_store)
            static_cast<double2*>(A.w.s_store)[((int64_t)(t - A.t_begin) * 3 + part) * nodes + q] = make_double2(sr, si);
          if constexpr (kRc) s2v *= shape_product(ch, rw, g, k, part, q, GV, nd, A.fp.rolloff);
        }
        acc += nd.w * nd.gprod * s2v;
        ++evaluated;
      }
      __syncthreads();
    }
    acc = wave_sum(acc);
    const double cnt = wave_sum((double)evaluated);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) A.w.tiles[t] = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    if ((tid & 63) == 0 && cnt > 0) atomicAdd(A.w.nodes, (unsigned long long)cnt);
  }
}

__global__ void k_zero_counter(unsigned int* c, unsigned long long* nodes) {
  *c = 0u;
  if (nodes) *nodes = 0ull;
}

// ---------------------------------------------------------------------------- reduction
// One wave per channel: P_NLI,i = 16/27 gamma_i^2 R_i sum_k tile(i,k) (eq. gain_fin times R_i),
// eta_i = P_NLI,i / P_i^3, P_ASE,i = NF_i h f_i R_i / rho(L, f_i), SNR_i (eq. loss).
__global__ void k_reduce(PlanView pv, const double* __restrict__ P, const double* __restrict__ nf, double snr_trx,
                         Work w, double* eta, double* pnli_out, double* snr_out, int g_begin, int g_end,
                         int n_spans) {
  const int g = g_begin + blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (g >= g_end) return;
  const int b = plan_of_channel(pv, g), o = pv.off[b], n = pv.off[b + 1] - o, i = g - o, J = pv.nli;
  const double* row = w.tiles + pv.toff[b] + (int64_t)i * n * J;
  double s = 0.0;
  if (J == 1) {
    for (int k = lane; k < n; k += 64) s += row[k];
  } else {  // the within-channel rule: tiles of point j weighted by w_j
    for (int j = 0; j < J; ++j) {
      double sj = 0.0;
      for (int k = lane; k < n; k += 64) sj += row[(int64_t)j * n + k];
      s += pv.wpt[(size_t)g * J + j] * sj;
    }
  }
  s = wave_sum(s);
  if (lane != 0) return;
  const double gm = pv.gamma[g], R = pv.R[g], f = pv.f[g], p = P[g];
  const double pn = (16.0 / 27.0) * gm * gm * R * s;
  w.pnli[g] = pn;
  if (pnli_out) pnli_out[g] = pn;
  if (eta) eta[g] = p > 0.0 ? pn / (p * p * p) : __builtin_nan("");
  if (nf) {  // SNR only when noise figures are given (isrsgn_eta passes none)
    double sn = 0.0;
    if (p > 0.0) {
      const double pase = nf[g] * kH * f * R * exp(-w.ellL[g]) * n_spans;  // one amplifier per span
      sn = p / (pn + pase);
      if (snr_trx > 0.0) sn = 1.0 / (1.0 / sn + 1.0 / snr_trx);
    }
    w.snr[g] = sn;
    if (snr_out) snr_out[g] = sn;
  }
}

// Throughput per plan: T_b = sum over P_i > 0 of 2 R_i log2(1 + SNR_i).
__global__ void k_throughput(PlanView pv, const double* __restrict__ P, Work w, double* thr) {
  __shared__ double red[16];
  const int b = blockIdx.x, o = pv.off[b], n = pv.off[b + 1] - o;
  double s = 0.0;
  for (int c = threadIdx.x; c < n; c += blockDim.x)
    if (P[o + c] > 0.0) s += 2.0 * pv.R[o + c] * log2(1.0 + w.snr[o + c]);
  s = block_sum(s, red);
  if (threadIdx.x == 0) thr[b] = s;
}

// Input rules of the boundary: launch powers finite and >= 0, noise figures (when given)
// finite and >= 0.  One block: out[0] invalid entries, out[1] first bad power, out[2] first bad
// noise figure (n when none).
__global__ void __launch_bounds__(1024) k_check_inputs(const double* __restrict__ P, const double* __restrict__ nf,
                                                       int n, int* out) {
  __shared__ int red[3][16];
  int bad = 0, first_p = n, first_nf = n;
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    const double p = P[c];
    if (!(p >= 0.0) || !(p <= 1.7976931348623157e308)) { ++bad; first_p = min(first_p, c); }
    if (nf) {
      const double v = nf[c];
      if (!(v >= 0.0) || !(v <= 1.7976931348623157e308)) { ++bad; first_nf = min(first_nf, c); }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    bad += __shfl_xor(bad, o, 64);
    first_p = min(first_p, __shfl_xor(first_p, o, 64));
    first_nf = min(first_nf, __shfl_xor(first_nf, o, 64));
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) { red[0][wid] = bad; red[1][wid] = first_p; red[2][wid] = first_nf; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < nw; ++q) {
      bad += red[0][q];
      first_p = min(first_p, red[1][q]);
      first_nf = min(first_nf, red[2][q]);
    }
    out[0] = bad;
    out[1] = first_p;
    out[2] = first_nf;
  }
}

__global__ void k_copy(double* __restrict__ dst, const double* __restrict__ src, int64_t n) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
    dst[q] = src[q];
}

// The caller's tile blocks [i][k] = sum_j w_j tile(i, j, k) (plan b's output block at toff[b] / nli).
__global__ void k_fold_tiles(PlanView pv, Work w, double* __restrict__ out) {
  const int J = pv.nli;
  const int64_t total = pv.n_tiles / J;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = pv.n_batch;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (pv.toff[mid] / J <= q) lo = mid; else hi = mid;
    }
    const int o = pv.off[lo], n = pv.off[lo + 1] - o;
    const int64_t loc = q - pv.toff[lo] / J;
    const int i = (int)(loc / n), k = (int)(loc % n);
    const double* src = w.tiles + pv.toff[lo] + (int64_t)i * n * J + k;
    double v = 0.0;
    for (int j = 0; j < J; ++j) v += pv.wpt[(size_t)(o + i) * J + j] * src[(int64_t)j * n];
    out[q] = v;
  }
}

__global__ void k_put_words(unsigned long long* __restrict__ dst, WordChunk c) {
  const int q = threadIdx.x;
  if (q < c.n) dst[q] = c.w[q];
}

__global__ void k_copy_profile(PlanView pv, FibreParams fp, Work w, double* zm, double* dz, double* ell,
                               double* ellL) {
  const int M = fp.n_steps;
  const int64_t nz = (int64_t)pv.n_batch * M, ne = (int64_t)M * pv.n_total;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < ne + nz + pv.n_total;
       q += (int64_t)gridDim.x * blockDim.x) {
    if (q < nz) {
      if (zm) zm[q] = w.zm[q];
      if (dz) dz[q] = w.dz[q];
    } else if (q < nz + ne) {
      if (ell) ell[q - nz] = w.ell64[q - nz];
    } else {
      if (ellL) ellL[q - nz - ne] = w.ellL[q - nz - ne];
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------- launchers

hipError_t launch_channel_setup(const PlanView& pv, const FibreParams& fp, hipStream_t s) {
  hipLaunchKernelGGL(k_channel_setup, dim3((pv.n_total + 255) / 256), dim3(256), 0, s, pv, fp);
  return hipGetLastError();
}

hipError_t launch_steps(const PlanView& pv, const FibreParams& fp, const double* P, const Work& w, hipStream_t s) {
  hipLaunchKernelGGL(k_steps, dim3(pv.n_batch), dim3(256), 0, s, pv, fp, P, w);
  return hipGetLastError();
}

hipError_t launch_profile(const PlanView& pv, const FibreParams& fp, const double* P, const Work& w,
                          bool keep_states, hipStream_t s) {
  if (fp.profile == 0) {
    hipLaunchKernelGGL(k_profile_closed_form, dim3(fp.n_steps + 1, pv.n_batch), dim3(256), 0, s, pv, fp, P, w);
  } else {
    hipLaunchKernelGGL(k_profile_ode, dim3(pv.n_batch), dim3(1024), 0, s, pv, fp, P, w, keep_states ? 1 : 0);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (fp.precision == 0) {
    const int64_t total = (int64_t)fp.n_steps * pv.n_total;
    const int blocks = (int)((total + 255) / 256 < 65536 ? (total + 255) / 256 : 65536);
    hipLaunchKernelGGL(k_table32, dim3(blocks), dim3(256), 0, s, pv, fp, w);
    e = hipGetLastError();
    if (e == hipSuccess && fp.profile != 0) {
      hipLaunchKernelGGL(k_lowrank, dim3(pv.n_batch), dim3(1024), sizeof(double) * fp.n_steps, s, pv, fp, w);
      e = hipGetLastError();
    }
  }
  return e;
}

namespace {

// Tile-kernel variants (step-loop unroll, minimum waves per SIMD), chosen by the host autotuner.
using TileKernel = void (*)(TileArgs);
#define ISRSGN_TILE_VARIANTS(P, L)                                                                 \
  {k_tiles<P, L, 1, 0>, k_tiles<P, L, 2, 0>, k_tiles<P, L, 2, 5>, k_tiles<P, L, 1, 4>, k_tiles<P, L, 2, 4>, \
   k_tiles<P, L, 4, 3>}
const TileKernel kTileKernels[2][2][kTileVariants] = {{ISRSGN_TILE_VARIANTS(0, false), ISRSGN_TILE_VARIANTS(0, true)},
                                                     {ISRSGN_TILE_VARIANTS(1, false), ISRSGN_TILE_VARIANTS(1, true)}};
const char* const kTileVariantNames[kTileVariants] = {"unroll1", "unroll2", "unroll2-w5", "unroll1-w4", "unroll2-w4",
                                                       "unroll4-w3"};
// raised-cosine spectra: one kernel for every variant index (unroll 2; the FP32 form at least 5
// waves per SIMD like the rectangular kernels' usual pick, the FP64 form with no occupancy hint)
const TileKernel kTileKernelsRc[2][2] = {{k_tiles<0, false, 2, 5, true>, k_tiles<0, true, 2, 5, true>},
                                         {k_tiles<1, false, 2, 0, true>, k_tiles<1, true, 2, 0, true>}};

TileKernel tile_kernel(const FibreParams& fp, int variant) {
  const int v = variant < 0 || variant >= kTileVariants ? 0 : variant;
  if (fp.rolloff > 0.0) return kTileKernelsRc[fp.precision ? 1 : 0][fp.profile == 0 ? 1 : 0];
  return kTileKernels[fp.precision ? 1 : 0][fp.profile == 0 ? 1 : 0][v];
}

}  // namespace

const char* tile_variant_name(int variant) {
  return variant >= 0 && variant < kTileVariants ? kTileVariantNames[variant] : "?";
}

size_t tile_lds(const FibreParams& fp, int nmax) { return tile_lds_bytes(nmax, fp.grid_s, fp.n_steps, tile_lowrank(fp)); }

int tile_blocks_per_cu(const FibreParams& fp, int nmax, int variant) {
  int nb = 0;
  const size_t shm = tile_lds_bytes(nmax, fp.grid_s, fp.n_steps, tile_lowrank(fp));
  const void* k = reinterpret_cast<const void*>(tile_kernel(fp, variant));
  // above 64 KiB the kernel must opt in before the occupancy query counts its blocks
  if (shm > 65536) (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kTileBlock, shm);
  if (e != hipSuccess || nb < 1) nb = 1;
  return nb;
}

hipError_t launch_tiles(const PlanView& pv, const FibreParams& fp, const double* P, const Work& w, int nmax,
                        int grid, int variant, unsigned int t_begin, unsigned int t_end, bool reset_nodes,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(1), 0, s, w.counter, reset_nodes ? w.nodes : nullptr);
  TileArgs a{pv, fp, P, w, nmax, t_begin, t_end};
  const size_t shm = tile_lds_bytes(nmax, fp.grid_s, fp.n_steps, tile_lowrank(fp));
  const void* k = reinterpret_cast<const void*>(tile_kernel(fp, variant));
  if (shm > 65536) (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  void* args[] = {&a};
  hipError_t e = hipLaunchKernel(k, dim3(grid), dim3(kTileBlock), args, shm, s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_reduce_rows(const PlanView& pv, const FibreParams& fp, const double* P, const double* nf,
                              double snr_trx, const Work& w, double* eta, double* pnli_out, double* snr_out,
                              int g_begin, int g_end, hipStream_t s) {
  if (g_end <= g_begin) return hipSuccess;
  hipLaunchKernelGGL(k_reduce, dim3((g_end - g_begin + 3) / 4), dim3(256), 0, s, pv, P, nf, snr_trx, w, eta,
                     pnli_out, snr_out, g_begin, g_end, fp.n_spans);
  return hipGetLastError();
}

hipError_t launch_throughput(const PlanView& pv, const double* P, const Work& w, double* thr_out, hipStream_t s) {
  hipLaunchKernelGGL(k_throughput, dim3(pv.n_batch), dim3(256), 0, s, pv, P, w, thr_out);
  return hipGetLastError();
}

hipError_t launch_reduce(const PlanView& pv, const FibreParams& fp, const double* P, const double* nf,
                         double snr_trx, const Work& w, double* eta, double* pnli_out, double* snr_out,
                         double* thr_out, hipStream_t s) {
  (void)fp;
  hipError_t e = launch_reduce_rows(pv, fp, P, nf, snr_trx, w, eta, pnli_out, snr_out, 0, pv.n_total, s);
  if (e != hipSuccess || !thr_out) return e;
  return launch_throughput(pv, P, w, thr_out, s);
}

hipError_t launch_check_inputs(const double* P, const double* nf, int n, int* out, hipStream_t s) {
  hipLaunchKernelGGL(k_check_inputs, dim3(1), dim3(1024), 0, s, P, nf, n, out);
  return hipGetLastError();
}

hipError_t launch_copy(double* dst, const double* src, int64_t n, hipStream_t s) {
  const int64_t blocks = (n + 255) / 256 < 2048 ? (n + 255) / 256 : 2048;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)(blocks < 1 ? 1 : blocks)), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}

hipError_t launch_fold_tiles(const PlanView& pv, const Work& w, double* out, hipStream_t s) {
  const int64_t total = pv.n_tiles / pv.nli, blocks = (total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096;
  hipLaunchKernelGGL(k_fold_tiles, dim3((unsigned)(blocks < 1 ? 1 : blocks)), dim3(256), 0, s, pv, w, out);
  return hipGetLastError();
}

hipError_t launch_put_words(unsigned long long* dst, const WordChunk& c, hipStream_t s) {
  hipLaunchKernelGGL(k_put_words, dim3(1), dim3(256), 0, s, dst, c);
  return hipGetLastError();
}

hipError_t launch_copy_profile(const PlanView& pv, const FibreParams& fp, const Work& w, double* zm, double* dz,
                               double* ell, double* ellL, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_profile, dim3(256), dim3(256), 0, s, pv, fp, w, zm, dz, ell, ellL);
  return hipGetLastError();
}

}  // namespace isrsgn
