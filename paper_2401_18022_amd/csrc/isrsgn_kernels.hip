// HIP kernels of libisrsgn.so for gfx950 (MI355X): setup, distance steps, power
// profile, COI x interferer pair integrals, and the NLI / SNR / throughput reduction.
//
// Model: arXiv:2401.18022 -- eq. (new_gn_model) with the step sum of eq. (slow_vary),
// the power term of eq. (pk), the phase mismatch of eq. (phi), hyperbolic coordinates
// of eqs. (q1)-(q4), assembly eqs. (gain_fin)/(psi_fin), cost eq. (loss).
#include "isrsgn_internal.h"

#include <hip/hip_runtime.h>

namespace isrsgn {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kC = 299792458.0;
constexpr double kH = 6.62607015e-34;
constexpr double kLn10 = 2.302585092994045684;
constexpr double kHalfLog2e = 0.72134752044448170368;  // log2(e) / 2

// ---------------------------------------------------------------------------- reductions

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over a block of `nthreads` (multiple of 64); fixed order, result on every thread.
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = 0.0;
  for (int q = 0; q < nw; ++q) t += red[q];
  __syncthreads();
  return t;
}

__device__ inline double tab_at(int n, const double* xs, const double* ys, double x) {
  if (n == 1 || x <= xs[0]) return ys[0];
  if (x >= xs[n - 1]) return ys[n - 1];
  int lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (xs[mid] <= x) lo = mid; else hi = mid;
  }
  return ys[lo] + (x - xs[lo]) / (xs[hi] - xs[lo]) * (ys[hi] - ys[lo]);
}

__device__ inline int plan_of_channel(const PlanView& pv, int g) {
  int lo = 0, hi = pv.n_batch;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (pv.off[mid] <= g) lo = mid; else hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------------------- setup (Sec. II)

__global__ void k_channel_setup(PlanView pv, FibreParams fp) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= pv.n_total) return;
  double f = pv.f[c];
  double a = tab_at(fp.n_tab, fp.tab_f, fp.tab_alpha, f);
  double ae = tab_at(fp.n_tab, fp.tab_f, fp.tab_aeff, f);
  pv.alpha[c] = a;
  pv.aeff[c] = ae;
  pv.gamma[c] = fp.gamma_const > 0 ? fp.gamma_const : 2.0 * kPi * fp.n2 * f / (kC * ae);  // eq. (gamma)
  pv.cr[c] = fp.cr * fp.aeff_ref / ae;  // Raman gain scaled by A_eff at the channel frequency
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
  }
}

// ---------------------------------------------------------------------------- power profile
// Closed form (linear Raman slope over a rectangular spectrum, uniform loss):
//   ln rho(z,F) = -alpha z - a (F - f_ref) - ln sum_j (P_j/P_tot) exp(-a (f_j - f_ref)) sinhc(a R_j/2)
//   a = P_tot C_r L_eff(z).  Grid (M + 1, n_batch): row M is the span end.
__device__ inline double sinhc(double x) {
  if (fabs(x) < 1e-4) { double x2 = x * x; return 1.0 + x2 / 6.0 + x2 * x2 / 120.0; }
  return sinh(x) / x;
}

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
      s += P[o + c] / pt * exp(-a * (pv.f[o + c] - fp.f_ref)) * sinhc(0.5 * a * pv.R[o + c]);
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
struct OdeShared {
  double sA[kMaxChannels], sB[kMaxChannels], sC[kMaxChannels];
  double wt[3][16];
};

__device__ void block_scan3(double& a, double& bb, double& c, OdeShared& sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    double ta = __shfl_up(a, o, 64), tb = __shfl_up(bb, o, 64), tc = __shfl_up(c, o, 64);
    if (lane >= o) { a += ta; bb += tb; c += tc; }
  }
  if (lane == 63) { sh.wt[0][wid] = a; sh.wt[1][wid] = bb; sh.wt[2][wid] = c; }
  __syncthreads();
  double pa = 0.0, pb = 0.0, pc = 0.0;
  for (int q = 0; q < wid; ++q) { pa += sh.wt[0][q]; pb += sh.wt[1][q]; pc += sh.wt[2][q]; }
  a += pa; bb += pb; c += pc;
  (void)nw;
}

struct OdeChan {
  double f, ft, alpha, cr, p0;
  int glo, ghi;  // gain window (c, ghi]: j in [c+1, ghi]
  int llo;       // loss window [llo, c)
};

__device__ double ode_rhs(const OdeChan& ch, int c, int n, double ell, bool active, int photon, OdeShared& sh) {
  double p = active ? ch.p0 * exp(ell) : 0.0;
  double a = p, bb = ch.ft * p, cc = active ? p / ch.f : 0.0;
  block_scan3(a, bb, cc, sh);
  __syncthreads();
  if (active) { sh.sA[c] = a; sh.sB[c] = bb; sh.sC[c] = cc; }
  __syncthreads();
  double r = 0.0;
  if (active) {
    // gain from (c, ghi]
    double gA = 0.0, gB = 0.0;
    if (ch.ghi > c) { gA = sh.sA[ch.ghi] - sh.sA[c]; gB = sh.sB[ch.ghi] - sh.sB[c]; }
    double lA = 0.0, lB = 0.0, lC = 0.0;
    if (c > ch.llo) {
      double baseA = ch.llo > 0 ? sh.sA[ch.llo - 1] : 0.0;
      double baseB = ch.llo > 0 ? sh.sB[ch.llo - 1] : 0.0;
      double baseC = ch.llo > 0 ? sh.sC[ch.llo - 1] : 0.0;
      lA = sh.sA[c - 1] - baseA; lB = sh.sB[c - 1] - baseB; lC = sh.sC[c - 1] - baseC;
    }
    double gain = ch.cr * (gB - ch.ft * gA);
    double loss = photon ? ch.cr * ch.f * (ch.f * lC - lA) : ch.cr * (ch.ft * lA - lB);
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
  OdeChan ch{};
  const double fmid = 0.5 * (pv.f[o] + pv.f[o + n - 1]);
  if (active) {
    ch.f = pv.f[o + c];
    ch.ft = ch.f - fmid;
    ch.alpha = pv.alpha[o + c];
    ch.cr = pv.cr[o + c];
    ch.p0 = P[o + c];
    const double cut = fp.cutoff;
    // gain window: last j with f_j - f_c <= cut
    int lo = c, hi = n;  // invariant: f[lo] - f_c <= cut (lo = c), f[hi] beyond
    if (cut <= 0) lo = n - 1;
    else {
      while (hi - lo > 1) { int mid = (lo + hi) >> 1; if (pv.f[o + mid] - ch.f <= cut) lo = mid; else hi = mid; }
    }
    ch.ghi = lo;
    // loss window: first j with f_c - f_j <= cut
    int l2 = -1, h2 = c;  // invariant: f[h2] within, f[l2] beyond
    if (cut <= 0) h2 = 0;
    else {
      while (h2 - l2 > 1) { int mid = (l2 + h2) >> 1; if (ch.f - pv.f[o + mid] <= cut) h2 = mid; else l2 = mid; }
    }
    ch.llo = h2;
  }
  double ell = 0.0;
  double* st = keep_states ? w.states + w.state_off[b] : nullptr;
  const int sub = fp.ode_sub;
  int step = 0;
  for (int m = 0; m < M; ++m) {
    const double h = w.dz[b * M + m] / (2.0 * sub);
    for (int half = 0; half < 2; ++half) {
      for (int q = 0; q < sub; ++q) {
        if (st && active) st[(size_t)step * n + c] = ell;
        double k1 = ode_rhs(ch, c, n, ell, active, fp.photon_ratio, sh);
        double k2 = ode_rhs(ch, c, n, ell + 0.5 * h * k1, active, fp.photon_ratio, sh);
        double k3 = ode_rhs(ch, c, n, ell + 0.5 * h * k2, active, fp.photon_ratio, sh);
        double k4 = ode_rhs(ch, c, n, ell + h * k3, active, fp.photon_ratio, sh);
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

// ---------------------------------------------------------------------------- tile geometry
// Parts of tile (i,k) in offsets (x, y) = (f1 - f_i, f2 - f_i) with x + y in [slo, shi):
//   Q1: x = r e^v, y = r e^-v, v >= 0 (fold about x = y)
//   Q3: x = -r e^v, y = -r e^-v, v >= 0 (fold)
//   Q4: x = r e^v, y = -r e^-v (stands for the mirror part Q2 as well)
// r = sqrt(|x y|) = e^(s/2).  sup|x y| fixes the top of the s window.
enum { kQ1 = 0, kQ3 = 1, kQ4 = 2 };

__device__ bool part_umax(int part, double slo, double shi, double xp, double xn, double* umax) {
  if (part == kQ1) {
    if (shi <= 0 || xp <= 0) return false;
    double lo = fmax(slo, 0.0);
    if (lo >= 2.0 * xp) return false;
    double m = fmin(0.5 * shi, xp);
    *umax = m * m;
    return *umax > 0;
  }
  if (part == kQ3) {
    if (slo >= 0 || xn <= 0) return false;
    double lo = fmax(-shi, 0.0), hi = -slo;
    if (lo >= 2.0 * xn) return false;
    double m = fmin(0.5 * hi, xn);
    *umax = m * m;
    return *umax > 0;
  }
  if (xp <= 0 || xn <= 0) return false;
  double best = 0.0;
  double ulo = fmax(0.0, xp - shi), uhi = fmin(xn, xp - slo);
  if (uhi > ulo) best = fmax(best, xp * uhi);
  double xlo = fmax(0.0, xn + slo), xhi = fmin(xp, xn + shi);
  if (xhi > xlo) best = fmax(best, xhi * xn);
  if (!(best > 0)) return false;
  *umax = best;
  return true;
}

__device__ bool part_vrange(int part, double r, double slo, double shi, double xp, double xn, double* vlo,
                            double* vhi) {
  if (part == kQ1 || part == kQ3) {
    const double lo = part == kQ1 ? fmax(slo, 0.0) : fmax(-shi, 0.0);
    const double hi = part == kQ1 ? shi : -slo;
    const double lim = part == kQ1 ? xp : xn;
    const double chi = hi / (2.0 * r);
    if (!(chi > 1.0)) return false;
    const double clo = lo / (2.0 * r);
    *vlo = clo > 1.0 ? acosh(clo) : 0.0;
    *vhi = fmin(acosh(chi), log(lim / r));
    return *vhi > *vlo;
  }
  *vlo = fmax(asinh(slo / (2.0 * r)), log(r / xn));
  *vhi = fmin(asinh(shi / (2.0 * r)), log(xp / r));
  return *vhi > *vlo;
}

// Shared state of a tile workgroup: channel data of the current plan and the row layout of
// the current part, carved out of dynamic LDS (sized for the largest plan and grid_s).
struct TileShared {
  double* lo_edge;  // f_c - R_c/2
  double* hi_edge;  // f_c + R_c/2
  double* fc;
  double* psd;      // G_c = P_c / R_c
  double *row_vlo, *row_dv, *row_r, *row_w;
  double* red;      // [4]
  unsigned int* tile;
};

__host__ __device__ inline size_t tile_lds_bytes(int nmax, int gs) {
  return sizeof(double) * (4 * (size_t)nmax + 4 * (size_t)gs + 4) + 16;
}

__device__ inline TileShared carve_lds(char* base, int nmax, int gs) {
  double* d = reinterpret_cast<double*>(base);
  TileShared sh;
  sh.lo_edge = d; d += nmax;
  sh.hi_edge = d; d += nmax;
  sh.fc = d; d += nmax;
  sh.psd = d; d += nmax;
  sh.row_vlo = d; d += gs;
  sh.row_dv = d; d += gs;
  sh.row_r = d; d += gs;
  sh.row_w = d; d += gs;
  sh.red = d; d += 4;
  sh.tile = reinterpret_cast<unsigned int*>(d);
  return sh;
}

// Channel whose band [f_c - R_c/2, f_c + R_c/2) holds F, or -1.
__device__ inline int find_channel(const TileShared& sh, int n, double F) {
  if (F < sh.lo_edge[0]) return -1;
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (sh.lo_edge[mid] <= F) lo = mid; else hi = mid;
  }
  return F < sh.hi_edge[lo] ? lo : -1;
}

// Interpolation segment and weight of ln rho at F, given the channel c that holds F.
__device__ inline void segment(const TileShared& sh, int n, int c, double F, int* seg, double* t) {
  if (n == 1) { *seg = 0; *t = 0.0; return; }
  int s = F >= sh.fc[c] ? c : c - 1;
  s = s < 0 ? 0 : (s > n - 2 ? n - 2 : s);
  *seg = s;
  *t = (F - sh.fc[s]) / (sh.fc[s + 1] - sh.fc[s]);
}

// eq. (phi): phase mismatch per metre for offsets x, y and COI offset w from f_ref.
__device__ inline double phase_mismatch(double x, double y, double w, double b2, double b3, double b4) {
  const double p4 = x * x + 1.5 * x * y + y * y + 3.0 * x * w + 3.0 * y * w + 3.0 * w * w;
  return -4.0 * kPi * kPi * x * y * (b2 + kPi * b3 * (x + y + 2.0 * w) + (2.0 * kPi * kPi / 3.0) * b4 * p4);
}

struct TileArgs {
  PlanView pv;
  FibreParams fp;
  const double* P;
  Work w;
  int nmax;  // largest plan
};

// Decode a global tile index into (plan, COI, interferer).
__device__ inline void decode_tile(const PlanView& pv, unsigned int t, int* b, int* i, int* k) {
  int lo = 0, hi = pv.n_batch;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (pv.toff[mid] <= (int64_t)t) lo = mid; else hi = mid;
  }
  const int n = pv.off[lo + 1] - pv.off[lo];
  const int64_t loc = (int64_t)t - pv.toff[lo];
  *b = lo;
  *i = (int)(loc / n);
  *k = (int)(loc % n);
}

// |S|^2 of eq. (psi_fin) at one node: S = sum_m p_m dz_m exp(j phi z_m) sinc(phi dz_m / 2).
// FP32 form: the phase phi z_m is formed in FP64 and reduced to [-1/2, 1/2] revolutions before
// the FP32 hardware sine/cosine; the sinc factor uses a Taylor polynomial while |phi dz/2| < 1/2.
// p_m = exp(ln rho terms of eq. pk) from the FP32 table (general) or rho(z_m, f3) (linear profile,
// where ln rho(f1) + ln rho(f2) - ln rho(f_i) = ln rho(f3) exactly).
template <bool kLinear>
__device__ inline double node_s2_fp32(double phr, const double* __restrict__ zm, const float* __restrict__ hdz,
                                      const double* __restrict__ dz, const float2* __restrict__ tab, int n, int M,
                                      int s1, float t1, int s2, float t2, int s3, float t3, int ci) {
  const float phrf = (float)phr;
  const float inv_piphr = 1.0f / ((float)kPi * phrf);
  float sr = 0.0f, si = 0.0f;
  for (int m = 0; m < M; ++m) {
    const double tt = phr * zm[m];
    const float fr = (float)(tt - rint(tt));
    const float sn = __builtin_amdgcn_sinf(fr);
    const float cs = __builtin_amdgcn_cosf(fr);
    const float hh = phrf * hdz[m];
    const float u = 2.0f * (float)kPi * hh;
    const float u2 = u * u;
    const float dzm = 2.0f * hdz[m];
    const float apoly = dzm * (1.0f + u2 * (-1.0f / 6.0f + u2 * (1.0f / 120.0f - u2 * (1.0f / 5040.0f))));
    const float asn = __builtin_amdgcn_sinf(hh - rintf(hh)) * inv_piphr;
    const float amp0 = fabsf(u) < 0.5f ? apoly : asn;
    const float2* row = tab + (size_t)m * n;
    float e2;
    if (kLinear) {
      const float2 l3 = row[s3];
      e2 = 2.0f * (l3.x + t3 * l3.y);
    } else {
      const float2 l1 = row[s1], l2 = row[s2], l3 = row[s3];
      e2 = (l1.x + t1 * l1.y) + (l2.x + t2 * l2.y) + (l3.x + t3 * l3.y) - row[ci].x;
    }
    const float amp = __builtin_amdgcn_exp2f(e2) * amp0;
    sr = fmaf(amp, cs, sr);
    si = fmaf(amp, sn, si);
  }
  return (double)sr * sr + (double)si * si;
}

// FP64 form of the same sum (ocml sincospi/sinpi/exp).
template <bool kLinear>
__device__ inline double node_s2_fp64(double phr, const double* __restrict__ zm, const double* __restrict__ dz,
                                      const double* __restrict__ tab, int n, int M, int s1, double t1, int s2,
                                      double t2, int s3, double t3, int ci) {
  double sr = 0.0, si = 0.0;
  for (int m = 0; m < M; ++m) {
    const double tt = phr * zm[m];
    double sn, cs;
    sincospi(2.0 * (tt - rint(tt)), &sn, &cs);
    const double hh = 0.5 * phr * dz[m];
    const double amp0 = hh == 0.0 ? dz[m] : sinpi(2.0 * (hh - rint(hh))) / (kPi * phr);
    const double* row = tab + (size_t)m * n;
    double e;
    if (kLinear) {
      e = row[s3] + t3 * (row[s3 + (n > 1 ? 1 : 0)] - row[s3]);
    } else {
      const int d = n > 1 ? 1 : 0;
      e = 0.5 * ((row[s1] + t1 * (row[s1 + d] - row[s1])) + (row[s2] + t2 * (row[s2 + d] - row[s2])) +
                 (row[s3] + t3 * (row[s3 + d] - row[s3])) - row[ci]);
    }
    const double amp = exp(e) * amp0;
    sr = fma(amp, cs, sr);
    si = fma(amp, sn, si);
  }
  return sr * sr + si * si;
}

// Forward pair-integral kernel.  Persistent: each workgroup takes tiles (b, i, k) from a
// work counter; per tile it lays out the rows of each part in LDS, then strides the
// part's grid_s x grid_v nodes across its 256 lanes (a wave covers consecutive nodes of a
// row), accumulates node values in FP64 and reduces over the workgroup in a fixed order.
template <int kPrec, bool kLinear>
__global__ void __launch_bounds__(kTileBlock) k_tiles(TileArgs A) {
  extern __shared__ __align__(16) char smem_raw[];
  const TileShared sh = carve_lds(smem_raw, A.nmax, A.fp.grid_s);
  const PlanView& pv = A.pv;
  const FibreParams& fp = A.fp;
  const int M = fp.n_steps, GS = fp.grid_s, GV = fp.grid_v, tid = threadIdx.x;
  int cur_b = -1;
  for (;;) {
    if (tid == 0) *sh.tile = atomicAdd(A.w.counter, 1u);
    __syncthreads();
    const unsigned int t = *sh.tile;
    if ((int64_t)t >= pv.n_tiles) break;
    int b, i, k;
    decode_tile(pv, t, &b, &i, &k);
    const int o = pv.off[b], n = pv.off[b + 1] - o;
    if (b != cur_b) {
      for (int c = tid; c < n; c += kTileBlock) {
        const double f = pv.f[o + c], R = pv.R[o + c];
        sh.fc[c] = f;
        sh.lo_edge[c] = f - 0.5 * R;
        sh.hi_edge[c] = f + 0.5 * R;
        sh.psd[c] = A.P[o + c] / R;
      }
      cur_b = b;
    }
    __syncthreads();
    const double fi = sh.fc[i];
    const double xp = sh.hi_edge[n - 1] - fi, xn = fi - sh.lo_edge[0];
    const double slo = sh.lo_edge[k] - fi, shi = sh.hi_edge[k] - fi;
    const double wi = fi - fp.f_ref, gk = sh.psd[k];
    const double* zm = A.w.zm + (size_t)b * M;
    const double* dz = A.w.dz + (size_t)b * M;
    const float* hdz = A.w.hdz32 + (size_t)b * M;
    double acc = 0.0;
    unsigned int evaluated = 0;
    for (int part = kQ1; part <= kQ4; ++part) {
      double umax;
      if (!part_umax(part, slo, shi, xp, xn, &umax)) continue;
      const double smax = log(umax), smin = smax - fp.s_decades * kLn10, ds = (smax - smin) / GS;
      for (int a = tid; a < GS; a += kTileBlock) {
        const double s = smin + (a + 0.5) * ds, r = exp(0.5 * s);
        double vlo, vhi;
        if (part_vrange(part, r, slo, shi, xp, xn, &vlo, &vhi)) {
          const double dv = (vhi - vlo) / GV;
          sh.row_vlo[a] = vlo;
          sh.row_dv[a] = dv;
          sh.row_r[a] = r;
          sh.row_w[a] = 2.0 * exp(s) * ds * dv;
        } else {
          sh.row_dv[a] = 0.0;
        }
      }
      __syncthreads();
      const int64_t nodes = (int64_t)GS * GV;
      for (int64_t q = tid; q < nodes; q += kTileBlock) {
        const int a = (int)(q / GV), bb = (int)(q % GV);
        const double dv = sh.row_dv[a];
        if (dv == 0.0) continue;
        const double v = sh.row_vlo[a] + (bb + 0.5) * dv, r = sh.row_r[a];
        const double ev = exp(v);
        double x = r * ev, y = r / ev;
        if (part == kQ3) { x = -x; y = -y; }
        else if (part == kQ4) { y = -y; }
        const int c1 = find_channel(sh, n, fi + x);
        const int c2 = find_channel(sh, n, fi + y);
        if (c1 < 0 || c2 < 0) continue;
        const double gprod = sh.psd[c1] * sh.psd[c2] * gk;
        const double phr = phase_mismatch(x, y, wi, fp.b2, fp.b3, fp.b4) * (0.5 / kPi);
        int s1, s2, s3;
        double t1, t2, t3;
        segment(sh, n, c1, fi + x, &s1, &t1);
        segment(sh, n, c2, fi + y, &s2, &t2);
        segment(sh, n, k, fi + x + y, &s3, &t3);
        double s2v;
        if (kPrec == 0) {
          s2v = node_s2_fp32<kLinear>(phr, zm, hdz, dz, A.w.lt32 + (size_t)M * o, n, M, s1, (float)t1, s2,
                                      (float)t2, s3, (float)t3, i);
        } else {
          s2v = node_s2_fp64<kLinear>(phr, zm, dz, A.w.ell64 + (size_t)M * o, n, M, s1, t1, s2, t2, s3, t3, i);
        }
        acc += sh.row_w[a] * gprod * s2v;
        ++evaluated;
      }
      __syncthreads();
    }
    acc = wave_sum(acc);
    const double cnt = wave_sum((double)evaluated);
    if ((tid & 63) == 0) sh.red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) A.w.tiles[t] = (sh.red[0] + sh.red[1]) + (sh.red[2] + sh.red[3]);
    __syncthreads();
    if ((tid & 63) == 0 && cnt > 0) atomicAdd(A.w.nodes, (unsigned long long)cnt);
  }
}

__global__ void k_zero_counter(unsigned int* c, unsigned long long* nodes) {
  *c = 0u;
  *nodes = 0ull;
}

// ---------------------------------------------------------------------------- reduction
// One wave per channel: P_NLI,i = 16/27 gamma_i^2 R_i sum_k tile(i,k) (eq. gain_fin times R_i),
// eta_i = P_NLI,i / P_i^3, P_ASE,i = NF_i h f_i R_i / rho(L, f_i), SNR_i (eq. loss).
__global__ void k_reduce(PlanView pv, const double* __restrict__ P, const double* __restrict__ nf, double snr_trx,
                         Work w, double* eta, double* pnli_out, double* snr_out) {
  const int g = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (g >= pv.n_total) return;
  const int b = plan_of_channel(pv, g), o = pv.off[b], n = pv.off[b + 1] - o, i = g - o;
  const double* row = w.tiles + pv.toff[b] + (int64_t)i * n;
  double s = 0.0;
  for (int k = lane; k < n; k += 64) s += row[k];
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
      const double pase = nf[g] * kH * f * R * exp(-w.ellL[g]);
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
  }
  return e;
}

int tile_blocks_per_cu(const FibreParams& fp, int nmax, bool adjoint) {
  (void)adjoint;
  int nb = 0;
  const size_t shm = tile_lds_bytes(nmax, fp.grid_s);
  hipError_t e;
  if (fp.precision == 0)
    e = fp.profile == 0 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiles<0, true>, kTileBlock, shm)
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiles<0, false>, kTileBlock, shm);
  else
    e = fp.profile == 0 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiles<1, true>, kTileBlock, shm)
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiles<1, false>, kTileBlock, shm);
  if (e != hipSuccess || nb < 1) nb = 1;
  return nb;
}

hipError_t launch_tiles(const PlanView& pv, const FibreParams& fp, const double* P, const Work& w, int nmax,
                        int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(1), 0, s, w.counter, w.nodes);
  TileArgs a{pv, fp, P, w, nmax};
  const size_t shm = tile_lds_bytes(nmax, fp.grid_s);
  if (fp.precision == 0) {
    if (fp.profile == 0) hipLaunchKernelGGL((k_tiles<0, true>), dim3(grid), dim3(kTileBlock), shm, s, a);
    else hipLaunchKernelGGL((k_tiles<0, false>), dim3(grid), dim3(kTileBlock), shm, s, a);
  } else {
    if (fp.profile == 0) hipLaunchKernelGGL((k_tiles<1, true>), dim3(grid), dim3(kTileBlock), shm, s, a);
    else hipLaunchKernelGGL((k_tiles<1, false>), dim3(grid), dim3(kTileBlock), shm, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_reduce(const PlanView& pv, const FibreParams& fp, const double* P, const double* nf,
                         double snr_trx, const Work& w, double* eta, double* pnli_out, double* snr_out,
                         double* thr_out, hipStream_t s) {
  (void)fp;
  hipLaunchKernelGGL(k_reduce, dim3((pv.n_total + 3) / 4), dim3(256), 0, s, pv, P, nf, snr_trx, w, eta, pnli_out,
                     snr_out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !thr_out) return e;
  hipLaunchKernelGGL(k_throughput, dim3(pv.n_batch), dim3(256), 0, s, pv, P, w, thr_out);
  return hipGetLastError();
}

hipError_t launch_copy_profile(const PlanView& pv, const FibreParams& fp, const Work& w, double* zm, double* dz,
                               double* ell, double* ellL, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_profile, dim3(256), dim3(256), 0, s, pv, fp, w, zm, dz, ell, ellL);
  return hipGetLastError();
}

}  // namespace isrsgn
