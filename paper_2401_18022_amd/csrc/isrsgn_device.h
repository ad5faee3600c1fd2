// Device helpers shared by the forward and adjoint kernels of libisrsgn.so (internal).
//
// Model: arXiv:2401.18022 -- step sum eq. (slow_vary) inside eq. (psi_fin), power term
// eq. (pk), phase mismatch eq. (phi), hyperbolic coordinates eqs. (q1)-(q4).
#pragma once

#include <hip/hip_runtime.h>

#include "isrsgn_internal.h"

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

// Sum over the block (a multiple of 64 threads); fixed order, result on every thread.
__device__ inline double block_sum(double v, double* red) {
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

__device__ inline double sinhc(double x) {
  if (fabs(x) < 1e-4) { double x2 = x * x; return 1.0 + x2 / 6.0 + x2 * x2 / 120.0; }
  return sinh(x) / x;
}

// d sinhc / dx
__device__ inline double sinhc_d(double x) {
  if (fabs(x) < 1e-3) { double x2 = x * x; return x / 3.0 + x * x2 / 30.0 + x * x2 * x2 / 840.0; }
  return (x * cosh(x) - sinh(x)) / (x * x);
}

// ---------------------------------------------------------------------------- ODE helpers
// Block of 1024 threads, thread c owning channel c of the plan.
struct OdeShared {
  double sA[kMaxChannels], sB[kMaxChannels], sC[kMaxChannels];
  double wt[3][16];
};

// Inclusive block-wide prefix sums of three values (fixed order).
__device__ inline void block_scan3(double& a, double& bb, double& c, OdeShared& sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
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
}

// Per-channel constants of the Raman ODEs and the index windows of its gain and loss sums:
// channel c gains from j in (c, ghi] (0 < f_j - f_c <= cut) and feeds j in [llo, c).
struct OdeChan {
  double f, ft, alpha, cr, p0;
  int ghi, llo;
};

__device__ inline OdeChan ode_chan(const PlanView& pv, const FibreParams& fp, const double* P, int o, int n, int c,
                                   double fmid) {
  OdeChan ch{};
  ch.f = pv.f[o + c];
  ch.ft = ch.f - fmid;
  ch.alpha = pv.alpha[o + c];
  ch.cr = pv.cr[o + c];
  ch.p0 = P[o + c];
  const double cut = fp.cutoff;
  int lo = c, hi = n;  // last j with f_j - f_c <= cut
  if (cut <= 0) lo = n - 1;
  else
    while (hi - lo > 1) { int mid = (lo + hi) >> 1; if (pv.f[o + mid] - ch.f <= cut) lo = mid; else hi = mid; }
  ch.ghi = lo;
  int l2 = -1, h2 = c;  // first j with f_c - f_j <= cut
  if (cut <= 0) h2 = 0;
  else
    while (h2 - l2 > 1) { int mid = (l2 + h2) >> 1; if (ch.f - pv.f[o + mid] <= cut) h2 = mid; else l2 = mid; }
  ch.llo = h2;
  return ch;
}

// Window sums of the prefix arrays: (c, ghi] and [llo, c).
__device__ inline void window_above(const OdeShared& sh, const OdeChan& ch, int c, double* A, double* B, double* Cc) {
  *A = *B = *Cc = 0.0;
  if (ch.ghi > c) {
    *A = sh.sA[ch.ghi] - sh.sA[c];
    *B = sh.sB[ch.ghi] - sh.sB[c];
    *Cc = sh.sC[ch.ghi] - sh.sC[c];
  }
}
__device__ inline void window_below(const OdeShared& sh, const OdeChan& ch, int c, double* A, double* B, double* Cc) {
  *A = *B = *Cc = 0.0;
  if (c > ch.llo) {
    const double bA = ch.llo > 0 ? sh.sA[ch.llo - 1] : 0.0;
    const double bB = ch.llo > 0 ? sh.sB[ch.llo - 1] : 0.0;
    const double bC = ch.llo > 0 ? sh.sC[ch.llo - 1] : 0.0;
    *A = sh.sA[c - 1] - bA;
    *B = sh.sB[c - 1] - bB;
    *Cc = sh.sC[c - 1] - bC;
  }
}

// ---------------------------------------------------------------------------- tile geometry
// Parts of tile (i,k) in offsets (x, y) = (f1 - f_i, f2 - f_i) with x + y in [slo, shi):
//   Q1: x = r e^v, y = r e^-v, v >= 0 (fold about x = y)
//   Q3: x = -r e^v, y = -r e^-v, v >= 0 (fold)
//   Q4: x = r e^v, y = -r e^-v (stands for the mirror part Q2 as well)
// r = sqrt(|x y|) = e^(s/2).  sup|x y| fixes the top of the s window.
enum { kQ1 = 0, kQ3 = 1, kQ4 = 2 };

__device__ inline bool part_umax(int part, double slo, double shi, double xp, double xn, double* umax) {
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

__device__ inline bool part_vrange(int part, double r, double slo, double shi, double xp, double xn, double* vlo,
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

// Channel data of the current plan in LDS.
struct ChanLds {
  double* fc;
  double* hw;   // (1 + beta) R_c/2: half the width of the spectrum's support
  double* psd;  // P_c / R_c: the flat part of the PSD
  // the support's edges (the same FP64 operations wherever they are formed)
  __device__ double lo(int c) const { return fc[c] - hw[c]; }
  __device__ double hi(int c) const { return fc[c] + hw[c]; }
};

// Row layout of the current part in LDS: v_lo, dv (0: empty row), r, node weight.
struct RowLds {
  double *vlo, *dv, *r, *w;
};

__device__ inline void load_channels(const ChanLds& ch, const PlanView& pv, const double* P, int o, int n,
                                     double beta) {
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    const double f = pv.f[o + c], R = pv.R[o + c], hw = beta > 0.0 ? 0.5 * (1.0 + beta) * R : 0.5 * R;
    ch.fc[c] = f;
    ch.hw[c] = hw;
    ch.psd[c] = P[o + c] / R;
  }
}

// Raised-cosine spectrum relative to its flat part: 1 for |u| <= (1-beta) R/2, then
// (1 + cos(pi (|u| - (1-beta) R/2) / (beta R))) / 2 to the support edge (u = F - f_c; beta > 0).
__device__ inline double rc_shape(double u, double R, double beta) {
  const double a = fabs(u), flat = 0.5 * (1.0 - beta) * R;
  if (a <= flat) return 1.0;
  return 0.5 * (1.0 + cospi((a - flat) / (beta * R)));
}

// The shape of channel c at F (its symbol rate from the support's half-width (1 + beta) R/2).
__device__ inline double shape_at(const ChanLds& ch, int c, double F, double beta) {
  return rc_shape(F - ch.fc[c], 2.0 * ch.hw[c] / (1.0 + beta), beta);
}

// Laplace transform M(a) = int g(u) exp(-a u) du of the unit-area raised cosine (rectangle: beta = 0):
// sinhc(a R/2) cosh(a beta R/2) / (1 + (a beta R / pi)^2), and its derivative in a.
__device__ inline double spectrum_m(double a, double R, double beta) {
  const double s = sinhc(0.5 * a * R);
  if (!(beta > 0.0)) return s;
  const double h = 0.5 * beta * R, c = beta * R / kPi, ac = a * c;
  return s * cosh(a * h) / (1.0 + ac * ac);
}
__device__ inline double spectrum_md(double a, double R, double beta) {
  const double s = sinhc(0.5 * a * R), sd = 0.5 * R * sinhc_d(0.5 * a * R);
  if (!(beta > 0.0)) return sd;
  const double h = 0.5 * beta * R, c = beta * R / kPi, ac = a * c, d = 1.0 + ac * ac;
  const double ch = cosh(a * h), shd = h * sinh(a * h);
  return (sd * ch + s * shd) / d - s * ch * (2.0 * ac * c) / (d * d);
}

// Interpolation segment and weight of ln rho at F, given the channel c that holds F.  kT32: the
// weight for the FP32 form, which uses it in FP32 (offset in FP64, then an FP32 quotient).
template <bool kT32 = false>
__device__ inline void segment(const ChanLds& ch, int n, int c, double F, int* seg, double* t) {
  if (n == 1) { *seg = 0; *t = 0.0; return; }
  int s = F >= ch.fc[c] ? c : c - 1;
  s = s < 0 ? 0 : (s > n - 2 ? n - 2 : s);
  *seg = s;
  if constexpr (kT32)
    *t = (double)((float)(F - ch.fc[s]) * __builtin_amdgcn_rcpf((float)(ch.fc[s + 1] - ch.fc[s])));
  else
    *t = (F - ch.fc[s]) / (ch.fc[s + 1] - ch.fc[s]);
}

// The f term of eq. (pk) at the NLI frequency F of COI i (fc: the plan's centres): the centre
// itself (segment i, weight 0, exact for every i) or the interpolation segment holding F,
// extrapolated with the end segments like f1 and f2.
__device__ inline void nli_segment(const double* fc, int n, int i, double F, int* seg, double* t) {
  if (F == fc[i] || n == 1) { *seg = i; *t = 0.0; return; }
  int s = F >= fc[i] ? i : i - 1;
  s = s < 0 ? 0 : (s > n - 2 ? n - 2 : s);
  *seg = s;
  *t = (F - fc[s]) / (fc[s + 1] - fc[s]);
}

// eq. (phi): phase mismatch per metre for offsets x, y and COI offset w from f_ref.
__device__ inline double phase_mismatch(double x, double y, double w, double b2, double b3, double b4) {
  const double p4 = x * x + 1.5 * x * y + y * y + 3.0 * x * w + 3.0 * y * w + 3.0 * w * w;
  return -4.0 * kPi * kPi * x * y * (b2 + kPi * b3 * (x + y + 2.0 * w) + (2.0 * kPi * kPi / 3.0) * b4 * p4);
}

// Decode a global tile index into (plan, COI, COI point, interferer): plan b's tiles are [i][j][k].
__device__ inline void decode_tile(const PlanView& pv, unsigned int t, int* b, int* i, int* j, int* k) {
  int lo = 0, hi = pv.n_batch;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (pv.toff[mid] <= (int64_t)t) lo = mid; else hi = mid;
  }
  const int n = pv.off[lo + 1] - pv.off[lo];
  const int64_t loc = (int64_t)t - pv.toff[lo], row = loc / n;
  *b = lo;
  *i = (int)(row / pv.nli);
  *j = (int)(row % pv.nli);
  *k = (int)(loc % n);
}

// Geometry of tile (i, j, k) of the current plan: fi is the NLI frequency of point j of COI i
// (the centre f_i with one point).
struct TileGeo {
  double fi, xp, xn, slo, shi, wi, gk;
  double lo0;  // lower edge of the plan's first channel
  float cinv;  // channels per Hz of the plan's lower edges, on average (0 for one channel)
};

__device__ inline TileGeo tile_geo(const ChanLds& ch, int n, double fnli, int k, double f_ref) {
  TileGeo g;
  g.fi = fnli;
  g.xp = ch.hi(n - 1) - g.fi;
  g.xn = g.fi - ch.lo(0);
  g.slo = ch.lo(k) - g.fi;
  g.shi = ch.hi(k) - g.fi;
  g.wi = g.fi - f_ref;
  g.gk = ch.psd[k];
  g.lo0 = ch.lo(0);
  g.cinv = n > 1 ? (float)((double)(n - 1) / (ch.lo(n - 1) - g.lo0)) : 0.0f;
  return g;
}

// The tile geometry is the same for every lane but comes from LDS loads, which the compiler
// keeps in vector registers; moving it to scalar registers frees 14 VGPRs per lane.
__device__ inline double uniform_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffLL));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline TileGeo uniform_geo(TileGeo g) {
  g.fi = uniform_f64(g.fi);
  g.xp = uniform_f64(g.xp);
  g.xn = uniform_f64(g.xn);
  g.slo = uniform_f64(g.slo);
  g.shi = uniform_f64(g.shi);
  g.wi = uniform_f64(g.wi);
  g.gk = uniform_f64(g.gk);
  g.lo0 = uniform_f64(g.lo0);
  g.cinv = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(g.cinv)));
  return g;
}

// Lays out the rows of one part in LDS (all threads of the block); false if the part is empty.
__device__ inline bool layout_rows(const RowLds& rw, const TileGeo& g, int part, int gs, int gv, double s_decades) {
  double umax;
  if (!part_umax(part, g.slo, g.shi, g.xp, g.xn, &umax)) return false;
  const double smax = log(umax), smin = smax - s_decades * kLn10, ds = (smax - smin) / gs;
  for (int a = threadIdx.x; a < gs; a += blockDim.x) {
    const double s = smin + (a + 0.5) * ds, r = exp(0.5 * s);
    double vlo, vhi;
    if (part_vrange(part, r, g.slo, g.shi, g.xp, g.xn, &vlo, &vhi)) {
      const double dv = (vhi - vlo) / gv;
      rw.vlo[a] = vlo;
      rw.dv[a] = dv;
      rw.r[a] = r;
      rw.w[a] = 2.0 * exp(s) * ds * dv;
    } else {
      rw.dv[a] = 0.0;
    }
  }
  return true;
}

// Channel whose band [f_c - R_c/2, f_c + R_c/2) holds F, or -1.  The index is first estimated
// from the plan's mean spacing and then walked to the last lower edge at or below F: one or two
// LDS reads on a regular grid.  After four steps the walk gives way to a binary search, so any
// spacing gives the same channel as the search alone.
__device__ inline int find_channel(const ChanLds& ch, int n, double F, const TileGeo& g) {
  if (F < g.lo0) return -1;
  int c = (int)((float)(F - g.lo0) * g.cinv);
  c = c < 0 ? 0 : (c > n - 1 ? n - 1 : c);
  int steps = 0;
  while (c > 0 && ch.lo(c) > F && steps < 4) { --c; ++steps; }
  while (c + 1 < n && ch.lo(c + 1) <= F && steps < 4) { ++c; ++steps; }
  if (steps >= 4) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (ch.lo(mid) <= F) lo = mid; else hi = mid;
    }
    c = lo;
  }
  return F < ch.hi(c) ? c : -1;
}

// One node of a part: offsets, channels, interpolation segments, phase rate (revolutions per m).
struct Node {
  double w, gprod, phr;
  int c1, c2, s1, s2, s3;
  double t1, t2, t3;
};

// n identical spans: the spans' fields differ by the phase phi (k-1) L, so |S|^2 gains the
// phased-array factor |sum_k e^(j phi (k-1) L)|^2 = sin^2(n phi L/2) / sin^2(phi L/2) (App. A).
// x = phi L / (2 pi) in revolutions; the factor has period 1 in x and tends to n^2 at integers.
__device__ inline double span_array_factor(double x, int n) {
  const double r = x - rint(x);
  if (fabs(r) < 1e-12) return (double)n * n;
  const double q = sinpi(n * r) / sinpi(r);
  return q * q;
}

// kT32: segment weights for the FP32 form
template <bool kT32 = false>
__device__ inline bool make_node(const ChanLds& ch, const RowLds& rw, const TileGeo& g, int n, int k, int part,
                                 int a, int bcol, const FibreParams& fp, Node* nd) {
  const double dv = rw.dv[a];
  if (dv == 0.0) return false;
  const double v = rw.vlo[a] + (bcol + 0.5) * dv, r = rw.r[a];
  const double ev = exp(v);
  double x = r * ev, y = r / ev;
  if (part == kQ3) { x = -x; y = -y; }
  else if (part == kQ4) { y = -y; }
  const int c1 = find_channel(ch, n, g.fi + x, g);
  const int c2 = find_channel(ch, n, g.fi + y, g);
  if (c1 < 0 || c2 < 0) return false;
  nd->w = rw.w[a];
  nd->c1 = c1;
  nd->c2 = c2;
  nd->gprod = ch.psd[c1] * ch.psd[c2] * g.gk;
  nd->phr = phase_mismatch(x, y, g.wi, fp.b2, fp.b3, fp.b4) * (0.5 / kPi);
  if (fp.n_spans > 1) nd->w *= span_array_factor(nd->phr * fp.span, fp.n_spans);
  segment<kT32>(ch, n, c1, g.fi + x, &nd->s1, &nd->t1);
  segment<kT32>(ch, n, c2, g.fi + y, &nd->s2, &nd->t2);
  segment<kT32>(ch, n, k, g.fi + x + y, &nd->s3, &nd->t3);
  return true;
}

// Raised-cosine shapes of a node's f1, f2 and f3 relative to the flat PSDs (Node::gprod holds the
// flat ones), recomputed from the node's row and column; called after the node's step sum, where
// few registers are live (rolloff > 0 only).
__device__ inline void node_shapes(const ChanLds& ch, const RowLds& rw, const TileGeo& g, int k, int part, int a,
                                   int bcol, int c1, int c2, double beta, double* sh1, double* sh2, double* sh3) {
  const double v = rw.vlo[a] + (bcol + 0.5) * rw.dv[a], r = rw.r[a];
  const double ev = exp(v);
  double x = r * ev, y = r / ev;
  if (part == kQ3) { x = -x; y = -y; }
  else if (part == kQ4) { y = -y; }
  *sh1 = shape_at(ch, c1, g.fi + x, beta);
  *sh2 = shape_at(ch, c2, g.fi + y, beta);
  *sh3 = shape_at(ch, k, g.fi + x + y, beta);
}

// ---------------------------------------------------------------------------- step terms
// Term m of S = sum_m p_m dz_m exp(j phi z_m) sinc(phi dz_m / 2) (eq. slow_vary), returned as
// (re, im).  p_m = exp(E_m), E_m = [ln rho(f1) + ln rho(f2) + ln rho(f3) - ln rho(f_i)] / 2 (eq. pk);
// with a profile linear in f (the closed form) E_m = ln rho(f3) exactly.
//
// FP32 form: the phase phi z_m is formed in FP64 and reduced to [0, 1) revolutions before
// the FP32 hardware sine/cosine (which take revolutions); the sinc factor uses its Taylor
// polynomial while |phi dz_m / 2| < 1/2 and the edge form beyond; E_m comes from an FP32 table of
// ln rho log2(e)/2 (Gather32) or from its low-rank form (LowRank32).
// Per-step data of a plan, read with wave-uniform addresses.  k_steps writes the plan's records to
// global memory; the forward tile kernel stages them in LDS, and the adjoint reads the global copy
// through the constant address space (scalar loads into SGPRs, no VGPRs or LDS traffic).
struct StepRec {
  double zm;   // step midpoint z_m
  double zu;   // upper edge z_m + dz_m / 2 (the lower edge of step 0 is z = 0)
  float hdz;   // dz_m / 2
  float zmf;   // z_m in FP32 (the FP32-phase form)
  float dz;    // dz_m
  float c2;    // (2 pi dz_m / 2)^2: the sinc argument squared is phr^2 c2
};

__host__ __device__ inline StepRec step_record(double zm, double dz, float hdz) {
  StepRec v;
  v.zm = zm;
  v.zu = zm + 0.5 * dz;
  v.hdz = hdz;
  v.zmf = (float)zm;
  v.dz = 2.0f * hdz;
  const float c = 2.0f * (float)kPi * hdz;
  v.c2 = c * c;
  return v;
}

// Step m from the LDS copy or from the global one (field by field: no copy constructor binds to
// the constant address space); the step functions below take either pointer kind (SP).
using ConstStep = const __attribute__((address_space(4))) StepRec;
__device__ inline StepRec step_at(const StepRec* st, int m) { return st[m]; }
__device__ inline StepRec step_at(ConstStep* st, int m) {
  StepRec v;
  v.zm = st[m].zm;
  v.zu = st[m].zu;
  v.hdz = st[m].hdz;
  v.zmf = st[m].zmf;
  v.dz = st[m].dz;
  v.c2 = st[m].c2;
  return v;
}

// Per-tile table columns for the f3 and f_i terms of E_m, staged in LDS.  f3 lies in channel k,
// so its interpolation segment is A = clamp(k-1) or B = clamp(k); per step:
//   general profile: (L_A - L_i, dL_A, L_B - L_i, dL_B)   (L = ln rho log2(e)/2, dL to the next centre)
//   linear profile:  (2 L_A, 2 dL_A, 2 L_B, 2 dL_B)
struct Col4 {
  float ax, ay, bx, by;
};

struct Term32 {
  double phr;
  float phrf, phrf2, inv_piphr, t1, t2, t3;
  unsigned o1, o2;  // byte offsets of the f1 / f2 segments within a table row
  bool up3;         // f3 uses segment B
};

__device__ inline Term32 term32_setup(const Node& nd, int k, int n) {
  Term32 q;
  q.phr = nd.phr;
  q.phrf = (float)nd.phr;
  q.phrf2 = q.phrf * q.phrf;
  q.inv_piphr = 1.0f / ((float)kPi * q.phrf);
  q.t1 = (float)nd.t1;
  q.t2 = (float)nd.t2;
  q.t3 = (float)nd.t3;
  q.o1 = (unsigned)nd.s1 * (unsigned)sizeof(float2);
  q.o2 = (unsigned)nd.s2 * (unsigned)sizeof(float2);
  const int segb = k < n - 2 ? k : (n - 2 > 0 ? n - 2 : 0);
  q.up3 = nd.s3 == segb;
  return q;
}

// Column segments of tile (i,k): A = clamp(k-1, 0, n-2), B = clamp(k, 0, n-2).
__device__ inline void col_segments(int k, int n, int* sa, int* sb) {
  const int hi = n - 2 > 0 ? n - 2 : 0;
  *sa = k - 1 < 0 ? 0 : (k - 1 > hi ? hi : k - 1);
  *sb = k > hi ? hi : k;
}

// sf, tf: the f term's segment and weight (nli_segment)
template <bool kLinear>
__device__ inline void load_cols(Col4* col, const float2* __restrict__ tab, int n, int M, int sf, double tf, int k) {
  int sa, sb;
  col_segments(k, n, &sa, &sb);
  for (int m = threadIdx.x; m < M; m += blockDim.x) {
    const float2* row = tab + (size_t)m * n;
    const float2 A = row[sa], B = row[sb];
    Col4 c;
    if (kLinear) {
      c.ax = 2.0f * A.x; c.ay = 2.0f * A.y; c.bx = 2.0f * B.x; c.by = 2.0f * B.y;
    } else {
      const float li = fmaf((float)tf, row[sf].y, row[sf].x);
      c.ax = A.x - li; c.ay = A.y; c.bx = B.x - li; c.by = B.y;
    }
    col[m] = c;
  }
}

__device__ inline void load_steps(StepRec* st, const double* __restrict__ zm, const double* __restrict__ dz,
                                  const float* __restrict__ hdz, int M) {
  for (int m = threadIdx.x; m < M; m += blockDim.x) st[m] = step_record(zm[m], dz[m], hdz[m]);
}

// The plan's FP32 profile table [m][c] (float2: scaled ln rho and the slope to the next
// channel) behind a raw buffer descriptor: per step the row offset is a scalar and each
// node's segment offsets are fixed vector offsets, so the loads need no per-step vector
// address arithmetic.  3rd-dword 0x00020000: raw 32-bit data format on gfx9.
struct Tab32 {
  __amdgpu_buffer_rsrc_t r;
};

__device__ inline Tab32 make_tab32(const float2* tab, int n, int M) {
  return Tab32{__builtin_amdgcn_make_buffer_rsrc(const_cast<float2*>(tab), (short)0,
                                                 (int)((unsigned)n * (unsigned)M * (unsigned)sizeof(float2)),
                                                 0x00020000)};
}

__device__ inline float2 tab32_at(const Tab32& t, unsigned voff, unsigned soff) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(t.r, voff, soff, 0);
  return make_float2(__uint_as_float(v[0]), __uint_as_float(v[1]));
}

// Evaluation forms of the FP32 step term.  Along the steps dz_m grows (equal power decrement),
// so each node has a first step m_s from which |phi dz_m / 2| >= 1/2 ("sine steps"); before it
// the sinc factor is its Taylor polynomial.  A wave runs its nodes' steps in up to three ranges,
// each in one form for all lanes (m_lo, m_hi: the smallest and largest m_s of the wave):
//   kTierSmall: every node has |phi| z_max < 1/4 revolution and no sine step: phase formed in
//               FP32 (error < 5e-8 revolutions), polynomial sinc -- no FP64;
//   kTierPoly:  steps [0, m_lo): FP64 phase, polynomial sinc;
//   kTierMixed: steps [m_lo, m_hi): FP64 phase, polynomial or sine chosen per lane;
//   edge form:  steps [m_hi, M): every lane is past m_s.  Since z_m is the step midpoint,
//               dz_m sinc(phi dz_m / 2) e^(j phi z_m) = (E_(m+1) - E_m) / (j phi) with the edge
//               phasors E = e^(j phi z) at z_m -+ dz_m / 2 (the exact integral of e^(j phi z)
//               over the step), so one sine/cosine pair per step, carried from step to step,
//               replaces the phase pair and the sinc sine.
enum { kTierMixed = 0, kTierSmall = 1, kTierPoly = 2 };

// Sources of the f1 + f2 part of log2 p_m (eq. pk) for the FP32 step terms.
//   Gather32:  the scaled profile table, interpolated at the node's f1 and f2 segments;
//   LowRank32: the plan's low-rank form of that table, L(m, c) ~ sum_r a_r(m) b_r(c): per node
//              c_r = b_r(f1) + b_r(f2) + b_r(f3) - b_r(f_i) (interpolated like the table --
//              interpolation commutes with the factorisation), per step sum_r a_r(m) c_r with
//              a_r(m) from LDS: the whole exponent, with no memory gathers and no column reads.
struct Gather32 {
  static constexpr bool kAllTerms = false;  // the f3, f_i terms come from the tile's columns
  Tab32 tab;
  int n;
  __device__ float e12(const Term32& q, int m) const {
    const unsigned row = (unsigned)m * (unsigned)n * (unsigned)sizeof(float2);
    const float2 l1 = tab32_at(tab, q.o1, row), l2 = tab32_at(tab, q.o2, row);
    return fmaf(q.t1, l1.y, l1.x) + fmaf(q.t2, l2.y, l2.x);
  }
};

// Global memory that no kernel writes while the reading kernel runs (the constant address space):
// wave-uniform loads from it become scalar loads into SGPRs.
using ConstF32 = const __attribute__((address_space(4))) float;
__device__ inline ConstF32* const_f32(const float* p) { return (ConstF32*)p; }

struct LowRank32 {
  static constexpr bool kAllTerms = true;
  // the plan's a_r(m), [M][kRank] in global memory: every lane of a wave reads the same step, so
  // the reads are scalar loads and the factors sit in SGPRs (no LDS traffic, no VGPRs)
  ConstF32* a;
  float c[kRank];
  // b: the plan's [channel][kRank] (b_r, b_r(next channel) - b_r); b3: the same row of the
  // node's f3 segment, one of the tile's column pair (LDS); bf: the tile's f term b_r at its NLI
  // frequency (LDS); both from lowrank_tile_terms
  // kB3Vec4: b3s is 16-byte aligned (a row of b in global memory), read as float4
  template <bool kB3Vec4 = false>
  __device__ void setup(const Term32& q, const float2* __restrict__ b, const float2* b3s, const float* bf) {
    const float4* b1 = reinterpret_cast<const float4*>(b + (size_t)(q.o1 / sizeof(float2)) * kRank);
    const float4* b2 = reinterpret_cast<const float4*>(b + (size_t)(q.o2 / sizeof(float2)) * kRank);
#pragma unroll
    for (int j = 0; j < kRank / 2; ++j) {
      const float4 u = b1[j], v = b2[j];
      float2 w0, w1;  // (the LDS rows are only 8-byte aligned)
      if constexpr (kB3Vec4) {
        const float4 w = reinterpret_cast<const float4*>(b3s)[j];
        w0 = make_float2(w.x, w.y);
        w1 = make_float2(w.z, w.w);
      } else {
        w0 = b3s[2 * j];
        w1 = b3s[2 * j + 1];
      }
      c[2 * j] = (fmaf(q.t1, u.y, u.x) + fmaf(q.t2, v.y, v.x)) + (fmaf(q.t3, w0.y, w0.x) - bf[2 * j]);
      c[2 * j + 1] = (fmaf(q.t1, u.w, u.z) + fmaf(q.t2, v.w, v.z)) + (fmaf(q.t3, w1.y, w1.x) - bf[2 * j + 1]);
    }
  }
  // smallest terms first; the same order as the factorisation's FP32 check
  __device__ float e12(const Term32&, int m) const {
    float e = 0.0f;
#pragma unroll
    for (int j = kRank / 4 - 1; j >= 0; --j) {
      ConstF32* v = a + m * kRank + 4 * j;
      e = fmaf(v[3], c[4 * j + 3], e);
      e = fmaf(v[2], c[4 * j + 2], e);
      e = fmaf(v[1], c[4 * j + 1], e);
      e = fmaf(v[0], c[4 * j], e);
    }
    return e;
  }
};

// Per-tile terms of the low-rank exponent in LDS, t[5 kRank] (kRank + 2 kRank float2):
//   t[0, kRank): the f term bf_r = b_r(sf) + tf (b_r(sf + 1) - b_r(sf)) (b_r(sf) itself at a
//   channel centre); then the rows (b_r, next - b_r) of the tile's two f3 segments A = sa, B = sb.
// Written by the first 3 kRank threads.
constexpr int kLrTileFloats = 5 * kRank;

// The f term alone (the first kRank floats of lowrank_tile_terms), by the first kRank threads.
__device__ inline void lowrank_f_term(const float2* __restrict__ b, int sf, float tf, float* bf) {
  if (threadIdx.x < kRank) {
    const float2 x = b[(size_t)sf * kRank + threadIdx.x];
    bf[threadIdx.x] = tf == 0.0f ? x.x : fmaf(tf, x.y, x.x);
  }
}
__device__ inline void lowrank_tile_terms(const float2* __restrict__ b, int sf, float tf, int sa, int sb, float* t) {
  const int r = threadIdx.x;
  if (r < kRank) {
    const float2 x = b[(size_t)sf * kRank + r];
    t[r] = tf == 0.0f ? x.x : fmaf(tf, x.y, x.x);
  } else if (r < 3 * kRank) {
    const int q = r - kRank;
    reinterpret_cast<float2*>(t + kRank)[q] = b[(size_t)(q < kRank ? sa : sb) * kRank + q % kRank];
  }
}

template <bool kLinear, class Src>
__device__ inline float log2p32(const Term32& q, int m, float2 cab, const Src& src) {
  if constexpr (!kLinear && Src::kAllTerms) return src.e12(q, m);
  const float e3 = fmaf(q.t3, cab.y, cab.x);
  if (kLinear) return e3;
  return src.e12(q, m) + e3;
}

// Column pair of step m for this node: the f3 term uses one of the two segments (fixed per node).
__device__ inline float2 col_pair(const Term32& q, const Col4* __restrict__ col, int m) {
  return reinterpret_cast<const float2*>(col + m)[q.up3 ? 1 : 0];
}

// Amplitude of step m's term in the midpoint forms: p_m dz_m sinc(phi dz_m / 2).
template <bool kLinear, int kTier, class Src>
__device__ inline float amp32(const Term32& q, int m, const StepRec& sv, float2 cab, const Src& src) {
  const float u2 = q.phrf2 * sv.c2;
  float amp0 = sv.dz * fmaf(u2, fmaf(u2, fmaf(u2, -1.0f / 5040.0f, 1.0f / 120.0f), -1.0f / 6.0f), 1.0f);
  if (kTier == kTierMixed) {  // both forms, then a per-lane select (no branch)
    const float hh = q.phrf * sv.hdz;
    const float as = __builtin_amdgcn_sinf(hh - rintf(hh)) * q.inv_piphr;
    amp0 = u2 < 0.25f ? amp0 : as;
  }
  return __builtin_amdgcn_exp2f(log2p32<kLinear>(q, m, cab, src)) * amp0;
}

template <bool kLinear, int kTier, class Src, class SP>
__device__ inline float2 term32(const Term32& q, int m, SP st, const Col4* __restrict__ col,
                                const Src& src) {
  const StepRec sv = step_at(st, m);
  const float2 cab = col_pair(q, col, m);
  float fr;
  if (kTier == kTierSmall) {
    fr = q.phrf * sv.zmf;  // |phr z_m| < 1/4 at every step in this form: already reduced
  } else {
    // fract(phr z_m) in [0, 1): one product and fract in FP64, then the conversion (the hardware
    // sine and cosine take any argument within 256 revolutions, equally accurate on [0, 1))
    fr = (float)__builtin_amdgcn_fract(q.phr * sv.zm);
  }
  const float sn = __builtin_amdgcn_sinf(fr);
  const float cs = __builtin_amdgcn_cosf(fr);
  const float amp = amp32<kLinear, kTier>(q, m, sv, cab, src);
  return make_float2(amp * cs, amp * sn);
}

// (cos, sin) of 2 pi phr z at a step edge, the FP64 phase reduced to [0, 1) revolutions.
__device__ inline float2 edge_phasor32(double phr, double z) {
  const float fr = (float)__builtin_amdgcn_fract(phr * z);
  return make_float2(__builtin_amdgcn_cosf(fr), __builtin_amdgcn_sinf(fr));
}

// Phasor at the lower edge of step m.
template <class SP>
__device__ inline float2 lower_edge_phasor32(double phr, SP st, int m) {
  return m > 0 ? edge_phasor32(phr, st[m - 1].zu) : make_float2(1.0f, 0.0f);
}

// Step m in edge form, as 2 pi phr times its term: p_m (E_(m+1) - E_m) / j.  e holds E_m on
// entry and E_(m+1) on return.
template <bool kLinear, class Src, class SP>
__device__ inline float2 term32_edge(const Term32& q, int m, SP st,
                                     const Col4* __restrict__ col, const Src& src, float2& e) {
  const double zu = st[m].zu;
  const float2 cab = col_pair(q, col, m);
  const float2 e1 = edge_phasor32(q.phr, zu);
  const float p = __builtin_amdgcn_exp2f(log2p32<kLinear>(q, m, cab, src));
  const float2 r = make_float2(p * (e1.y - e.y), p * (e.x - e1.x));
  e = e1;
  return r;
}

// First sine step m_s of a node (M if none): the same test as the mixed form's select.
template <class SP>
__device__ inline int sine_step(const Term32& q, SP st, int M) {
  if (q.phrf2 * st[0].c2 >= 0.25f) return 0;
  if (q.phrf2 * st[M - 1].c2 < 0.25f) return M;
  int lo = 1, hi = M - 1;  // the answer lies in [1, M - 1]
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (q.phrf2 * st[mid].c2 < 0.25f) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Whether a node qualifies for the FP32-phase form (plan's last step: largest z and dz).
template <class SP>
__device__ inline bool node_small(const Term32& q, SP st, int M) {
  const float ap = fabsf(q.phrf), tp = 2.0f * (float)kPi;
  return ap * st[M - 1].zmf < 0.25f && tp * ap * st[M - 1].hdz < 0.5f;
}

// The wave's ranges.  Every lane of the wave must be active; lanes without a node pass
// active = false and do not restrict the result.
struct Split32 {
  bool small;      // kTierSmall for all steps
  int m_lo, m_hi;  // 0 <= m_lo <= m_hi <= M
};

template <class SP>
__device__ inline Split32 wave_split(bool active, const Term32& q, SP st, int M) {
  Split32 r;
  r.small = __all(!active || node_small(q, st, M));
  if (r.small) {
    r.m_lo = r.m_hi = M;
    return r;
  }
  int lo = M, hi = 0;
  if (active) lo = hi = sine_step(q, st, M);
#pragma unroll
  for (int sh = 1; sh < 64; sh <<= 1) {
    lo = min(lo, __shfl_xor(lo, sh));
    hi = max(hi, __shfl_xor(hi, sh));
  }
  // equal in every lane after the butterfly: scalar registers, so the range loops are uniform
  // (their table loads keep a scalar row offset)
  lo = __builtin_amdgcn_readfirstlane(lo);
  hi = __builtin_amdgcn_readfirstlane(hi);
  r.m_lo = lo;
  r.m_hi = hi > lo ? hi : lo;
  return r;
}

// Sum of the step terms over [m0, m1) in form kTier (not the edge form).
template <bool kLinear, int kTier, int kUnroll, class Src, class SP>
__device__ inline void accumulate_range32(const Term32& q, SP st, const Col4* __restrict__ col,
                                          const Src& src, int m0, int m1, float* a, float* b) {
  float x = 0.0f, y = 0.0f;
#pragma unroll kUnroll
  for (int m = m0; m < m1; ++m) {
    const float2 t = term32<kLinear, kTier>(q, m, st, col, src);
    x += t.x;
    y += t.y;
  }
  *a += x;
  *b += y;
}

// S of one node: the wave's ranges in order, the edge range scaled by 1 / (2 pi phr) at the end.
template <bool kLinear, int kUnroll, class Src, class SP>
__device__ inline void accumulate32(const Term32& q, const Split32& sp, SP st,
                                    const Col4* __restrict__ col, const Src& src, int M, float* sr, float* si) {
  float a = 0.0f, b = 0.0f;
  if (sp.small) {
    accumulate_range32<kLinear, kTierSmall, kUnroll>(q, st, col, src, 0, M, &a, &b);
  } else {
    if (sp.m_lo > 0) accumulate_range32<kLinear, kTierPoly, kUnroll>(q, st, col, src, 0, sp.m_lo, &a, &b);
    if (sp.m_hi > sp.m_lo) accumulate_range32<kLinear, kTierMixed, kUnroll>(q, st, col, src, sp.m_lo, sp.m_hi, &a, &b);
    if (sp.m_hi < M) {
      float2 e = lower_edge_phasor32(q.phr, st, sp.m_hi);
      float x = 0.0f, y = 0.0f;
#pragma unroll kUnroll
      for (int m = sp.m_hi; m < M; ++m) {
        const float2 t = term32_edge<kLinear>(q, m, st, col, src, e);
        x += t.x;
        y += t.y;
      }
      const float h = 0.5f * q.inv_piphr;
      a = fmaf(h, x, a);
      b = fmaf(h, y, b);
    }
  }
  *sr = a;
  *si = b;
}

// FP64 form of the same term (ocml sincospi / sinpi / exp on the FP64 table).
struct Term64 {
  double phr, t1, t2, t3;
  int s1, s2, s3;
};

// The tile's f term of eq. (pk) per step (FP64 form): ln rho(z_m) at its NLI frequency, in LDS.
__device__ inline void load_fcol64(double* lf, const double* __restrict__ tab, int n, int M, int sf, double tf) {
  const int d = n > 1 ? 1 : 0;
  for (int m = threadIdx.x; m < M; m += blockDim.x) {
    const double* row = tab + (size_t)m * n;
    lf[m] = tf == 0.0 ? row[sf] : row[sf] + tf * (row[sf + d] - row[sf]);
  }
}

__device__ inline Term64 term64_setup(const Node& nd) {
  Term64 q;
  q.phr = nd.phr;
  q.t1 = nd.t1;
  q.t2 = nd.t2;
  q.t3 = nd.t3;
  q.s1 = nd.s1;
  q.s2 = nd.s2;
  q.s3 = nd.s3;

  return q;
}

// lf: the tile's f-term column (load_fcol64)
template <bool kLinear>
__device__ inline double2 term64(const Term64& q, int m, const double* __restrict__ zm, const double* __restrict__ dz,
                                 const double* __restrict__ tab, int n, const double* lf) {
  const double tt = q.phr * zm[m];
  double sn, cs;
  sincospi(2.0 * (tt - rint(tt)), &sn, &cs);
  const double hh = 0.5 * q.phr * dz[m];
  const double amp0 = hh == 0.0 ? dz[m] : sinpi(2.0 * (hh - rint(hh))) / (kPi * q.phr);
  const double* row = tab + (size_t)m * n;
  const int d = n > 1 ? 1 : 0;
  double e;
  if (kLinear) {
    e = row[q.s3] + q.t3 * (row[q.s3 + d] - row[q.s3]);
  } else {
    e = 0.5 * ((row[q.s1] + q.t1 * (row[q.s1 + d] - row[q.s1])) + (row[q.s2] + q.t2 * (row[q.s2 + d] - row[q.s2])) +
               (row[q.s3] + q.t3 * (row[q.s3 + d] - row[q.s3])) - lf[m]);
  }
  const double amp = exp(e) * amp0;
  return make_double2(amp * cs, amp * sn);
}

}  // namespace
}  // namespace isrsgn
