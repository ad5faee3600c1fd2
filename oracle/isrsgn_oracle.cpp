// ISRS GN numerical-integral model: plain FP64 CPU oracle.
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference
// that the GPU library is checked against.  Only tests/, the smoke check and the
// CPU-baseline leg of the benchmark may load it; the product path never does.
// It shares no code, header or table with the GPU library.
//
// Model (Jarmolovicius et al., "Optimising O-to-U Band Transmission Using Fast
// ISRS Gaussian Noise Numerical Integral Model", arXiv:2401.18022):
//   * NLI PSD at the COI, eq. (new_gn_model) / (gain_fin) with (psi_fin):
//       G(f) = 16/27 gamma(f)^2  Int Int G(f1) G(f2) G(f1+f2-f) |S(f1,f2)|^2
//       S    = sum_m p(f1,f2,z_m) dz_m exp(j phi z_m) sinc(phi dz_m / 2)
//   * power-profile term p, eq. (pk): sqrt(rho(f1) rho(f2) rho(f1+f2-f) / rho(f))
//   * phase mismatch with beta2..beta4, eq. (phi)
//   * quadrants and hyperbolic coordinates, eqs. (q1a)-(q4d) and (q1)-(q4)
//   * throughput cost, eq. (loss), and C = 2 B_ch (-L)  (Sec. IV)
//   * gamma(lambda) = 2 pi n2 / (lambda A_eff), eq. (gamma)
//   * beta2/beta3/beta4 from D, S, dS/dlambda, eqs. (d), (d_slope), (d_curve)
//
// Readings where the paper is silent (all shared, as definitions, with the GPU
// library; the code is not shared):
//   * the double integral is partitioned into COI x interferer tiles by the
//     channel that f1+f2-f falls in; each tile is integrated in three parts
//     (Q1 folded about x=y, Q3 folded, Q4 which also stands for Q2) on a
//     log-spaced upsilon1 grid (D decades below the part's sup|xy|) with a
//     uniform upsilon2 grid between the exact per-row limits;
//   * distance steps have equal power decrement under the mean loss of the
//     occupied channels, evaluated at their midpoints;
//   * P1 profile = closed-form ISRS solution for a linear gain slope;
//     P2 profile = RK4 on the Raman ODEs (triangular gain with cut-off,
//     photon-number ratio, A_eff scaling), ln rho interpolated linearly in f
//     between channel centres;
//   * transmit spectra: unit-area raised-cosine shape of roll-off beta (the PSD of an RRC-filtered
//     signal; beta = 0 is the paper's rectangle), G_Tx = P_c g_c(f - f_c) on |f - f_c| < (1+beta) R_c/2;
//   * noise powers are PSDs integrated against the receiver's power response R_i g_i(f - f_i)
//     (unit passband, noise bandwidth R_i): ASE = NF h f G_amp R with G_amp = 1/rho(L, f); NLI by a
//     normalised midpoint rule over nli_points points across the COI's support, whose one-point
//     form is the locally-white R_i G(f_i);
//   * n identical spans: each amplifier restores the launch power, so every span has the same
//     power profile and adds the same ASE; span k's field carries the phase phi (k-1) L.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <thread>
#include <vector>

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kC = 299792458.0;        // m/s
constexpr double kH = 6.62607015e-34;     // J s
constexpr double kLn10 = 2.302585092994045684;

// ---------------------------------------------------------------------------
// Forward-mode dual number: value and derivative along one direction of P.
struct Dual {
  double v, d;
  Dual() : v(0), d(0) {}
  Dual(double x) : v(x), d(0) {}
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) { return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)}; }
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline Dual& operator*=(Dual& a, Dual b) { a = a * b; return a; }

inline double Val(double x) { return x; }
inline double Val(Dual x) { return x.v; }
inline double Exp(double x) { return std::exp(x); }
inline Dual Exp(Dual x) { double e = std::exp(x.v); return {e, e * x.d}; }
inline double Log(double x) { return std::log(x); }
inline Dual Log(Dual x) { return {std::log(x.v), x.d / x.v}; }
inline double Sinh(double x) { return std::sinh(x); }
inline Dual Sinh(Dual x) { return {std::sinh(x.v), std::cosh(x.v) * x.d}; }
inline double Cosh(double x) { return std::cosh(x); }
inline Dual Cosh(Dual x) { return {std::cosh(x.v), std::sinh(x.v) * x.d}; }
inline double Log2(double x) { return std::log2(x); }
inline Dual Log2(Dual x) { return {std::log2(x.v), x.d / (x.v * std::log(2.0))}; }

// Forward-mode dual number carrying kDirs directions at once: the value (and every
// transcendental of it) is computed once, each direction's derivative by the chain rule.
constexpr int kDirs = 16;
struct DualN {
  double v;
  double d[kDirs];
  DualN() : v(0) { for (int q = 0; q < kDirs; ++q) d[q] = 0; }
  DualN(double x) : v(x) { for (int q = 0; q < kDirs; ++q) d[q] = 0; }
};
inline DualN operator+(const DualN& a, const DualN& b) {
  DualN r(a.v + b.v);
  for (int q = 0; q < kDirs; ++q) r.d[q] = a.d[q] + b.d[q];
  return r;
}
inline DualN operator-(const DualN& a, const DualN& b) {
  DualN r(a.v - b.v);
  for (int q = 0; q < kDirs; ++q) r.d[q] = a.d[q] - b.d[q];
  return r;
}
inline DualN operator-(const DualN& a) {
  DualN r(-a.v);
  for (int q = 0; q < kDirs; ++q) r.d[q] = -a.d[q];
  return r;
}
inline DualN operator*(const DualN& a, const DualN& b) {
  DualN r(a.v * b.v);
  for (int q = 0; q < kDirs; ++q) r.d[q] = a.d[q] * b.v + a.v * b.d[q];
  return r;
}
inline DualN operator/(const DualN& a, const DualN& b) {
  DualN r(a.v / b.v);
  for (int q = 0; q < kDirs; ++q) r.d[q] = (a.d[q] * b.v - a.v * b.d[q]) / (b.v * b.v);
  return r;
}
// products and sums with a constant (its derivative is zero)
inline DualN operator*(const DualN& a, double b) {
  DualN r(a.v * b);
  for (int q = 0; q < kDirs; ++q) r.d[q] = a.d[q] * b;
  return r;
}
inline DualN operator*(double a, const DualN& b) { return b * a; }
inline DualN operator+(const DualN& a, double b) {
  DualN r = a;
  r.v += b;
  return r;
}
inline DualN operator+(double a, const DualN& b) { return b + a; }
inline DualN& operator+=(DualN& a, const DualN& b) { a = a + b; return a; }
inline DualN& operator-=(DualN& a, const DualN& b) { a = a - b; return a; }
inline DualN& operator*=(DualN& a, const DualN& b) { a = a * b; return a; }
// f(a) with f'(a.v) = fp: the chain rule applied to every direction
inline DualN Chain(const DualN& a, double f, double fp) {
  DualN r(f);
  for (int q = 0; q < kDirs; ++q) r.d[q] = fp * a.d[q];
  return r;
}
inline double Val(const DualN& x) { return x.v; }
inline DualN Exp(const DualN& x) { double e = std::exp(x.v); return Chain(x, e, e); }
inline DualN Log(const DualN& x) { return Chain(x, std::log(x.v), 1.0 / x.v); }
inline DualN Sinh(const DualN& x) { return Chain(x, std::sinh(x.v), std::cosh(x.v)); }
inline DualN Cosh(const DualN& x) { return Chain(x, std::cosh(x.v), std::sinh(x.v)); }
inline DualN Log2(const DualN& x) { return Chain(x, std::log2(x.v), 1.0 / (x.v * std::log(2.0))); }

// Derivative outputs: direction q of x goes to out[idx * stride + q].
inline void PutDer(double, double* out, size_t idx) { out[idx] = 0.0; }
inline void PutDer(const Dual& x, double* out, size_t idx) { out[idx] = x.d; }
inline void PutDer(const DualN& x, double* out, size_t idx) {
  for (int q = 0; q < kDirs; ++q) out[idx * kDirs + q] = x.d[q];
}

// sinh(x)/x with its limit 1 at x = 0.
template <class T> T Sinhc(T x) {
  if (std::fabs(Val(x)) < 1e-4) {
    T x2 = x * x;
    return T(1.0) + x2 * (1.0 / 6.0) + x2 * x2 * (1.0 / 120.0);
  }
  return Sinh(x) / x;
}

// Two-sided Laplace transform M(a) = int g(u) exp(-a u) du of the unit-area raised-cosine
// spectrum g of symbol rate R and roll-off beta.  g is the rectangle of width R (transform
// sinhc(a R/2)) convolved with the unit half-cosine lobe (pi / (2 beta R)) cos(pi v / (beta R)) on
// |v| <= beta R/2 (transform cosh(a beta R/2) / (1 + (a beta R/pi)^2)); beta = 0 leaves sinhc.
template <class T> T Spectrum(T a, double R, double beta) {
  T m = Sinhc(a * (0.5 * R));
  if (beta > 0) {
    const double h = 0.5 * beta * R, c = beta * R / 3.14159265358979323846;
    T ac = a * c;
    m = m * Cosh(a * h) / (T(1.0) + ac * ac);
  }
  return m;
}

}  // namespace

extern "C" {

// Problem description handed over from Python (all SI units; host arrays).
typedef struct {
  double span_m, f_ref_hz, beta2, beta3, beta4;
  int n_tab;
  const double *tab_f_hz, *tab_alpha_per_m, *tab_aeff_m2;
  double n2, gamma_const, cr, aeff_ref, raman_cutoff;
  int profile, photon_ratio;
  int n_steps, grid_s, grid_v;
  double s_decades;
  int ode_sub;
  int n_ch;
  const double *f_hz, *rs_hz, *p_w, *nf_lin;
  double snr_trx;
  const double* dp;  // direction of the dual numbers (NULL: plain FP64 pass)
  int n_threads;
  int unfold;  // 1: evaluate both sides of each fold explicitly (symmetry check)
  int mode;    // 0: model integrand; 1: unit integrand; 2: unit integrand on the channel support
  int n_spans;  // identical spans (App. A, eq. gain: sum over spans k with offsets (k-1) L)
  double rolloff;   // raised-cosine roll-off of every transmit spectrum (0: rectangular)
  int nli_points;   // points of the within-channel NLI rule (1: locally white at the centre)
} orc_problem;

}  // extern "C"

namespace {

// ---------------------------------------------------------------------------
// Setup (Sec. II).

// Linear interpolation in f through a table, held constant beyond its ends.
double table_at(int n, const double* xs, const double* ys, double x) {
  if (n == 1 || x <= xs[0]) return ys[0];
  if (x >= xs[n - 1]) return ys[n - 1];
  int lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (xs[mid] <= x) lo = mid; else hi = mid;
  }
  double t = (x - xs[lo]) / (xs[hi] - xs[lo]);
  return ys[lo] + t * (ys[hi] - ys[lo]);
}

struct Channels {
  int n;
  double beta;  // roll-off of the transmit spectra
  std::vector<double> f, R, alpha, aeff, gamma, cr, nf;
  // half-width of channel c's support
  double half(int c) const { return 0.5 * (1.0 + beta) * R[c]; }
  // unit-area spectral shape of channel c at absolute frequency F: the raised cosine
  // (1/R) on |u| <= (1-beta) R/2, (1/R) (1 + cos(pi (|u| - (1-beta) R/2) / (beta R))) / 2 up to
  // (1+beta) R/2, zero beyond (u = F - f_c); beta = 0 is the rectangle of width R
  double shape(int c, double F) const {
    const double u = std::fabs(F - f[c]), r = R[c];
    if (u >= half(c)) return 0.0;
    const double flat = 0.5 * (1.0 - beta) * r;
    if (u <= flat) return 1.0 / r;
    return 0.5 * (1.0 + std::cos(kPi * (u - flat) / (beta * r))) / r;
  }
};

Channels make_channels(const orc_problem& pb) {
  Channels ch;
  ch.n = pb.n_ch;
  ch.beta = pb.rolloff;
  for (int c = 0; c < pb.n_ch; ++c) {
    double f = pb.f_hz[c];
    ch.f.push_back(f);
    ch.R.push_back(pb.rs_hz[c]);
    double a = table_at(pb.n_tab, pb.tab_f_hz, pb.tab_alpha_per_m, f);
    double ae = table_at(pb.n_tab, pb.tab_f_hz, pb.tab_aeff_m2, f);
    ch.alpha.push_back(a);
    ch.aeff.push_back(ae);
    // eq. (gamma) with lambda = c/f: gamma = 2 pi n2 f / (c A_eff)
    ch.gamma.push_back(pb.gamma_const > 0 ? pb.gamma_const : 2.0 * kPi * pb.n2 * f / (kC * ae));
    // Raman gain scaled by the effective area at the channel frequency (Sec. II, App. A)
    ch.cr.push_back(pb.cr * pb.aeff_ref / ae);
    ch.nf.push_back(pb.nf_lin ? pb.nf_lin[c] : 1.0);
  }
  return ch;
}

// ---------------------------------------------------------------------------
// Distance steps (Sec. III-A, eq. slow_vary0-slow_vary): logarithmically growing
// steps with (approximately) equal power change per step; evaluated at midpoints.
struct Steps {
  std::vector<double> edge, zm, dz;
};

Steps make_steps(double alpha_bar, double L, int n) {
  Steps s;
  s.edge.resize(n + 1);
  double q = -std::expm1(-alpha_bar * L);  // 1 - exp(-alpha L): total power fraction lost
  for (int j = 0; j <= n; ++j) {
    if (alpha_bar * L < 1e-12) s.edge[j] = L * j / n;
    else s.edge[j] = -std::log1p(-q * j / (double)n) / alpha_bar;
  }
  s.edge[n] = L;
  for (int j = 0; j < n; ++j) {
    s.zm.push_back(0.5 * (s.edge[j] + s.edge[j + 1]));
    s.dz.push_back(s.edge[j + 1] - s.edge[j]);
  }
  return s;
}

double mean_loss(const Channels& ch, const double* p) {
  double sum = 0; int cnt = 0;
  for (int c = 0; c < ch.n; ++c) if (p[c] > 0) { sum += ch.alpha[c]; ++cnt; }
  if (cnt == 0) { for (int c = 0; c < ch.n; ++c) sum += ch.alpha[c]; cnt = ch.n; }
  return sum / cnt;
}

// ---------------------------------------------------------------------------
// Normalised power profile rho(z, f) (App. A; link function of eq. pk).
template <class T>
struct Profile {
  int kind;              // 0: closed form, 1: ODE table
  int M, N;
  double alpha, f_ref;   // closed form: uniform loss and reference frequency
  std::vector<T> a_m, lnnorm_m;  // closed form per step: slope and log-normaliser
  T a_L, lnnorm_L;
  std::vector<double> zm;
  double L;
  std::vector<T> ell;    // ODE: ln rho at (z_m, f_c), [m*N + c]
  std::vector<T> ell_L;  // ODE: ln rho at (L, f_c)
  const std::vector<double>* fc;

  // ln rho at step m (m < 0: span end) and absolute frequency F.
  T lnrho(int m, double F) const {
    if (kind == 0) {
      double z = m < 0 ? L : zm[m];
      const T& a = m < 0 ? a_L : a_m[m];
      const T& ln = m < 0 ? lnnorm_L : lnnorm_m[m];
      return T(-alpha * z) - a * (F - f_ref) - ln;
    }
    const std::vector<double>& f = *fc;
    const T* row = m < 0 ? ell_L.data() : ell.data() + (size_t)m * N;
    if (N == 1) return row[0];
    int c = 0;
    if (F >= f[N - 1]) c = N - 2;
    else if (F > f[0]) {
      int lo = 0, hi = N - 1;
      while (hi - lo > 1) { int mid = (lo + hi) / 2; if (f[mid] <= F) lo = mid; else hi = mid; }
      c = lo;
    }
    double t = (F - f[c]) / (f[c + 1] - f[c]);
    return row[c] + (row[c + 1] - row[c]) * t;
  }
};

// P1: closed-form ISRS solution for a linear Raman gain slope (the draft-comment expression of
// App. A, Zirngibl 1998), for rectangular spectra:
//   rho(z,F) = exp(-alpha z) exp(-a (F - f_ref)) / sum_j (P_j/P_tot) exp(-a (f_j - f_ref)) sinhc(a R_j / 2)
// and for raised-cosine spectra with sinhc(a R_j/2) replaced by the spectrum's transform M_j(a)
//   a(z) = P_tot C_r L_eff(z),  L_eff(z) = (1 - exp(-alpha z)) / alpha
template <class T>
void closed_form_at(const Channels& ch, const std::vector<T>& P, double alpha, double cr, double f_ref,
                    double z, T* a_out, T* lnnorm_out) {
  T ptot(0.0);
  for (int j = 0; j < ch.n; ++j) ptot += P[j];
  if (!(Val(ptot) > 0)) { *a_out = T(0.0); *lnnorm_out = T(0.0); return; }
  double leff = alpha > 0 ? -std::expm1(-alpha * z) / alpha : z;
  T a = ptot * (cr * leff);
  T norm(0.0);
  for (int j = 0; j < ch.n; ++j)
    norm += P[j] / ptot * Exp(-a * (ch.f[j] - f_ref)) * Spectrum(a, ch.R[j], ch.beta);
  *a_out = a;
  *lnnorm_out = Log(norm);
}

// P2: Raman power-evolution ODEs, integrated for ell_k = ln(P_k(z)/P_k(0)):
//   d ell_k / dz = -alpha_k + sum_j g_kj P_j exp(ell_j)
//   g_kj = +C_r,k Tri(f_j - f_k)                 (f_j > f_k: k gains from j)
//   g_kj = -C_r,k Tri(f_k - f_j) (f_k / f_j)^pr  (f_j < f_k: k feeds j; pr = photon ratio)
//   Tri(d) = d for d <= cut-off, 0 beyond (no cut-off when cut-off <= 0).
// Classical RK4; each distance step is split into 2*ode_sub equal sub-steps so
// that the step midpoints and the span end are grid points.
template <class T>
void ode_profile(const Channels& ch, const std::vector<T>& P, const Steps& st, double cutoff,
                 int photon_ratio, int ode_sub, std::vector<T>* ell, std::vector<T>* ell_L) {
  const int N = ch.n, M = (int)st.dz.size();
  std::vector<double> g((size_t)N * N, 0.0);
  for (int k = 0; k < N; ++k)
    for (int j = 0; j < N; ++j) {
      double d = ch.f[j] - ch.f[k];
      if (j == k) continue;
      if (d > 0 && (cutoff <= 0 || d <= cutoff)) g[(size_t)k * N + j] = ch.cr[k] * d;
      if (d < 0 && (cutoff <= 0 || -d <= cutoff))
        g[(size_t)k * N + j] = -ch.cr[k] * (-d) * (photon_ratio ? ch.f[k] / ch.f[j] : 1.0);
    }
  auto rhs = [&](const std::vector<T>& l, std::vector<T>& out) {
    std::vector<T> pw(N);
    for (int j = 0; j < N; ++j) pw[j] = P[j] * Exp(l[j]);
    for (int k = 0; k < N; ++k) {
      T s(-ch.alpha[k]);
      for (int j = 0; j < N; ++j) {
        double gk = g[(size_t)k * N + j];
        if (gk != 0.0) s += pw[j] * gk;
      }
      out[k] = s;
    }
  };
  std::vector<T> l(N, T(0.0)), k1(N), k2(N), k3(N), k4(N), tmp(N);
  auto rk4 = [&](double h) {
    rhs(l, k1);
    for (int c = 0; c < N; ++c) tmp[c] = l[c] + k1[c] * (0.5 * h);
    rhs(tmp, k2);
    for (int c = 0; c < N; ++c) tmp[c] = l[c] + k2[c] * (0.5 * h);
    rhs(tmp, k3);
    for (int c = 0; c < N; ++c) tmp[c] = l[c] + k3[c] * h;
    rhs(tmp, k4);
    for (int c = 0; c < N; ++c) l[c] = l[c] + (k1[c] + k2[c] * 2.0 + k3[c] * 2.0 + k4[c]) * (h / 6.0);
  };
  ell->assign((size_t)M * N, T(0.0));
  ell_L->assign(N, T(0.0));
  for (int m = 0; m < M; ++m) {
    double h = st.dz[m] / (2.0 * ode_sub);
    for (int s = 0; s < ode_sub; ++s) rk4(h);
    for (int c = 0; c < N; ++c) (*ell)[(size_t)m * N + c] = l[c];
    for (int s = 0; s < ode_sub; ++s) rk4(h);
  }
  for (int c = 0; c < N; ++c) (*ell_L)[c] = l[c];
}

template <class T>
Profile<T> make_profile(const orc_problem& pb, const Channels& ch, const std::vector<T>& P, const Steps& st) {
  Profile<T> pr;
  pr.kind = pb.profile == 0 ? 0 : 1;
  pr.M = (int)st.zm.size();
  pr.N = ch.n;
  pr.zm = st.zm;
  pr.L = pb.span_m;
  pr.fc = &ch.f;
  pr.f_ref = pb.f_ref_hz;
  pr.alpha = ch.alpha[0];
  if (pr.kind == 0) {
    double cr = ch.cr[0];
    pr.a_m.resize(pr.M);
    pr.lnnorm_m.resize(pr.M);
    for (int m = 0; m < pr.M; ++m) closed_form_at(ch, P, pr.alpha, cr, pr.f_ref, st.zm[m], &pr.a_m[m], &pr.lnnorm_m[m]);
    closed_form_at(ch, P, pr.alpha, cr, pr.f_ref, pb.span_m, &pr.a_L, &pr.lnnorm_L);
  } else {
    ode_profile(ch, P, st, pb.raman_cutoff, pb.photon_ratio, pb.ode_sub, &pr.ell, &pr.ell_L);
  }
  return pr;
}

// ---------------------------------------------------------------------------
// Phase mismatch, eq. (phi): x, y are the offsets of f1, f2 from the COI and w the
// COI offset from the reference frequency of the dispersion Taylor series.
double phase_mismatch(double x, double y, double w, double b2, double b3, double b4) {
  double poly4 = x * x + 1.5 * x * y + y * y + 3.0 * x * w + 3.0 * y * w + 3.0 * w * w;
  return -4.0 * kPi * kPi * x * y * (b2 + kPi * b3 * (x + y + 2.0 * w) + (2.0 * kPi * kPi / 3.0) * b4 * poly4);
}

// Channel whose spectrum's support [f_c - (1+beta) R_c/2, f_c + (1+beta) R_c/2) holds F, or -1.
int channel_of(const Channels& ch, double F) {
  int lo = 0, hi = ch.n;  // find the last channel whose lower edge <= F
  if (F < ch.f[0] - ch.half(0)) return -1;
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (ch.f[mid] - ch.half(mid) <= F) lo = mid; else hi = mid;
  }
  return F < ch.f[lo] + ch.half(lo) ? lo : -1;
}

// Points and weights of the within-channel NLI rule of COI i: n midpoints across the support
// [f_i - (1+beta) R_i/2, f_i + (1+beta) R_i/2], weights proportional to the receiver's power
// response R_i g_i(f - f_i) and normalised to its noise bandwidth R_i (so a flat NLI PSD is
// integrated exactly, and one point is the locally-white R_i G(f_i)).
void nli_points(const Channels& ch, int i, int n, std::vector<double>* f, std::vector<double>* q) {
  f->assign(n, 0.0);
  q->assign(n, 0.0);
  const double d = 2.0 * ch.half(i) / n;
  double sum = 0.0;
  for (int j = 0; j < n; ++j) {
    (*f)[j] = ch.f[i] + (j + 0.5 - 0.5 * n) * d;
    (*q)[j] = ch.R[i] * ch.shape(i, (*f)[j]);
    sum += (*q)[j];
  }
  for (int j = 0; j < n; ++j) (*q)[j] *= ch.R[i] / sum;
}

// Transmit PSD of channel c at F: P_c / R_c for the rectangle, P_c g_c(F - f_c) in general.
template <class T>
T density(const Channels& ch, const std::vector<T>& P, int c, double F) {
  if (ch.beta == 0.0) return P[c] / ch.R[c];
  return P[c] * ch.shape(c, F);
}

// gamma at an arbitrary frequency: eq. (gamma) with A_eff interpolated from the table, or the constant.
double gamma_at(const orc_problem& pb, double f) {
  double ae = table_at(pb.n_tab, pb.tab_f_hz, pb.tab_aeff_m2, f);
  return pb.gamma_const > 0 ? pb.gamma_const : 2.0 * kPi * pb.n2 * f / (kC * ae);
}

// ---------------------------------------------------------------------------
// Tile geometry: hyperbolic coordinates upsilon1 = x y (stored as s = ln|x y|) and
// upsilon2 = v = ln sqrt(|x/y|) (eqs. q1-q4; unit Jacobian).  Parts:
//   Q1: x = r e^v,  y = r e^-v   (x, y > 0; folded to v >= 0, factor 2)
//   Q3: x = -r e^v, y = -r e^-v  (x, y < 0; folded to v >= 0, factor 2)
//   Q4: x = r e^v,  y = -r e^-v  (x > 0 > y; stands for Q2 as well, factor 2)
// with r = sqrt(upsilon1).  A tile (i,k) is the part of the band square where
// F3 = f_i + x + y lies in channel k: x + y in [S_lo, S_hi).
enum { kQ1 = 0, kQ3 = 1, kQ4 = 2 };

bool part_umax(int part, double slo, double shi, double xp, double xn, double* umax) {
  if (part == kQ1) {
    if (shi <= 0 || xp <= 0) return false;
    double lo = std::max(slo, 0.0);
    if (lo >= 2 * xp) return false;
    double m = std::min(0.5 * shi, xp);
    *umax = m * m;
    return *umax > 0;
  }
  if (part == kQ3) {
    if (slo >= 0 || xn <= 0) return false;
    double lo = std::max(-shi, 0.0), hi = -slo;
    if (lo >= 2 * xn) return false;
    double m = std::min(0.5 * hi, xn);
    *umax = m * m;
    return *umax > 0;
  }
  if (xp <= 0 || xn <= 0) return false;
  double best = 0;
  double ulo = std::max(0.0, xp - shi), uhi = std::min(xn, xp - slo);   // along x = xp
  if (uhi > ulo) best = std::max(best, xp * uhi);
  double xlo = std::max(0.0, xn + slo), xhi = std::min(xp, xn + shi);   // along -y = xn
  if (xhi > xlo) best = std::max(best, xhi * xn);
  if (!(best > 0)) return false;
  *umax = best;
  return true;
}

bool part_vrange(int part, double r, double slo, double shi, double xp, double xn, double* vlo, double* vhi) {
  if (part == kQ1 || part == kQ3) {
    double lo = part == kQ1 ? std::max(slo, 0.0) : std::max(-shi, 0.0);
    double hi = part == kQ1 ? shi : -slo;
    double lim = part == kQ1 ? xp : xn;
    double chi = hi / (2 * r);
    if (!(chi > 1)) return false;
    double clo = lo / (2 * r);
    *vlo = clo > 1 ? std::acosh(clo) : 0.0;
    *vhi = std::min(std::acosh(chi), std::log(lim / r));
    return *vhi > *vlo;
  }
  *vlo = std::max(std::asinh(slo / (2 * r)), std::log(r / xn));
  *vhi = std::min(std::asinh(shi / (2 * r)), std::log(xp / r));
  return *vhi > *vlo;
}

void part_map(int part, double r, double v, double* x, double* y) {
  double ev = std::exp(v), emv = std::exp(-v);
  if (part == kQ1) { *x = r * ev; *y = r * emv; }
  else if (part == kQ3) { *x = -r * ev; *y = -r * emv; }
  else { *x = r * ev; *y = -r * emv; }
}

struct Model {
  const orc_problem* pb;
  Channels ch;
  Steps st;
};

// Psi of eq. (psi_fin) at NLI frequency fi: G_Tx(f1) G_Tx(f2) G_Tx(f1+f2-fi) |S|^2, offsets x, y
// from fi.  P: channel powers (G_Tx = P_c times the channel's unit shape).
template <class T>
T psi(const Model& md, const Profile<T>& pr, const std::vector<T>& P, double fi, double x, double y) {
  const Channels& ch = md.ch;
  const orc_problem& pb = *md.pb;
  int c1 = channel_of(ch, fi + x), c2 = channel_of(ch, fi + y), c3 = channel_of(ch, fi + x + y);
  if (pb.mode == 1) return T(1.0);
  if (c1 < 0 || c2 < 0 || c3 < 0) return T(0.0);
  if (pb.mode == 2) return T(1.0);
  T gprod = density(ch, P, c1, fi + x) * density(ch, P, c2, fi + y) * density(ch, P, c3, fi + x + y);
  double phi = phase_mismatch(x, y, fi - pb.f_ref_hz, pb.beta2, pb.beta3, pb.beta4);
  T sre(0.0), sim(0.0);
  // eq. (psi_fin): sum over the n identical spans (offset (k-1) L, the same power profile in
  // each: the amplifiers restore the launch power) and over the steps of a span
  const int n_spans = pb.n_spans > 0 ? pb.n_spans : 1;
  for (int k = 0; k < n_spans; ++k) {
    const double off = k * pb.span_m;
    for (int m = 0; m < (int)md.st.zm.size(); ++m) {
      // eq. (pk): p = sqrt(rho(f1) rho(f2) rho(f1+f2-f) / rho(f))
      T p = Exp((pr.lnrho(m, fi + x) + pr.lnrho(m, fi + y) + pr.lnrho(m, fi + x + y) - pr.lnrho(m, fi)) * 0.5);
      double dz = md.st.dz[m], zm = md.st.zm[m];
      double u = phi * dz / 2;
      double sinc = u == 0.0 ? 1.0 : std::sin(u) / u;
      T amp = p * (dz * sinc);
      sre += amp * std::cos(phi * (off + zm));
      sim += amp * std::sin(phi * (off + zm));
    }
  }
  return gprod * (sre * sre + sim * sim);
}

// tile(fi, k): Riemann sum of Psi at NLI frequency fi over the part of the band square where
// f1 + f2 - fi lies in channel k (without the 16/27 gamma^2 factor).
template <class T>
T tile_integral(const Model& md, const Profile<T>& pr, const std::vector<T>& P, double fi, int k) {
  const Channels& ch = md.ch;
  const orc_problem& pb = *md.pb;
  const int n = ch.n;
  double xp = (ch.f[n - 1] + ch.half(n - 1)) - fi;
  double xn = fi - (ch.f[0] - ch.half(0));
  double delta = ch.f[k] - fi;
  double slo = delta - ch.half(k), shi = delta + ch.half(k);
  T total(0.0);
  for (int part = kQ1; part <= kQ4; ++part) {
    double umax;
    if (!part_umax(part, slo, shi, xp, xn, &umax)) continue;
    double smax = std::log(umax), smin = smax - pb.s_decades * kLn10;
    double ds = (smax - smin) / pb.grid_s;
    for (int a = 0; a < pb.grid_s; ++a) {
      double s = smin + (a + 0.5) * ds, r = std::exp(0.5 * s);
      double vlo, vhi;
      if (!part_vrange(part, r, slo, shi, xp, xn, &vlo, &vhi)) continue;
      double dv = (vhi - vlo) / pb.grid_v;
      for (int b = 0; b < pb.grid_v; ++b) {
        double v = vlo + (b + 0.5) * dv;
        double x, y;
        part_map(part, r, v, &x, &y);
        double w = std::exp(s) * ds * dv;
        if (pb.unfold) {  // the fold partner (y, x) evaluated explicitly
          total += (psi(md, pr, P, fi, x, y) + psi(md, pr, P, fi, y, x)) * w;
        } else {
          total += psi(md, pr, P, fi, x, y) * (2.0 * w);
        }
      }
    }
  }
  return total;
}

// Paper-literal quadrants of eqs. (q1)-(q4) at NLI frequency fi over the whole band square,
// same node rule (D decades below the quadrant's sup|x y|, uniform in upsilon2).
double paper_quadrant(const Model& md, const Profile<double>& pr, const std::vector<double>& P, double fi, int q) {
  const Channels& ch = md.ch;
  const orc_problem& pb = *md.pb;
  const int n = ch.n;
  double bp = (ch.f[n - 1] + ch.half(n - 1)) - fi;  // the paper's B - f
  double bm = fi - (ch.f[0] - ch.half(0));          // the paper's B + f
  // (f1 limit, f2 limit, sign of f1, sign of f2) per quadrant
  double l1[4] = {bp, bm, bm, bp}, l2[4] = {bp, bp, bm, bm};
  double s1[4] = {+1, -1, -1, +1}, s2[4] = {+1, +1, -1, -1};
  double umax = l1[q] * l2[q];
  if (!(umax > 0)) return 0.0;
  double smax = std::log(umax), smin = smax - pb.s_decades * kLn10;
  double ds = (smax - smin) / pb.grid_s;
  double total = 0;
  for (int a = 0; a < pb.grid_s; ++a) {
    double s = smin + (a + 0.5) * ds, r = std::exp(0.5 * s);
    double vlo = -std::log(l2[q] / r), vhi = std::log(l1[q] / r);  // g1 <= l1, g2 <= l2
    if (!(vhi > vlo)) continue;
    double dv = (vhi - vlo) / pb.grid_v;
    for (int b = 0; b < pb.grid_v; ++b) {
      double v = vlo + (b + 0.5) * dv;
      double g1 = r * std::exp(v), g2 = r * std::exp(-v);
      total += psi(md, pr, P, fi, s1[q] * g1, s2[q] * g2) * (std::exp(s) * ds * dv);
    }
  }
  return total;
}

// ---------------------------------------------------------------------------
template <class T>
std::vector<T> powers(const orc_problem& pb) {
  std::vector<T> P(pb.n_ch);
  for (int c = 0; c < pb.n_ch; ++c) P[c] = T(pb.p_w[c]);
  return P;
}
template <>
std::vector<Dual> powers<Dual>(const orc_problem& pb) {
  std::vector<Dual> P(pb.n_ch);
  for (int c = 0; c < pb.n_ch; ++c) P[c] = Dual(pb.p_w[c], pb.dp ? pb.dp[c] : 0.0);
  return P;
}
// pb.dp holds kDirs directions, row-major [q][c]
template <>
std::vector<DualN> powers<DualN>(const orc_problem& pb) {
  std::vector<DualN> P(pb.n_ch);
  for (int c = 0; c < pb.n_ch; ++c) {
    P[c] = DualN(pb.p_w[c]);
    for (int q = 0; q < kDirs; ++q) P[c].d[q] = pb.dp ? pb.dp[(size_t)q * pb.n_ch + c] : 0.0;
  }
  return P;
}

int n_workers(const orc_problem& pb) {
  int n = pb.n_threads > 0 ? pb.n_threads : (int)std::thread::hardware_concurrency();
  return std::max(1, n);
}

template <class F>
void parallel_for(int count, int workers, F&& fn) {
  std::atomic<int> next(0);
  auto body = [&]() {
    for (int t = next.fetch_add(1); t < count; t = next.fetch_add(1)) fn(t);
  };
  workers = std::min(workers, std::max(1, count));
  std::vector<std::thread> pool;
  for (int w = 1; w < workers; ++w) pool.emplace_back(body);
  body();
  for (auto& t : pool) t.join();
}

bool valid(const orc_problem* pb) {
  if (!pb || pb->n_ch < 1 || pb->n_steps < 1 || pb->grid_s < 1 || pb->grid_v < 1 || pb->ode_sub < 1) return false;
  if (pb->profile == 0 && pb->n_tab != 1) return false;  // the closed form needs uniform loss
  if (!(pb->rolloff >= 0.0 && pb->rolloff <= 1.0) || pb->nli_points < 1) return false;
  for (int c = 0; c + 1 < pb->n_ch; ++c)  // spectra may touch but not overlap
    if (pb->f_hz[c + 1] - pb->f_hz[c] < 0.5 * (1.0 + pb->rolloff) * (pb->rs_hz[c] + pb->rs_hz[c + 1])) return false;
  return true;
}

// Forward model for a list of COIs.  Outputs per listed COI: the tile row, P_NLI, eta,
// SNR (and their derivatives along dp when T = Dual).  thr = sum over listed COIs.
template <class T>
int forward_impl(const orc_problem* pb, int n_coi, const int* coi, double* tiles, double* dtiles,
                 double* pnli, double* dpnli, double* eta, double* deta, double* snr, double* dsnr,
                 double* thr, double* dthr, double* ell_out, double* ell_L_out) {
  if (!valid(pb)) return -1;
  Model md;
  md.pb = pb;
  md.ch = make_channels(*pb);
  md.st = make_steps(mean_loss(md.ch, pb->p_w), pb->span_m, pb->n_steps);
  std::vector<T> P = powers<T>(*pb);
  Profile<T> pr = make_profile(*pb, md.ch, P, md.st);
  const int N = pb->n_ch;
  if (ell_out)
    for (int m = 0; m < pb->n_steps; ++m)
      for (int c = 0; c < N; ++c) ell_out[(size_t)m * N + c] = Val(pr.lnrho(m, md.ch.f[c]));
  if (ell_L_out)
    for (int c = 0; c < N; ++c) ell_L_out[c] = Val(pr.lnrho(-1, md.ch.f[c]));
  if (n_coi <= 0) return 0;
  // the within-channel rule: per COI q and point j the NLI frequency and the weight that turns
  // tile(f_ij, k) into the COI's tile row: q_j gamma(f_ij)^2 / (gamma_i^2 R_i), so that
  // P_NLI,i = 16/27 gamma_i^2 R_i sum_k row(k) (one point, rectangle: weight 1, f_i0 = f_i)
  const int J = pb->nli_points;
  std::vector<double> fpt((size_t)n_coi * J), wpt((size_t)n_coi * J);
  for (int q = 0; q < n_coi; ++q) {
    const int i = coi[q];
    std::vector<double> fj, qj;
    nli_points(md.ch, i, J, &fj, &qj);
    for (int j = 0; j < J; ++j) {
      const double gr = md.ch.gamma[i] > 0 ? gamma_at(*pb, fj[j]) / md.ch.gamma[i] : 1.0;
      fpt[(size_t)q * J + j] = fj[j];
      wpt[(size_t)q * J + j] = qj[j] * gr * gr / md.ch.R[i];
    }
  }
  std::vector<T> tp((size_t)n_coi * J * N);
  parallel_for(n_coi * J * N, n_workers(*pb), [&](int t) {
    tp[t] = tile_integral(md, pr, P, fpt[t / N], t % N);
  });
  std::vector<T> tl((size_t)n_coi * N);
  for (int q = 0; q < n_coi; ++q)
    for (int k = 0; k < N; ++k) {
      T v(0.0);
      for (int j = 0; j < J; ++j)
        v += tp[((size_t)q * J + j) * N + k] * wpt[(size_t)q * J + j];
      tl[(size_t)q * N + k] = v;
    }
  T tsum(0.0);
  for (int q = 0; q < n_coi; ++q) {
    int i = coi[q];
    T row(0.0);
    for (int k = 0; k < N; ++k) {
      row += tl[(size_t)q * N + k];
      if (tiles) tiles[(size_t)q * N + k] = Val(tl[(size_t)q * N + k]);
      if (dtiles) PutDer(tl[(size_t)q * N + k], dtiles, (size_t)q * N + k);
    }
    const Channels& ch = md.ch;
    // eq. (gain_fin) integrated over the COI's band by the within-channel rule
    T pn = row * ((16.0 / 27.0) * ch.gamma[i] * ch.gamma[i] * ch.R[i]);
    T pi = P[i];
    T et = Val(pi) > 0 ? pn / (pi * pi * pi) : T(std::numeric_limits<double>::quiet_NaN());
    // ASE: NF h f G_amp R with the amplifier restoring the launch power, G_amp = 1/rho(L, f_i),
    // one amplifier per span
    T pase = Exp(-pr.lnrho(-1, ch.f[i])) * (ch.nf[i] * kH * ch.f[i] * ch.R[i] * (pb->n_spans > 0 ? pb->n_spans : 1));
    T sn(0.0);
    if (Val(pi) > 0) {
      sn = pi / (pn + pase);
      if (pb->snr_trx > 0) sn = T(1.0) / (T(1.0) / sn + T(1.0 / pb->snr_trx));
      tsum += Log2(T(1.0) + sn) * (2.0 * ch.R[i]);  // eq. (loss) and C = 2 B_ch (-L)
    }
    if (pnli) pnli[q] = Val(pn);
    if (dpnli) PutDer(pn, dpnli, q);
    if (eta) eta[q] = Val(et);
    if (deta) PutDer(et, deta, q);
    if (snr) snr[q] = Val(sn);
    if (dsnr) PutDer(sn, dsnr, q);
  }
  if (thr) *thr = Val(tsum);
  if (dthr) PutDer(tsum, dthr, 0);
  return 0;
}

}  // namespace

extern "C" {

// eqs. (d), (d_slope), (d_curve): beta2, beta3, beta4 at lambda from D, S, dS/dlambda (SI).
int orc_beta_from_dispersion(double lambda, double D, double S, double Sdot, double* out3) {
  double w = 2.0 * kPi * kC;
  out3[0] = -D * lambda * lambda / w;
  out3[1] = lambda * lambda * lambda / (w * w) * (2.0 * D + S * lambda);
  out3[2] = -std::pow(lambda, 4) / (w * w * w) * (6.0 * D + 6.0 * S * lambda + Sdot * lambda * lambda);
  return 0;
}

double orc_phi(double x, double y, double w, double b2, double b3, double b4) {
  return phase_mismatch(x, y, w, b2, b3, b4);
}

int orc_steps(double alpha_bar, double L, int n, double* edge, double* zm, double* dz) {
  if (n < 1) return -1;
  Steps s = make_steps(alpha_bar, L, n);
  for (int j = 0; j <= n; ++j) edge[j] = s.edge[j];
  for (int j = 0; j < n; ++j) { zm[j] = s.zm[j]; dz[j] = s.dz[j]; }
  return 0;
}

// Step table of a problem, the mean loss used for it, and the profile at the channel centres.
int orc_profile(const orc_problem* pb, double* alpha_bar, double* edge, double* zm, double* dz,
                double* ell, double* ell_L) {
  if (!valid(pb)) return -1;
  Channels ch = make_channels(*pb);
  double ab = mean_loss(ch, pb->p_w);
  if (alpha_bar) *alpha_bar = ab;
  orc_steps(ab, pb->span_m, pb->n_steps, edge, zm, dz);
  return forward_impl<double>(pb, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                              nullptr, nullptr, nullptr, nullptr, ell, ell_L);
}

// ln rho at arbitrary (step m, frequency F) points; m = -1 is the span end.
int orc_lnrho(const orc_problem* pb, int n, const int* m, const double* F, double* out) {
  if (!valid(pb)) return -1;
  Model md;
  md.pb = pb;
  md.ch = make_channels(*pb);
  md.st = make_steps(mean_loss(md.ch, pb->p_w), pb->span_m, pb->n_steps);
  std::vector<double> P = powers<double>(*pb);
  Profile<double> pr = make_profile(*pb, md.ch, P, md.st);
  for (int q = 0; q < n; ++q) out[q] = pr.lnrho(m[q], F[q]);
  return 0;
}

// Plain FP64 forward for the listed COIs (n_coi = n_ch with coi = 0..n-1 for everything).
int orc_forward(const orc_problem* pb, int n_coi, const int* coi, double* tiles, double* pnli,
                double* eta, double* snr, double* thr) {
  return forward_impl<double>(pb, n_coi, coi, tiles, nullptr, pnli, nullptr, eta, nullptr, snr, nullptr,
                              thr, nullptr, nullptr, nullptr);
}

// tile(i,k) of eq. (gain_fin) (without 16/27 gamma^2 R_i) for a list of (COI, interferer) pairs.
int orc_tiles(const orc_problem* pb, int n_pairs, const int* coi, const int* intf, double* out) {
  if (!valid(pb)) return -1;
  for (int q = 0; q < n_pairs; ++q)
    if (coi[q] < 0 || coi[q] >= pb->n_ch || intf[q] < 0 || intf[q] >= pb->n_ch) return -1;
  Model md;
  md.pb = pb;
  md.ch = make_channels(*pb);
  md.st = make_steps(mean_loss(md.ch, pb->p_w), pb->span_m, pb->n_steps);
  std::vector<double> P = powers<double>(*pb);
  Profile<double> pr = make_profile(*pb, md.ch, P, md.st);
  parallel_for(n_pairs, n_workers(*pb), [&](int q) { out[q] = tile_integral(md, pr, P, md.ch.f[coi[q]], intf[q]); });
  return 0;
}

// tile(f[q], k[q]) at arbitrary NLI frequencies f inside the band (the within-channel rule's points).
int orc_tiles_at(const orc_problem* pb, int n, const double* f, const int* k, double* out) {
  if (!valid(pb)) return -1;
  for (int q = 0; q < n; ++q)
    if (k[q] < 0 || k[q] >= pb->n_ch) return -1;
  Model md;
  md.pb = pb;
  md.ch = make_channels(*pb);
  md.st = make_steps(mean_loss(md.ch, pb->p_w), pb->span_m, pb->n_steps);
  std::vector<double> P = powers<double>(*pb);
  Profile<double> pr = make_profile(*pb, md.ch, P, md.st);
  parallel_for(n, n_workers(*pb), [&](int q) { out[q] = tile_integral(md, pr, P, f[q], k[q]); });
  return 0;
}

// Same, in forward-mode dual numbers along pb->dp: values and directional derivatives.
int orc_forward_dual(const orc_problem* pb, int n_coi, const int* coi, double* tiles, double* dtiles,
                     double* pnli, double* dpnli, double* snr, double* dsnr, double* thr, double* dthr) {
  if (!pb || !pb->dp) return -1;
  return forward_impl<Dual>(pb, n_coi, coi, tiles, dtiles, pnli, dpnli, nullptr, nullptr, snr, dsnr,
                            thr, dthr, nullptr, nullptr);
}

// The same with up to kDirs directions in one pass: dirs is [n_dirs][n_ch] (the rest zero);
// dtiles [n_coi * n_ch][kDirs], dpnli and dsnr [n_coi][kDirs], dthr [kDirs].
int orc_forward_dualn(const orc_problem* pb, int n_dirs, const double* dirs, int n_coi, const int* coi,
                      double* tiles, double* dtiles, double* pnli, double* dpnli, double* snr, double* dsnr,
                      double* thr, double* dthr) {
  if (!pb || !dirs || n_dirs < 1 || n_dirs > kDirs) return -1;
  std::vector<double> d((size_t)kDirs * pb->n_ch, 0.0);
  std::copy(dirs, dirs + (size_t)n_dirs * pb->n_ch, d.begin());
  orc_problem local = *pb;
  local.dp = d.data();
  return forward_impl<DualN>(&local, n_coi, coi, tiles, dtiles, pnli, dpnli, nullptr, nullptr, snr, dsnr,
                             thr, dthr, nullptr, nullptr);
}

int orc_max_dirs(void) { return kDirs; }

// Integrand Psi(x, y) for COI i (G products included), for symmetry checks.
int orc_psi(const orc_problem* pb, int i, int n, const double* x, const double* y, double* out) {
  if (!valid(pb) || i < 0 || i >= pb->n_ch) return -1;
  Model md;
  md.pb = pb;
  md.ch = make_channels(*pb);
  md.st = make_steps(mean_loss(md.ch, pb->p_w), pb->span_m, pb->n_steps);
  std::vector<double> P = powers<double>(*pb);
  Profile<double> pr = make_profile(*pb, md.ch, P, md.st);
  for (int q = 0; q < n; ++q) out[q] = psi(md, pr, P, md.ch.f[i], x[q], y[q]);
  return 0;
}

// The paper's four quadrant integrals Q1..Q4 for COI i (no tiles); sum(q) * 16/27 gamma^2 R_i = P_NLI.
int orc_paper_quadrants(const orc_problem* pb, int i, double* q4) {
  if (!valid(pb) || i < 0 || i >= pb->n_ch) return -1;
  Model md;
  md.pb = pb;
  md.ch = make_channels(*pb);
  md.st = make_steps(mean_loss(md.ch, pb->p_w), pb->span_m, pb->n_steps);
  std::vector<double> P = powers<double>(*pb);
  Profile<double> pr = make_profile(*pb, md.ch, P, md.st);
  parallel_for(4, n_workers(*pb), [&](int q) { q4[q] = paper_quadrant(md, pr, P, md.ch.f[i], q); });
  return 0;
}

// The same four quadrants at an arbitrary NLI frequency f inside the band (no tiles):
// sum(q4) * 16/27 gamma(f)^2 is the NLI PSD G(f) of eq. (new_gn_model).
int orc_paper_quadrants_at(const orc_problem* pb, double f, double* q4) {
  if (!valid(pb)) return -1;
  Model md;
  md.pb = pb;
  md.ch = make_channels(*pb);
  md.st = make_steps(mean_loss(md.ch, pb->p_w), pb->span_m, pb->n_steps);
  std::vector<double> P = powers<double>(*pb);
  Profile<double> pr = make_profile(*pb, md.ch, P, md.st);
  parallel_for(4, n_workers(*pb), [&](int q) { q4[q] = paper_quadrant(md, pr, P, f, q); });
  return 0;
}

// The within-channel rule of channel c: points f_out[n] and weights q_out[n] (Hz).
int orc_nli_points(const orc_problem* pb, int c, double* f_out, double* q_out) {
  if (!valid(pb) || c < 0 || c >= pb->n_ch) return -1;
  Channels ch = make_channels(*pb);
  std::vector<double> f, q;
  nli_points(ch, c, pb->nli_points, &f, &q);
  for (int j = 0; j < pb->nli_points; ++j) { f_out[j] = f[j]; q_out[j] = q[j]; }
  return 0;
}

// Transmit PSD of channel c at frequencies F[n] (W/Hz) and gamma at those frequencies.
int orc_psd(const orc_problem* pb, int c, int n, const double* F, double* psd_out, double* gamma_out) {
  if (!valid(pb) || c < 0 || c >= pb->n_ch) return -1;
  Channels ch = make_channels(*pb);
  std::vector<double> P = powers<double>(*pb);
  for (int q = 0; q < n; ++q) {
    if (psd_out) psd_out[q] = std::fabs(F[q] - ch.f[c]) < ch.half(c) ? density(ch, P, c, F[q]) : 0.0;
    if (gamma_out) gamma_out[q] = gamma_at(*pb, F[q]);
  }
  return 0;
}

// The spectrum's Laplace transform M(a) of the closed-form profile (pins).
double orc_spectrum_laplace(double a, double R, double beta) { return Spectrum(a, R, beta); }

// gamma per channel (eq. gamma) for a problem.
int orc_gamma(const orc_problem* pb, double* out) {
  if (!pb) return -1;
  Channels ch = make_channels(*pb);
  for (int c = 0; c < pb->n_ch; ++c) out[c] = ch.gamma[c];
  return 0;
}

}  // extern "C"
