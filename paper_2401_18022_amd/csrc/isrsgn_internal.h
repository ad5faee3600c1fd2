// Internal interface between the host runtime (isrsgn_api.cpp) and the HIP kernels
// (isrsgn_kernels.hip) of libisrsgn.so.  Not installed; not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace isrsgn {

constexpr int kMaxChannels = 1024;  // per plan (one ODE workgroup of 1024 threads per plan)
constexpr int kMaxGridS = 1024;     // rows per part held in LDS by the tile kernels
constexpr int kTileBlock = 256;     // threads per tile workgroup (4 wave64)
constexpr int kTileVariants = 6;    // forward tile-kernel variants for the autotuner
constexpr int kRank = 8;            // terms of the low-rank FP32 profile table (a multiple of 4)

// Device view of one (possibly batched) channel plan.
struct PlanView {
  int n_batch;
  int n_total;           // channels over all plans
  int nli;               // points of the within-channel NLI rule per COI
  int64_t n_tiles;       // sum over plans of N_b^2 nli: tiles (i, j, k), j the COI's point
  const int* off;        // [n_batch + 1] channel offsets
  const int64_t* toff;   // [n_batch + 1] tile offsets
  const double* f;       // [n_total] centres
  const double* R;       // [n_total] symbol rates (rectangular PSD widths)
  double* alpha;         // [n_total] loss at the centre
  double* aeff;          // [n_total] effective area at the centre
  double* gamma;         // [n_total] nonlinear coefficient
  double* cr;            // [n_total] Raman slope scaled by A_ref / A_eff
  double* fpt;           // [n_total * nli] NLI frequency of point j of COI c
  double* wpt;           // [n_total * nli] its weight q_j gamma(f_j)^2 / (gamma_c^2 R_c) in the tile row
};

struct FibreParams {
  double span, f_ref, b2, b3, b4;
  double n2, gamma_const, cr, aeff_ref, cutoff;
  int profile, photon_ratio, n_steps, grid_s, grid_v, ode_sub, precision;
  int n_spans;  // identical spans: phased-array factor per node, n-fold ASE
  int lowrank;  // most terms of the low-rank profile table (kRank; ISRSGN_LOWRANK=N caps it, 0: table reads)
  int adj_wide;  // the sixteen-wave adjoint where its LDS fits (1; ISRSGN_ADJOINT_WAVES=4 keeps four waves)
  double rolloff;  // raised-cosine roll-off of every transmit spectrum (0: rectangular)
  int nli;         // points of the within-channel NLI rule
  double s_decades;
  int n_tab;
  const double* tab_f;      // device copies of the tables
  const double* tab_alpha;
  const double* tab_aeff;
};

// Per-call device workspace (sized for the plan by the host runtime).
struct Work {
  double* abar;     // [n_batch] mean loss of the occupied channels
  double* zm;       // [n_batch * M] step midpoints
  double* dz;       // [n_batch * M] step widths
  float* hdz32;     // [n_batch * M] half widths in FP32
  double* step_rec; // [n_batch * M] step records (StepRec, 32 bytes each)
  double* ell64;    // [M * n_total] ln rho(z_m, f_c): plan b block at M * off[b], row-major [m][c]
  float2* lt32;     // same layout: (ell * log2(e)/2, next - this) for the FP32 integrand
  // low-rank form of lt32's values (ODE profile, FP32 form): lr_a [n_batch][M][kRank] (FP32),
  // lr_b [n_total][kRank] (b_r, next channel's b_r - b_r), lr_rank [n_batch] (terms used; -1:
  // the tile kernels read lt32), FP64 workspace lr_res [M * n_total] and lr_b64 [n_total][kRank]
  float* lr_a;
  float2* lr_b;
  int* lr_rank;
  double* lr_res;
  double* lr_b64;
  double* ellL;     // [n_total] ln rho(L, f_c)
  double* tiles;    // [n_tiles]: plan b at toff[b], [i][j][k]
  double* pnli;     // [n_total]
  double* snr;      // [n_total]
  unsigned int* counter;  // work counter of the persistent tile kernels
  unsigned long long* nodes;  // nodes evaluated by the last forward tile launch
  // gradient: S of every node of the current row batch, written by the forward tile kernel
  // and read by the adjoint ([tile - t_begin][part][node]; float2 in the FP32 form, double2
  // in the FP64 form), or null
  void* s_store;
  // adjoint
  double* states;   // ODE states, plan b at sstate_off[b]: [(M*2*ode_sub + 1) * N_b]
  const int64_t* state_off;
  double* lam;      // [n_total] dT/dP_NLI,i * 16/27 gamma_i^2 R_i  (weight of tile row i)
  double* gG;       // [n_total] dT/dG_c accumulated by the adjoint tile kernel
  double* gL;       // [M * n_total] dT/d ell(m, c), same layout as ell64
  double* gLL;      // [n_total] dT/d ell(L, c)
  double* gP;       // [n_total] gradient assembly scratch
};

// Launchers (isrsgn_kernels.hip).  All enqueue on `s` and return the launch status.
hipError_t launch_channel_setup(const PlanView& pv, const FibreParams& fp, hipStream_t s);
hipError_t launch_steps(const PlanView& pv, const FibreParams& fp, const double* P, const Work& w, hipStream_t s);
hipError_t launch_profile(const PlanView& pv, const FibreParams& fp, const double* P, const Work& w,
                          bool keep_states, hipStream_t s);
// tiles [t_begin, t_end); reset_nodes clears the evaluated-node counter first (a call's first launch)
hipError_t launch_tiles(const PlanView& pv, const FibreParams& fp, const double* P, const Work& w,
                        int nmax, int grid, int variant, unsigned int t_begin, unsigned int t_end, bool reset_nodes,
                        hipStream_t s);
const char* tile_variant_name(int variant);
hipError_t launch_reduce(const PlanView& pv, const FibreParams& fp, const double* P, const double* nf,
                         double snr_trx, const Work& w, double* eta, double* pnli_out, double* snr_out,
                         double* thr_out, hipStream_t s);
// P_NLI, eta and SNR of the global channels [g_begin, g_end) (their tile rows must be complete)
hipError_t launch_reduce_rows(const PlanView& pv, const FibreParams& fp, const double* P, const double* nf,
                              double snr_trx, const Work& w, double* eta, double* pnli_out, double* snr_out,
                              int g_begin, int g_end, hipStream_t s);
hipError_t launch_throughput(const PlanView& pv, const double* P, const Work& w, double* thr_out, hipStream_t s);
hipError_t launch_copy_profile(const PlanView& pv, const FibreParams& fp, const Work& w, double* zm,
                               double* dz, double* ell, double* ellL, hipStream_t s);
// The gradient in pieces (row batches): clear dT/d ell and dT/dG; upstream weights of the
// channels [g_begin, g_end); the adjoint of tiles [t_begin, t_end) (stored: S comes from
// w.s_store instead of a recomputing sweep); profile adjoint and assembly.
hipError_t launch_grad_init(const PlanView& pv, const FibreParams& fp, const Work& w, hipStream_t s);
hipError_t launch_grad_rows(const PlanView& pv, const FibreParams& fp, const double* P, const double* nf,
                            double snr_trx, const Work& w, int g_begin, int g_end, hipStream_t s);
// lds_max: LDS one workgroup may allocate (picks the sixteen-wave form where it fits)
hipError_t launch_adjoint_tiles(const PlanView& pv, const FibreParams& fp, const double* P, const Work& w, int nmax,
                                int grid, unsigned int t_begin, unsigned int t_end, bool stored, size_t lds_max,
                                hipStream_t s);
hipError_t launch_grad_finish(const PlanView& pv, const FibreParams& fp, const double* P, const Work& w,
                              double* coef, double* dthr, hipStream_t s);
size_t adjoint_lds(int nmax, int gs, int M, int prec);  // the four-wave form's (the smallest)
size_t tile_lds(const FibreParams& fp, int nmax);
int adjoint_blocks_per_cu(const FibreParams& fp, int nmax, bool stored, size_t lds_max);
int tile_blocks_per_cu(const FibreParams& fp, int nmax, int variant);
hipError_t launch_copy(double* dst, const double* src, int64_t n, hipStream_t s);
// The caller's N_b x N_b tile blocks from tiles (i, j, k): sum over the points j with their weights.
hipError_t launch_fold_tiles(const PlanView& pv, const Work& w, double* out, hipStream_t s);
// Up to kChunkWords 8-byte words carried to the device in the kernel's arguments (no copy from
// host memory, so a captured launch keeps its values): dst[q] = words[q] for q < n.
constexpr int kChunkWords = 240;
struct WordChunk {
  unsigned long long w[kChunkWords];
  int n;
};
hipError_t launch_put_words(unsigned long long* dst, const WordChunk& c, hipStream_t s);
// out[0] invalid entries of P (finite, >= 0) and nf (when given: finite, >= 0); out[1], out[2]
// the first bad index of each (n when none)
hipError_t launch_check_inputs(const double* P, const double* nf, int n, int* out, hipStream_t s);

}  // namespace isrsgn
