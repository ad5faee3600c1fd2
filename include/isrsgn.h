/*
 * isrsgn.h -- C ABI of the MI355X ISRS Gaussian-noise numerical-integral engine.
 *
 * The library evaluates the nonlinear-interference (NLI) model of
 * Jarmolovicius et al., "Optimising O-to-U Band Transmission Using Fast ISRS
 * Gaussian Noise Numerical Integral Model" (arXiv:2401.18022):
 *
 *   - the NLI PSD at a channel of interest (COI), eq. (new_gn_model), solved as
 *     in App. A: distance-step sum eq. (slow_vary), power-profile term eq. (pk),
 *     phase mismatch with beta2..beta4 eq. (phi), quadrants eqs. (q1a)-(q4d) and
 *     hyperbolic coordinates eqs. (q1)-(q4), assembled by eqs. (gain_fin)/(psi_fin);
 *   - the link cost eq. (loss) and the throughput C = 2 B_ch (-L) of Sec. IV;
 *   - its gradient with respect to every launch power (hand-written adjoint).
 *
 * Discretisation (the paper leaves node placement open; these definitions are
 * part of the interface):
 *   * tile (i,k) is the part of the (f1, f2) plane, offsets x = f1 - f_i and
 *     y = f2 - f_i within the band, where f1 + f2 - f_i falls in channel k;
 *     tile(i,k) = sum over parts Q1 (x,y>0, folded about x=y), Q3 (x,y<0, folded)
 *     and Q4 (x>0>y, standing for Q2 too) of a Riemann sum in s = ln|x y| and
 *     v = ln sqrt|x/y|: grid_s midpoints over [ln U - s_decades ln 10, ln U]
 *     (U = sup|x y| over the part) and grid_v midpoints between the exact
 *     per-row v limits; node weight 2 e^s ds dv (unit Jacobian);
 *   * distance steps: n_steps steps with equal power decrement under the mean
 *     loss of the occupied channels, the power term evaluated at the midpoints;
 *   * ln rho(z, f) is interpolated linearly in f between channel centres;
 *   * transmit spectra (eq. new_gn_model's G_Tx): P_c times a unit-area raised cosine of roll-off
 *     beta (the PSD of an RRC-filtered signal), flat to (1-beta) R_c/2 and zero from (1+beta) R_c/2;
 *     beta = 0 (the default) is the rectangle of width R_c;
 *   * noise powers are noise PSDs integrated against the receiver's power response R_i g_i(f - f_i)
 *     (unit passband, noise bandwidth R_i).  For the NLI, nli_points midpoints of equal parts of
 *     the COI's support, weights proportional to the response and normalised to R_i, each point f_j
 *     with its own tiles (i, j, k) (NLI frequency f_j in place of f_i in the offsets, the phase and
 *     the f term of eq. pk) and gamma(f_j)^2; one point (the default) is the locally-white R_i G(f_i);
 *   * P_NLI,i = 16/27 gamma_i^2 R_i sum_k tile(i,k), tile(i,k) = sum_j w_j tile(i,j,k),
 *     w_j = q_j gamma(f_j)^2 / (gamma_i^2 R_i) (w = 1 with one point); eta_i = P_NLI,i / P_i^3;
 *     P_ASE,i = NF_i h f_i R_i / rho(L, f_i);  SNR_i = P_i / (P_NLI,i + P_ASE,i)
 *     (combined with a transceiver SNR as 1/(1/SNR + 1/SNR_trx) when given);
 *     T = sum over P_i > 0 of 2 R_i log2(1 + SNR_i).
 *
 * Conventions: SI units everywhere (Hz, W, m, s).  All arrays are FP64.
 * Arrays named *_dev are device pointers owned by the caller (e.g. torch
 * tensors); everything else is host memory, read during the call only.
 * Work is enqueued on the given HIP stream (NULL = the default stream).  A handle
 * must not be used by two host threads at once.  Every call returns ISRSGN_OK or a
 * negative error code and leaves a message for isrsgn_last_error().
 *
 * Input rules (Sec. IV, eq. loss): launch powers P_k must be finite and >= 0, P_k = 0
 * marking an empty (guard) channel of the set A; noise figures must be finite and >= 0.
 * With the checks on (the default, isrsgn_set_checks) every call first runs a small
 * validation kernel on P (and NF) and waits on the host for its verdict -- so for the
 * stream's earlier work too -- and returns ISRSGN_EINVAL, naming the first bad index,
 * before any output is written; the calls are otherwise asynchronous.  The wait is
 * skipped while the stream is being captured into a graph.  With the checks off (or
 * under capture) nothing is validated: NaN propagates into the outputs and a negative
 * power enters the PSD products as a negative density.  Errors found on the host
 * (arguments, plans) leave the outputs untouched; a HIP error in the middle of a call
 * may leave them partly written.
 */
#ifndef ISRSGN_H
#define ISRSGN_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct isrsgn_fibre isrsgn_fibre; /* opaque: fibre tables, device workspace, caches */

enum {
  ISRSGN_OK = 0,
  ISRSGN_EINVAL = -1,      /* invalid argument (message says which) */
  ISRSGN_ENOMEM = -2,      /* device allocation failed; the handle stays usable */
  ISRSGN_EDEVICE = -3,     /* HIP runtime error (message carries the HIP error string) */
  ISRSGN_EUNSUPPORTED = -4 /* a combination the library does not provide */
};

enum { ISRSGN_FP32 = 0, ISRSGN_FP64 = 1 };
enum { ISRSGN_PROFILE_CLOSED_FORM = 0, ISRSGN_PROFILE_ODE = 1 };

/* Fibre and discretisation (Sec. II, Table I, App. A).  Deep-copied by
 * isrsgn_setup_fibre; the caller may free it on return. */
typedef struct {
  double span_m;            /* span length L */
  double f_ref_hz;          /* reference frequency of the dispersion Taylor series (w_i = f_i - f_ref) */
  double beta2, beta3, beta4; /* s^2/m, s^3/m, s^4/m at f_ref; used when disp_from_d == 0 */
  int disp_from_d;          /* 1: betas from D, S, dS/dlambda at lambda = c/f_ref, eqs. (d)-(d_curve) */
  double d_s_per_m2, s_s_per_m3, sdot_s_per_m4;
  int n_tab;                /* >= 1 points of loss and effective area vs frequency (ascending), */
  const double* tab_f_hz;   /*   interpolated linearly in f and held constant beyond the ends    */
  const double* alpha_per_m;
  const double* aeff_m2;
  double n2_m2_per_w;       /* gamma(f) = 2 pi n2 f / (c A_eff(f)), eq. (gamma) */
  double gamma_const_per_w_m; /* > 0 overrides gamma(f) with a constant */
  double cr_per_w_m_hz;     /* Raman gain slope C_r at aeff_ref_m2; channel k uses C_r A_ref / A_eff(f_k) */
  double aeff_ref_m2;
  double raman_cutoff_hz;   /* triangular gain: zero beyond this offset; <= 0: linear over the band */
  int profile;              /* ISRSGN_PROFILE_CLOSED_FORM (needs n_tab == 1) or ISRSGN_PROFILE_ODE */
  int photon_ratio;         /* ODE: the higher-frequency channel loses f_k/f_j times the power gained */
  int n_steps;              /* distance steps N_M, 1..4096 */
  int grid_s, grid_v;       /* nodes per part: grid_s (2..1024) rows x grid_v (2..65536) per row */
  double s_decades;         /* depth of the ln|xy| window below sup|xy|, > 0 (14 is ample) */
  int ode_sub;              /* ODE: RK4 sub-steps per half distance step, 1..64 */
  int precision;            /* ISRSGN_FP32 or ISRSGN_FP64.  FP32: step terms and the step sum S of each
                               node in FP32, the phase argument phi z_m formed and reduced in FP64,
                               node values |S|^2 w G1 G2 G3 and every later sum in FP64.
                               With the ODE profile the FP32 forward takes ln rho(z_m, f) from a
                               low-rank form of the profile table, checked per call to stay within
                               1e-6 of the FP64 table at every entry (else the table is read);
                               ISRSGN_LOWRANK=N in the environment at setup caps the terms at N
                               (at most 8; 0 always reads the table) */
  int n_spans;              /* identical spans, each followed by an amplifier restoring the launch
                             * power (App. A, eq. gain summed over spans), 1..100000: every node's
                             * |S|^2 carries the phased-array factor sin^2(n phi L/2)/sin^2(phi L/2)
                             * and the ASE is n times one span's */
  double rolloff;           /* raised-cosine roll-off of every transmit spectrum, 0..1 (0: rectangular);
                             * the closed-form profile then uses the spectrum's Laplace transform
                             * sinhc(aR/2) cosh(a beta R/2) / (1 + (a beta R/pi)^2) for sinhc(aR/2) */
  int nli_points;           /* points of the within-channel NLI rule, 1..64 (1: locally white); the
                             * pair-integral work grows in proportion */
} isrsgn_fibre_desc;

/* One or more channel plans, concatenated CSR-style (host memory).
 * Plan b owns channels [ch_offsets[b], ch_offsets[b+1]); each plan is sorted by
 * frequency with non-overlapping spectra (f_{k+1} - f_k >= (1 + rolloff) (R_k + R_{k+1})/2),
 * 1..1024 channels.  Device copies are cached by content. */
typedef struct {
  int n_batch;
  const int* ch_offsets;    /* n_batch + 1 entries, ch_offsets[0] == 0 */
  const double* f_hz;       /* channel centres */
  const double* rs_hz;      /* symbol rates = rectangular PSD widths (Sec. III) */
} isrsgn_plan;

/* Creates a handle.  Validates desc (EINVAL), converts the dispersion, copies the
 * tables.  *out is set only on success; release it with isrsgn_destroy. */
int isrsgn_setup_fibre(const isrsgn_fibre_desc* desc, isrsgn_fibre** out);

/* NLI of every channel of every plan: eq. (gain_fin) times R_i.
 *   P_w_dev[n_ch_total]     launch powers (>= 0; 0 marks an empty channel, the set A of eq. loss)
 *   eta_dev[n_ch_total]     eta_i = P_NLI,i / P_i^3 (NaN where P_i == 0)
 *   pnli_w_dev[n_ch_total]  P_NLI,i in W (may be NULL)
 *   tile_dev_or_null        per plan an N_b x N_b row-major block [i][k] of tile integrals
 *                           (W^3/Hz^3 * Hz^2 * m^2; with several NLI points the weighted sum over
 *                           them, so P_NLI,i = 16/27 gamma_i^2 R_i sum_k tile(i,k) holds), blocks
 *                           concatenated in plan order; may be NULL */
int isrsgn_eta(isrsgn_fibre* h, const isrsgn_plan* plan, const double* P_w_dev, double* eta_dev,
               double* pnli_w_dev, double* tile_dev_or_null, void* hip_stream);

/* SNR per channel and throughput per plan (eq. loss, Sec. IV).
 *   nf_lin_dev[n_ch_total]  amplifier noise figure (linear)
 *   snr_trx_lin             transceiver back-to-back SNR (linear); 0 = ideal transceiver
 *   snr_dev[n_ch_total]     linear SNR (0 where P_i == 0)
 *   thr_bps_dev[n_batch]    throughput in bit/s */
int isrsgn_snr(isrsgn_fibre* h, const isrsgn_plan* plan, const double* P_w_dev, const double* nf_lin_dev,
               double snr_trx_lin, double* snr_dev, double* thr_bps_dev, void* hip_stream);

/* isrsgn_snr plus the exact gradient of each plan's throughput with respect to every
 * launch power, through the PSD products and the power profile (adjoint method).
 *   dthr_dP_dev[n_ch_total] d thr_b / d P_k in bit/s/W for k in plan b
 * Workspace: the forward keeps S of eq. (psi_fin) per integration node (8 bytes per node in
 * the FP32 form, 16 in the FP64 form) for one batch of COI rows at a time, so the adjoint
 * does not evaluate the step terms twice.  The handle allocates it per plan on the first
 * gradient call for that plan, at most ISRSGN_STORE_MB MiB (environment; 0 keeps no store;
 * by default half of the device memory free at that call), and splits the rows into as many
 * batches as that bound needs; it lives until isrsgn_destroy.  If a row does not fit or the allocation fails, the adjoint
 * recomputes S instead (same result, slower).  ISRSGN_ENOMEM if the adjoint's other
 * buffers (O(n_ch_total * n_steps) doubles) cannot be allocated.  The FP32 form's adjoint with
 * the store runs sixteen-wave workgroups where their LDS fits the device (plans up to about
 * 1400 channels at grid 128 x 128, 112 steps), else four-wave ones; ISRSGN_ADJOINT_WAVES=4 in
 * the environment at setup keeps four (same result to the rounding of FP64 atomics). */
int isrsgn_snr_grad(isrsgn_fibre* h, const isrsgn_plan* plan, const double* P_w_dev, const double* nf_lin_dev,
                    double snr_trx_lin, double* snr_dev, double* thr_bps_dev, double* dthr_dP_dev,
                    void* hip_stream);

/* isrsgn_snr for callers that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same arguments, input rules and results as
 * isrsgn_snr (a single call also accepts several plans).  It calls no allocator: the plan's device
 * copy and the call's whole workspace (distance steps, power-profile tables, tile integrals,
 * reductions) live in one static device array of ISRSGN_NOALLOC_SCRATCH_BYTES, of which every GPU
 * the library runs on holds its own copy until the process ends (its address is looked up at
 * isrsgn_setup_fibre).  The plan reaches the device in kernel arguments, not through a copy from
 * host memory, so a captured call replays with the plan it was captured with.
 *   Limit: the call's workspace must fit the array, else ISRSGN_EINVAL stating the need.  In bytes,
 *   each section rounded up to 256: per plan about 8 N_b^2 (tiles) plus 8 N_ch n_steps (FP64
 *   table), 8 N_ch n_steps more in the FP32 form and 8 N_ch n_steps more with the FP32 form and the
 *   ODE profile, plus O(N_ch + n_batch n_steps) small arrays: 4.3 MiB for 589 channels at 112 steps,
 *   10.8 MiB for 1024 channels.
 *   Sharing: every call on a GPU uses that GPU's one array, which keeps the last call's contents;
 *   calls that overlap on one GPU (several streams, handles or host threads) race and give wrong
 *   results, so the caller serialises them.
 * The tile-kernel variant is the autotuner's earlier choice for the discretisation (or
 * ISRSGN_TILE_VARIANT), else a fixed default; results agree with isrsgn_snr to the precision
 * form's rounding.  Stage timers and work counters do not cover this call, and isrsgn_destroy does
 * not wait for it: synchronise its stream before destroying the handle. */
#define ISRSGN_NOALLOC_SCRATCH_BYTES (32 * 1024 * 1024)
int isrsgn_snr_noalloc(isrsgn_fibre* h, const isrsgn_plan* plan, const double* P_w_dev, const double* nf_lin_dev,
                       double snr_trx_lin, double* snr_dev, double* thr_bps_dev, void* hip_stream);

/* The distance steps and the power profile on their own (App. A, eq. pk):
 *   z_mid_dev[n_batch * n_steps], dz_dev[n_batch * n_steps]  step midpoints and widths per plan
 *   ell_dev   per plan an n_steps x N_b row-major block of ln rho(z_m, f_c)
 *   ell_L_dev[n_ch_total]     ln rho(L, f_c)
 * Any output may be NULL. */
int isrsgn_profile(isrsgn_fibre* h, const isrsgn_plan* plan, const double* P_w_dev, double* z_mid_dev,
                   double* dz_dev, double* ell_dev, double* ell_L_dev, void* hip_stream);

/* Graph mode (a9).  When enabled, each (plan, entry point, transceiver SNR) is captured once
 * into a HIP graph on the handle's own non-blocking stream, over device buffers the plan
 * owns; every later call copies P and NF in with a kernel, launches the graph on the
 * caller's stream and copies the outputs out (no memset or memcpy nodes).  The first call
 * for a discretisation runs eagerly so the autotuner can time the tile-kernel variants.
 * Results are identical to eager calls.  Stage timers report only the whole call. */
int isrsgn_set_graph(isrsgn_fibre* h, int enabled);

/* Stage timers.  When enabled, every call records HIP events around its stages on
 * its stream.  isrsgn_stage_times waits for the last call and writes milliseconds
 * for: [0] steps+profile, [1] pair integrals (forward tile kernel), [2] reduction,
 * [3] adjoint tile kernel, [4] profile adjoint + gradient assembly, [5] whole call;
 * stages that did not run read 0.  n is the capacity of ms_out (up to 6). */
int isrsgn_set_timing(isrsgn_fibre* h, int enabled);
int isrsgn_stage_times(isrsgn_fibre* h, double* ms_out, int n);

/* Work done by the last call's forward pair integrals on the most recently used plan
 * (waits for it): [0] nodes evaluated (nodes on the channel support of non-empty rows),
 * [1] node-steps = nodes * n_steps, [2] tiles, [3] index of the tile-kernel variant the
 * autotuner chose (ISRSGN_TILE_VARIANT in the environment forces one; ISRSGN_TUNE_CACHE
 * names a file that keeps the choices across processes), [4] batches of COI rows of a
 * gradient with the per-node store (0: the adjoint recomputed S; the store is bounded by
 * ISRSGN_STORE_MB in the environment, by default half of the free device memory, 0 disables it), [5] plans whose FP32
 * step terms used the low-rank form of the ODE profile table (the rest read the table), [6] the
 * most terms any of them needed.  n is the capacity of out (up to 7). */
int isrsgn_work_counts(isrsgn_fibre* h, double* out, int n);

/* Input checks (default on): see "Input rules" above.  Off: no validation kernel and no host
 * wait, for callers that guarantee valid inputs (serving loops, graph capture). */
int isrsgn_set_checks(isrsgn_fibre* h, int enabled);

/* Frees the handle and its device memory.  Waits for the last call on every stream the handle
 * was given (not for unrelated work; the runtime's own free may still wait for the device).
 * NULL is allowed. */
void isrsgn_destroy(isrsgn_fibre* h);

/* Message of the last failed call on this thread ("" if none). Valid until the next call. */
const char* isrsgn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ISRSGN_H */
