/* fstat.h -- coherent F-statistic over a grid of sky positions and spindowns,
 * on one AMD Instinct MI355X (gfx950).
 *
 * The method is the narrow-band all-sky search of Astone, Borkowski,
 * Jaranowski, Krolak and Pietka, "Data analysis of gravitational-wave signals
 * from spinning neutron stars. V": for every grid node (sky position alpha,
 * delta and spindown fdot) the data are demodulated and resampled to the
 * solar-system-barycentre time (Sec. VI A, Eqs. Bt and ia), multiplied by the
 * amplitude-modulation functions a(t), b(t) (Sec. II, Eq. patt), Fourier
 * transformed (Sec. VI B, Eq. DFT) into the two correlations F_a, F_b of
 * Eqs. (Fab), and combined into the F-statistic of Eq. (OS) on every Fourier
 * bin of the band.
 *
 * Conventions
 *   - Every call returns fstat_status: FSTAT_OK (0) or a negative error code.
 *     Arguments are validated before any device work; on error nothing is
 *     launched and the outputs are left untouched.  No call aborts, throws or
 *     exits.
 *   - Pointers marked "host" are read during the call and may be freed when it
 *     returns.  Pointers marked "device" are device memory of the plan's GPU,
 *     owned by the caller (e.g. torch tensors); the library writes them
 *     asynchronously on the caller's stream (hip_stream = hipStream_t, NULL for
 *     the default stream).
 *   - A plan is immutable after creation, except for its workspace; calls on
 *     one plan must not overlap in time (they share the workspace): serialise
 *     them on one stream.
 *   - Frequencies are band-relative: the data are real narrow-band samples of
 *     the band [f_ref, f_ref + 1/(2 dt)); a band-relative frequency f is the
 *     physical frequency f_ref + f.  Bin k of an nfft-point transform is
 *     f_k = k / (nfft dt); the bins of the band are 0 <= k < nfft/2.
 *   - Times: t is segment time in seconds (0 at the first sample, which is also
 *     the spindown reference time, Eq. pha3); the ephemeris clock is
 *     T = t0 + t.
 */
#ifndef FSTAT_H
#define FSTAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fstat_status;
#define FSTAT_OK 0
#define FSTAT_EINVAL (-1)        /* a null pointer, a size or a value out of range */
#define FSTAT_ENOTINTDAYS (-2)   /* n dt is not n_sidereal_days sidereal days (within dt/2) */
#define FSTAT_ENOMEM (-3)        /* device or pinned-host allocation failed */
#define FSTAT_EDEVICE (-4)       /* a HIP runtime call failed (no device, launch error) */
#define FSTAT_EUNSUPPORTED (-5)  /* valid but not supported: nfft not a power of two in
                                    [2^10, 2^22] or below n; n below 16 */

/* Interpolation used to resample onto the barycentric time grid (Sec. VI A). */
#define FSTAT_NEAREST 0     /* nearest neighbour ("stroboscopic") resampling */
#define FSTAT_LINEAR_UP2 1  /* two-step: 2x Fourier upsampling, then a degree-1 spline */
#define FSTAT_CUBIC_UP2 2   /* two-step: 2x Fourier upsampling, then the periodic cubic spline */

/* Arithmetic of the node path.  In both modes the barycentric time, the Roemer
 * delay and the demodulation phase are evaluated in FP64. */
#define FSTAT_FP32 0  /* resampled data, FFTs and F combination in FP32 */
#define FSTAT_FP64 1  /* everything in FP64 */

/* Output modes of fstat_grid. */
#define FSTAT_OUT_MAP 0        /* F on every bin of [k_lo, k_hi) */
#define FSTAT_OUT_MAX 1        /* per node: the largest F in [k_lo, k_hi) and its bin */
#define FSTAT_OUT_CROSSINGS 2  /* every (node, bin) with F above a threshold */

/* Detector (Sec. II; Sec. V for the Earth radius). Angles in radians. */
typedef struct {
  double lat_rad;    /* geodetic latitude */
  double lon_rad;    /* east longitude */
  double gamma_rad;  /* arm bisector, measured counter-clockwise from local East */
  double zeta_rad;   /* angle between the arms (pi/2); only scales injected signals */
  double radius_m;   /* distance of the site from the Earth's centre (spherical Earth) */
} fstat_detector;

/* Analytic ephemeris standing in for the DE405-based astrometry of Sec. V: the
 * Earth's centre on a circular orbit in the ecliptic plane (the R_ES term of
 * Eq. pha5), the site rotating at the sidereal rate (the R_E term). */
typedef struct {
  double obliquity_rad;    /* obliquity of the ecliptic, Eq. (pha4) */
  double orbit_radius_m;   /* SSB -> Earth-centre distance */
  double orbit_omega;      /* orbital angular rate, rad/s */
  double orbit_phase0;     /* orbital angle at T = 0, rad */
  double sidereal_day_s;   /* rotation period (86164 s in the workloads) */
  double gmst0_rad;        /* sidereal angle of Greenwich at T = 0 */
} fstat_ephemeris;

/* One data segment.  The observation time n dt must be a whole number of
 * sidereal days (the assumption under which <ab> = 0 and Eq. (OS) holds,
 * Sec. III A). */
typedef struct {
  const double *x;          /* host [n]: real narrow-band samples */
  int64_t n;                /* samples, >= 16 */
  double dt;                /* sampling interval, s */
  int32_t n_sidereal_days;  /* n dt / sidereal_day_s, >= 1 */
  double t0;                /* ephemeris time of the first sample, s */
  const uint8_t *mask;      /* host [n] or NULL: 0 marks a gap (sample ignored); at least
                               one sample must be kept (FSTAT_EINVAL otherwise) */
  double f_ref_hz;          /* lower band edge */
  double sigma2;            /* noise variance per sample; <= 0: estimated from the
                               data outside gaps (unbiased sample variance) */
  int64_t nfft;             /* FFT length: power of two, n <= nfft <= 2^22;
                               0 = smallest power of two >= 2n */
} fstat_segment;

typedef struct {
  int32_t interp;    /* FSTAT_NEAREST / FSTAT_LINEAR_UP2 / FSTAT_CUBIC_UP2 */
  int32_t prec;      /* FSTAT_FP32 / FSTAT_FP64 */
  int32_t device;    /* HIP device ordinal */
  int32_t max_batch; /* nodes per FFT batch; 0 = library default (or the tuned value) */
  int32_t autotune;  /* 1: at plan time, time the candidate FFT splits nfft = R x C
                        (C = 1024, 2048, 4096 columns where valid), node-batch sizes
                        (FP32: 32, 64, 128, 256; FP64: 2, 4, 8) and stream modes (1, 2; see
                        fstat_plan_schedule) of every segment on a sample grid of 64 sky
                        positions (FP64: 8) x 16 spindowns, in two sweeps (in order, then
                        reversed), and keep the fastest (the default schedule unless
                        another is at least 3 % faster); one
                        tuning per distinct (n, nfft), shared by the segments of that
                        size.  The choice is cached in the file named by the
                        environment variable FSTAT_TUNE_CACHE if it is set.
                        0: fixed defaults. */
  int32_t launch;    /* FSTAT_LAUNCH_PASSES or FSTAT_LAUNCH_PERSISTENT */
} fstat_options;

/* How fstat_grid (and a recorded graph) runs a call. */
#define FSTAT_LAUNCH_PASSES 0      /* a sequence of launches per sky batch and node batch: sky
                                      preparation, first FFT pass, second FFT pass (default) */
#define FSTAT_LAUNCH_PERSISTENT 1  /* the whole call in one launch of a persistent kernel: a work
                                      queue of tiles (sky preparation of each sky batch, pass 1
                                      and pass 2 of each node), segments ordered by FFT length
                                      (longest first), each tile started once what it reads is
                                      complete.  Used for FP32 plans on calls whose segments all
                                      have 2^18 <= nfft <= 2^22 (the plan then splits them with
                                      C = 4096 columns) and no interbinning; other calls run as
                                      FSTAT_LAUNCH_PASSES.  Every wait inside the kernel is
                                      bounded: if one expires the kernel stops early and the
                                      plan's error flag is set (fstat_plan_status).  The
                                      outputs equal those of FSTAT_LAUNCH_PASSES bit for bit
                                      (the same tile code runs in both). */
/* Environment: FSTAT_STREAMS=1 (or 2) at plan creation fixes the stream mode
 * of every segment (see fstat_plan_schedule) instead of the default or tuned
 * one; meant for per-kernel timing.  FSTAT_PERSIST_SLOTS (3..128, default
 * 128: spill slots of nfft x 16 bytes each) and FSTAT_PERSIST_CHUNK (a
 * divisor of 64, default 32: tiles a workgroup claims at once) set the
 * pipeline of FSTAT_LAUNCH_PERSISTENT; the outputs do not depend on them.
 * FSTAT_PERSIST_SPIN_TICKS lowers the bound of the persistent kernel's waits
 * (wall-clock ticks, default 2 s worth; 0: a wait not satisfied at once
 * expires): a way to exercise the error path of fstat_plan_status. */

typedef struct fstat_plan_s *fstat_plan_t;

/* Create a plan: copies the segments to the device and does the
 * node-independent preparation of Sec. VI A: gap mask, noise variance (the
 * sigma^2 of the normalisation S0 = 2 sigma^2 dt of Eq. OS for white noise),
 * and, for the two-step interpolations, the 2x Fourier upsampling of the data
 * and its spline.  The observation time of every segment must be a whole
 * number of sidereal days (Sec. III A, the condition under which <ab> = 0 and
 * F takes the form of Eq. OS): FSTAT_ENOTINTDAYS otherwise.  With
 * opt->autotune the FFT schedule of every segment size is timed and chosen
 * (see fstat_options).  Synchronous.  On success *out receives the plan,
 * which owns device copies of the segments; release it with fstat_destroy.
 * Errors: FSTAT_EINVAL (NULL pointers, nseg <= 0, options out of range,
 * non-finite data or geometry, a segment made only of gaps),
 * FSTAT_EUNSUPPORTED (n < 16, nfft not a power of two in [max(n, 2^10),
 * 2^22]), FSTAT_ENOMEM, FSTAT_EDEVICE (no device, or opt->device out of
 * range gives FSTAT_EINVAL). */
fstat_status fstat_plan(const fstat_segment *segs, int32_t nseg, const fstat_detector *det,
                        const fstat_ephemeris *eph, const fstat_options *opt, fstat_plan_t *out);

/* A grid node: sky position, spindown (Hz/s), segment index, and the offset of
 * its line of Fourier bins.  Output bin k of a node is the band-relative
 * frequency (k + bin_offset) / (nfft dt): the nodes of a lattice grid lie on
 * lines parallel to the frequency axis spaced by one Fourier bin, each line
 * shifted by a fraction of a bin (Sec. IV, Eq. avec).  0 gives the plain
 * Fourier frequencies; |bin_offset| < 1 (FSTAT_EINVAL otherwise). */
typedef struct {
  double alpha;       /* right ascension, rad */
  double delta;       /* declination, rad */
  double fdot;        /* first spindown, Hz/s */
  int32_t seg;        /* segment of the plan */
  float bin_offset;   /* in Fourier bins */
} fstat_node;

/* A threshold crossing (output mode FSTAT_OUT_CROSSINGS). */
typedef struct {
  int64_t node;   /* index into the node array of the call */
  int64_t k;      /* Fourier bin */
  double F;
} fstat_crossing;

/* Output descriptor of fstat_grid.  The element type of F and Fmax is float
 * for an FSTAT_FP32 plan and double for an FSTAT_FP64 plan. */
typedef struct {
  int32_t mode;             /* FSTAT_OUT_MAP / _MAX / _CROSSINGS */
  int32_t interbin;         /* 0: the Fourier bins k only.  1: also the half bins k + 1/2 by
                               interbinning, Eq. (intbin) of Sec. VI B:
                               S(k + 1/2) ~ (S(k+1) - S(k)) / sqrt(2) for S_a and S_b, then
                               F as below.  Every output then covers 2 (k_hi - k_lo) points
                               indexed 2k + h (h = 1 for k + 1/2): the map is
                               [n_nodes][2 (k_hi - k_lo)], kmax and the crossings' k are in
                               half-bin units.  Meant for nfft = nextpow2(n) (no padding). */
  int64_t k_lo, k_hi;       /* bins 0 <= k_lo < k_hi <= nfft/2 of every node's segment */
  double threshold;         /* mode CROSSINGS: report F > threshold */
  void *F;                  /* device [n_nodes][k_hi - k_lo] (mode MAP; twice as wide with interbin) */
  void *Fmax;               /* device [n_nodes] (mode MAX) */
  int64_t *kmax;            /* device [n_nodes] (mode MAX); ties go to the lowest bin */
  fstat_crossing *crossings;      /* device [max_crossings] (mode CROSSINGS), unordered */
  unsigned long long *n_crossings;/* device [1]: number of crossings found (may exceed
                                     max_crossings; records beyond it are dropped) */
  int64_t max_crossings;
} fstat_out;

/* F-statistic of Eq. (OS) on the Fourier bins of every node (Sec. VI):
 *   F_k = (B |S_a,k|^2 + A |S_b,k|^2 - 2 C Re(S_a,k S_b,k*)) / (sigma^2 (A B - C^2)),
 *   S_a,k = sum_j x(t_j) a(t_j) e^{-i phi_s(t_j)} e^{-2 pi i j k / nfft},
 * with t_j the detector time of barycentric time t_b0 + j dt, A, B, C the sums
 * of a^2, b^2, ab over the detector samples outside gaps (C vanishes for
 * whole sidereal days without gaps, which gives Eq. OS exactly).
 * nodes: host [n_nodes].  The F values are written on hip_stream; the call
 * returns once the work is enqueued. */
fstat_status fstat_grid(fstat_plan_t p, const fstat_node *nodes, int64_t n_nodes, const fstat_out *out,
                        void *hip_stream);

/* The batched grid of Sec. VI as one replayable launch: records the whole
 * launch sequence of fstat_grid(p, nodes, n_nodes, out) -- every segment and
 * sky batch of the node list, both FFT passes -- into a HIP graph with a device
 * workspace of its own.  Arguments and errors as for fstat_grid; synchronous.
 * The node list is copied; the output buffers named in *out are the ones every
 * launch writes.  The graph reads the plan's segment data, so destroy it before
 * the plan.  *g receives the graph. */
typedef struct fstat_graph_s *fstat_graph_t;
fstat_status fstat_graph_create(fstat_plan_t p, const fstat_node *nodes, int64_t n_nodes, const fstat_out *out,
                                fstat_graph_t *g);
/* Enqueue one replay on hip_stream: the outputs are rewritten exactly as a
 * fstat_grid call with the recorded arguments would write them.  Replays of one
 * graph that overlap in time (on different streams) race on its workspace. */
fstat_status fstat_graph_launch(fstat_graph_t g, void *hip_stream);
/* Waits for the device, then frees the graph and its workspace. */
void fstat_graph_destroy(fstat_graph_t g);

/* F at continuous parameters by the same resampling method (the sum over the
 * barycentric grid with e^{-2 pi i f j dt} in place of the FFT kernel), for
 * candidate refinement off the grid.  All FP64.
 *   params: device [n][4] = (f band-relative Hz, fdot Hz/s, alpha rad, delta rad)
 *   seg:    device [n] segment indices, or NULL for segment 0
 *   F:      device [n]
 *   state:  device [n][FSTAT_STATE] or NULL: what fstat_adjoint needs
 *           (S_a, S_b, A, B, C) */
#define FSTAT_STATE 8
fstat_status fstat_eval(fstat_plan_t p, const double *params, const int32_t *seg, int64_t n, double *F,
                        double *state, void *hip_stream);

/* Reverse-mode (adjoint) pass of fstat_eval: dparams[i][:] = gF[i] * dF_i/d(f, fdot,
 * alpha, delta), recomputing the resampled series rather than storing it.
 * Differentiates through t_b0(alpha, delta), the implicit relation
 * t_j + phi_m(t_j) = t_b0 + j dt, the interpolant (zero for FSTAT_NEAREST),
 * a(t_j), b(t_j), the phase, and A, B, C.
 *   state: device [n][FSTAT_STATE] from fstat_eval with the same params
 *   gF:    device [n] upstream gradient, or NULL for ones
 *   dparams: device [n][4] */
fstat_status fstat_adjoint(fstat_plan_t p, const double *params, const int32_t *seg, int64_t n,
                           const double *state, const double *gF, double *dparams, void *hip_stream);

/* Second step of the maximum-likelihood estimation (Sec. III): at the
 * candidates' (f, fdot, alpha, delta), the estimators of the four amplitudes
 * (Eq. amle0; with gaps, the 2 x 2 normal equations in A, B, C that reduce to it
 * when C = 0) and their inversion to h0, cos(iota), psi, phi0 (Eqs. ampone,
 * h0iota).  The phase 2 pi (f_ref + f) phi_m(0) that F does not need is
 * restored, so phi0 refers to the signal phase of Eq. (pha3) at t = 0.
 *   state: device [n][FSTAT_STATE] from fstat_eval with the same params
 *   out:   device [n][8]: the amplitudes A1..A4 of Eq. (ampone) (the data's
 *          amplitudes divided by sin zeta), h0, cos(iota), psi in [0, pi/2),
 *          phi0 in [0, 2 pi) ((psi + pi/2, phi0 + pi) describes the same wave;
 *          for cos(iota) = +-1 only 2 psi +- phi0 is determined).
 * Invalid segment indices give NaN rows. */
fstat_status fstat_amplitudes(fstat_plan_t p, const double *params, const int32_t *seg, int64_t n,
                              const double *state, double *out, void *hip_stream);

/* F at the candidates' (f, fdot, alpha, delta) without resampling: Eqs. (OS)-(Fab)
 * summed directly on the detector samples t_i = i dt with the phase of Eq. (pha3)
 * (less the heterodyne) at the detector time, as the paper's fine search
 * evaluates it (Sec. VII).  FP64.  params, seg, F as for fstat_eval. */
fstat_status fstat_eval_exact(fstat_plan_t p, const double *params, const int32_t *seg, int64_t n, double *F,
                              void *hip_stream);

/* Fine search (Sec. VI C): from each candidate, a Nelder-Mead simplex search for
 * the maximum of F over (f, fdot, alpha, delta), all candidates in one launch
 * (one workgroup each).  Coordinates are scaled by scale[] (the initial simplex is
 * the start plus one step scale[d] along each axis); the search stops when every
 * vertex lies within tol scale units (per axis) of the best one, or after
 * max_evals evaluations of F.  Coefficients: reflection 1, expansion 2,
 * contraction 1/2, shrink 1/2. */
typedef struct {
  double scale[4];    /* > 0, in the units of f (Hz), fdot (Hz/s), alpha, delta (rad) */
  double tol;         /* > 0, in scale units */
  int32_t max_evals;  /* 5 .. 100000 */
  int32_t exact;      /* 1: F of fstat_eval_exact; 0: F of fstat_eval (resampling method) */
} fstat_refine_options;
/*   params:     device [n][4] starting points (e.g. the coarse-grid maxima)
 *   params_out: device [n][4] best vertex;  F_out: device [n] its F
 *   evals_out:  device [n] F evaluations used, or NULL.  Invalid segments give NaN. */
fstat_status fstat_refine(fstat_plan_t p, const double *params, const int32_t *seg, int64_t n,
                          const fstat_refine_options *opt, double *params_out, double *F_out, int32_t *evals_out,
                          void *hip_stream);

/* Detection threshold F0 for a false-alarm probability alpha over n_cells
 * independent cells: inverts Eq. (FP), alpha = 1 - (1 - P_F(F0))^N_c, with
 * P_F(F0) = (1 + F0) e^{-F0} of Eq. (PF) (2F chi-square with 4 degrees of
 * freedom).  Host computation; 0 < alpha < 1, n_cells >= 1.  The expected number
 * of false alarms is N_c P_F(F0) (Eq. NF). */
fstat_status fstat_threshold(double alpha, double n_cells, double *F0);

/* ---- The lattice grid of Sec. IV (host computations, no device) --------------
 * Phase parameters of the linear model with one spindown (Sec. III B, Eqs.
 * philin, albe, siglin): xi = (omega_0 [rad/s], omega_1 [rad/s^2], alpha_1,
 * alpha_2 [rad/s]) with the known functions m = (t, t^2/2, mu_1(t), mu_2(t)),
 * mu_1 = (R^y_ES + R^y_E cos eps)/c, mu_2 = (R^x_ES + R^x_E)/c, t the segment
 * time.  alpha_1 = omega (n_y), alpha_2 = omega (n_x) in the ecliptic frame. */

/* Reduced Fisher matrix of Eq. (redFm-def), G_kl = <m_k m_l> - <m_k><m_l>, the
 * average over the kept samples t_j = j dt of one segment (its x is not read).
 *   gamma: host [4][4] row-major, written.
 * FSTAT_EINVAL: a NULL pointer, n < 2, dt <= 0, fewer than 2 kept samples. */
fstat_status fstat_lattice_fisher(const fstat_segment *seg, const fstat_detector *det, const fstat_ephemeris *eph,
                                  double gamma[16]);

/* A covering lattice of the correlation hyperellipsoid G(tau, tau) = 1 - C0
 * (Eq. hype): A4* (Eq. gen, thickness 1.7655) with covering radius
 * R = sqrt(1 - C0) in whitened coordinates, shrunk by mu along a lattice vector
 * l and expanded by nu across it so that l maps onto a0 = (dp0, 0, 0, 0)
 * (Eqs. avec, opt), then turned about a0 so that a second basis vector has no
 * sky components (Eqs. constraint2, opt2).  Every parameter point lies within
 * correlation C0 (in the linear model) of a lattice point. */
typedef struct {
  double basis[16];    /* rows a0..a3 (row-major [4][4], xi coordinates): a0 = (dp0, 0, 0, 0);
                          a1 = (a10, a11, 0, 0); a2, a3 the sky vectors, their sky projections
                          Lagrange-Gauss reduced, |omega_1 part| <= |a11|/2, |omega_0 part| <= dp0/2 */
  double gamma[16];    /* the reduced Fisher matrix it was built for */
  double dp0;          /* angular frequency spacing of the Fourier bins, 2 pi / (nfft dt) */
  double c0;           /* minimal correlation C0 */
  double R;            /* sqrt(1 - C0) */
  double mu, nu;       /* shrink along l, expansion across it */
  double theta;        /* thickness 1.7655 / (mu nu^3) */
  double margin_w1;    /* half-width of a covering ellipsoid's shadow on the omega_1 axis */
  double margin_sky;   /* its largest half-width in the (alpha_1, alpha_2) plane */
  int32_t rule;        /* the rule for nu it was built with */
  int32_t reserved;
} fstat_lattice;

/* The expansion factor nu.  The paper defines it by the covering radius
 * staying R; its worked two-dimensional example (nu = sqrt(108 - pi^2)/9,
 * theta = 1.8171) and the Virgo thickness (about 20 % above A4*) follow
 * another rule, the largest nu keeping the images of the starting lattice's
 * deep holes within R.  Both give coverings; the first is thinner (2-D
 * example: theta 1.219; 2-day segment at nfft = 2^20: 1.838 against 2.094). */
#define FSTAT_NU_DEEP_HOLES 0  /* the worked example's rule: closed form, microseconds */
#define FSTAT_NU_COVERING 1    /* the definition: bisection on the covering radius, ~1 s */

/*   gamma: host [4][4] symmetric positive definite; dp0 > 0; 0 < c0 < 1;
 *   rule: FSTAT_NU_DEEP_HOLES or FSTAT_NU_COVERING.
 * FSTAT_EINVAL: arguments out of range, gamma not positive definite or too
 * ill-conditioned for the constraints to hold to 1e-9. */
fstat_status fstat_lattice_build(const double gamma[16], double dp0, double c0, int32_t rule,
                                 fstat_lattice *out);

/* The lattice of one segment: fstat_lattice_fisher over its kept samples, then
 * fstat_lattice_build with the angular resolution of its Fourier bins,
 * dp0 = 2 pi / (nfft dt) (nfft = seg->nfft, or the smallest power of two
 * >= 2n when 0: the plan's FFT length).  Errors as for the two calls, and
 * FSTAT_EINVAL for an nfft that is not a power of two >= n. */
fstat_status fstat_lattice_segment(const fstat_segment *seg, const fstat_detector *det, const fstat_ephemeris *eph,
                                   double c0, int32_t rule, fstat_lattice *out);

/* A sky region and spindown range to cover. */
typedef struct {
  double f_sky_hz;      /* frequency of the sky mapping, omega_s = 2 pi f_sky (the top of the band:
                           the finest sky resolution the band needs) */
  double fdot_lo, fdot_hi;            /* spindown range, Hz/s */
  double sky_c1, sky_c2, sky_radius;  /* a disk in the (alpha_1, alpha_2) plane, rad/s;
                                         sky_radius <= 0: the whole sky disk |alpha| <= omega_s */
  int32_t hemisphere;   /* +1 / -1: ecliptic north / south only; 0: both */
  int32_t seg;          /* written into every node */
} fstat_lattice_region;

/* The grid nodes of a lattice over a region: every lattice point whose covering
 * ellipsoid reaches the region (the ranges widened by the margins), one node per
 * (sky point, spindown); the node's Fourier bins k are the lattice points
 * k a0 + (its omega_0), so its bin_offset is frac(omega_0 / dp0) (a float32; a
 * value that rounds to 1 is 0).  A sky point inside the disk gives both
 * directions n_z = +-sqrt(1 - n_x^2 - n_y^2) (the linear model does not tell
 * them apart) unless hemisphere selects one; one outside it is put on the
 * ecliptic (n scaled to unit length).  Order: sky points (k2 outer, k3 inner),
 * then direction, then k1.
 *   nodes: host [capacity] or NULL when capacity = 0; coef: host [capacity][3]
 *   lattice coefficients (k1, k2, k3) of a1, a2, a3, or NULL.
 *   *count receives the number of nodes of the region; min(count, capacity)
 *   are written.  The obliquity is the ephemeris's. */
fstat_status fstat_lattice_nodes(const fstat_lattice *lat, const fstat_lattice_region *reg,
                                 const fstat_ephemeris *eph, fstat_node *nodes, int32_t *coef, int64_t capacity,
                                 int64_t *count);

/* F and its gradient for the gradient refinement of candidates off the coarse
 * grid (the fine search of Sec. VI C, by ascent instead of a simplex): F of
 * fstat_eval at params and, if dF != NULL, dF/d(f, fdot, alpha, delta) of
 * fstat_adjoint with unit upstream weights, in one call.
 *   params: device [n][4] as for fstat_eval; seg: device [n] or NULL
 *   F: device [n]; dF: device [n][4] or NULL (then F only)
 * The forward state between the two kernels lives in the plan's workspace
 * (n x FSTAT_STATE doubles, grown on demand: the call may allocate device
 * memory, and overlapping calls on one plan race on it).  Invalid segment
 * indices give NaN.  FSTAT_EINVAL for NULL params/F or n <= 0. */
fstat_status fstat_grad(fstat_plan_t p, const double *params, const int32_t *seg, int64_t n, double *F,
                        double *dF, void *hip_stream);

/* fstat_grad without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc).  The same kernels and results as fstat_grad; the forward state
 * lives in a fixed device array of the library (FSTAT_GRAD_STATIC_MAX x
 * FSTAT_STATE doubles, 4 MiB, held by each GPU the library runs on until the
 * process ends) instead of the plan's workspace.  Every call on one GPU
 * shares that array: calls that overlap in time on one GPU (any plan, any
 * stream) race on it and must be serialised.  dF is required.
 *   params: device [n][4]; seg: device [n] or NULL; F: device [n];
 *   dF: device [n][4]
 * FSTAT_EUNSUPPORTED for n > FSTAT_GRAD_STATIC_MAX; FSTAT_EINVAL for NULL
 * params, F, dF or n <= 0. */
#define FSTAT_GRAD_STATIC_MAX 65536
fstat_status fstat_grad_static(fstat_plan_t p, const double *params, const int32_t *seg, int64_t n, double *F,
                               double *dF, void *hip_stream);

/* The continuous parameters of output bins of grid nodes, for fstat_eval,
 * fstat_grad, fstat_refine and fstat_amplitudes: node i and its output index
 * k[i] (a map column plus k_lo, a kmax, or a crossing's k; with interbin = 1
 * the interbinned index 2k + h, h = 1 for the half bin k + 1/2 of Eq. intbin)
 * give the band-relative frequency f = (k + bin_offset) / (nfft dt) of the
 * node's segment (Eq. DFT: Fourier frequency k / (nfft dt), shifted by the
 * node's lattice line, Eq. avec), and its fdot, alpha, delta.
 *   nodes: host [n]; k: host [n], 0 <= k < nfft/2 (interbin: < nfft)
 *   params: host [n][4] (f, fdot, alpha, delta), written; seg: host [n] or
 *   NULL, the nodes' segment indices, written.
 * FSTAT_EINVAL: NULL pointers, n < 0, interbin not 0/1, a node's segment or
 * bin out of range (nothing is written then). */
fstat_status fstat_bin_params(fstat_plan_t p, const fstat_node *nodes, const int64_t *k, int64_t n,
                              int32_t interbin, double *params, int32_t *seg);

/* Waits for the plan's device, then reports and clears the plan's error flag:
 * FSTAT_EDEVICE if a persistent launch (FSTAT_LAUNCH_PERSISTENT) stopped early
 * since the last call (a wait inside the kernel outlived its bound; the
 * outputs of that call are incomplete), FSTAT_OK otherwise.  The flag stays
 * set until this call clears it: persistent launches of the plan made in
 * between stop at once, with incomplete outputs, and are reported by the same
 * FSTAT_EDEVICE. */
fstat_status fstat_plan_status(fstat_plan_t p);

/* Plan facts.  Host outputs; any pointer may be NULL. */
fstat_status fstat_plan_info(fstat_plan_t p, int32_t seg, int64_t *n, int64_t *nfft, double *sigma2,
                             int32_t *fft_R, int32_t *fft_C);

/* The schedule in use for a segment (defaults or autotuned): FFT split
 * nfft = R x C, columns per second-pass workgroup B2, nodes per batch, and
 * the stream mode: 1 = both FFT passes of a batch on the caller's stream, one
 * after the other (the default); 2 = the second pass on a plan-owned side
 * stream, overlapping the first pass of the next batch.  Host outputs; any
 * pointer may be NULL. */
fstat_status fstat_plan_schedule(fstat_plan_t p, int32_t seg, int32_t *R, int32_t *C, int32_t *B2,
                                 int32_t *batch, int32_t *streams);

/* Diagnostic: the demodulated, resampled, a/b-weighted series z_a, z_b of one
 * node (the input of the FFTs, natural order), as FP64 device [n][4] =
 * (Re z_a, Im z_a, Re z_b, Im z_b), computed in the plan's precision, with the
 * node's bin offset applied as the factor e^{-2 pi i bin_offset j / nfft}. */
fstat_status fstat_demod_series(fstat_plan_t p, const fstat_node *node, double *out, void *hip_stream);

/* Kernel timing (a tracing aid, off by default).  While enabled, every kernel
 * launch of fstat_grid is bracketed by two HIP events on the caller's stream.
 * fstat_profile(p, 1) enables and resets the counters, fstat_profile(p, 0)
 * disables.  fstat_profile_read synchronises the device and returns, for one
 * kernel kind, the number of launches, their summed duration in milliseconds
 * and their summed algorithmic HBM bytes (the bytes the launch must move:
 *   FSTAT_K_PASS1: 4 complex values of the working precision per FFT bin
 *                  written (the a- and b-spectra between the passes), plus the
 *                  per-sample sky record read (4 reals per sample);
 *   FSTAT_K_PASS2: the same spectra read back, plus one real per output bin
 *                  written;
 *   FSTAT_K_SKY:   the sky records written, 4 reals per sample.)
 * Any output pointer may be NULL. */
#define FSTAT_K_SKY 0
#define FSTAT_K_PASS1 1
#define FSTAT_K_PASS2 2
#define FSTAT_K_OTHER 3
fstat_status fstat_profile(fstat_plan_t p, int32_t enable);
fstat_status fstat_profile_read(fstat_plan_t p, int32_t kind, int64_t *launches, double *ms, double *bytes);

void fstat_destroy(fstat_plan_t p);
const char *fstat_strerror(fstat_status s);

/* Measurement aid: copy `bytes` from src to dst (both device, 16-byte aligned,
 * not overlapping; bytes a multiple of 16) with a grid-stride kernel of
 * `blocks` workgroups of 256 threads (0: up to 8192) and streaming accesses,
 * enqueued on hip_stream.  Timing it gives the bandwidth the memory system
 * sustains for one read and one write of every byte, the reference for the
 * grid path's own.  FSTAT_EINVAL for bad arguments. */
fstat_status fstat_copy_probe(void *dst, const void *src, int64_t bytes, int32_t blocks, void *hip_stream);

/* Measurement aid: the store pattern of the first FFT pass alone, enqueued on
 * hip_stream.  For each of `nodes` nodes (dst: nodes x R x C elements of 16
 * bytes, 16-byte aligned) and each column r < R, one workgroup of C/16
 * threads writes the C elements of row r, thread t the elements k2 = t +
 * q C/16 (q < 16), at [k2 / b2][r][k2 % b2] within the node (b2 a power of two
 * <= C: the blocked spill layout) or [r][k2] (b2 = 0: row-major), with
 * streaming 16-byte stores of (r, node, 0, 1) as floats.  Timing it gives the
 * rate the pass's write pattern can reach without its transform.  C in
 * {1024, 2048, 4096}, 1 <= nodes <= 65535; FSTAT_EINVAL otherwise. */
fstat_status fstat_spill_write_probe(void *dst, int64_t nodes, int32_t R, int32_t C, int32_t b2, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* FSTAT_H */
