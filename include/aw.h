/*
 * aw.h -- C ABI of libaw, the MI355X (gfx950) ensemble mapper for the
 * Arnold-web model of arXiv:1107.4107 ("Mapping the Arnold web with a
 * GPU-supercomputer", Seibert, Denisov, Ponomarev, Hanggi).
 *
 * Model (eqs. 1-2): H(P, X) = |P|^2 / 2 + eps * Hp(X),
 *                   Hp(x, y, z) = cos x cos y (1 + cos 2z),   M = 3.
 * Propagation (section "Computational method"): a symplectic map with step h.
 * The paper's 6th-order scheme is taken as the triple-jump composition
 * S6(h) = S4(d1 h) S4(d0 h) S4(d1 h), S4(t) = S2(g1 t) S2(g0 t) S2(g1 t),
 * S2(t) = D(t/2) K(t) D(t/2) with d1 = 1/(2 - 2^(1/5)), g1 = 1/(2 - 2^(1/3));
 * its first-order member K(h) then D(h) is the coupled standard map that the
 * model section names.  Drift D(t): X += t P.  Kick K(t): P -= t eps grad Hp(X).
 *
 * Conventions for every entry point:
 *  - Pointers named *_dev are device memory of the current HIP device, owned
 *    by the caller; the library never frees or reallocates them.  Pointers to
 *    descriptors (aw_ensemble, aw_image_spec, aw_tuning) are host memory and
 *    are read before the call returns.
 *  - Arrays are structure-of-arrays, float64 unless stated: a "[R][N]" array
 *    holds row r of orbit n at offset r*N + n.  Orbit n of a GRID2 slice is
 *    n = j*nx + i (i along axis[0]).
 *  - All work is enqueued on `stream` (a hipStream_t, NULL = default stream);
 *    no entry point synchronises the host except where stated.
 *  - Arguments are validated before anything is enqueued.  On a non-AW_OK
 *    return nothing was enqueued (AW_EDEVICE: a launch failed) and
 *    aw_last_error() gives a message.  No C++ exception crosses the ABI.
 *  - Asynchronous device faults surface at the caller's next synchronisation.
 *  - Internal scratch (histogram items and sort buffers, batch tables) is
 *    one area per (device, stream), allocated by the library on first use and
 *    kept until aw_release() or process exit, so calls on different streams
 *    may overlap.  An area too small for a call is replaced by one at least
 *    twice its size; the old one is retired (earlier work on the stream may
 *    still use it) and freed by aw_release().  The call path never frees
 *    device memory (hipFree waits for the device) and never waits for the
 *    device: to keep it from allocating at all, size the stream's area up
 *    front with aw_image_workspace() and aw_reserve().  Batch tables travel
 *    through pinned host buffers that are reused once their copies are done.
 *    A stream handle's area is tied to the handle's value: destroy a stream
 *    only after its work has finished before reusing the handle.
 */
#ifndef AW_H
#define AW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AW_OK = 0,
  AW_EINVAL = 1,        /* an argument is out of range or inconsistent */
  AW_EUNSUPPORTED = 2,  /* a well-formed request the library does not do (e.g. M != 3) */
  AW_EDEVICE = 3,       /* a HIP call or kernel launch failed */
  AW_ENOMEM = 4,        /* internal scratch could not be allocated */
  AW_EWORKSPACE = 5     /* caller workspace too small */
} aw_status;

/* Text of the last non-AW_OK status returned on this host thread. */
const char *aw_last_error(void);
/* Library version string. */
const char *aw_version(void);
/* Frees the library's internal scratch, retired areas and staging buffers on
 * the current device (synchronises it). */
aw_status aw_release(void);

/* Map forms (section "Computational method"): the first-order coupled
 * standard map (kick then drift), and symmetric compositions of the
 * drift-kick-drift step S2: order 2 (S2), 4 and 6 by triple jumps (S4, S6:
 * 9 kicks per step), and the 7-stage symmetric composition of order 6 (Y6:
 * 7 kicks per step, weights solved from the order conditions). */
typedef enum { AW_MAP_STDMAP = 1, AW_MAP_S2 = 2, AW_MAP_S4 = 4, AW_MAP_S6 = 6, AW_MAP_Y6 = 7 } aw_map_form;

/* Initial conditions of an ensemble (sections "Main results", Figs. 2-4).
 *  GRID2:    a 2-D slice: s = base; s[axis[0]] = lo[0] + i * ((hi[0]-lo[0])/nx),
 *            s[axis[1]] = lo[1] + j * ((hi[1]-lo[1])/ny)  (left edges).
 *  BOX:      s_k = box_lo[k] + (box_hi[k]-box_lo[k]) * U(seed_ic, 16 n + k).
 *  EXPLICIT: the caller's ic_dev[6][N].
 *  SPHERE:   fixed energy (Figs. 2-3): X_k = box_lo[k] + (box_hi[k]-box_lo[k])
 *            U(seed_ic, 16 n + k) for k < 3 (the torus); the direction of P
 *            uniform in area on the sphere segment phi in [window[0], window[1]),
 *            mu = cos(theta) in [window[2], window[3]):
 *            mu = window[2] + (window[3]-window[2]) U(seed_ic, 16 n + 3),
 *            phi = window[0] + (window[1]-window[0]) U(seed_ic, 16 n + 4),
 *            P = |P| (sqrt(1-mu^2) cos phi, sqrt(1-mu^2) sin phi, mu) with
 *            |P| = sqrt(2 (energy - eps Hp(X))), so H = energy (eq. 1).
 *            Needs energy > 2|eps| and -pi <= window[0] < window[1] <= pi,
 *            -1 <= window[2] < window[3] <= 1.
 * U(seed, c) = (SplitMix64 output number c of the stream seeded with `seed`,
 * i.e. mix(seed + (c+1)*0x9E3779B97F4A7C15)) >> 11, times 2^-53.
 * The tangent start of orbit n is w0 = u/|u|, u_k = 2 U(seed_tangent, 16 n + k) - 1,
 * for every ic_kind.  Coordinate order is (x, y, z, px, py, pz).
 *  CLOUD:    the injected cloud of Fig. 4: velocity components
 *            vx = cloud[0] + cloud[2] g1, vy = cloud[1] + cloud[3] g2 with a
 *            Box-Muller pair g1 = r cos(2 pi u2), g2 = r sin(2 pi u2),
 *            r = sqrt(-2 ln(1 - u1)), u1 = U(seed_ic, 128 n + 120),
 *            u2 = U(seed_ic, 128 n + 121); X uniform on the box (first three
 *            coordinates) drawn at attempt a = 0, 1, ... < 40 from
 *            U(seed_ic, 128 n + 3 a + k), taking the first X with
 *            R = 2 (energy - eps Hp(X)) - vx^2 - vy^2 >= 0 (after 40 failed
 *            attempts the last X with R clamped to 0); vz = s sqrt(R) with
 *            s = -1 if U(seed_ic, 128 n + 122) < 1/2 else +1.  H = energy.
 *            Needs energy > 2|eps| and finite cloud values. */
typedef enum { AW_IC_GRID2 = 0, AW_IC_BOX = 1, AW_IC_EXPLICIT = 2, AW_IC_SPHERE = 3, AW_IC_CLOUD = 4 } aw_ic_kind;

/* flags */
#define AW_F_TANGENT 1u  /* propagate the tangent vector (L, lambda, chi, class) */
#define AW_F_WINDOW 2u   /* "remained within the area" (section "Main results", Fig. 3):
                          * test after every step (and at the start) that the direction
                          * of P, phi = atan2(py, px), mu = pz/|P|, lies in the closed
                          * window [window[0], window[1]] x [window[2], window[3]];
                          * orbits that ever leave get bit 1 of their class byte set and
                          * are left out of the HIST images.  Same window limits as SPHERE. */

/* Rows of the per-orbit output orbit_out[AW_NOUT][N]:
 *  L      = ln(|w_T| / |w_0|), the tangent-vector growth (FTLE numerator);
 *  LAMBDA = L / (T h);         CHI = L / ln(1 + T h);
 *  V      = (X_T - X_0) / (T h) on unwrapped X, the finite-time mean velocity
 *           of section "Main results" with Delta t = T h;
 *  DP2    = |P_T - P_0|^2, the momentum drift of the model section;
 *  J      = (1/T) sum_{k=1..T} |P_k - P_0|^2;
 *  DE     = H(s_T) - H(s_0).
 * Without AW_F_TANGENT the rows L, LAMBDA, CHI hold NaN and class bit 0 is 0.
 * Class byte: bit 0 = chi > chi_threshold, bit 1 = left the window (AW_F_WINDOW). */
enum {
  AW_OUT_L = 0, AW_OUT_LAMBDA, AW_OUT_CHI, AW_OUT_VX, AW_OUT_VY, AW_OUT_VZ,
  AW_OUT_DP2, AW_OUT_J, AW_OUT_DE, AW_NOUT
};

typedef struct {
  int32_t M;              /* degrees of freedom; only 3 is defined (eq. 2) */
  int32_t map_form;       /* aw_map_form */
  double eps;             /* eps of eq. 1 (finite) */
  double h;               /* step (finite, non-zero; the paper: 0.01 * 2 pi) */
  int64_t n_steps;        /* T >= 1 */
  int32_t ic_kind;        /* aw_ic_kind */
  int32_t axis[2];        /* GRID2: the two varied coordinates, 0..5, distinct */
  double lo[2], hi[2];    /* GRID2: ranges */
  int64_t nx, ny;         /* GRID2: grid size (>= 1) */
  double base[6];         /* GRID2: the fixed coordinates */
  double box_lo[6], box_hi[6]; /* BOX */
  int64_t n_orbits;       /* BOX and EXPLICIT: N (>= 0); GRID2: ignored (N = nx*ny) */
  uint64_t seed_ic;       /* BOX */
  uint64_t seed_tangent;  /* tangent start */
  double chi_threshold;   /* class = chi > chi_threshold */
  uint32_t flags;         /* AW_F_* */
  double energy;          /* SPHERE, CLOUD: total energy E of eq. 1 */
  double window[4];       /* SPHERE segment / AW_F_WINDOW area: phi_lo, phi_hi, mu_lo, mu_hi */
  double cloud[4];        /* CLOUD: centre (vx, vy) and standard deviations (sigma_x, sigma_y) */
} aw_ensemble;

/* Launch shape.  NULL or zero fields = defaults (automatic block, one orbit
 * per lane, step loop not unrolled, renormalisation every 8 steps).  block in
 * {0, 64, 128, 256, 512}: the kernels hold a 64 KB sine/cosine table per
 * block, so blocks of 512 lanes are needed for a full CU; 0 picks 512 when
 * the ensemble gives every CU at least one such block, else the largest of
 * 256, 128 and 64 that still does.  The window-test and time-window
 * propagation and the batched persistent launch run a block above 256 (or
 * automatic) as 256.  orbits_per_lane in {1, 2}; unroll in {1, 2};
 * renorm_every in {1, 2, 4, 8, 16}.  persistent_wgs: workgroups of the batched
 * persistent launch (0 = auto).  lanes_per_orbit in {0, 1, 2}: tangent-free
 * launches that end before n_steps (aw_map_ensemble_steps) or bin time windows
 * (aw_window_density), without AW_F_WINDOW, can run one orbit on two lanes (u
 * and p_u on one, v and p_v on the other, in the rotated frame); 0 does so
 * when one lane per orbit would leave SIMDs without a wave (fewer than
 * 64 x 4 x CUs orbits).  Results are bitwise the same either way. */
typedef struct {
  int32_t block;
  int32_t orbits_per_lane;
  int32_t unroll;
  int32_t renorm_every;
  int32_t persistent_wgs;
  int32_t lanes_per_orbit;
} aw_tuning;

/* Number of orbits of an ensemble (nx*ny for GRID2), or -1 if invalid. */
int64_t aw_ensemble_size(const aw_ensemble *ens);

/* Writes the initial state ic_dev[6][N] and the tangent start w0_dev[6][N]
 * (either may be NULL) of an ensemble: the exact values the propagation
 * starts from.  EXPLICIT ensembles copy ic_dev from ic_in_dev. */
aw_status aw_generate_ic(const aw_ensemble *ens, const double *ic_in_dev,
                         double *ic_dev, double *w0_dev, void *stream);

/* Propagate ensembles for their n_steps and write per-orbit outputs.
 * n_ens >= 1 descriptors; with n_ens > 1 every ensemble must share map_form
 * and flags, and all of them run in ONE persistent launch whose workgroups
 * take (ensemble, tile) items, longest first, from a device queue.
 *   ic_dev[e]        EXPLICIT: [6][N_e], else ignored (the array may be NULL)
 *   orbit_out_dev[e] [AW_NOUT][N_e] or NULL
 *   state_out_dev[e] [12][N_e] (X, P, unit tangent) or NULL
 *   cls_dev[e]       uint8 [N_e] (1 = chi > chi_threshold) or NULL
 * Per-orbit results are bitwise independent of the tuning and of batching. */
aw_status aw_map_ensemble(const aw_ensemble *ens, int32_t n_ens,
                          const double *const *ic_dev, double *const *orbit_out_dev,
                          double *const *state_out_dev, uint8_t *const *cls_dev,
                          const aw_tuning *tuning, void *stream);

/* Rows of the resumable carry[AW_NCARRY][N], the propagation's own state in
 * its rotated frame (u = x + y, v = x - y, z; momenta and tangent alike): X,
 * P, tangent (scaled), X0 (original frame), P0, twice the J sum, tangent scale
 * exponent, steps done, left-the-window flag.  Only the library reads it. */
#define AW_NCARRY 22

/* Resumable form of aw_map_ensemble for one ensemble: runs global steps
 * [k_begin, k_end) with 0 <= k_begin < k_end <= n_steps.  k_begin == 0 starts
 * from the initial conditions; otherwise the state is read from carry_dev.
 * If k_end < n_steps the state is written to carry_dev; if k_end == n_steps
 * the outputs are written as by aw_map_ensemble.  A chain of calls covering
 * [0, n_steps) gives results bitwise equal to one aw_map_ensemble call. */
aw_status aw_map_ensemble_steps(const aw_ensemble *ens, const double *ic_dev,
                                double *carry_dev, int64_t k_begin, int64_t k_end,
                                double *orbit_out_dev, double *state_out_dev,
                                uint8_t *cls_dev, const aw_tuning *tuning, void *stream);

/* Images (section "Main results"; Figs. 2-4).
 *  IC_GRID:   GRID2 ensembles only; image[j][i] = orbit_out row `field` of
 *             orbit j*nx + i (W = nx, H = ny; W = H = 0 takes every
 *             ensemble's own nx, ny, so one batch may mix grid sizes).  counts, if non-NULL, is one
 *             uint32: the number of orbits with class 1 (needs AW_F_TANGENT).
 *  HIST_P0:   key = initial coordinates (key_axis[0], key_axis[1]); bin
 *             floor((a - lo)/(hi - lo) * W) per axis, half-open ranges, items
 *             outside dropped; image = per-bin mean of row `field` (0 where
 *             empty), counts = per-bin count.
 *  HIST_VDIR: the density F of the direction of V on the momentum sphere:
 *             phi = atan2(Vy, Vx) over [lo[0], hi[0]] (W bins), mu = Vz/|V|
 *             over [lo[1], hi[1]] (H bins), closed at the top; all four zero
 *             means the whole sphere [-pi, pi] x [-1, 1] (a zoom otherwise);
 *             image = count / (N dphi dmu) with N the ensemble size,
 *             counts = per-bin count.  A zero V is dropped, and so are
 *             orbits that left the window under AW_F_WINDOW.
 * Histograms are built by a counting sort of items by image tile followed by
 * per-tile LDS accumulation; counts are exact and deterministic, float sums
 * may differ in the last bits between runs. */
typedef enum { AW_IMG_IC_GRID = 0, AW_IMG_HIST_P0 = 1, AW_IMG_HIST_VDIR = 2 } aw_image_kind;

typedef struct {
  int32_t kind;        /* aw_image_kind */
  int32_t field;       /* AW_OUT_* row imaged (IC_GRID) or averaged (HIST_P0) */
  int32_t W, H;        /* image size; IC_GRID requires W = nx, H = ny */
  int32_t key_axis[2]; /* HIST_P0: key coordinates, 0..5 */
  double lo[2], hi[2]; /* HIST_P0: key ranges (lo < hi) */
} aw_image_spec;

/* Propagate and reduce to an image, per ensemble:
 *   image_dev[e]  [H][W] float64;  counts_dev[e] [H][W] uint32 (or NULL; see above)
 *   cls_dev[e]    uint8 [N_e] or NULL.
 * n_ens > 1 runs the propagation as one persistent launch (as aw_map_ensemble). */
aw_status aw_indicator_image(const aw_ensemble *ens, int32_t n_ens, const aw_image_spec *spec,
                             double *const *image_dev, uint32_t *const *counts_dev,
                             uint8_t *const *cls_dev, const aw_tuning *tuning, void *stream);

/* Bytes of library scratch that one aw_indicator_image call over these
 * ensembles and spec takes on its stream (spec = NULL: one aw_map_ensemble
 * call over them; 0 for a single ensemble).  Validates like the call. */
aw_status aw_image_workspace(const aw_ensemble *ens, int32_t n_ens, const aw_image_spec *spec, size_t *bytes);
/* Grows the library scratch of `stream` on the current device to at least
 * `bytes` now (an allocation; it does not wait for the device), so that later
 * calls on the stream that need no more allocate nothing. */
aw_status aw_reserve(size_t bytes, void *stream);

/* Time-window density of Fig. 4 (section "Main results"): F averaged over the
 * windows between two plots.  Runs n_windows consecutive windows of
 * window_steps map steps each, starting at global step k_begin (0 = from the
 * initial conditions, else from carry_dev), for one ensemble.  For every
 * window w the mean velocity V_w = (X(end) - X(start)) / (window_steps h) of
 * each orbit is binned as in HIST_VDIR (spec->kind must be AW_IMG_HIST_VDIR;
 * spec->lo/hi zoom as there) and ADDED to counts_accum_dev [H][W] (uint32;
 * the caller zeroes it once); orbits that left the window under AW_F_WINDOW
 * are not added.  The state after the last window is left in carry_dev
 * [AW_NCARRY][N] (required), so consecutive calls continue the run; the
 * averaged density is counts / (n_windows_total N dphi dmu).  Needs
 * k_begin + n_windows window_steps <= n_steps.  The per-window results are
 * bitwise independent of how the windows are split over calls. */
aw_status aw_window_density(const aw_ensemble *ens, const double *ic_dev, double *carry_dev,
                            int64_t k_begin, int64_t n_windows, int64_t window_steps,
                            const aw_image_spec *spec, uint32_t *counts_accum_dev,
                            const aw_tuning *tuning, void *stream);

/* The histogram reduction on its own, over caller keys a_dev[N], b_dev[N] and
 * values v_dev[N] (v_dev may be NULL: the sums are then zero): bin along
 * each axis floor((key - lo)/(hi - lo) * W); closed_upper = 0: half-open
 * ranges, out-of-range and non-finite keys dropped; closed_upper = 1: a key
 * equal to hi goes to the last bin.  counts_dev [H][W] uint32, sums_dev
 * [H][W] float64 (NULL allowed), dropped_dev one uint64 (NULL allowed). */
aw_status aw_histogram2d(int64_t N, const double *a_dev, const double *b_dev, const double *v_dev,
                         double lo0, double hi0, double lo1, double hi1, int32_t W, int32_t H,
                         int32_t closed_upper, uint32_t *counts_dev, double *sums_dev,
                         uint64_t *dropped_dev, void *stream);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the same
 * histogram as aw_histogram2d (same arguments, results and errors), with its
 * scratch in a fixed device array of AW_NOALLOC_SCRATCH_BYTES instead of the
 * stream's library scratch.  It calls no hipMalloc, hipFree or allocating
 * routine; the array is a file-scope device variable that every GPU the
 * library runs on holds (its own copy) until the process ends.  The first
 * call on a device looks up that device's address of the array (the HIP
 * runtime may place the array in device memory then); later calls change
 * nothing in the device's memory use.  Scratch a
 * call needs, each part rounded up to 256 bytes: 4 N (bins) + 2 N (sorted
 * local bins), with values (v_dev != NULL) + 8 N (sorted values); tile tables
 * of 4 T G + 4 G + 4 (2 T + 1) + 8 (T + 1) + 4 (T + B) bytes; and partial
 * tiles of 8192 B bytes, with values + 16384 B; where T = ceil(W/32)
 * ceil(H/32), G = ceil(N/8192) and B = min(ceil(N/16384), max(ceil(T/2),
 * 256)) (N = 0 counts as 1).  For a 512 x 512 image that allows about
 * 4.3e6 items with values or 1.06e7 without.  A larger request returns
 * AW_EWORKSPACE and enqueues nothing.
 * Every call on a GPU shares that GPU's array, and the array keeps the last
 * call's contents (each call writes every part it reads before reading it):
 * calls on one stream are ordered and safe, but calls that overlap on one
 * GPU -- on different streams, or from host threads that do not order their
 * streams -- race on the array and give wrong results. */
#define AW_NOALLOC_SCRATCH_BYTES (64u << 20)
aw_status aw_histogram2d_noalloc(int64_t N, const double *a_dev, const double *b_dev, const double *v_dev,
                                 double lo0, double hi0, double lo1, double hi1, int32_t W, int32_t H,
                                 int32_t closed_upper, uint32_t *counts_dev, double *sums_dev,
                                 uint64_t *dropped_dev, void *stream);

/* Equal-area keys of the direction of V[3][N]: phi = atan2(Vy, Vx),
 * mu = Vz / |V|; NaN for a zero V. */
aw_status aw_vdir_keys(int64_t N, const double *V_dev, double *phi_dev, double *mu_dev, void *stream);

/* Gradient of J = (1/T) sum_{k=1..T} |P_k - P_0|^2 (the step-averaged momentum
 * drift of the model section) by a hand-written adjoint: one forward pass that
 * stores a state checkpoint every ckpt_every steps, then, segment by segment
 * from the end, a recompute of the segment's step states and a reverse sweep
 * that inverts each stage.  ens->ic_kind must be EXPLICIT (ic_dev[6][N]).
 *   grad_J_dev [N]: upstream dL/dJ_n (NULL = all ones)
 *   J_out_dev [N] or NULL; grad_ic_dev [6][N]: dL/d(initial x..pz);
 *   grad_eps_dev [N]: per-orbit dL/deps contributions (sum them for the scalar).
 * The recompute keeps the state at the end of every 4th step (global count)
 * and of the segment's last step; the sweep rebuilds the steps in between by
 * inverting their stages from the next kept state.
 * Requires a caller workspace of aw_indicator_grad_workspace() bytes: the
 * n_seg = ceil(T / ckpt_every) checkpoints, the final state and the kept step
 * states of one segment (at most floor((ck + 2)/4) + 1 with ck =
 * min(ckpt_every, T)), 6 doubles per orbit each.  With ckpt_every >= T (one
 * segment) the forward pass keeps the step states itself and the backward
 * pass sweeps them without a recompute: about T*N*12 bytes of workspace.
 * The result is bitwise the same for every ckpt_every that is a multiple of 4
 * and for ckpt_every >= T (the same states are kept); other intervals keep
 * more states and agree to rounding. */
aw_status aw_indicator_grad_workspace(const aw_ensemble *ens, int64_t ckpt_every, size_t *bytes);
aw_status aw_indicator_grad(const aw_ensemble *ens, const double *ic_dev, const double *grad_J_dev,
                            int64_t ckpt_every, double *J_out_dev, double *grad_ic_dev,
                            double *grad_eps_dev, void *workspace_dev, size_t ws_bytes,
                            const aw_tuning *tuning, void *stream);

/* The same gradient by a reversible sweep: the forward pass is the same, but
 * the backward pass neither recomputes the segments nor stores step states.
 * It sweeps each segment back from the exact state at its end (the next
 * checkpoint, or the final state), undoing the steps one after the other by
 * inverting their stages.  This relies on the map being a composition of
 * invertible stages; the reconstructed states carry the rounding of the
 * inversion, which restarts from an exact state at every checkpoint.  The
 * result agrees with aw_indicator_grad to rounding, not bitwise.  Same
 * arguments; the workspace holds only the checkpoints and the final state:
 * aw_indicator_grad_reversible_workspace() bytes (aw_indicator_grad_workspace()
 * bytes are enough too). */
aw_status aw_indicator_grad_reversible_workspace(const aw_ensemble *ens, int64_t ckpt_every, size_t *bytes);
aw_status aw_indicator_grad_reversible(const aw_ensemble *ens, const double *ic_dev, const double *grad_J_dev,
                                       int64_t ckpt_every, double *J_out_dev, double *grad_ic_dev,
                                       double *grad_eps_dev, void *workspace_dev, size_t ws_bytes,
                                       const aw_tuning *tuning, void *stream);

/* Gradient of the tangent-growth indicator L = ln(|w_T| / |w_0|) -- the
 * finite-time Lyapunov exponent that the conclusions name as the indicator to
 * compare with, before its division by T h -- with respect to the initial
 * state and eps, at a fixed tangent start.  A second-order adjoint: a forward
 * pass with the tangent stores (state, tangent) every ckpt_every steps; then,
 * segment by segment from the end, the segment is recomputed and swept
 * backwards, each stage inverted, with the adjoint of state and tangent
 * propagated through the kick's second and third derivatives of eq. 2's Hp.
 * ens->ic_kind must be EXPLICIT.
 *   ic_dev [6][N], w0_dev [6][N] (the tangent start; need not be unit);
 *   grad_L_dev [N]: upstream dF/dL_n (NULL = all ones);
 *   L_out_dev [N] or NULL: L per orbit;
 *   grad_ic_dev [6][N]: dF/d(initial x..pz);
 *   grad_eps_dev [N]: per-orbit dF/deps contributions (sum for the scalar).
 * lambda = L/(T h) and chi = L/ln(1 + T h) scale the same gradients.  On
 * chaotic orbits the derivative grows like exp(lambda T h) and is only
 * meaningful where the trajectory is.  As for aw_indicator_grad, the
 * recompute keeps (state, tangent) at the end of every 4th step and of the
 * segment's last step, and the sweep inverts the steps in between.
 * Requires a caller workspace of aw_ftle_grad_workspace() bytes: 12 doubles
 * per orbit per checkpoint, for the final state and per kept step of a
 * segment, then one 16-bit rescale exponent per orbit per 8 steps.  As for
 * aw_indicator_grad, ckpt_every >= T keeps the step states in the forward pass
 * and skips the recompute (about T*N*24 bytes); the result is bitwise the same
 * for ckpt_every a multiple of 4 and for ckpt_every >= T. */
aw_status aw_ftle_grad_workspace(const aw_ensemble *ens, int64_t ckpt_every, size_t *bytes);
aw_status aw_ftle_grad(const aw_ensemble *ens, const double *ic_dev, const double *w0_dev,
                       const double *grad_L_dev, int64_t ckpt_every, double *L_out_dev,
                       double *grad_ic_dev, double *grad_eps_dev, void *workspace_dev, size_t ws_bytes,
                       const aw_tuning *tuning, void *stream);

/* The same gradient by a reversible sweep: no segment recompute and no stored
 * step states.  Each segment is swept back from the exact state at its end,
 * inverting the stages of state and tangent step after step, and undoing
 * every tangent rescale with the exponent the forward pass recorded.  The
 * result agrees with aw_ftle_grad to rounding, not bitwise: the reconstructed
 * states carry the inversion's rounding, and on chaotic orbits the tangent's
 * reconstruction error grows like exp(2 lambda h ckpt_every) within a
 * segment.  Same arguments; the workspace holds the checkpoints, the final
 * state and the rescale exponents: aw_ftle_grad_reversible_workspace() bytes
 * (aw_ftle_grad_workspace() bytes are enough too). */
aw_status aw_ftle_grad_reversible_workspace(const aw_ensemble *ens, int64_t ckpt_every, size_t *bytes);
aw_status aw_ftle_grad_reversible(const aw_ensemble *ens, const double *ic_dev, const double *w0_dev,
                                  const double *grad_L_dev, int64_t ckpt_every, double *L_out_dev,
                                  double *grad_ic_dev, double *grad_eps_dev, void *workspace_dev, size_t ws_bytes,
                                  const aw_tuning *tuning, void *stream);

/* A captured HIP graph of aw_indicator_image over n_ens ensembles: the
 * class-counter clears, one persistent launch (one plain launch for a single
 * ensemble) and, for HIST_P0 and HIST_VDIR images, every ensemble's histogram
 * reduction.  The graph owns its scratch area and batch tables (allocated
 * here, freed by aw_graph_destroy); caller buffers are bound at creation and
 * the descriptors copied.  Every launch status of the capture is checked: on
 * a failure the capture is ended, nothing is returned in *out and the status
 * is AW_EDEVICE.  Launching replays the whole batch; replays on different
 * streams must not overlap (they share the graph's scratch). */
typedef struct aw_graph aw_graph;
aw_status aw_graph_create(const aw_ensemble *ens, int32_t n_ens, const aw_image_spec *spec,
                          double *const *image_dev, uint32_t *const *counts_dev,
                          uint8_t *const *cls_dev, const aw_tuning *tuning, aw_graph **out);
aw_status aw_graph_launch(aw_graph *g, void *stream);
void aw_graph_destroy(aw_graph *g);

/* Kernel timing for measurement: when enabled, HIP events are recorded on the
 * launch stream around every propagation kernel.  aw_timing_read() waits for
 * the recorded events, returns the summed kernel milliseconds and the number
 * of launches since the last read, and clears the record. */
aw_status aw_timing_enable(int32_t on);
aw_status aw_timing_read(double *ms, int64_t *launches);

/* FP64 operations per map step of the propagation kernel as built, for the
 * roofline: counts of fma, mul and add/sub instructions (per orbit-step,
 * excluding the per-orbit prologue/epilogue); flops = 2 fma + mul + add. */
aw_status aw_step_op_counts(int32_t map_form, int32_t tangent, int64_t *fma, int64_t *mul,
                            int64_t *add);

#ifdef __cplusplus
}
#endif
#endif /* AW_H */
