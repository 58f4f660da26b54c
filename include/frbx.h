/*
 * frbx -- cross-spectrum fast-radio-burst search on AMD MI355X (gfx950).
 *
 * C ABI of libfrbx.so.  The method is that of Liu et al. 2018, "A Fast Radio
 * Burst Search Method for VLBI Observation" (arXiv:1801.02391): per-baseline
 * incoherent dedispersion of millisecond complex cross spectra over a grid of
 * DM trials (Sec. 2.2, Eqs. 1-3), a fringe search of every half-overlapped
 * time segment over single-band delay, multiband delay and delay rate
 * (Sec. 2.3, Eqs. 4-5; Sec. 5.1), normalisation and threshold of each
 * baseline's power series (Eq. 6, Sec. 2.4.1), the multi-window filter,
 * best-DM selection (Sec. 5.3) and cross-baseline matching (Sec. 2.4.1).
 *
 * Conventions used by every entry point
 *   Units: MHz, ms, microseconds (MHz * us = cycles), pc cm^-3; rates in s/s.
 *   Arrays are row-major; "[A][B]" means A is the slowest index.
 *   Every call returns frbx_status and never throws.  On failure the context
 *   (when there is one) keeps a message readable with frbx_last_error().
 *   Output buffers are owned by the caller.  A call taking (cap, *n) writes at
 *   most cap records, sets *n to the number available and returns
 *   FRBX_E_RANGE when cap < *n (cap = 0 is a size query).
 *   One context belongs to one host thread and one HIP stream.
 *   Device memory is allocated only by the entry points that size a
 *   workspace (frbx_load*, frbx_run, frbx_stream_begin/push, frbx_power_sum,
 *   frbx_refine_begin, frbx_dump_segment, frbx_calibrate) and by those that
 *   build the grid tables on the device after a grid changed
 *   (frbx_get_segments, frbx_get_lattice, frbx_get_ap_offsets,
 *   frbx_refine_cells); it is reused across calls and freed by
 *   frbx_destroy.  The table builders also load, once per process, device
 *   and lattice, the run-time compiled float32 kernel (see
 *   frbx_set_specialisation), whose code stays loaded until the process
 *   ends.  frbx_run_cube_noalloc allocates nothing (it runs in a
 *   fixed per-GPU workspace).  No entry point frees memory the caller owns.
 */
#ifndef FRBX_H
#define FRBX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct frbx_ctx frbx_ctx;

typedef enum {
  FRBX_OK = 0,
  FRBX_E_INVAL = 1,  /* an argument or a grid is invalid                    */
  FRBX_E_STATE = 2,  /* call out of order (e.g. results before frbx_run)     */
  FRBX_E_RANGE = 3,  /* output capacity too small; *n holds the size needed  */
  FRBX_E_NOMEM = 4,  /* an allocation failed                                 */
  FRBX_E_DEVICE = 5  /* a HIP runtime call or a kernel launch failed         */
} frbx_status;

/* Data layout of the cross spectra S(n, j, k) of Sec. 2.2: IF n in [0, N)
 * with sky frequency if_freq_mhz[n] (lower edge, upper sideband), frequency
 * point j in [0, J) at baseband frequency j * chan_bw_mhz, accumulation
 * period (AP) k in [0, K) of t_ap_ms.  The pointer is read during
 * frbx_create only.  One work-group searches one segment, one lane per
 * (IF, channel group): N may be at most 128, 64, 64, 32, 32, 16 for J = 8,
 * 16, 32, 64, 128, 256, and the segment's LDS plan (which grows with N, J,
 * sbd_pad and n_mbd) must fit 150 KiB; a larger shape is refused with
 * FRBX_E_INVAL when the grids are first used (frbx_run, frbx_get_segments,
 * ...). */
typedef struct {
  int32_t n_baselines;        /* B >= 1                          */
  int32_t n_if;               /* N >= 1                          */
  int32_t n_chan;             /* J: 8, 16, 32, 64, 128 or 256    */
  int64_t n_frames;           /* K >= 1                          */
  double t_ap_ms;             /* AP duration, > 0                */
  double chan_bw_mhz;         /* frequency-point spacing, > 0    */
  const double *if_freq_mhz;  /* [N] IF sky frequencies          */
} frbx_layout;

/* One record per threshold crossing (Sec. 2.4.1 step a) or per single-pulse
 * detection (steps b-d and Sec. 5.3).  k0 is the first AP of the segment on
 * the dedispersion reference frequency (the top of the band); the segment
 * covers APs [k0, k0 + window_len - 1]. */
typedef struct {
  int32_t baseline;
  int32_t dm_index;
  int32_t window_index;
  int32_t window_len;
  int64_t segment;      /* q: k0 = q * hop                                  */
  int64_t k0;
  double dm;            /* pc cm^-3                                         */
  double power;         /* |G| at the peak (Eq. 5 amplitude)               */
  double power_norm;    /* Eq. 6                                            */
  int32_t rate_idx;     /* r: rate = (r - R/2) * rate_step                  */
  int32_t sbd_idx;      /* s: sbd  = (s - PJ/2) / (PJ * chan_bw)            */
  int32_t mbd_idx;      /* m: mbd  = (m - M/2) * mbd_step                   */
  int32_t n_windows;    /* detections: distinct windows in its group, else 0 */
  double rate;          /* s/s                                              */
  double sbd_us;
  double mbd_us;
  int32_t group_id;     /* detections: cross-baseline group, else -1        */
  int32_t reserved;
} frbx_candidate;

/* Cross-baseline matching group (Sec. 2.4.1, cross matching). */
typedef struct {
  int32_t group_id;
  int32_t n_baselines;  /* distinct baselines among its detections          */
  int64_t k_start;      /* earliest AP covered by a member                  */
  int64_t k_end;        /* latest AP covered by a member                    */
  int32_t best;         /* index (into the detection list) of the member
                           with the highest normalised power               */
  int32_t reported;     /* n_baselines >= n_bl_min                          */
} frbx_group;

/* Library version string (static storage). */
const char *frbx_version(void);

/* Create a search context on HIP device `device`, bound to `hip_stream`
 * (a hipStream_t; NULL = the device's null stream).  Validates the layout;
 * FRBX_E_INVAL for an unsupported shape, FRBX_E_DEVICE if the device cannot
 * be selected.  Default grids: one DM trial at 0, sbd_pad 4, M = 256 on the
 * default lattice, R = 1, windows {2, 4}, threshold 3, N_win,min 3,
 * N_bl,min 2. */
frbx_status frbx_create(const frbx_layout *layout, int device, void *hip_stream,
                        frbx_ctx **out);

/* Release every resource of the context (NULL is ignored). */
void frbx_destroy(frbx_ctx *ctx);

/* Text of the last error on this context (empty if none). */
const char *frbx_last_error(const frbx_ctx *ctx);

/* Channel-delay and initial-phase calibration of Eq. 5 (Sec. 2.3): every
 * point is rotated by exp(-i [2 pi (f_j - f_bw/2) tau0 + phi0]) with
 * f_bw = J * chan_bw before the fit.  tau0_us, phi0_rad: [B][N] host
 * arrays (NULL = zeros). */
frbx_status frbx_set_calibration(frbx_ctx *ctx, const double *tau0_us, const double *phi0_rad);

/* DM trials DM_d = dm_lo + d * dm_step, d in [0, n_dm) (coarse DM bins of
 * Sec. 5.3).  k_dm: dispersion constant of Eq. 1 in ms MHz^2 (<= 0 selects
 * 4.149e6).  The AP offsets follow Eqs. 1-2 with the reference at the highest
 * channel frequency. */
frbx_status frbx_set_dm_grid(frbx_ctx *ctx, double dm_lo, double dm_step, int32_t n_dm,
                             double k_dm);

/* Delay grids of the fringe search (Eq. 5, Sec. 5.1).  SBD: PJ = sbd_pad * J
 * points, sbd_pad in {1, 2, 4, 8}.  MBD: n_mbd in {16, 32, 64, 128, 256}
 * points of step mbd_step_us; mbd_step_us <= 0 selects T/M with T = 1/g the
 * MBD ambiguity, g the gcd of the IF offsets from IF 0 in whole kHz.  Any
 * step must place every IF on the transform lattice (f0^n - f0^0) * step * M
 * integral, distinct modulo M; FRBX_E_INVAL otherwise.  f_ref_fit_mhz is the
 * fit reference frequency (NaN = f0^0); it only rotates the phase of G. */
frbx_status frbx_set_delay_grid(frbx_ctx *ctx, int32_t sbd_pad, int32_t n_mbd,
                                double mbd_step_us, double f_ref_fit_mhz);

/* Delay-rate bins of Eq. 4: rate_r = (r - floor(R/2)) * rate_step, R in
 * [1, 64].  rate_step <= 0 selects 1 / (2 f_max l_max t_ap) (half the
 * fringe-rate resolution of the longest window at the top frequency).  The
 * rate phase is taken about the window centre of the dedispersed APs. */
frbx_status frbx_set_rate_grid(frbx_ctx *ctx, int32_t n_rate, double rate_step);

/* Window lengths in APs (Sec. 2.4.1), 1 <= n <= 8, distinct, each >= 1.
 * Segments of window l start every hop = max(1, l/2) APs. */
frbx_status frbx_set_windows(frbx_ctx *ctx, const int32_t *len_frames, int32_t n);

/* Detection parameters: threshold on the Eq. 6 normalised power (strict >),
 * minimum number of windows per single pulse (step d) and of baselines per
 * reported cross-matching group. */
frbx_status frbx_set_detection(frbx_ctx *ctx, double threshold, int32_t n_win_min,
                               int32_t n_bl_min);

/* Device memory for the dedispersed DM tiles of frbx_run / frbx_stream_push,
 * in bytes: the DM trials are dedispersed floor(bytes / tile) at a time, one
 * trial's tile being (K - dk_max) x N x J x 8 bytes (K: the APs of the run or
 * of the stream buffer).  0 (default) = 6 GiB, at least one trial per tile.
 * A positive budget below one trial's tile makes the search fail with
 * FRBX_E_NOMEM (the message gives both sizes); an allocation that the device
 * refuses returns FRBX_E_NOMEM as well.  FRBX_E_INVAL for bytes < 0. */
frbx_status frbx_set_tile_budget(frbx_ctx *ctx, int64_t bytes);

/* Arithmetic of the fringe transform.
 *   FRBX_PREC_F32       float32 segment sums, SBD and MBD transforms on the
 *                       vector ALUs (in-register FFTs).  When every IF's MBD
 *                       lattice position lies within one row of the first
 *                       MBD pass (16 positions at n_mbd = 256) after a
 *                       common shift, that pass is skipped (a phase factor
 *                       on G; |G| is unchanged).
 *   FRBX_PREC_F16X3     float32 segment sums and SBD transform; the MBD
 *                       transform on the matrix cores as three float16
 *                       products (high x high + high x low + low x high of a
 *                       float16 high/low split of both operands, float32
 *                       accumulation): products good to ~2^-21 relative.
 *   FRBX_PREC_F16       one float16 product (inputs and DFT matrices
 *                       rounded once to float16, float32 accumulation); the
 *                       SBD transform as in FRBX_PREC_F16X3, or on the
 *                       matrix cores too (frbx_set_sbd_matrix_cores).
 * The matrix-core forms need n_mbd = 256, n_chan >= 16 and n_if <= 32
 * (FRBX_E_INVAL at frbx_run otherwise); their operands are scaled by a
 * power of two chosen from the largest input component so that float16
 * cannot overflow.  In every form the peak power keeps 19 mantissa bits of
 * |G|^2 (the low bits carry the peak's position). */
typedef enum { FRBX_PREC_F32 = 0, FRBX_PREC_F16X3 = 1, FRBX_PREC_F16 = 2 } frbx_precision;

frbx_status frbx_set_precision(frbx_ctx *ctx, int32_t precision);

/* FRBX_PREC_F16 with n_chan <= 64: enable = 1 runs the SBD transform on the
 * matrix cores as well: per SBD sub-grid a real-embedded J-point DFT GEMM of
 * the rotated segment sums (float32 sums, float16 operands), eight waves per
 * segment.  Default 0 (the float32 SBD transform of FRBX_PREC_F16X3, which
 * measured faster: 110 against 122 ms per launch on the VGOS-shaped
 * workload).  Same accuracy bar either way; takes effect at the next
 * frbx_run. */
frbx_status frbx_set_sbd_matrix_cores(frbx_ctx *ctx, int enable);

/* Kernel specialisation (not a step of the paper).  In FRBX_PREC_F32,
 * when the IF lattice of Eq. 5 is not compact (the general form of the
 * fringe kernel), the kernel is compiled at run time (hipRTC, gfx950, about
 * 2 s once per process, device, n_chan, n_mbd and row set) for the rows of
 * its first MBD pass that hold an IF, which that pass then alone reads and
 * transforms.  It computes the same sums as the statically built kernel;
 * as a separate compilation its multiply-add fusion may differ, so powers
 * agree to float32 rounding (a few parts in 10^6).  enable = 0 keeps the
 * statically built kernel; default 1.  Takes effect at the next frbx_run. */
frbx_status frbx_set_specialisation(frbx_ctx *ctx, int enable);

/* The row set of the kernel the last frbx_run used (bit i1 for lattice
 * positions (n_mbd / A) i1 + i2, A the first pass's row count); 0 for the
 * statically built kernel.  *why (may be NULL) receives the reason the
 * specialised kernel could not be built, or "" (valid until the next
 * frbx_run on this context). */
frbx_status frbx_get_specialisation(const frbx_ctx *ctx, uint32_t *rows, const char **why);

/* Float32 re-evaluation of the crossings of the matrix-core forms (not a
 * step of the paper; it gives their threshold decisions and crossing peaks
 * float32 arithmetic).  With band > 0, after the search in FRBX_PREC_F16X3
 * or FRBX_PREC_F16 (frbx_run or frbx_stream_push), every segment whose
 * Eq. 6 normalised power exceeds threshold - band is searched again by the
 * float32 kernel (its segment sums gathered straight from the input with
 * the AP offsets), its power and index are replaced in the cube, and the
 * statistics, crossings and detections are taken from the updated cube.
 * That cube keeps the matrix-core powers of every segment outside the
 * band, so the Eq. 6 mean and deviation, and with them every normalised
 * power, differ from a float32 search's by about the form's power error
 * (up to 2.3e-3 in P_norm measured on the precision workload): crossings
 * that close to the threshold can still differ.
 * band = 0 (default) turns it off; ignored in FRBX_PREC_F32; FRBX_E_INVAL
 * for band < 0.  Its launch is not among the kernel times of
 * frbx_get_timing (the run's wall time includes it). */
frbx_status frbx_set_recheck(frbx_ctx *ctx, double band);

/* The current band and the number of segments re-evaluated by the last
 * frbx_run / frbx_stream_push (either pointer may be NULL). */
frbx_status frbx_get_recheck(const frbx_ctx *ctx, double *band, int64_t *n_last);

/* Hand the cross spectra to the context: complex64 (re, im float32 pairs)
 * with layout [B][N][J][K].  is_device = 1: `vis` is a device pointer on the
 * context's device; it is borrowed and must stay valid and unchanged until
 * the next frbx_load or frbx_destroy.  is_device = 0: host memory, copied. */
frbx_status frbx_load(frbx_ctx *ctx, const void *vis, int is_device);

/* As frbx_load for cross spectra stored as complex32: (re, im) float16
 * pairs, layout [B][N][J][K] (the storage form of the precision workloads).
 * The search reads them into float32. */
frbx_status frbx_load_f16(frbx_ctx *ctx, const void *vis, int is_device);

/* The cross spectra as OCP FP8 e4m3 (e4m3fn) byte pairs (re, im)
 * [B][N][J][K][2] with one float32 scale per (baseline, IF, channel)
 * [B][N][J] (value = decoded code x scale), both on the host (copied) or
 * both on the device (read during the call).  The library decodes them
 * exactly into a complex64 copy that it owns and searches that.  Errors as
 * for frbx_load. */
frbx_status frbx_load_e4m3(frbx_ctx *ctx, const void *codes, const float *scale, int is_device);

/* Run the whole search on the context's stream and wait for it: dedispersion
 * and segment sums, fringe search and peak of every (baseline, DM trial,
 * window, segment), Eq. 6 statistics and threshold on the device; the
 * multi-window filter, best-DM merge and cross-baseline matching on the
 * host. */
frbx_status frbx_run(frbx_ctx *ctx);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the device
 * part of frbx_run -- dedispersion and the fringe search of every (baseline,
 * DM trial, segment) -- with no allocation, enqueued on the context's stream
 * without waiting.  It writes the power cube as frbx_get_power_cube returns
 * it after frbx_run: power float32 and idx int32, both DEVICE buffers of the
 * caller, [B][D][segments] with cap elements each (cap < needed:
 * FRBX_E_RANGE with *n = needed; cap = 0 is a size query).  No statistics,
 * crossings or detections, no float32 re-evaluation, no timing.
 * The dedispersed DM tiles go through a fixed workspace of 64 MiB that the
 * library holds on every GPU it runs on until the process ends (looked up
 * at frbx_create); one DM trial's tile, (K - dk_max) x N x J x 8 bytes, must
 * fit in it, else FRBX_E_INVAL.  Every call on one GPU shares that
 * workspace: calls that overlap on one GPU (two streams, two threads) race
 * and must be serialised by the caller.  The input must be loaded and the
 * grid tables built after the last setter (frbx_get_segments or frbx_run):
 * FRBX_E_STATE otherwise, since building them allocates.  The results equal
 * frbx_run's cube bit for bit. */
frbx_status frbx_run_cube_noalloc(frbx_ctx *ctx, float *power, int32_t *idx, int64_t cap,
                                  int64_t *n);

/* Segment layout of the current grids: dk_max (largest AP offset over all DM
 * trials), per window its hop and segment count Q (arrays of the number of
 * windows, may be NULL), and cube_len = sum of Q (segments per (b, d)). */
frbx_status frbx_get_segments(const frbx_ctx *ctx, int64_t *dk_max, int32_t *hop,
                              int64_t *n_seg, int64_t *cube_len);

/* MBD lattice of the Eq. 5 MBD term for the current grids: q[n] (array of N,
 * may be NULL) = the lattice position of IF n, ((f0^n - f0^0) mbd_step M)
 * mod M; *mbd_step_us the MBD grid step (may be NULL); *compact_shift (may
 * be NULL) = the common shift s with every (q[n] - s) mod M inside one row
 * of the first MBD pass, for which the float32 transform runs in one pass,
 * or -1 when it runs the general two-pass form. */
frbx_status frbx_get_lattice(const frbx_ctx *ctx, int64_t *q, double *mbd_step_us,
                             int32_t *compact_shift);

/* The same lattice for a layout without a context (host only, no device):
 * n_mbd in {16, 32, 64, 128, 256}, mbd_step_us <= 0 for T/M; FRBX_E_INVAL
 * for a layout or grid that frbx_set_delay_grid / frbx_run would refuse
 * (offsets not on the lattice, two IFs on one point). */
frbx_status frbx_mbd_lattice(const frbx_layout *layout, int32_t n_mbd, double mbd_step_us, int64_t *q,
                             double *mbd_step_out, int32_t *compact_shift);

/* AP offsets of Eq. 2 for the current DM grid: [D][N][J] int32 (host). */
frbx_status frbx_get_ap_offsets(const frbx_ctx *ctx, int32_t *out, int64_t cap, int64_t *n);

/* Power cube: power[b][d][seg] = max |G| of the segment and idx = packed
 * (r * PJ + s) * M + m of its lowest-index maximum; seg runs over the windows
 * in order, each window's segments consecutive.  Host buffers, cap in
 * elements; either pointer may be NULL.  A segment whose data hold a NaN or
 * an infinity gets a power that is not finite (NaN with idx -1 when a cell
 * is not a number); it takes no part in Eq. 6 and never crosses.  Among
 * cells equal to within the 19 kept mantissa bits the lowest index wins
 * within one (rate, SBD sub-grid); across sub-grids the float32 search keeps
 * the sub-grid whose largest cell is largest in all bits. */
frbx_status frbx_get_power_cube(const frbx_ctx *ctx, float *power, int32_t *idx,
                                int64_t cap, int64_t *n);

/* Device pointers of the power cube (valid until the next run/destroy). */
frbx_status frbx_get_power_cube_device(const frbx_ctx *ctx, const float **power,
                                       const int32_t **idx);

/* Eq. 6 statistics per (b, d, window): mean, population std and the number
 * of finite segment powers they were taken over. */
frbx_status frbx_get_stats(const frbx_ctx *ctx, double *mean, double *stdev,
                           int64_t *count, int64_t cap, int64_t *n);

/* Threshold crossings (Sec. 2.4.1 step a), sorted by (b, d, window, q). */
frbx_status frbx_get_crossings(const frbx_ctx *ctx, frbx_candidate *out, int64_t cap,
                               int64_t *n);

/* Single-pulse detections after steps b-d and the best-DM merge, ordered by
 * (baseline, k0); group_id names their cross-matching group. */
frbx_status frbx_get_candidates(const frbx_ctx *ctx, frbx_candidate *out, int64_t cap,
                                int64_t *n);

/* Cross-matching groups (all of them; `reported` marks n_baselines >=
 * N_bl,min), in creation order. */
frbx_status frbx_get_groups(const frbx_ctx *ctx, frbx_group *out, int64_t cap, int64_t *n);

/* ---- Streaming (chunked) search ------------------------------------------
 * The search of a long observation in chunks of chunk_frames APs.  The
 * library keeps, per baseline and channel, the last dk_max + l_max - 1 APs
 * of the data seen so far (the DM-overlap carry) so that every segment of
 * every window and DM trial is searched exactly once, by the first push that
 * completes it; segment q of window l covers APs [q hop, q hop + l - 1] on the
 * global AP axis, as in frbx_run.  The grids must be set before
 * frbx_stream_begin and not changed until the next begin.
 * After each push the per-push results are read with the usual getters:
 * frbx_get_power_cube (the segments completed by this push, [B][D][S_push],
 * windows in order), frbx_get_stats (Eq. 6 over this push's segments of each
 * window: the statistics are per chunk), frbx_get_crossings (this push's
 * crossings, global segment index and k0); frbx_get_candidates and
 * frbx_get_groups cover all pushes since frbx_stream_begin. */
typedef enum {
  FRBX_IN_C64 = 0,   /* complex64 */
  FRBX_IN_C32 = 1,   /* (re, im) float16 pairs */
  FRBX_IN_E4M3 = 2   /* (re, im) OCP FP8 e4m3 byte pairs, value = decoded x scale[b][n][j] */
} frbx_input_kind;

frbx_status frbx_stream_begin(frbx_ctx *ctx, int64_t chunk_frames);

/* One chunk [B][N][J][chunk_frames] of `kind`; scale: float32 [B][N][J] for
 * FRBX_IN_E4M3 (else ignored), on the same side (host / device) as the
 * chunk.  Host chunks are copied; device chunks are read before the call
 * returns. */
frbx_status frbx_stream_push(frbx_ctx *ctx, const void *chunk, int32_t kind, const float *scale,
                             int is_device);

/* Stream position: APs pushed so far, and per window (arrays of the number
 * of windows, may be NULL) the global index of the first segment and the
 * number of segments of the last push. */
frbx_status frbx_stream_position(const frbx_ctx *ctx, int64_t *frames_in, int64_t *first_segment,
                                 int64_t *n_segments);

/* Multiple-baselines power summation scheme (Sec. 2.4.2), after frbx_run:
 * the powers of corresponding segments of the listed baselines are summed,
 * normalised per (DM trial, window) with Eq. 6, thresholded, and filtered
 * with steps b and d of Sec. 2.4.1 (step c is skipped: MBD has no meaning
 * for the combined baseline); then the best DM bin per pulse (Sec. 5.3).
 * baselines: host array of n_bl distinct indices.  Detections are written as
 * for frbx_get_candidates with baseline = -1 and the summed power in
 * `power`. */
frbx_status frbx_power_sum(frbx_ctx *ctx, const int32_t *baselines, int32_t n_bl,
                           frbx_candidate *out, int64_t cap, int64_t *n);

/* Initial-phase and channel-delay extraction of Appendix A on a calibrator
 * segment: APs [k0, k0 + len) of `baseline` summed without dedispersion or
 * calibration; the (SBD, MBD) cell of maximum |G| on the current delay
 * grids; per IF the channel delay tau0 maximising the amplitude of
 * sum_{j>=1} S(n,j) exp(-2 pi i f_j SBD) exp(-2 pi i (f_j - f_bw/2) tau)
 * (|tau| <= 1/(2 chan_bw), refined to ~1e-9 us) and the initial phase
 * phi0 = angle of sum_{j>=1} S(n,j) exp(-2 pi i [f_j SBD + (f0^n -
 * f_ref,fit) MBD + (f_j - f_bw/2) tau0]).  tau0_us, phi0_rad: host [N]
 * outputs, ready for frbx_set_calibration (row `baseline`). */
frbx_status frbx_calibrate(frbx_ctx *ctx, int32_t baseline, int64_t k0, int32_t len,
                           double *tau0_us, double *phi0_rad);

/* ---- Refinement of coarse peaks ------------------------------------------
 * |G| of one segment as a function of continuous parameters
 *   theta = (SBD tau_s [us], MBD tau_m [us], delay rate rho [s/s],
 *            DM [pc cm^-3], arrival offset t [APs]):
 *   G = sum_{n, j >= 1} C_b(n,j) exp(-2 pi i (f_j tau_s + (f0^n - f0^0) tau_m))
 *         sum_{u<l} exp(-2 pi i 1e3 f0^n rho t_ap (u - (l-1)/2))
 *                   V~_b(n, j, k0 + t + x_nj(DM) + u)
 * -- Eq. 5 with the rate term of Eq. 4 at continuous delays and rate, and
 * the frames of Eq. 3 taken at the unrounded Eq. 1 shift
 * x_nj(DM) = k_DM DM (f^-2 - f_ref^-2) / t_ap plus t, where V~ is Keys'
 * cubic interpolation (a = -1/2) of the frames of the channel (frames outside
 * the data count as zero).  The relaxation replaces the rounding of Eq. 2,
 * whose gradient in DM is zero; at DM = 0, t = 0 and grid delays and rate
 * P = |G| equals the coarse search's cell.  Sums in float32, phase
 * arguments in float64.  Needs input loaded with frbx_load /
 * frbx_load_f16 (not a stream); the input must stay resident.
 *
 * The ascent (frbx_refine_run) proposes, per step, a move of every
 * coordinate in grid cells z of -g/H (gradient over curvature of P in z)
 * where H < 0, else 0.5 cell along the gradient, clipped to +-0.5 cell, and
 * takes it within a trust radius.  Cells:
 * SBD 1/(P J chan_bw), MBD the MBD grid step, rate the rate step (held when
 * the grid has one rate), DM the DM step, t one AP.  A DM step moves t by
 * -xbar per unit DM (xbar = mean of dx/dDM over the fitted points), which
 * decorrelates DM from the arrival offset. */

/* The n_max crossings of the last frbx_run with the highest normalised
 * power (ties: baseline, DM trial, window, segment ascending), as
 * frbx_candidate records; cap = 0 is a size query (E_RANGE). */
frbx_status frbx_top_peaks(const frbx_ctx *ctx, int64_t n_max, frbx_candidate *out, int64_t cap,
                           int64_t *n);

/* Start a refinement of n peaks (host records: baseline, dm_index,
 * window_len, k0, rate_idx, sbd_idx, mbd_idx are read).  The start point of
 * each is its grid cell (tau_s[sbd_idx], tau_m[mbd_idx], rho[rate_idx],
 * DM[dm_index], 0); theta0 (host [n][5], may be NULL) receives it.  Device
 * buffers for n peaks are held by the context until the next begin. */
frbx_status frbx_refine_begin(frbx_ctx *ctx, const frbx_candidate *peaks, int64_t n, double *theta0);

/* n_steps ascent steps on the device (one launch each) from the begun grid
 * points, then the better of the last point and the best one with its P
 * (so P never ends below its start).  Each step is a trust-region Newton
 * step: a point that does not lower P below the best so far becomes the best
 * (its proposed move stored, the radius doubled up to 0.5 cell), otherwise
 * the radius is halved; the best point's move is taken clipped to the
 * radius.  Repeated runs restart from the begun points. */
frbx_status frbx_refine_run(frbx_ctx *ctx, int32_t n_steps);

/* Results of frbx_refine_run: theta host [n][5], power host [n] (either may
 * be NULL); cap = 0 is a size query. */
frbx_status frbx_refine_results(const frbx_ctx *ctx, double *theta, float *power, int64_t cap,
                                int64_t *n);

/* Forward, backward and curvature on the begun peaks, with device pointers
 * on the context stream (the pieces of a torch.autograd.Function):
 *   forward:   power[i] = P(theta_i)                      theta [n][5] f64, power [n] f32
 *   backward:  grad_theta[i][k] = grad_power[i] dP/dtheta_k (theta_i)
 *   curvature: curv[i][k] = d2P/dtheta_k^2 (k < 5), curv[i][5] = d2P/dDM dt */
frbx_status frbx_refine_forward(frbx_ctx *ctx, const double *theta, float *power);
frbx_status frbx_refine_backward(frbx_ctx *ctx, const double *theta, const float *grad_power,
                                 double *grad_theta);
frbx_status frbx_refine_curvature(frbx_ctx *ctx, const double *theta, double *curv);

/* The ascent's grid cells [5] and xbar (host outputs, either may be NULL). */
frbx_status frbx_refine_cells(frbx_ctx *ctx, double *cells, double *xbar);

/* |G|^2 of every cell of one segment, [R][PJ][M] float32 into a device
 * buffer of the caller (for element-wise checks of the fringe transform;
 * needs a loaded context with valid grids). */
frbx_status frbx_dump_segment(frbx_ctx *ctx, int32_t baseline, int32_t dm_index,
                              int32_t window_index, int64_t segment, float *dev_out);

/* Per-kernel timing of the last frbx_run, from HIP events recorded on the
 * context's stream around every launch (enable before the run; enabling adds
 * two event records per launch).  Times in milliseconds, summed over the
 * launches of each kernel; n_* are the launch counts and *_units the
 * segments (fringe) or dedispersed spectra (dedisperse) they processed. */
typedef struct {
  double fringe_ms;
  int64_t n_fringe;
  int64_t fringe_units;
  double dedisperse_ms;
  int64_t n_dedisperse;
  int64_t dedisperse_units;
  double stats_ms;
  int64_t n_stats;
  int64_t dedisperse_bytes;   /* algorithmic bytes of the dedispersion
                                 launches: every dedispersed spectrum written
                                 once, every channel's input span read once
                                 per group of DM trials */
  double refine_ms;           /* refinement launches of the last
                                 frbx_refine_run (timed like the others) */
  int64_t n_refine;
  int64_t refine_units;       /* peaks x launches */
} frbx_timing;

frbx_status frbx_set_timing(frbx_ctx *ctx, int enable);
frbx_status frbx_get_timing(const frbx_ctx *ctx, frbx_timing *out);

/* Host-only: the Eq. 2 AP-offset table for a layout and DM grid, [D][N][J]
 * int32; needs no device. */
frbx_status frbx_ap_offsets(const frbx_layout *layout, double dm_lo, double dm_step,
                            int32_t n_dm, double k_dm, int32_t *out);

/* Host-only: steps b-d per (baseline, DM), the best-DM merge and the
 * cross-baseline matching of Sec. 2.4.1 over a list of crossings (fields
 * baseline, dm_index, window_len, k0, power_norm, mbd_us are read; the rest
 * is carried).  t_amb_us is the MBD ambiguity.  use_mbd = 0 skips step c
 * (the power-summation scheme, Sec. 2.4.2).  Outputs as for
 * frbx_get_candidates / frbx_get_groups. */
frbx_status frbx_detect(const frbx_candidate *crossings, int64_t n_cross, double t_amb_us,
                        int32_t n_win_min, int32_t n_bl_min, int32_t use_mbd,
                        frbx_candidate *dets, int64_t det_cap, int64_t *n_dets,
                        frbx_group *groups, int64_t group_cap, int64_t *n_groups);

#ifdef __cplusplus
}
#endif

#endif /* FRBX_H */
