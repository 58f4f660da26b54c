// Internal interface between the host side of libfrbx and its HIP kernels.
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#else
// hipRTC declares the fixed-width integers in a namespace of its own
using __hip_internal::int32_t;
using __hip_internal::int64_t;
using __hip_internal::uint32_t;
using __hip_internal::uint64_t;
#endif

namespace frbx {

constexpr int kMaxWindows = 8;
constexpr int kBlock = 256;  // threads per work-group of every kernel

// One threshold crossing as written by the statistics kernel.
struct DevCrossing {
  int32_t row;    // (b * D + d) * n_windows + window
  int32_t q;      // segment index within the window
  float power;    // |G| peak
  int32_t idx;    // packed (r * PJ + s) * M + m
  double pnorm;   // Eq. 6
};

// Dedispersion of one baseline for a tile of DM trials (Eqs. 1-3): the
// dedispersed, calibrated AP sequence W[dl][k][c] = cal[c] * V[c][k + dk[d][c]]
// for k < k_eff and channel c = n * J + j.
struct DedisperseArgs {
  const void *vis;     // [NJ][K] of this baseline: complex64, or complex32
                       // (two float16) when in_f16
  int32_t in_f16;
  int64_t n_frames;    // K: APs available per channel
  int64_t row_stride;  // elements between channel rows (>= n_frames)
  const int32_t *dk;   // [D][NJ]
  int32_t d0;          // first DM trial of the tile
  int32_t n_dt;        // DM trials in the tile
  const float2 *cal;   // [NJ] of this baseline
  float2 *out;         // [n_dt][k_eff][NJ]
  int64_t k_eff;       // K - dk_max
  int32_t nj;          // N * J
  int32_t group;       // DM trials sharing one staged input tile (>= 1); the
                       // AP offsets of a group differ by < kDedispSpread
};

// Dedispersion tile: 16 channels x 256 APs, staged input span up to
// 256 + kDedispSpread APs per channel (the fastest of the tile shapes
// measured on MI355X).
constexpr int kDedispCh = 16;
constexpr int kDedispAp = 256;
constexpr int kDedispSpread = 128;
constexpr int kDedispMaxGroup = 64;   // DM trials per staged tile at most

// Fringe search of every segment of one baseline and DM tile (Sec. 2.3,
// Eq. 5 with the rate term of Eq. 4; Sec. 5.1): segment sums of W with rate
// rotation, zero-padded SBD transform per IF, MBD transform across the IF
// lattice, and the peak of |G| over (rate, SBD, MBD).
struct FringeArgs {
  const float2 *w;           // [n_dt][k_eff][NJ]
  int64_t w_dm_stride;       // k_eff * NJ
  int32_t n_if;              // N
  int32_t n_rate;            // R
  int32_t sbd_pad;           // P
  int32_t n_win;
  int32_t win_len[kMaxWindows];
  int32_t win_hop[kMaxWindows];
  int32_t win_off[kMaxWindows];   // first cube segment of the window
  int32_t win_k0[kMaxWindows];    // AP of the window's first segment (k0 = win_k0 + q hop)
  int32_t rate_off[kMaxWindows];  // offset (float2) of the window's [R][N][l] phasors
  int32_t seg_total;               // segments per (b, d)
  int32_t n_dt;                    // DM trials in this launch
  const float2 *rate_ph;
  const float2 *tw_sbd;      // [PJ]      exp(-2 pi i k / PJ)
  const float2 *pre_sbd;     // [P][JA]   exp(-2 pi i i1 c / (P JA))
  const float2 *tw_mbd;      // [M]       exp(-2 pi i k / M)
  const int32_t *mbd_row;    // [M]       IF on lattice position q, N if none
  const int32_t *mbd_pos;    // [N]       compact lattice: position of IF n less a common
                             //           shift, all < fringe_compact_rows(M); null: general form
  // list launches (re-evaluation of selected segments): one work-group per
  // (baseline, DM trial, segment) triple, the segment sums gathered straight
  // from the input with the AP offsets (no dedispersed copy); `power` and
  // `pidx` then point at the whole cube [B][D][seg_total]
  const int32_t *seg_list;   // [grid][3]
  const void *vis;           // [B][N J][vis_stride], complex64 or complex32
  int32_t vis_f16;
  int32_t n_dm;
  int64_t vis_stride;        // elements per channel row
  int64_t vis_frames;        // valid APs per row
  const int32_t *dk;         // [D][N J] AP offsets
  const float2 *cal;         // [B][N J] calibration phasors
  float *power;              // [n_dt][seg_total] cube rows of (b, d0)
  int32_t *pidx;
  float *dump;               // non-null: one segment, |G|^2 of every cell
  int32_t dump_dl;
  int32_t dump_seg;
  // matrix-core form of the MBD transform: the real-embedded DFT matrix
  // over the IF lattice as float16 MFMA B operands, [32 tiles][NK][64 lanes]
  // x 8 halves, high part and (split form) low part; inputs are scaled by a
  // power of two so that float16 cannot overflow
  const void *mfma_b_hi;
  const void *mfma_b_lo;
  float mfma_scale;
  // matrix-core SBD transform (float16 form): the real-embedded J-point DFT
  // matrix as MFMA A operands, [2J/16 row tiles][J/16 K chunks][64 lanes] x
  // 8 halves
  const void *sbd_a;
};

struct StatsArgs {
  const float *power;        // [B*D][seg_total]
  const int32_t *pidx;
  int32_t seg_total;
  int32_t n_win;
  int32_t win_off[kMaxWindows];
  int32_t win_q[kMaxWindows];
  double threshold;
  double *mean;              // [B*D*n_win]
  double *stdev;
  int64_t *count;
  DevCrossing *out;
  unsigned long long *n_out;
  int64_t cap;
};

#ifndef __HIPCC_RTC__
// Launch wrappers (defined in frbx_kernels.hip).  They return the HIP status
// of the launch.
hipError_t launch_dedisperse(const DedisperseArgs &a, hipStream_t s);
hipError_t launch_fringe(int n_chan, int n_mbd, const FringeArgs &a, size_t lds_bytes,
                         int grid, hipStream_t s);
size_t fringe_lds_bytes(int n_chan, int n_mbd, int n_if, int sbd_pad);
bool fringe_supported(int n_chan, int n_mbd, int n_if, int sbd_pad);
// Lattice rows of the compact MBD form for n_mbd points (0 if unsupported).
int fringe_compact_rows(int n_mbd);
// The float32 fringe search of the n (baseline, DM trial, segment) triples
// listed in a.seg_list (one work-group each), n_mbd = 256 only.
hipError_t launch_fringe_list(int n_chan, int n_mbd, const FringeArgs &a, size_t lds_bytes, int n,
                              hipStream_t s);
hipError_t launch_stats(const StatsArgs &a, int rows, hipStream_t s);

// matrix-core fringe kernel: n_pass = 1 (float16) or 3 (float16 high/low
// split, float32-grade products); supports n_mbd = 256, n_chan >= 16,
// n_if <= 32
// The 3-pass matrix-core form with 17-32 IFs and at most 64 channels forms
// each complex product of the MBD GEMM from three real products; its B
// table holds, per tile of 16 MBD columns, the matrices cos, -sin and
// cos - sin (K = IF).
constexpr bool mfma_three_real(int n_chan, int n_if, int n_pass) {
  return n_pass == 3 && n_if > 16 && n_if <= 32 && n_chan <= 64;
}
hipError_t launch_fringe_mfma(int n_chan, int n_if, int n_pass, const FringeArgs &a,
                              size_t lds_bytes, int grid, hipStream_t s);
size_t fringe_mfma_lds_bytes(int n_chan, int n_if, int sbd_pad, int n_pass);
bool fringe_mfma_supported(int n_chan, int n_mbd, int n_if, int sbd_pad, int n_pass);

// matrix-core fringe kernel with both transforms on the matrix cores
// (float16 form): 512 threads per segment; n_chan in {16, 32, 64, 128},
// n_mbd = 256, n_if <= 32
constexpr int kBlockGemm = 512;
hipError_t launch_fringe_gemm(int n_chan, int n_if, const FringeArgs &a, size_t lds_bytes, int grid,
                              hipStream_t s);
size_t fringe_gemm_lds_bytes(int n_chan, int n_if, int sbd_pad);
bool fringe_gemm_supported(int n_chan, int n_mbd, int n_if, int sbd_pad);

// out[d][s] = sum over the listed baselines of power[b][d][s]
hipError_t launch_cube_sum(const float *power, int64_t bl_stride, const int32_t *baselines,
                           int n_bl, float *out, int64_t n, hipStream_t s);

// Y[c] = sum_{k0 <= k < k0 + len} V[c][k] (complex64 or complex32 input),
// c over n_chan_total channels of one baseline
hipError_t launch_segment_sum(const void *vis, int in_f16, int64_t n_frames, int n_ch, int64_t k0,
                              int len, float2 *out, hipStream_t s);

// streaming input: dst[c][k0 + k] = complex64 of src[c][k] for k < n_frames
// (src complex64, complex32, or FP8 e4m3 pairs times scale[c]); channel c
// over n_ch, dst row stride dst_frames
hipError_t launch_ingest(const void *src, int src_kind, const float *scale, int64_t n_frames, int n_ch,
                         float2 *dst, int64_t dst_frames, int64_t k0, hipStream_t s);
// dst[c][k] = src[c][from + k] for k < n (the carry into the other buffer)
hipError_t launch_carry(const float2 *src, float2 *dst, int n_ch, int64_t frames, int64_t from, int64_t n,
                        hipStream_t s);

// Refinement of coarse peaks: |G| of one segment at continuous (SBD, MBD,
// rate, DM, arrival offset), Eq. 5 with the rate term of Eq. 4 and the frames
// of Eq. 3 taken at the unrounded Eq. 1 shift (Keys cubic interpolation).
struct RefineChan {   // per channel c = n * J + j
  double fj;          // j * chan_bw (MHz)
  double fm;          // f0^n - f0^0 (MHz)
  double wr;          // 1e3 f0^n t_ap: rate phase in cycles per unit rate and AP
  double dxd;         // k_DM (f^-2 - f_ref^-2) / t_ap: APs of shift per unit DM
};
struct RefineSeg {
  int32_t b;          // baseline
  int32_t l;          // window length (APs)
  int64_t k0;         // first AP of the segment at f_ref
};
enum RefineMode { kRefineForward = 0, kRefineBackward = 1, kRefineCurvature = 2, kRefineStep = 3,
                  kRefineFinal = 4 };
struct RefineArgs {
  const void *vis;           // [B][NJ][row_stride] complex64, or complex32 when in_f16
  int32_t in_f16;
  int64_t n_frames;          // APs per channel
  int64_t row_stride;
  int32_t nj, J;
  const RefineChan *chan;    // [NJ]
  const float2 *cal;         // [B][NJ]
  const RefineSeg *seg;      // [n]
  int32_t n;
  double *theta;             // [n][5] (sbd us, mbd us, rate, DM, t APs); updated by a step
  float *power;              // [n] |G| (forward; step: before the step)
  const float *grad_power;   // [n] backward: upstream gradient
  double *grad_theta;        // [n][5] backward: grad_power * dP/dtheta
  double *curv;              // [n][6] curvature: d2P/dtheta_i^2 (5), d2P/dDM dt
  double *theta_best;        // step / final: [n][5] best point so far
  double *step_best;         // step: [n][5] proposed move at the best point (grid cells)
  float *p_best;             // step / final: [n] |G| at the best point (-1: none yet)
  double *radius;            // step: [n] trust radius (grid cells)
  double cells[5];           // step: grid cell of each parameter (0: held)
  double dm_t;               // step: arrival-offset cells moved per DM cell (-xbar c_DM / c_t)
  double max_step;           // step: largest move per coordinate and largest radius, cells
};
hipError_t launch_refine(int mode, const RefineArgs &a, hipStream_t s);

// max(|re|, |im|) over n complex values (float32 or float16 pairs) into
// *out (float bits, caller zeroes it first)
hipError_t launch_absmax(const void *vis, int64_t n, int in_f16, unsigned int *out,
                         hipStream_t s);

// Workspace of the search variant that allocates nothing: a file-scope
// device array of kNoAllocBytes on every GPU the library runs on.
// noalloc_workspace(device) must be called with `device` current; the first
// call on a device looks up that device's copy of the array
// (hipGetSymbolAddress) and later calls return the same address.
constexpr size_t kNoAllocBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
hipError_t noalloc_workspace(int device, void **ptr);

// The float32 fringe kernel of the general MBD form specialised to the
// rows of its first MBD pass that hold an IF (bit i1 of `rows`), compiled
// at run time with hipRTC for the current device (defined in
// frbx_jit.cpp).  The first call for a (device, n_chan, n_mbd, rows)
// compiles and loads it; later calls return the loaded function.  nullptr
// with the reason in *err when it cannot be built.
hipFunction_t fringe_rows_kernel(int device, int n_chan, int n_mbd, unsigned rows, std::string *err);
hipError_t launch_fringe_rows(hipFunction_t fn, const FringeArgs &a, size_t lds_bytes, int grid,
                              hipStream_t s);
#endif  // !__HIPCC_RTC__

}  // namespace frbx
