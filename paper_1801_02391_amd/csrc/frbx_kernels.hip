// HIP kernels of the cross-spectrum FRB search for gfx950 (MI355X).
//
//   dedisperse_kernel  Eqs. 1-3 (Sec. 2.2) and the Eq. 5 calibration: shifts
//                      every channel by its AP offset for each DM trial of a
//                      tile and transposes to AP-major order, so that the
//                      segment sums of the fringe kernel read whole spectra.
//                      HBM-bound; LDS-tiled transpose, coalesced both ways.
//   fringe_kernel      Eq. 5 with the Eq. 4 rate term, Sec. 5.1: one
//                      work-group per segment; for each rate bin it forms the
//                      segment sums in registers, runs the zero-padded SBD
//                      transform per IF as P sub-DFTs of J points (two
//                      in-register passes with an LDS transpose), then the
//                      M-point MBD transform over the IF lattice for each SBD
//                      column (two in-register passes, wave-local LDS
//                      transpose; one pass for compact IF lattices) and
//                      keeps the peak of |G|^2.  VALU-bound.  List launches
//                      search selected segments, gathering their sums from
//                      the input (re-evaluation near the threshold).
//   fringe_mfma_kernel the same search with the MBD transform as a
//                      real-embedded complex GEMM on the matrix cores (float16
//                      operands, float32 accumulation; one product, or three
//                      of a high/low split for float32-grade results).
//   fringe_gemm_kernel the float16 form with the SBD transform on the matrix
//                      cores as well (a J-point DFT GEMM per SBD sub-grid),
//                      eight waves per segment.
//   stats_kernel       Eq. 6 and the threshold of Sec. 2.4.1 per (baseline,
//                      DM trial, window): float64 two-pass mean / population
//                      deviation, ordered compaction of the crossings.
//   cube_sum_kernel    power summation over a set of baselines (Sec. 2.4.2).
//   segment_sum_kernel a calibrator window sum for Appendix A.
//   ingest_kernel,     streaming input: decode a chunk (complex64, complex32,
//   carry_kernel       FP8 e4m3 x per-channel scale) behind the DM-overlap
//                      carry, and copy the carry between the two buffers.
//   refine_kernel      |G| of a segment at continuous delays, rate, DM and
//                      arrival offset (Eq. 5 with the Eq. 4 rate term, frames
//                      at the unrounded Eq. 1 shift by cubic interpolation),
//                      its gradient and curvature, and a trust-region Newton
//                      step of the ascent.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>

#include "frbx_internal.h"

// Workspace of the search variant that allocates nothing (dedispersed DM
// tiles): every GPU holds its own copy of this array, at its own address,
// from module load until the process ends.  In host code the name is only a
// host-side stand-in; the device address comes from noalloc_workspace().
static __device__ __align__(256) unsigned char scratch[frbx::kNoAllocBytes];

#include "frbx_fringe.h"

namespace frbx {
namespace {

// ---------------------------------------------------------------- kernels

// One work-group dedisperses a tile of 16 channels x 256 APs for a group of
// DM trials: each channel's input span (the 256 APs shifted by the group's
// smallest offset, plus the offset spread of the group) is read once,
// coalesced, into LDS, with the group's offsets relative to its first
// trial; every trial of the group then writes its 256 AP-major spectra from
// the staged span (16 channels = 128 contiguous bytes per AP), with the
// Eq. 5 calibration applied on the way.  The write loop reads nothing from
// global memory: a load there would make each wave wait for its earlier
// stores to complete (one counter covers both on this GPU).
template <bool F16>
__global__ __launch_bounds__(kBlock) void dedisperse_kernel(DedisperseArgs a) {
  constexpr int SW = kDedispAp + kDedispSpread + 1;   // staged APs per channel (+1 pad)
  __shared__ float2 tile[kDedispCh][SW];
  __shared__ int32_t shs[kDedispMaxGroup][kDedispCh];  // offset of trial g0 + j minus trial g0's
  const int64_t kt = int64_t(blockIdx.x) * kDedispAp;
  const int ct = blockIdx.y * kDedispCh;
  const int g0 = blockIdx.z * a.group;                  // first trial of the group (tile-local)
  const int ng = min(a.group, a.n_dt - g0);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int32_t *dk0 = a.dk + int64_t(a.d0 + g0) * a.nj;
  const int32_t *dk1 = a.dk + int64_t(a.d0 + g0 + ng - 1) * a.nj;
  for (int x = threadIdx.x; x < ng * kDedispCh; x += kBlock) {
    const int j = x / kDedispCh, i = x - j * kDedispCh;
    const int c = ct + i;
    shs[j][i] = c < a.nj ? a.dk[int64_t(a.d0 + g0 + j) * a.nj + c] - dk0[c] : 0;
  }
  // stage: wave w loads channels w, w + 4, ...; frames base .. base + span
  for (int i = w; i < kDedispCh; i += kBlock / 64) {
    const int c = ct + i;
    if (c >= a.nj) continue;
    const int64_t base = kt + dk0[c];
    const int span = kDedispAp + (dk1[c] - dk0[c]);
    const int64_t row = int64_t(c) * a.row_stride;
    for (int x = lane; x < span; x += 64) {
      const int64_t f = base + x;
      tile[i][x] = f < a.n_frames ? load_vis(a.vis, row + f, F16) : make_float2(0.f, 0.f);
    }
  }
  __syncthreads();
  // write: lane -> channel (kDedispCh consecutive lanes per AP)
  const int cl = lane & (kDedispCh - 1);
  const int c = ct + cl;
  const float2 cal = c < a.nj ? a.cal[c] : make_float2(0.f, 0.f);
  const int kr = threadIdx.x / kDedispCh;                // 0..15
  // full tiles (all but the last AP tile) store without a bounds test, so
  // that the staged reads of several APs are issued together
  const bool full = kt + kDedispAp <= a.k_eff && ct + kDedispCh <= a.nj;
  for (int j = 0; j < ng; ++j) {
    const int shift = shs[j][cl];
    float2 *outd = a.out + int64_t(g0 + j) * a.k_eff * a.nj;
    if (full) {
#pragma unroll 8
      for (int kk = kr; kk < kDedispAp; kk += kBlock / kDedispCh)
        outd[(kt + kk) * a.nj + c] = cmul(tile[cl][kk + shift], cal);
    } else {
      for (int kk = kr; kk < kDedispAp; kk += kBlock / kDedispCh) {
        const int64_t k = kt + kk;
        if (c < a.nj && k < a.k_eff) outd[k * a.nj + c] = cmul(tile[cl][kk + shift], cal);
      }
    }
  }
}

// Block-wide sum of a double (all threads get the result).
__device__ double block_sum(double v, double *sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < kBlock / 64; ++w) s += sh[w];
  return s;
}

__global__ __launch_bounds__(kBlock) void stats_kernel(StatsArgs a) {
  __shared__ double sh[kBlock / 64];
  __shared__ int wcount[kBlock / 64];
  __shared__ long long base_sh;
  const int row = blockIdx.x;
  const int wi = row % a.n_win;
  const int bd = row / a.n_win;
  const int Q = a.win_q[wi];
  const float *p = a.power + int64_t(bd) * a.seg_total + a.win_off[wi];
  const int32_t *pi = a.pidx + int64_t(bd) * a.seg_total + a.win_off[wi];
  double s = 0.0, cnt = 0.0;
  for (int q = threadIdx.x; q < Q; q += kBlock) {
    const float v = p[q];
    if (isfinite(v)) {
      s += v;
      cnt += 1.0;
    }
  }
  const double S = block_sum(s, sh);
  const double C = block_sum(cnt, sh);
  const double mu = C > 0 ? S / C : 0.0;
  double s2 = 0.0;
  for (int q = threadIdx.x; q < Q; q += kBlock) {
    const float v = p[q];
    if (isfinite(v)) {
      const double d = double(v) - mu;
      s2 += d * d;
    }
  }
  const double S2 = block_sum(s2, sh);
  const double sd = C > 0 ? sqrt(S2 / C) : 0.0;
  if (threadIdx.x == 0) {
    a.mean[row] = mu;
    a.stdev[row] = sd;
    a.count[row] = static_cast<int64_t>(C);
  }
  if (!(sd > 0.0)) return;
  // count, reserve, then write the crossings in q order
  int n_cross = 0;
  for (int q = threadIdx.x; q < Q; q += kBlock) {
    const float v = p[q];
    n_cross += (isfinite(v) && (double(v) - mu) / sd > a.threshold) ? 1 : 0;
  }
  const double tot = block_sum(double(n_cross), sh);
  if (tot == 0.0) return;
  if (threadIdx.x == 0) base_sh = (long long)atomicAdd(a.n_out, (unsigned long long)tot);
  __syncthreads();
  long long pos = base_sh;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int q0 = 0; q0 < Q; q0 += kBlock) {
    const int q = q0 + threadIdx.x;
    bool f = false;
    double pn = 0.0;
    if (q < Q) {
      const float v = p[q];
      pn = (double(v) - mu) / sd;
      f = isfinite(v) && pn > a.threshold;
    }
    const unsigned long long bal = __ballot(f);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wcount[wv] = __popcll(bal);
    __syncthreads();
    int woff = 0, all = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
      if (w < wv) woff += wcount[w];
      all += wcount[w];
    }
    if (f) {
      const long long o = pos + woff + before;
      if (o < a.cap) {
        DevCrossing cr;
        cr.row = row;
        cr.q = q;
        cr.power = p[q];
        cr.idx = pi[q];
        cr.pnorm = pn;
        a.out[o] = cr;
      }
    }
    pos += all;
    __syncthreads();
  }
}


// ------------------------------------------------ matrix-core fringe kernel
// The MBD transform of Eq. 5 as a real-embedded complex GEMM on the gfx950
// matrix cores: for each SBD column s, G(s, m) = sum_n X(n, s) w_M^{q_n m};
// with A[s][2n + {0,1}] = (Re, Im) X(n, s) and the constant B operand
// B[2n][m] = (cos, -sin), B[2n+1][m] = (sin, cos) (Re and Im column blocks),
// one v_mfma_f32_16x16x32_f16 per (16 SBD rows, 16 MBD columns, 32 K).
// The segment sum and the SBD transform are the float32 steps above; the
// SBD output is scaled (power of two), rounded to float16 (and, in the
// 3-pass form, its residual to a second float16) and staged in LDS in the
// A-operand layout.  Each of the 4 waves owns 64 MBD columns and keeps
// their B operands in registers for the kernel's life.
// With 17-32 IFs and at most 64 channels (where the larger A tiles still
// leave room for three work-groups per CU) the 3-pass form builds each
// complex product from three real ones (X W with W = c + i d: P1 = Re X c, P2 = Im X d, P3 = (Re X +
// Im X)(c + d); Re = P1 - P2, Im = P3 - P1 - P2): three GEMMs of K = 32
// over the IFs (A chunks Re X, Im X, Re X + Im X; B matrices c, d, c + d)
// in place of two of K = 64, a quarter fewer matrix-core instructions.
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef _Float16 h2_t __attribute__((ext_vector_type(2)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <int J, int NK>
__host__ __device__ inline void mfma_lds_plan(int n_if, int sbd_pad, int n_pass, int &t_off,
                                              int &a_off, int &total_bytes) {
  constexpr int JA = Split<J>::A, JB = Split<J>::B;
  const int AS = 32 * (mfma_three_real(J, 16 * NK, n_pass) ? 3 : NK) + 8;
  const int t_bytes = n_if * JA * (JB + 1) * 8;
  const int tw_bytes = sbd_pad * J * 8;
  t_off = t_bytes;                               // TW after the transpose scratch
  a_off = (t_bytes + tw_bytes + 15) & ~15;       // A tiles, 16-byte aligned
  total_bytes = a_off + (n_pass == 3 ? 2 : 1) * J * AS * 2;
}

// The three-product form runs three waves per SIMD (168 VGPRs, no spill).
template <int J, int NK, int NP, bool DUMP>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(mfma_three_real(J, 16 * NK, NP) && !DUMP ? 3 : 1)))
void fringe_mfma_kernel(FringeArgs a) {
  constexpr int M = 256;
  constexpr int JA = Split<J>::A, JB = Split<J>::B;
  constexpr bool K3 = mfma_three_real(J, 16 * NK, NP);  // three real products per complex one
  constexpr int NKA = K3 ? 3 : NK;          // A chunks of 32 per row
  constexpr int AS = 32 * NKA + 8;  // A row stride in halves (+16 B against bank conflicts)
  constexpr int NSB = J / 16;       // 16-row SBD blocks per tile
  extern __shared__ float2 lds[];
  __shared__ float red_v[kBlock / 64];
  __shared__ int32_t red_i[kBlock / 64];

  const int N = a.n_if, R = a.n_rate, P = a.sbd_pad;
  const int PJ = P * J;
  const int NJ = N * J;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;

  int dl, seg;
  block_segment(a, DUMP, dl, seg);
  int wi = 0;
  while (wi + 1 < a.n_win && a.win_off[wi + 1] <= seg) ++wi;
  const int l = a.win_len[wi];
  const int q = seg - a.win_off[wi];
  const int64_t k0 = a.win_k0[wi] + int64_t(q) * a.win_hop[wi];
  const float2 *wd = a.w + int64_t(dl) * a.w_dm_stride + k0 * NJ;
  const float2 *rph = a.rate_ph + a.rate_off[wi];

  int t_off, a_off, total;
  mfma_lds_plan<J, NK>(N, P, NP, t_off, a_off, total);
  float2 *Sc = lds;
  float2 *TW = reinterpret_cast<float2 *>(reinterpret_cast<char *>(lds) + t_off);
  _Float16 *Ahi = reinterpret_cast<_Float16 *>(reinterpret_cast<char *>(lds) + a_off);
  _Float16 *Alo = Ahi + J * AS;

  for (int i = t; i < PJ; i += kBlock) TW[i] = a.tw_sbd[i];
  for (int i = t; i < (NP == 3 ? 2 : 1) * J * AS; i += kBlock) Ahi[i] = _Float16(0.0f);

  // B operands of this wave: Re tiles 4 wave + p and Im tiles 16 + 4 wave + p;
  // K3: matrices c, d, c + d of tile 4 wave + p
  constexpr int NBT = K3 ? 4 : 8, NBK = K3 ? 3 : NK;
  h8_t bh[NBT][NBK], bl[NBT][NBK];
  {
    const h8_t *srch = static_cast<const h8_t *>(a.mfma_b_hi);
    const h8_t *srcl = static_cast<const h8_t *>(a.mfma_b_lo);
    static_for<0, NBT>([&](auto qq) {
      constexpr int p8 = decltype(qq)::value;
      const int tile = K3 ? 4 * wave + p8 : (p8 < 4 ? 4 * wave + p8 : 16 + 4 * wave + (p8 - 4));
      static_for<0, NBK>([&](auto kk) {
        constexpr int kc = decltype(kk)::value;
        bh[p8][kc] = srch[(tile * NBK + kc) * 64 + lane];
        if constexpr (NP == 3) bl[p8][kc] = srcl[(tile * NBK + kc) * 64 + lane];
      });
    });
  }
  const float scale = a.mfma_scale;

  const bool s_p1 = t < N * JB;
  const int n1 = t / JB, i2s = t - (t / JB) * JB;

  float best_v = -1.0f;
  int32_t best_i = 0x7fffffff;
  unsigned best_key = 0u;
  int best_blk = 0;

  for (int r = 0; r < R; ++r) {
    float2 y[JA];
    segment_sum<JA, JB>(y, wd, rph, r, N, J, l, R, s_p1, n1, i2s);
    for (int c = 0; c < P; ++c) {
      __syncthreads();
      sbd_pass1<JA, JB>(y, a.pre_sbd, TW, Sc, c, P, PJ, s_p1, n1, i2s);
      __syncthreads();
      // SBD pass 2 -> A rows a = k1 + JA k2 (SBD bin s' = c + P a), columns 2n, 2n+1
      for (int v = t; v < N * JA; v += kBlock) {
        const int n2 = v / JA, k1 = v - (v / JA) * JA;
        float2 z[JB];
        static_for<0, JB>([&](auto i) {
          constexpr int ii = decltype(i)::value;
          z[ii] = Sc[(n2 * JA + k1) * (JB + 1) + ii];
        });
        dft<JB>(z);
        static_for<0, JB>([&](auto k) {
          constexpr int kk = decltype(k)::value;
          const float xr = z[kk].x * scale, xi = z[kk].y * scale;
          if constexpr (K3) {
            // chunks Re X, Im X, Re X + Im X at K = n
            const int o = (k1 + JA * kk) * AS + n2;
            const float xs = xr + xi;
            const _Float16 hr = _Float16(xr), hi_ = _Float16(xi), hs = _Float16(xs);
            Ahi[o] = hr;
            Ahi[o + 32] = hi_;
            Ahi[o + 64] = hs;
            Alo[o] = _Float16(xr - float(hr));
            Alo[o + 32] = _Float16(xi - float(hi_));
            Alo[o + 64] = _Float16(xs - float(hs));
          } else {
            h2_t hi;
            hi.x = _Float16(xr);
            hi.y = _Float16(xi);
            const int o = (k1 + JA * kk) * AS + 2 * n2;
            *reinterpret_cast<h2_t *>(Ahi + o) = hi;
            if constexpr (NP == 3) {
              h2_t lo;
              lo.x = _Float16(xr - float(hi.x));
              lo.y = _Float16(xi - float(hi.y));
              *reinterpret_cast<h2_t *>(Alo + o) = lo;
            }
          }
        });
      }
      __syncthreads();
      // MBD on the matrix cores, 16 SBD rows at a time
      for (int sb = 0; sb < NSB; ++sb) {
        h8_t ah[NKA], al[NKA];
        const int arow = (16 * sb + (lane & 15)) * AS + 8 * (lane >> 4);
        static_for<0, NKA>([&](auto kk) {
          constexpr int kc = decltype(kk)::value;
          ah[kc] = *reinterpret_cast<const h8_t *>(Ahi + arow + 32 * kc);
          if constexpr (NP == 3) al[kc] = *reinterpret_cast<const h8_t *>(Alo + arow + 32 * kc);
        });
        // peak key of this lane's 16 cells: |G|^2 with its 4 lowest mantissa
        // bits replaced by (15 - slot), so one unsigned max keeps the value
        // (to 2^-19 relative) and the lowest slot among equal values
        unsigned kmax = 0u;
        static_for<0, 4>([&](auto pp) {
          constexpr int p = decltype(pp)::value;
          f4_t gr = {0.f, 0.f, 0.f, 0.f}, gi = {0.f, 0.f, 0.f, 0.f};
          if constexpr (K3) {
            f4_t p3 = {0.f, 0.f, 0.f, 0.f};
            // small products first, as below
            gr = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[0], bh[p][0], gr, 0, 0, 0);
            gi = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[1], bh[p][1], gi, 0, 0, 0);
            p3 = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[2], bh[p][2], p3, 0, 0, 0);
            gr = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[0], bl[p][0], gr, 0, 0, 0);
            gi = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[1], bl[p][1], gi, 0, 0, 0);
            p3 = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[2], bl[p][2], p3, 0, 0, 0);
            gr = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[0], bh[p][0], gr, 0, 0, 0);
            gi = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[1], bh[p][1], gi, 0, 0, 0);
            p3 = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[2], bh[p][2], p3, 0, 0, 0);
            // gr = P1, gi = P2 -> Re, Im
            static_for<0, 4>([&](auto ii) {
              constexpr int i = decltype(ii)::value;
              const float p1 = gr[i], p2 = gi[i];
              gr[i] = p1 - p2;
              gi[i] = (p3[i] - p1) - p2;
            });
          } else {
            static_for<0, NK>([&](auto kk) {
              constexpr int kc = decltype(kk)::value;
              if constexpr (NP == 3) {
                gr = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[kc], bh[p][kc], gr, 0, 0, 0);
                gi = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[kc], bh[4 + p][kc], gi, 0, 0, 0);
                gr = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[kc], bl[p][kc], gr, 0, 0, 0);
                gi = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[kc], bl[4 + p][kc], gi, 0, 0, 0);
              }
              gr = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[kc], bh[p][kc], gr, 0, 0, 0);
              gi = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[kc], bh[4 + p][kc], gi, 0, 0, 0);
            });
          }
          static_for<0, 4>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            const float v = gr[i] * gr[i] + gi[i] * gi[i];
            const unsigned key = (__float_as_uint(v) & 0xFFFFFFF0u) | unsigned(15 - (p * 4 + i));
            kmax = kmax > key ? kmax : key;
            if constexpr (DUMP) {
              const int arow_i = 16 * sb + 4 * (lane >> 4) + i;
              const int s = (c + P * arow_i + (PJ >> 1)) & (PJ - 1);
              const int m = (16 * (4 * wave + p) + (lane & 15) + (M >> 1)) & (M - 1);
              a.dump[(r * PJ + s) * M + m] = v / (scale * scale);
            }
          });
        });
        const float bv = __uint_as_float(kmax & 0xFFFFFFF0u);
        if (bv > best_v) {
          best_v = bv;
          best_key = kmax;
          best_blk = (r * P + c) * NSB + sb;
        }
      }
    }
  }
  // packed index of this lane's best cell
  if (best_v >= 0.0f) {
    const int slot = 15 - int(best_key & 15u);
    const int p = slot >> 2, i = slot & 3;
    const int sb = best_blk % NSB, rc = best_blk / NSB;
    const int c = rc % P, r = rc / P;
    const int arow_i = 16 * sb + 4 * (lane >> 4) + i;
    const int s = (c + P * arow_i + (PJ >> 1)) & (PJ - 1);
    const int m = (16 * (4 * wave + p) + (lane & 15) + (M >> 1)) & (M - 1);
    best_i = (r * PJ + s) * M + m;
  }

  for (int off = 32; off > 0; off >>= 1) {
    const float ov = __shfl_xor(best_v, off, 64);
    const int32_t oi = __shfl_xor(best_i, off, 64);
    if (ov > best_v || (ov == best_v && oi < best_i)) {
      best_v = ov;
      best_i = oi;
    }
  }
  if (lane == 0) {
    red_v[wave] = best_v;
    red_i[wave] = best_i;
  }
  __syncthreads();
  if (t == 0 && !DUMP) {
    float bv = red_v[0];
    int32_t bi = red_i[0];
    for (int w = 1; w < kBlock / 64; ++w) {
      if (red_v[w] > bv || (red_v[w] == bv && red_i[w] < bi)) {
        bv = red_v[w];
        bi = red_i[w];
      }
    }
    const int64_t o = int64_t(dl) * a.seg_total + seg;
    a.power[o] = bv >= 0.0f ? sqrtf(bv) / scale : __builtin_nanf("");
    a.pidx[o] = bv >= 0.0f ? bi : -1;
  }
}

// ------------------------------------- matrix-core fringe kernel, GEMM SBD
// The float16 form with both transforms of Eq. 5 on the matrix cores, eight
// waves per segment.
//   SBD (Sec. 5.1, f_j term): for each of the P sub-grids c of the
//   zero-padded transform (bins s' = c + P a), the J-point DFT over the
//   frequency points of the rotated, scaled segment sums,
//     X_c[a][n] = sum_j w_J^{j a} (w_PJ^{j c} scale Y(n, j)),
//   as a real-embedded GEMM: the constant DFT matrix is the A operand (rows
//   (a, Re/Im), K = (j, Re/Im), held in registers), the sums the B operand
//   (columns n, staged in LDS as float16).  One v_mfma_f32_16x16x32_f16 per
//   16 rows x 16 IFs x 32 K.
//   MBD (f0^n term): as in fringe_mfma_kernel, with each wave owning 32 MBD
//   columns (two Re and two Im tiles of the constant B operand).
// The SBD output goes from the accumulators to float16 A-operand rows of
// the MBD GEMM in LDS.  The sub-grids are taken `batch` at a time (as many
// as keep the LDS plan near 76 KiB, two work-groups per CU): two barriers per
// (rate, batch).
template <int J, int NK>
__host__ __device__ inline int gemm_batch(int sbd_pad) {
  constexpr int YB = 16 * NK * (2 * J + 8) * 2;   // bytes of one sub-grid's sums
  constexpr int AB = J * (32 * NK + 8) * 2;       // bytes of one sub-grid's MBD A rows
  int pb = sbd_pad;
  while (pb > 1 && sbd_pad * J * 8 + pb * (YB + AB) > 76 * 1024) pb >>= 1;
  return pb;
}

template <int J, int NK>
__host__ __device__ inline void gemm_lds_plan(int sbd_pad, int &y_off, int &a_off, int &total_bytes) {
  constexpr int YS = 2 * J + 8;     // sums row stride in halves (+16 B against bank conflicts)
  constexpr int AS = 32 * NK + 8;   // MBD A row stride in halves
  const int pb = gemm_batch<J, NK>(sbd_pad);
  y_off = sbd_pad * J * 8;          // after the scaled twiddles [PJ] float2
  a_off = y_off + pb * 16 * NK * YS * 2;
  total_bytes = a_off + pb * J * AS * 2;
}

template <int J, int NK, bool DUMP>
__global__ __launch_bounds__(kBlockGemm) void fringe_gemm_kernel(FringeArgs a) {
  constexpr int M = 256;
  constexpr int YS = 2 * J + 8, AS = 32 * NK + 8;
  constexpr int KC = J / 16;                  // 32-K chunks of the SBD GEMM (K = 2J)
  constexpr int SRT = 2 * J / 16;             // 16-row tiles of the SBD output (a, Re/Im)
  constexpr int RT = (SRT + 7) / 8;           // SBD row tiles per wave
  constexpr int JB = 16, JA = J / 16;         // segment-sum lanes: 16 per IF, J / 16 channels each
  constexpr int NW = kBlockGemm / 64;
  constexpr int YSUB = 16 * NK * YS, ASUB = J * AS;
  constexpr int NU = J / 16;                    // 16-row units of the MBD GEMM per sub-grid
  constexpr int CPU = 8;                        // cells per lane per unit
  extern __shared__ float2 lds[];
  __shared__ float red_v[NW];
  __shared__ int32_t red_i[NW];

  const int N = a.n_if, R = a.n_rate, P = a.sbd_pad;
  const int PJ = P * J;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;

  int dl, seg;
  block_segment(a, DUMP, dl, seg);
  int wi = 0;
  while (wi + 1 < a.n_win && a.win_off[wi + 1] <= seg) ++wi;
  const int l = a.win_len[wi];
  const int q = seg - a.win_off[wi];
  const int64_t k0 = a.win_k0[wi] + int64_t(q) * a.win_hop[wi];
  const float2 *wd = a.w + int64_t(dl) * a.w_dm_stride + k0 * (N * J);
  const float2 *rph = a.rate_ph + a.rate_off[wi];

  int y_off, a_off, total;
  gemm_lds_plan<J, NK>(P, y_off, a_off, total);
  const int PB = gemm_batch<J, NK>(P);   // sub-grids per batch
  float2 *TWs = lds;
  _Float16 *Yl = reinterpret_cast<_Float16 *>(reinterpret_cast<char *>(lds) + y_off);
  _Float16 *Am = reinterpret_cast<_Float16 *>(reinterpret_cast<char *>(lds) + a_off);
  const float scale = a.mfma_scale;
  for (int i = t; i < PJ; i += kBlockGemm) {
    const float2 w = a.tw_sbd[i];
    TWs[i] = make_float2(w.x * scale, w.y * scale);   // exact: scale is a power of two
  }
  // rows of IFs n >= N stay zero (K padding of the MBD GEMM, columns of the SBD GEMM)
  for (int i = t; i < PB * YSUB; i += kBlockGemm) Yl[i] = _Float16(0.0f);

  // constant operands, in registers for the kernel's life
  h8_t fa[RT][KC];
  {
    const h8_t *src = static_cast<const h8_t *>(a.sbd_a);
    static_for<0, RT>([&](auto kk) {
      constexpr int k = decltype(kk)::value;
      const int rt = wave + NW * k;
      static_for<0, KC>([&](auto cc) {
        constexpr int kc = decltype(cc)::value;
        if (rt < SRT) fa[k][kc] = src[(rt * KC + kc) * 64 + lane];
      });
    });
  }
  h8_t bm[4][NK];   // MBD: Re tiles 2 wave + {0, 1}, Im tiles 16 + 2 wave + {0, 1}
  {
    const h8_t *src = static_cast<const h8_t *>(a.mfma_b_hi);
    static_for<0, 4>([&](auto pp) {
      constexpr int p = decltype(pp)::value;
      const int tile = p < 2 ? 2 * wave + p : 16 + 2 * wave + (p - 2);
      static_for<0, NK>([&](auto cc) {
        constexpr int kc = decltype(cc)::value;
        bm[p][kc] = src[(tile * NK + kc) * 64 + lane];
      });
    });
  }

  // segment-sum lanes: IF n1, channels j = 16 i + i2 (i < J / 16)
  const bool s_act = t < N * JB;
  const int n1 = t / JB, i2 = t % JB;
  float2 y[JA];

  // B operands of the SBD GEMM for sub-grids c0 .. c0 + nb - 1:
  // w_PJ^{j c} scale Y(n, j) as float16
  auto sbd_operands = [&](int c0, int nb) {
    if (!s_act) return;
    for (int cb = 0; cb < nb; ++cb) {
      const int c = c0 + cb;
      _Float16 *Y = Yl + cb * YSUB;
      static_for<0, JA>([&](auto i) {
        constexpr int ii = decltype(i)::value;
        const int j = JB * ii + i2;
        const float2 z = cmul(y[ii], TWs[j * c]);
        h2_t h;
        h.x = _Float16(z.x);
        h.y = _Float16(z.y);
        *reinterpret_cast<h2_t *>(Y + n1 * YS + 2 * j) = h;
      });
    }
  };
  // SBD GEMM of nb sub-grids: rows (a, Re/Im) of this wave's tiles, columns n
  // -> float16 A rows of the MBD GEMM
  auto sbd_gemm = [&](int nb) {
    for (int cb = 0; cb < nb; ++cb) {
      const _Float16 *Y = Yl + cb * YSUB;
      _Float16 *A = Am + cb * ASUB;
      static_for<0, RT>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        const int rt = wave + NW * k;
        if (rt < SRT) {
          static_for<0, NK>([&](auto ct) {
            constexpr int cn = decltype(ct)::value;
            h8_t bb[KC];
            static_for<0, KC>([&](auto cc) {
              constexpr int kc = decltype(cc)::value;
              bb[kc] = *reinterpret_cast<const h8_t *>(Y + (16 * cn + (lane & 15)) * YS + 32 * kc +
                                                       8 * (lane >> 4));
            });
            f4_t x = {0.f, 0.f, 0.f, 0.f};
            static_for<0, KC>([&](auto cc) {
              constexpr int kc = decltype(cc)::value;
              x = __builtin_amdgcn_mfma_f32_16x16x32_f16(fa[k][kc], bb[kc], x, 0, 0, 0);
            });
            // rows 16 rt + 4 (lane / 16) + i: Re, Im of bins a0 and a0 + 1
            const int n = 16 * cn + (lane & 15);
            const int a0 = 8 * rt + 2 * (lane >> 4);
            h2_t h0, h1;
            h0.x = _Float16(x[0]);
            h0.y = _Float16(x[1]);
            h1.x = _Float16(x[2]);
            h1.y = _Float16(x[3]);
            *reinterpret_cast<h2_t *>(A + a0 * AS + 2 * n) = h0;
            *reinterpret_cast<h2_t *>(A + (a0 + 1) * AS + 2 * n) = h1;
          });
        }
      });
    }
  };
  // MBD GEMM of the 16 SBD rows of unit u of sub-grid buffer cb: Re and Im
  // of this wave's 32 MBD columns for the lane's CPU cells (slot 4 p + i:
  // column tile p, accumulator row i)
  auto mbd_unit = [&](int cb, int u, float (&gre)[CPU], float (&gim)[CPU]) {
    const _Float16 *A = Am + cb * ASUB;
    h8_t ah[NK];
    const int arow = (16 * u + (lane & 15)) * AS + 8 * (lane >> 4);
    static_for<0, NK>([&](auto cc) {
      constexpr int kc = decltype(cc)::value;
      ah[kc] = *reinterpret_cast<const h8_t *>(A + arow + 32 * kc);
    });
    static_for<0, 2>([&](auto pp) {
      constexpr int p = decltype(pp)::value;
      f4_t gr = {0.f, 0.f, 0.f, 0.f}, gi = {0.f, 0.f, 0.f, 0.f};
      static_for<0, NK>([&](auto cc) {
        constexpr int kc = decltype(cc)::value;
        gr = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[kc], bm[p][kc], gr, 0, 0, 0);
        gi = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[kc], bm[2 + p][kc], gi, 0, 0, 0);
      });
      static_for<0, 4>([&](auto ii) {
        constexpr int q4 = decltype(ii)::value;
        gre[4 * p + q4] = gr[q4];
        gim[4 * p + q4] = gi[q4];
      });
    });
  };
  // packed index of cell `slot` of the lane in unit u of sub-grid c, rate r
  auto cell_index = [&](int r, int c, int u, int slot) {
    const int arow_i = 16 * u + 4 * (lane >> 4) + (slot & 3);
    const int m = 16 * (2 * wave + (slot >> 2)) + (lane & 15);
    const int s = (c + P * arow_i + (PJ >> 1)) & (PJ - 1);
    return (r * PJ + s) * M + ((m + (M >> 1)) & (M - 1));
  };

  // ---- the search: per lane, the largest |G|^2 (as float bits: |G|^2 >= 0
  // orders like its bits, and a NaN cell outranks every number and is then
  // refused below) over each (rate, sub-grid), and the (rate, sub-grid) that
  // holds it; the cell itself is found again at the end.
  float best_v = -1.0f;
  int best_rc = 0x7fffffff;
  for (int r = 0; r < R; ++r) {
    // Eq. 3 segment sum with the Eq. 4 rate rotation (j = 0 not fitted)
    segment_sum<JA, JB>(y, wd, rph, r, N, J, l, R, s_act, n1, i2);
    for (int c0 = 0; c0 < P; c0 += PB) {
      sbd_operands(c0, PB);
      __syncthreads();
      sbd_gemm(PB);
      __syncthreads();
      for (int cb = 0; cb < PB; ++cb) {
        const int c = c0 + cb;
        unsigned m = 0u;
        static_for<0, NU>([&](auto uu) {
          constexpr int u = decltype(uu)::value;
          float gre[CPU], gim[CPU];
          mbd_unit(cb, u, gre, gim);
          unsigned bits[CPU];
          static_for<0, CPU>([&](auto e) {
            constexpr int k = decltype(e)::value;
            const float v = __builtin_fmaf(gim[k], gim[k], gre[k] * gre[k]);
            bits[k] = __float_as_uint(v);
            if constexpr (DUMP) a.dump[cell_index(r, c, u, k)] = v / (scale * scale);
          });
          static_for<0, CPU / 2>([&](auto e) {
            constexpr int k = decltype(e)::value;
            m = max(m, max(bits[2 * k], bits[2 * k + 1]));
          });
        });
        const float bv = __uint_as_float(m);
        if (bv > best_v) {
          best_v = bv;
          best_rc = r * P + c;
        }
      }
    }
  }
  if constexpr (DUMP) return;

  // ---- block maximum and its (rate, sub-grid): larger value, then lower
  // (rate, sub-grid)
  for (int off = 32; off > 0; off >>= 1) {
    const float ov = __shfl_xor(best_v, off, 64);
    const int orc = __shfl_xor(best_rc, off, 64);
    if (ov > best_v || (ov == best_v && orc < best_rc)) {
      best_v = ov;
      best_rc = orc;
    }
  }
  if (lane == 0) {
    red_v[wave] = best_v;
    red_i[wave] = best_rc;
  }
  __syncthreads();
  float vmax = red_v[0];
  int rc = red_i[0];
  for (int w = 1; w < NW; ++w) {
    if (red_v[w] > vmax || (red_v[w] == vmax && red_i[w] < rc)) {
      vmax = red_v[w];
      rc = red_i[w];
    }
  }
  const int64_t o = int64_t(dl) * a.seg_total + seg;
  if (!(vmax >= 0.0f)) {   // no finite cell (non-finite input)
    if (t == 0) {
      a.power[o] = __builtin_nanf("");
      a.pidx[o] = -1;
    }
    return;
  }
  // ---- find the cell: the (rate, sub-grid) that holds the maximum is
  // searched again with the same arithmetic, keeping the lowest packed
  // index among the largest cells (keys: |G|^2 with the 4 lowest mantissa
  // bits replaced by 15 - slot)
  const int r = rc / P, c = rc % P;
  segment_sum<JA, JB>(y, wd, rph, r, N, J, l, R, s_act, n1, i2);
  __syncthreads();   // the red_* reads above are done before they are reused
  sbd_operands(c, 1);
  __syncthreads();
  sbd_gemm(1);
  __syncthreads();
  float fv = -1.0f;
  int32_t fi = 0x7fffffff;
  static_for<0, NU>([&](auto uu) {
    constexpr int u = decltype(uu)::value;
    float gre[CPU], gim[CPU];
    mbd_unit(0, u, gre, gim);
    static_for<0, CPU>([&](auto e) {
      constexpr int k = decltype(e)::value;
      const float v = __builtin_fmaf(gim[k], gim[k], gre[k] * gre[k]);   // as in the scan
      const int32_t ci = cell_index(r, c, u, k);
      if (v > fv || (v == fv && ci < fi)) {
        fv = v;
        fi = ci;
      }
    });
  });
  for (int off = 32; off > 0; off >>= 1) {
    const float ov = __shfl_xor(fv, off, 64);
    const int32_t oi = __shfl_xor(fi, off, 64);
    if (ov > fv || (ov == fv && oi < fi)) {
      fv = ov;
      fi = oi;
    }
  }
  if (lane == 0) {
    red_v[wave] = fv;
    red_i[wave] = fi;
  }
  __syncthreads();
  if (t == 0) {
    float bv = red_v[0];
    int32_t bi = red_i[0];
    for (int w = 1; w < NW; ++w) {
      if (red_v[w] > bv || (red_v[w] == bv && red_i[w] < bi)) {
        bv = red_v[w];
        bi = red_i[w];
      }
    }
    a.power[o] = bv >= 0.0f ? sqrtf(bv) / scale : __builtin_nanf("");
    a.pidx[o] = bv >= 0.0f ? bi : -1;
  }
}

__global__ __launch_bounds__(kBlock) void cube_sum_kernel(const float *power, int64_t bl_stride,
                                                          const int32_t *bl, int n_bl, float *out,
                                                          int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock) {
    float acc = 0.f;
    for (int b = 0; b < n_bl; ++b) acc += power[int64_t(bl[b]) * bl_stride + i];
    out[i] = acc;
  }
}

// one wave per channel: lanes stride the APs, then a wave reduction
__global__ __launch_bounds__(kBlock) void segment_sum_kernel(const void *vis, int in_f16,
                                                             int64_t n_frames, int n_ch, int64_t k0,
                                                             int len, float2 *out) {
  const int c = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= n_ch) return;
  float2 acc = make_float2(0.f, 0.f);
  for (int u = lane; u < len; u += 64) acc = cadd(acc, load_vis(vis, int64_t(c) * n_frames + k0 + u, in_f16 != 0));
  for (int off = 32; off > 0; off >>= 1) {
    acc.x += __shfl_xor(acc.x, off, 64);
    acc.y += __shfl_xor(acc.y, off, 64);
  }
  if (lane == 0) out[c] = acc;
}

// OCP FP8 e4m3 (e4m3fn): sign, 4-bit exponent (bias 7), 3-bit mantissa, no
// infinities, 0x7f / 0xff are NaN; decoded exactly into float32.
__device__ __forceinline__ float fp8_e4m3(unsigned b) {
  const unsigned e = (b >> 3) & 15u, m = b & 7u;
  float v;
  if (e == 15u && m == 7u) v = __builtin_nanf("");
  else if (e == 0u) v = float(m) * 0.001953125f;           // m 2^-9
  else v = __uint_as_float(((e + 120u) << 23) | (m << 20));  // (1 + m/8) 2^(e-7)
  return (b & 128u) ? -v : v;
}

__global__ __launch_bounds__(kBlock) void ingest_kernel(const void *src, int kind, const float *scale,
                                                        int64_t n_frames, int n_ch, float2 *dst,
                                                        int64_t dst_frames, int64_t k0) {
  for (int c = blockIdx.y; c < n_ch; c += gridDim.y) {
    const float sc = kind == 2 ? scale[c] : 1.0f;
    float2 *d = dst + int64_t(c) * dst_frames + k0;
    for (int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x; k < n_frames;
         k += int64_t(gridDim.x) * kBlock) {
      const int64_t i = int64_t(c) * n_frames + k;
      float2 v;
      if (kind == 2) {
        const unsigned short w = static_cast<const unsigned short *>(src)[i];
        v = make_float2(fp8_e4m3(w & 255u) * sc, fp8_e4m3(w >> 8) * sc);
      } else {
        v = load_vis(src, i, kind == 1);
      }
      d[k] = v;
    }
  }
}

__global__ __launch_bounds__(kBlock) void carry_kernel(const float2 *src, float2 *dst, int n_ch, int64_t frames,
                                                       int64_t from, int64_t n) {
  for (int c = blockIdx.y; c < n_ch; c += gridDim.y) {
    const float2 *s = src + int64_t(c) * frames + from;
    float2 *d = dst + int64_t(c) * frames;
    for (int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x; k < n; k += int64_t(gridDim.x) * kBlock)
      d[k] = s[k];
  }
}

__global__ __launch_bounds__(kBlock) void absmax_kernel(const void *vis, int64_t n, int in_f16,
                                                        unsigned int *out) {
  float m = 0.f;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock) {
    const float2 v = load_vis(vis, i, in_f16 != 0);
    m = fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y)));
  }
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

// ------------------------------------------------------- refinement kernel
// exp(-2 pi i x) for x in cycles, reduced in float64 before the float sincos
__device__ __forceinline__ float2 cis_neg(double x) {
  const float f = float(x - rint(x));
  float sn, cs;
  sincospif(2.0f * f, &sn, &cs);
  return make_float2(cs, -sn);
}

// Keys cubic (a = -1/2) weights of the samples at -1, 0, 1, 2 for a point at
// fraction al of the way from sample 0 to sample 1, and (D >= 1) their first
// and (D >= 2) second derivatives with respect to the position.
template <int D>
__device__ __forceinline__ void keys_weights(float al, float (&w)[4], float (&w1)[4], float (&w2)[4]) {
  const float a2 = al * al, a3 = a2 * al;
  w[0] = 0.5f * (-a3 + 2.f * a2 - al);
  w[1] = 0.5f * (3.f * a3 - 5.f * a2 + 2.f);
  w[2] = 0.5f * (-3.f * a3 + 4.f * a2 + al);
  w[3] = 0.5f * (a3 - a2);
  if constexpr (D >= 1) {
    w1[0] = 0.5f * (-3.f * a2 + 4.f * al - 1.f);
    w1[1] = 0.5f * (9.f * a2 - 10.f * al);
    w1[2] = 0.5f * (-9.f * a2 + 8.f * al + 1.f);
    w1[3] = 0.5f * (3.f * a2 - 2.f * al);
  }
  if constexpr (D >= 2) {
    w2[0] = -3.f * al + 2.f;
    w2[1] = 9.f * al - 5.f;
    w2[2] = -9.f * al + 4.f;
    w2[3] = 3.f * al - 1.f;
  }
}

__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cfma(float2 acc, float2 a, float w) {
  return make_float2(fmaf(a.x, w, acc.x), fmaf(a.y, w, acc.y));
}

// One work-group per peak.  Every thread walks channels c = tid + 256 i,
// forms the rate-rotated window sum of the interpolated frames (and the
// derivative sums the mode needs), rotates by the delay phase and the
// calibration, and accumulates; a block reduction gives G and its
// derivatives, from which thread 0 writes the mode's output.
template <int MODE>
__global__ __launch_bounds__(kBlock) void refine_kernel(RefineArgs a) {
  constexpr int D = (MODE == kRefineForward || MODE == kRefineFinal) ? 0 : MODE == kRefineBackward ? 1 : 2;
  constexpr int NA = D == 0 ? 1 : D == 1 ? 6 : 12;
  const int p = blockIdx.x;
  const RefineSeg sg = a.seg[p];
  const double ts = a.theta[5 * p + 0], tm = a.theta[5 * p + 1], rho = a.theta[5 * p + 2];
  const double dm = a.theta[5 * p + 3], toff = a.theta[5 * p + 4];
  const int l = sg.l;
  const float uc = 0.5f * float(l - 1);
  const size_t esz = a.in_f16 ? 4 : 8;
  const void *vb = static_cast<const char *>(a.vis) + size_t(sg.b) * size_t(a.nj) * size_t(a.row_stride) * esz;
  const float2 *calb = a.cal + size_t(sg.b) * a.nj;
  float2 acc[NA];
  for (int i = 0; i < NA; ++i) acc[i] = make_float2(0.f, 0.f);

  for (int c = threadIdx.x; c < a.nj; c += kBlock) {
    if (c % a.J == 0) continue;  // the DC point is not fitted
    const RefineChan ch = a.chan[c];
    double pos = double(sg.k0) + toff + ch.dxd * dm;
    pos = fmin(fmax(pos, -8.0), double(a.n_frames) + 8.0);  // also maps NaN into range
    const double fl = floor(pos);
    const int64_t i0 = int64_t(fl) - 1;
    float w[4], w1[4], w2[4];
    keys_weights<D>(float(pos - fl), w, w1, w2);
    float2 S0 = make_float2(0.f, 0.f), S1 = S0, S11 = S0, S2 = S0, S3 = S0;
    const int64_t rowoff = int64_t(c) * a.row_stride;
    for (int u = 0; u < l; ++u) {
      const float du = float(u) - uc;
      const float2 r = cis_neg(rho * ch.wr * double(du));
      float2 val = make_float2(0.f, 0.f), d1 = val, d2 = val;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int64_t k = i0 + u + m;
        const float2 v = (k >= 0 && k < a.n_frames) ? load_vis(vb, rowoff + k, a.in_f16 != 0) : make_float2(0.f, 0.f);
        val = cfma(val, v, w[m]);
        if constexpr (D >= 1) d1 = cfma(d1, v, w1[m]);
        if constexpr (D >= 2) d2 = cfma(d2, v, w2[m]);
      }
      const float2 rv = cmul(r, val);
      S0 = cadd(S0, rv);
      if constexpr (D >= 1) {
        S1 = cfma(S1, rv, du);
        S2 = cadd(S2, cmul(r, d1));
      }
      if constexpr (D >= 2) {
        S11 = cfma(S11, rv, du * du);
        S3 = cadd(S3, cmul(r, d2));
      }
    }
    const float2 e = cmul(calb[c], cis_neg(ch.fj * ts + ch.fm * tm));
    const float2 term = cmul(e, S0);
    acc[0] = cadd(acc[0], term);
    if constexpr (D >= 1) {
      const float fj = float(ch.fj), fm = float(ch.fm), wr = float(ch.wr), dx = float(ch.dxd);
      const float2 eS2 = cmul(e, S2);
      acc[1] = cfma(acc[1], term, fj);
      acc[2] = cfma(acc[2], term, fm);
      acc[3] = cfma(acc[3], cmul(e, S1), wr);
      acc[4] = cfma(acc[4], eS2, dx);
      acc[5] = cadd(acc[5], eS2);
      if constexpr (D >= 2) {
        const float2 eS3 = cmul(e, S3);
        acc[6] = cfma(acc[6], term, fj * fj);
        acc[7] = cfma(acc[7], term, fm * fm);
        acc[8] = cfma(acc[8], cmul(e, S11), wr * wr);
        acc[9] = cfma(acc[9], eS3, dx * dx);
        acc[10] = cadd(acc[10], eS3);
        acc[11] = cfma(acc[11], eS3, dx);
      }
    }
  }

  // block reduction: wave shuffles, then one LDS row per wave
  __shared__ float2 red[kBlock / 64][NA];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    float2 v = acc[i];
    for (int off = 32; off > 0; off >>= 1) {
      v.x += __shfl_xor(v.x, off, 64);
      v.y += __shfl_xor(v.y, off, 64);
    }
    if (lane == 0) red[wv][i] = v;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double gr[NA], gi[NA];
  for (int i = 0; i < NA; ++i) {
    gr[i] = 0.0;
    gi[i] = 0.0;
    for (int k = 0; k < kBlock / 64; ++k) {
      gr[i] += double(red[k][i].x);
      gi[i] += double(red[k][i].y);
    }
  }
  const double P = sqrt(gr[0] * gr[0] + gi[0] * gi[0]);
  if constexpr (MODE == kRefineForward) {
    a.power[p] = float(P);
  } else if constexpr (MODE == kRefineFinal) {
    // the better of the last point and the best one
    const float Pf = float(P);
    if (Pf < a.p_best[p]) {
      for (int k = 0; k < 5; ++k) a.theta[5 * p + k] = a.theta_best[5 * p + k];
      a.power[p] = a.p_best[p];
    } else {
      a.power[p] = Pf;
    }
  } else {
    const double tp = 2.0 * M_PI, tp2 = tp * tp;
    // first derivatives: dG/dtau_s = -2 pi i sum f_j term, likewise MBD and rate
    double dr[5], di[5];
    for (int k = 0; k < 3; ++k) {
      dr[k] = tp * gi[1 + k];
      di[k] = -tp * gr[1 + k];
    }
    dr[3] = gr[4]; di[3] = gi[4];
    dr[4] = gr[5]; di[4] = gi[5];
    double g[5];
    for (int k = 0; k < 5; ++k) g[k] = P > 0.0 ? (gr[0] * dr[k] + gi[0] * di[k]) / P : 0.0;
    if constexpr (MODE == kRefineBackward) {
      const double up = double(a.grad_power[p]);
      for (int k = 0; k < 5; ++k) a.grad_theta[5 * p + k] = up * g[k];
    } else {
      double h[6] = {0, 0, 0, 0, 0, 0};
      if (P > 0.0) {
        double sr[6], si[6];
        for (int k = 0; k < 3; ++k) {  // (-2 pi i)^2 = -4 pi^2
          sr[k] = -tp2 * gr[6 + k];
          si[k] = -tp2 * gi[6 + k];
        }
        for (int k = 3; k < 6; ++k) {
          sr[k] = gr[6 + k];
          si[k] = gi[6 + k];
        }
        for (int k = 0; k < 5; ++k)
          h[k] = (dr[k] * dr[k] + di[k] * di[k] + gr[0] * sr[k] + gi[0] * si[k]) / P - g[k] * g[k] / P;
        h[5] = (dr[3] * dr[4] + di[3] * di[4] + gr[0] * sr[5] + gi[0] * si[5]) / P - g[3] * g[4] / P;
      }
      if constexpr (MODE == kRefineCurvature) {
        for (int k = 0; k < 6; ++k) a.curv[6 * p + k] = h[k];
      } else {
        // trust-region Newton ascent in grid cells (the DM coordinate carries
        // the arrival offset along, dm_t offset cells per DM cell): a point
        // that does not lower |G| below the best so far becomes the best, with
        // its proposed move (-g/H where the curvature is negative, else
        // max_step along the gradient) and a doubled radius; otherwise the
        // radius is halved.  The best point's move is then taken, clipped to
        // the radius.
        const double *c = a.cells;
        const double at = a.dm_t;
        const float Pf = float(P);
        double *tb = a.theta_best + 5 * p, *sb = a.step_best + 5 * p;
        double rad = a.radius[p];
        if (Pf >= a.p_best[p]) {
          double gz[5], hz[5];
          for (int k = 0; k < 5; ++k) {
            gz[k] = g[k] * c[k];
            hz[k] = h[k] * c[k] * c[k];
          }
          gz[3] += at * g[4] * c[4];
          hz[3] += 2.0 * at * h[5] * c[3] * c[4] + at * at * h[4] * c[4] * c[4];
          for (int k = 0; k < 5; ++k) {
            double s = hz[k] < 0.0 ? -gz[k] / hz[k] : a.max_step * double((gz[k] > 0.0) - (gz[k] < 0.0));
            s = fmin(fmax(s, -a.max_step), a.max_step);
            sb[k] = c[k] > 0.0 ? s : 0.0;
            tb[k] = a.theta[5 * p + k];
          }
          a.p_best[p] = Pf;
          rad = fmin(a.max_step, 2.0 * rad);
        } else {
          rad *= 0.5;
        }
        a.radius[p] = rad;
        double st[5];
        for (int k = 0; k < 5; ++k) st[k] = fmin(fmax(sb[k], -rad), rad);
        st[4] += at * st[3];
        for (int k = 0; k < 5; ++k) a.theta[5 * p + k] = tb[k] + c[k] * st[k];
        a.power[p] = float(P);
      }
    }
  }
}

}  // namespace

// ---------------------------------------------------------------- launchers
hipError_t launch_dedisperse(const DedisperseArgs &a, hipStream_t s) {
  (void)hipGetLastError();
  if (a.group < 1 || a.group > kDedispMaxGroup) return hipErrorInvalidValue;
  dim3 grid(unsigned((a.k_eff + kDedispAp - 1) / kDedispAp), unsigned((a.nj + kDedispCh - 1) / kDedispCh),
            unsigned((a.n_dt + a.group - 1) / a.group));
  if (a.in_f16)
    hipLaunchKernelGGL(dedisperse_kernel<true>, grid, dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(dedisperse_kernel<false>, grid, dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <int J, int M, bool DUMP, bool CL, bool LIST = false>
static hipError_t launch_fringe_t(const FringeArgs &a, size_t lds, int grid, hipStream_t s) {
  (void)hipGetLastError();  // start from a clean error state
  if (lds > 64 * 1024) {
    const hipError_t e =
        hipFuncSetAttribute(reinterpret_cast<const void *>(&fringe_kernel<J, M, DUMP, CL, LIST>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((fringe_kernel<J, M, DUMP, CL, LIST>), dim3(grid), dim3(kBlock), lds, s, a);
  return hipGetLastError();
}

#define FRBX_FOR_M(J)                                              \
  switch (n_mbd) {                                                 \
    case 16: return fn.template operator()<J, 16>();               \
    case 32: return fn.template operator()<J, 32>();               \
    case 64: return fn.template operator()<J, 64>();               \
    case 128: return fn.template operator()<J, 128>();             \
    case 256: return fn.template operator()<J, 256>();             \
    default: return fn.fail();                                     \
  }

template <typename Fn>
static auto dispatch(int n_chan, int n_mbd, Fn &&fn) {
  switch (n_chan) {
    case 8: FRBX_FOR_M(8)
    case 16: FRBX_FOR_M(16)
    case 32: FRBX_FOR_M(32)
    case 64: FRBX_FOR_M(64)
    case 128: FRBX_FOR_M(128)
    case 256: FRBX_FOR_M(256)
    default: return fn.fail();
  }
}

struct LaunchFn {
  const FringeArgs &a;
  size_t lds;
  int grid;
  hipStream_t s;
  template <int J, int M> hipError_t operator()() {
    if (a.mbd_pos)
      return a.dump ? launch_fringe_t<J, M, true, true>(a, lds, grid, s)
                    : launch_fringe_t<J, M, false, true>(a, lds, grid, s);
    return a.dump ? launch_fringe_t<J, M, true, false>(a, lds, grid, s)
                  : launch_fringe_t<J, M, false, false>(a, lds, grid, s);
  }
  hipError_t fail() { return hipErrorInvalidValue; }
};

struct LdsFn {
  int n_if, sbd_pad;
  template <int J, int M> size_t operator()() {
    int xo, so, to, tot;
    fringe_lds_plan<J, M>(n_if, sbd_pad, xo, so, to, tot);
    return size_t(tot) * sizeof(float2);
  }
  size_t fail() { return 0; }
};

struct SupportFn {
  int n_if, sbd_pad;
  template <int J, int M> bool operator()() {
    using S = FringeShape<J, M>;
    int xo, so, to, tot;
    fringe_lds_plan<J, M>(n_if, sbd_pad, xo, so, to, tot);
    return n_if * S::JB <= kBlock && size_t(tot) * sizeof(float2) <= 150 * 1024;
  }
  bool fail() { return false; }
};

hipError_t launch_fringe(int n_chan, int n_mbd, const FringeArgs &a, size_t lds_bytes, int grid,
                         hipStream_t s) {
  return dispatch(n_chan, n_mbd, LaunchFn{a, lds_bytes, grid, s});
}

size_t fringe_lds_bytes(int n_chan, int n_mbd, int n_if, int sbd_pad) {
  return dispatch(n_chan, n_mbd, LdsFn{n_if, sbd_pad});
}

bool fringe_supported(int n_chan, int n_mbd, int n_if, int sbd_pad) {
  return dispatch(n_chan, n_mbd, SupportFn{n_if, sbd_pad});
}

template <int J>
static hipError_t launch_fringe_list_t(const FringeArgs &a, size_t lds, int n, hipStream_t s) {
  return a.mbd_pos ? launch_fringe_t<J, 256, false, true, true>(a, lds, n, s)
                   : launch_fringe_t<J, 256, false, false, true>(a, lds, n, s);
}

hipError_t launch_fringe_list(int n_chan, int n_mbd, const FringeArgs &a, size_t lds_bytes, int n,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n_mbd != 256 || !a.seg_list || n > 2147483647) return hipErrorInvalidValue;
  switch (n_chan) {
    case 16: return launch_fringe_list_t<16>(a, lds_bytes, n, s);
    case 32: return launch_fringe_list_t<32>(a, lds_bytes, n, s);
    case 64: return launch_fringe_list_t<64>(a, lds_bytes, n, s);
    case 128: return launch_fringe_list_t<128>(a, lds_bytes, n, s);
    case 256: return launch_fringe_list_t<256>(a, lds_bytes, n, s);
    default: return hipErrorInvalidValue;
  }
}

int fringe_compact_rows(int n_mbd) {
  switch (n_mbd) {
    case 16: return Split<16>::B;
    case 32: return Split<32>::B;
    case 64: return Split<64>::B;
    case 128: return Split<128>::B;
    case 256: return Split<256>::B;
    default: return 0;
  }
}

hipError_t launch_stats(const StatsArgs &a, int rows, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  (void)hipGetLastError();
  hipLaunchKernelGGL(stats_kernel, dim3(rows), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}


template <int J, int NK, int NP>
static hipError_t launch_mfma_t(const FringeArgs &a, size_t lds, int grid, hipStream_t s) {
  (void)hipGetLastError();
  if (a.dump) {
    if (lds > 64 * 1024) {
      const hipError_t e = hipFuncSetAttribute(
          reinterpret_cast<const void *>(&fringe_mfma_kernel<J, NK, NP, true>),
          hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((fringe_mfma_kernel<J, NK, NP, true>), dim3(grid), dim3(kBlock), lds, s, a);
  } else {
    if (lds > 64 * 1024) {
      const hipError_t e = hipFuncSetAttribute(
          reinterpret_cast<const void *>(&fringe_mfma_kernel<J, NK, NP, false>),
          hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((fringe_mfma_kernel<J, NK, NP, false>), dim3(grid), dim3(kBlock), lds, s, a);
  }
  return hipGetLastError();
}

template <int J>
static hipError_t launch_mfma_j(int nk, int np, const FringeArgs &a, size_t lds, int grid,
                                hipStream_t s) {
  if (nk == 1) return np == 3 ? launch_mfma_t<J, 1, 3>(a, lds, grid, s) : launch_mfma_t<J, 1, 1>(a, lds, grid, s);
  if (nk == 2) return np == 3 ? launch_mfma_t<J, 2, 3>(a, lds, grid, s) : launch_mfma_t<J, 2, 1>(a, lds, grid, s);
  return hipErrorInvalidValue;
}

static int mfma_nk(int n_if) { return n_if <= 16 ? 1 : n_if <= 32 ? 2 : 0; }

hipError_t launch_fringe_mfma(int n_chan, int n_if, int n_pass, const FringeArgs &a, size_t lds,
                              int grid, hipStream_t s) {
  const int nk = mfma_nk(n_if);
  switch (n_chan) {
    case 16: return launch_mfma_j<16>(nk, n_pass, a, lds, grid, s);
    case 32: return launch_mfma_j<32>(nk, n_pass, a, lds, grid, s);
    case 64: return launch_mfma_j<64>(nk, n_pass, a, lds, grid, s);
    case 128: return launch_mfma_j<128>(nk, n_pass, a, lds, grid, s);
    case 256: return launch_mfma_j<256>(nk, n_pass, a, lds, grid, s);
    default: return hipErrorInvalidValue;
  }
}

size_t fringe_mfma_lds_bytes(int n_chan, int n_if, int sbd_pad, int n_pass) {
  int to, ao, tot;
  const int nk = mfma_nk(n_if);
  auto plan = [&](auto jc) {
    constexpr int J = decltype(jc)::value;
    if (nk == 1) mfma_lds_plan<J, 1>(n_if, sbd_pad, n_pass, to, ao, tot);
    else mfma_lds_plan<J, 2>(n_if, sbd_pad, n_pass, to, ao, tot);
  };
  switch (n_chan) {
    case 16: plan(std::integral_constant<int, 16>{}); break;
    case 32: plan(std::integral_constant<int, 32>{}); break;
    case 64: plan(std::integral_constant<int, 64>{}); break;
    case 128: plan(std::integral_constant<int, 128>{}); break;
    case 256: plan(std::integral_constant<int, 256>{}); break;
    default: return 0;
  }
  return size_t(tot);
}

bool fringe_mfma_supported(int n_chan, int n_mbd, int n_if, int sbd_pad, int n_pass) {
  if (n_mbd != 256 || (n_pass != 1 && n_pass != 3) || mfma_nk(n_if) == 0) return false;
  if (n_chan < 16 || n_chan > 256) return false;
  const int JB = n_chan >= 256 ? 16 : n_chan >= 64 ? 8 : 4;
  if (n_if * JB > kBlock) return false;
  const size_t b = fringe_mfma_lds_bytes(n_chan, n_if, sbd_pad, n_pass);
  return b > 0 && b <= 150 * 1024;
}

template <int J, int NK>
static hipError_t launch_gemm_t(const FringeArgs &a, size_t lds, int grid, hipStream_t s) {
  (void)hipGetLastError();
  auto go = [&](auto kern) -> hipError_t {
    if (lds > 64 * 1024) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlockGemm), lds, s, a);
    return hipGetLastError();
  };
  return a.dump ? go(&fringe_gemm_kernel<J, NK, true>) : go(&fringe_gemm_kernel<J, NK, false>);
}

template <int J>
static hipError_t launch_gemm_j(int nk, const FringeArgs &a, size_t lds, int grid, hipStream_t s) {
  if (nk == 1) return launch_gemm_t<J, 1>(a, lds, grid, s);
  if (nk == 2) return launch_gemm_t<J, 2>(a, lds, grid, s);
  return hipErrorInvalidValue;
}

hipError_t launch_fringe_gemm(int n_chan, int n_if, const FringeArgs &a, size_t lds, int grid,
                              hipStream_t s) {
  const int nk = mfma_nk(n_if);
  if (!a.sbd_a || n_if * 16 > kBlockGemm) return hipErrorInvalidValue;
  switch (n_chan) {
    case 16: return launch_gemm_j<16>(nk, a, lds, grid, s);
    case 32: return launch_gemm_j<32>(nk, a, lds, grid, s);
    case 64: return launch_gemm_j<64>(nk, a, lds, grid, s);
    default: return hipErrorInvalidValue;
  }
}

size_t fringe_gemm_lds_bytes(int n_chan, int n_if, int sbd_pad) {
  int yo, ao, tot;
  const int nk = mfma_nk(n_if);
  auto plan = [&](auto jc) {
    constexpr int J = decltype(jc)::value;
    if (nk == 1) gemm_lds_plan<J, 1>(sbd_pad, yo, ao, tot);
    else gemm_lds_plan<J, 2>(sbd_pad, yo, ao, tot);
  };
  switch (n_chan) {
    case 16: plan(std::integral_constant<int, 16>{}); break;
    case 32: plan(std::integral_constant<int, 32>{}); break;
    case 64: plan(std::integral_constant<int, 64>{}); break;
    default: return 0;
  }
  return size_t(tot);
}

bool fringe_gemm_supported(int n_chan, int n_mbd, int n_if, int sbd_pad) {
  if (n_mbd != 256 || mfma_nk(n_if) == 0) return false;
  // J = 128 would hold a 2 x 8-chunk DFT operand per wave (213 VGPRs, one
  // work-group per CU) and measured slower than the vector-ALU SBD
  if (n_chan != 16 && n_chan != 32 && n_chan != 64) return false;
  // 16 segment-sum lanes per IF
  if (n_if * 16 > kBlockGemm) return false;
  const size_t b = fringe_gemm_lds_bytes(n_chan, n_if, sbd_pad);
  return b > 0 && b <= 150 * 1024;
}

hipError_t launch_cube_sum(const float *power, int64_t bl_stride, const int32_t *baselines, int n_bl,
                           float *out, int64_t n, hipStream_t s) {
  (void)hipGetLastError();
  const int64_t blocks = std::min<int64_t>(8192, (n + kBlock - 1) / kBlock);
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(cube_sum_kernel, dim3(unsigned(blocks)), dim3(kBlock), 0, s, power, bl_stride,
                     baselines, n_bl, out, n);
  return hipGetLastError();
}

hipError_t launch_segment_sum(const void *vis, int in_f16, int64_t n_frames, int n_ch, int64_t k0, int len,
                              float2 *out, hipStream_t s) {
  (void)hipGetLastError();
  const int blocks = (n_ch + kBlock / 64 - 1) / (kBlock / 64);
  hipLaunchKernelGGL(segment_sum_kernel, dim3(blocks), dim3(kBlock), 0, s, vis, in_f16, n_frames, n_ch,
                     k0, len, out);
  return hipGetLastError();
}

hipError_t launch_ingest(const void *src, int src_kind, const float *scale, int64_t n_frames, int n_ch,
                         float2 *dst, int64_t dst_frames, int64_t k0, hipStream_t s) {
  (void)hipGetLastError();
  if (n_frames <= 0 || n_ch <= 0) return hipSuccess;
  const int64_t bx = std::min<int64_t>(64, (n_frames + kBlock - 1) / kBlock);
  const unsigned gy = unsigned(std::min(n_ch, 65535));   // the kernel strides over the rest
  hipLaunchKernelGGL(ingest_kernel, dim3(unsigned(bx), gy), dim3(kBlock), 0, s, src, src_kind,
                     scale, n_frames, n_ch, dst, dst_frames, k0);
  return hipGetLastError();
}

hipError_t launch_carry(const float2 *src, float2 *dst, int n_ch, int64_t frames, int64_t from, int64_t n,
                        hipStream_t s) {
  (void)hipGetLastError();
  if (n <= 0 || n_ch <= 0) return hipSuccess;
  if (src == dst) return hipErrorInvalidValue;
  const int64_t bx = std::min<int64_t>(64, (n + kBlock - 1) / kBlock);
  const unsigned gy = unsigned(std::min(n_ch, 65535));
  hipLaunchKernelGGL(carry_kernel, dim3(unsigned(bx), gy), dim3(kBlock), 0, s, src, dst, n_ch, frames,
                     from, n);
  return hipGetLastError();
}

hipError_t noalloc_workspace(int device, void **ptr) {
  static std::mutex mu;
  static void *addr[kMaxDevices] = {};
  if (!ptr || device < 0 || device >= kMaxDevices) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;   // the caller makes `device` current
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[device] = p;
  }
  *ptr = addr[device];
  return hipSuccess;
}

hipError_t launch_absmax(const void *vis, int64_t n, int in_f16, unsigned int *out, hipStream_t s) {
  (void)hipGetLastError();
  const int64_t blocks = std::min<int64_t>(4096, (n + kBlock - 1) / kBlock);
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(absmax_kernel, dim3(unsigned(blocks)), dim3(kBlock), 0, s, vis, n, in_f16, out);
  return hipGetLastError();
}

hipError_t launch_refine(int mode, const RefineArgs &a, hipStream_t s) {
  (void)hipGetLastError();
  if (a.n <= 0) return hipSuccess;
  switch (mode) {
    case kRefineForward: hipLaunchKernelGGL(refine_kernel<kRefineForward>, dim3(a.n), dim3(kBlock), 0, s, a); break;
    case kRefineBackward: hipLaunchKernelGGL(refine_kernel<kRefineBackward>, dim3(a.n), dim3(kBlock), 0, s, a); break;
    case kRefineCurvature: hipLaunchKernelGGL(refine_kernel<kRefineCurvature>, dim3(a.n), dim3(kBlock), 0, s, a); break;
    case kRefineStep: hipLaunchKernelGGL(refine_kernel<kRefineStep>, dim3(a.n), dim3(kBlock), 0, s, a); break;
    case kRefineFinal: hipLaunchKernelGGL(refine_kernel<kRefineFinal>, dim3(a.n), dim3(kBlock), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace frbx
