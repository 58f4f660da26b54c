// Device code of the float32 fringe search (Eq. 5 with the Eq. 4 rate term,
// Sec. 5.1) and the helpers it shares with the other kernels: compile-time
// twiddles, in-register DFTs (dense, and pruned to a compile-time set of
// non-zero inputs), the segment sums of Eq. 3, the SBD pass and the MBD peak.
// Included by frbx_kernels.hip and, for kernels specialised to an IF lattice
// at run time, compiled by hipRTC (which provides the HIP device environment
// itself: no runtime or standard headers then).
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "frbx_internal.h"
#endif

namespace frbx {

// ---------------------------------------------------------------- helpers
// A compile-time loop index (value usable in constant expressions).
template <int I>
struct Index {
  static constexpr int value = I;
};

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (I < N) {
    f(Index<I>{});
    static_for<I + 1, N>(f);
  }
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n >> 1); }

constexpr int bitrev(int i, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
  return r;
}

// Compile-time sine/cosine of (pi/2) * x, x in [0, 1), by Taylor series in
// double; used only for the fixed twiddles of the in-register DFTs.
constexpr double kHalfPi = 1.57079632679489661923;
constexpr double taylor_sin(double t) {
  double term = t, sum = t;
  for (int i = 1; i < 18; ++i) {
    term *= -t * t / ((2.0 * i) * (2.0 * i + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double taylor_cos(double t) {
  double term = 1.0, sum = 1.0;
  for (int i = 1; i < 18; ++i) {
    term *= -t * t / ((2.0 * i - 1.0) * (2.0 * i));
    sum += term;
  }
  return sum;
}
// exp(-2 pi i k / n) = (c, s): quadrant reduction on the integers first.
constexpr double tw_re(int k, int n) {
  k = ((k % n) + n) % n;
  const int q = (4 * k) / n;
  const double t = kHalfPi * double(4 * k - q * n) / double(n);
  const double c = taylor_cos(t), s = taylor_sin(t);
  return q == 0 ? c : q == 1 ? -s : q == 2 ? -c : s;
}
constexpr double tw_im(int k, int n) {
  k = ((k % n) + n) % n;
  const int q = (4 * k) / n;
  const double t = kHalfPi * double(4 * k - q * n) / double(n);
  const double c = taylor_cos(t), s = taylor_sin(t);
  const double sn = q == 0 ? s : q == 1 ? c : q == 2 ? -s : -c;  // sin(2 pi k / n)
  return -sn;
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// a * exp(-2 pi i K / N) with the twiddle known at compile time.
template <int K, int N>
__device__ __forceinline__ float2 twmul(float2 a) {
  constexpr int k = ((K % N) + N) % N;
  if constexpr (k == 0) {
    return a;
  } else if constexpr (4 * k == N) {
    return make_float2(a.y, -a.x);
  } else if constexpr (2 * k == N) {
    return make_float2(-a.x, -a.y);
  } else if constexpr (4 * k == 3 * N) {
    return make_float2(-a.y, a.x);
  } else {
    constexpr float c = static_cast<float>(tw_re(k, N));
    constexpr float s = static_cast<float>(tw_im(k, N));
    return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
  }
}

// In-register forward DFT of NP points, X[k] = sum_i x[i] exp(-2 pi i ik/NP):
// radix-2 decimation in frequency, natural order in and out.
template <int NP>
__device__ __forceinline__ void dft(float2 (&x)[NP]) {
  constexpr int L = ilog2(NP);
  static_for<0, L>([&](auto st) {
    constexpr int span = NP >> (decltype(st)::value + 1);
    static_for<0, NP / 2>([&](auto bi) {
      constexpr int b = decltype(bi)::value;
      constexpr int grp = b / span, pos = b % span;
      constexpr int i0 = grp * 2 * span + pos, i1 = i0 + span;
      const float2 a = x[i0], c = x[i1];
      x[i0] = cadd(a, c);
      x[i1] = twmul<pos * (NP / (2 * span)), NP>(csub(a, c));
    });
  });
  float2 y[NP];
  static_for<0, NP>([&](auto i) {
    constexpr int ii = decltype(i)::value;
    y[bitrev(ii, L)] = x[ii];
  });
  static_for<0, NP>([&](auto i) { x[decltype(i)::value] = y[decltype(i)::value]; });
}

// Inputs of the radix-2 decimation-in-frequency DFT below that can be non-
// zero before stage `stage`, given those of the input (bit i: x[i]): a
// butterfly's two outputs are zero exactly when both its inputs are.
constexpr unsigned dft_stage_mask(int np, unsigned mask, int stage) {
  for (int st = 0; st < stage; ++st) {
    const int span = np >> (st + 1);
    unsigned out = 0u;
    for (int b = 0; b < np / 2; ++b) {
      const int grp = b / span, pos = b % span;
      const int i0 = grp * 2 * span + pos, i1 = i0 + span;
      if (((mask >> i0) | (mask >> i1)) & 1u) out |= (1u << i0) | (1u << i1);
    }
    mask = out;
  }
  return mask;
}

// dft<NP> for an input that is zero outside the compile-time set MASK (bit
// i: x[i] may be non-zero; the others must hold +0): butterflies with two
// zero inputs are skipped and those with one skip the addition.  The
// results equal dft<NP>'s (adding an exact zero changes nothing but, at
// most, the sign of a zero).
template <int NP, unsigned MASK>
__device__ __forceinline__ void dft_masked(float2 (&x)[NP]) {
  constexpr int L = ilog2(NP);
  static_for<0, L>([&](auto st) {
    constexpr int stage = decltype(st)::value;
    constexpr unsigned nz = dft_stage_mask(NP, MASK, stage);
    constexpr int span = NP >> (stage + 1);
    static_for<0, NP / 2>([&](auto bi) {
      constexpr int b = decltype(bi)::value;
      constexpr int grp = b / span, pos = b % span;
      constexpr int i0 = grp * 2 * span + pos, i1 = i0 + span;
      constexpr bool z0 = !((nz >> i0) & 1u), z1 = !((nz >> i1) & 1u);
      constexpr int tk = pos * (NP / (2 * span));
      if constexpr (z0 && z1) {
        // both zero: so are both outputs
      } else if constexpr (z1) {
        x[i1] = twmul<tk, NP>(x[i0]);
      } else if constexpr (z0) {
        // x[i0] holds an exact +0: 0 - c, as in dft<NP>, keeps the product
        // and its rounding the same as the dense transform's (the compiler
        // may not fold it into a negation)
        const float2 c = x[i1];
        x[i1] = twmul<tk, NP>(csub(x[i0], c));
        x[i0] = c;
      } else {
        const float2 a = x[i0], c = x[i1];
        x[i0] = cadd(a, c);
        x[i1] = twmul<tk, NP>(csub(a, c));
      }
    });
  });
  float2 y[NP];
  static_for<0, NP>([&](auto i) {
    constexpr int ii = decltype(i)::value;
    y[bitrev(ii, L)] = x[ii];
  });
  static_for<0, NP>([&](auto i) { x[decltype(i)::value] = y[decltype(i)::value]; });
}

// Make the LDS writes of this wave visible to its other lanes before they
// read, and keep the compiler from moving LDS accesses across the point.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Size split of an F-point transform into (A in-register points of pass 1)
// x (B lanes of pass 1).
template <int F> struct Split;
template <> struct Split<8> { static constexpr int A = 4, B = 2; };
template <> struct Split<16> { static constexpr int A = 4, B = 4; };
template <> struct Split<32> { static constexpr int A = 8, B = 4; };
template <> struct Split<64> { static constexpr int A = 8, B = 8; };
template <> struct Split<128> { static constexpr int A = 16, B = 8; };
template <> struct Split<256> { static constexpr int A = 16, B = 16; };

template <int J, int M>
struct FringeShape {
  static constexpr int JA = Split<J>::A, JB = Split<J>::B;
  static constexpr int MA = Split<M>::A, MB = Split<M>::B;
  static constexpr int G = MA > MB ? MA : MB;    // lanes per MBD column group
  static constexpr int COLS = kBlock / G;        // columns per round
  static constexpr int SG = MA * MB + 16;        // float2 per group scratch
};

// LDS plan (float2 units): X tile [N+1][J+1] (rows of IFs, the last kept
// zero), or [max(N+1, MB)][J+1] in the compact form (rows of lattice
// positions, those without an IF kept zero), a scratch area shared by the
// SBD transpose and the MBD transposes, and the PJ-point SBD twiddle table.
// The host sizes the launch with the larger plan (CL = true).
template <int J, int M, bool CL = true>
__host__ __device__ inline void fringe_lds_plan(int n_if, int sbd_pad, int &x_off, int &s_off,
                                                int &t_off, int &total) {
  using S = FringeShape<J, M>;
  const int xs = J + 1;
  const int x_rows = CL && S::MB > n_if + 1 ? S::MB : n_if + 1;
  const int x_sz = x_rows * xs;
  const int t_sz = n_if * S::JA * (S::JB + 1);
  const int m_sz = S::COLS * S::SG;
  const int s_sz = t_sz > m_sz ? t_sz : m_sz;
  x_off = 0;
  s_off = x_sz;
  t_off = x_sz + s_sz;
  total = t_off + sbd_pad * J;
}


// ------------------------------------------------------- shared fringe steps
// Which segment a work-group handles.  Work-groups are dealt to the 8 XCDs
// round-robin; when the grid splits evenly, XCD x gets the contiguous range
// [x nb/8, (x+1) nb/8) so that overlapping segments share an L2.
__device__ __forceinline__ void block_segment(const FringeArgs &a, bool dump, int &dl, int &seg) {
  if (dump) {
    dl = a.dump_dl;
    seg = a.dump_seg;
    return;
  }
  const int nb = gridDim.x;
  const int bx = blockIdx.x;
  const int lb = (nb & 7) == 0 ? (bx & 7) * (nb >> 3) + (bx >> 3) : bx;
  dl = lb / a.seg_total;
  seg = lb - dl * a.seg_total;
}

// Segment sum of Eq. 3 with the Eq. 4 rate rotation about the window centre
// for rate bin r: y[i1] = sum_u ph[r][n1][u] W[k0 + u][n1][JB i1 + i2], with
// the j = 0 point excluded from the fit (Sec. 2.3).
template <int JA, int JB>
__device__ __forceinline__ void segment_sum(float2 (&y)[JA], const float2 *wd, const float2 *rph,
                                            int r, int N, int J, int l, int R, bool act, int n1,
                                            int i2s) {
  static_for<0, JA>([&](auto i) { y[decltype(i)::value] = make_float2(0.f, 0.f); });
  if (!act) return;
  const int NJ = N * J;
  const float2 *src = wd + n1 * J + i2s;
  const float2 *ph = rph + (r * N + n1) * l;
  // (the rate test inside the AP loop: with it outside, the compiler issues
  // the loads of an AP one at a time, each waited for)
  for (int u = 0; u < l; ++u) {
    if (R > 1) {
      const float2 p = ph[u];
      static_for<0, JA>([&](auto i) {
        constexpr int ii = decltype(i)::value;
        const float2 v = src[int64_t(u) * NJ + JB * ii];
        y[ii] = cadd(y[ii], cmul(v, p));
      });
    } else {
      static_for<0, JA>([&](auto i) {
        constexpr int ii = decltype(i)::value;
        y[ii] = cadd(y[ii], src[int64_t(u) * NJ + JB * ii]);
      });
    }
  }
  if (i2s == 0) y[0] = make_float2(0.f, 0.f);
}

// SBD pass 1 of tile c: x[i1] = y[i1] w_{P JA}^{i1 c}; JA-point DFT over i1;
// twiddle w_PJ^{i2 (c + P k1)}; store transposed T[n][k1][i2].
__device__ __forceinline__ float2 load_vis(const void *p, int64_t i, bool f16) {
  if (f16) {
    const _Float16 *h = static_cast<const _Float16 *>(p) + 2 * i;
    return make_float2(float(h[0]), float(h[1]));
  }
  return static_cast<const float2 *>(p)[i];
}

// The same segment sum gathered straight from the input of baseline b at DM
// trial d: W[k][c] = cal[c] V[c][k + dk[d][c]] (zero past the last AP),
// formed and accumulated in the same order as the dedispersed path.
template <int JA, int JB>
__device__ __forceinline__ void segment_sum_direct(float2 (&y)[JA], const FringeArgs &a, int b, int d,
                                                   int64_t k0, const float2 *rph, int r, int N, int J,
                                                   int l, int R, bool act, int n1, int i2s) {
  static_for<0, JA>([&](auto i) { y[decltype(i)::value] = make_float2(0.f, 0.f); });
  if (!act) return;
  const int NJ = N * J;
  const float2 *ph = rph + (r * N + n1) * l;
  static_for<0, JA>([&](auto i) {
    constexpr int ii = decltype(i)::value;
    const int c = n1 * J + JB * ii + i2s;
    const float2 cal = a.cal[int64_t(b) * NJ + c];
    const int64_t row = (int64_t(b) * NJ + c) * a.vis_stride;
    const int64_t f0 = k0 + a.dk[int64_t(d) * NJ + c];
    for (int u = 0; u < l; ++u) {
      const int64_t f = f0 + u;
      const float2 v = f < a.vis_frames ? load_vis(a.vis, row + f, a.vis_f16 != 0) : make_float2(0.f, 0.f);
      const float2 w = cmul(v, cal);
      y[ii] = R > 1 ? cadd(y[ii], cmul(w, ph[u])) : cadd(y[ii], w);
    }
  });
  if (i2s == 0) y[0] = make_float2(0.f, 0.f);
}

template <int JA, int JB>
__device__ __forceinline__ void sbd_pass1(const float2 (&y)[JA], const float2 *pre,
                                          const float2 *TW, float2 *Sc, int c, int P, int PJ,
                                          bool act, int n1, int i2s) {
  if (!act) return;
  float2 x[JA];
  static_for<0, JA>([&](auto i) {
    constexpr int ii = decltype(i)::value;
    x[ii] = cmul(y[ii], pre[c * JA + ii]);
  });
  dft<JA>(x);
  static_for<0, JA>([&](auto k) {
    constexpr int kk = decltype(k)::value;
    const float2 w = TW[(i2s * (c + P * kk)) & (PJ - 1)];
    Sc[(n1 * JA + kk) * (JB + 1) + i2s] = cmul(x[kk], w);
  });
}

// Peak of one MBD column after the last MBD pass: lane k1 holds
// z[k2] = G(s', k1 + MA k2) for SBD bin s' = c + P col.  The key of a cell
// is |G|^2 with its 4 lowest mantissa bits replaced by (15 - k2), so one
// unsigned max keeps the value (to 2^-19 relative) and the lowest MBD bin
// among equal values; the running best keeps the lowest packed index.
template <int M, int MA, int MB, bool DUMP>
__device__ __forceinline__ void mbd_column_peak(const float2 (&z)[MB], int r, int c, int col, int k1,
                                                int P, int PJ, float *dump, float &best_v,
                                                int32_t &best_i) {
  // shifted bins: s = (s' + PJ/2) mod PJ, m = k1 + MA ((k2 + MB/2) mod MB)
  const int sp = c + P * col;
  const int s = (sp + (PJ >> 1)) & (PJ - 1);
  const int32_t base = (r * PJ + s) * M + k1;
  unsigned kmax = 0u;
  static_for<0, MB / 2>([&](auto kk) {
    constexpr int ka = 2 * decltype(kk)::value, kb = ka + 1;
    constexpr int k2a = (ka + MB / 2) & (MB - 1), k2b = (kb + MB / 2) & (MB - 1);
    const float va = z[k2a].x * z[k2a].x + z[k2a].y * z[k2a].y;
    const float vb = z[k2b].x * z[k2b].x + z[k2b].y * z[k2b].y;
    const unsigned ua = (__float_as_uint(va) & 0xFFFFFFF0u) | unsigned(15 - ka);
    const unsigned ub = (__float_as_uint(vb) & 0xFFFFFFF0u) | unsigned(15 - kb);
    kmax = max(kmax, max(ua, ub));
    if constexpr (DUMP) {
      dump[base + MA * ka] = va;
      dump[base + MA * kb] = vb;
    }
  });
  const float cv = __uint_as_float(kmax & 0xFFFFFFF0u);
  const int ck = 15 - int(kmax & 15u);
  const int32_t ci = base + MA * ck;
  if (cv > best_v || (cv == best_v && ci < best_i)) {
    best_v = cv;
    best_i = ci;
  }
}

// Largest |G|^2 of one MBD column into blk, as float bits: |G|^2 >= 0
// orders like its bits, and a cell that is not a number outranks every
// number (its bits are above those of +inf).
template <int MB>
__device__ __forceinline__ void mbd_column_max(const float2 (&z)[MB], unsigned &blk) {
  unsigned m = blk;
  static_for<0, MB / 2>([&](auto kk) {
    constexpr int ka = 2 * decltype(kk)::value, kb = ka + 1;
    const float va = z[ka].x * z[ka].x + z[ka].y * z[ka].y;
    const float vb = z[kb].x * z[kb].x + z[kb].y * z[kb].y;
    m = max(m, max(__float_as_uint(va), __float_as_uint(vb)));
  });
  blk = m;
}

// CL (compact lattice): every IF sits at a lattice position below MB once
// the positions are shifted by a common offset (which changes only the phase
// of G, not |G|).  The first MBD pass then has one non-zero input per lane
// and reduces to the identity: X holds one row per position, and each lane
// of the second pass reads the MB rows of its column directly, twiddles them
// and transforms; the first pass and its LDS transpose drop out.
// LIST: one work-group per entry of a.seg_list instead of per segment of the
// tile (re-evaluation of selected segments).
// ROWS (general form): the rows i1 of the first MBD pass that hold an IF
// (bit i1 for lattice positions MB i1 + i2), 0 for all; the pass then
// reads and transforms only those rows (a kernel specialised to the IF
// lattice when the search starts; the same sums).
template <int J, int M, bool DUMP, bool CL, bool LIST = false, unsigned ROWS = 0u>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(J <= 64 && !DUMP && !LIST ? 3 : 1)))
void fringe_kernel(FringeArgs a) {
  using S = FringeShape<J, M>;
  constexpr int JA = S::JA, JB = S::JB, MA = S::MA, MB = S::MB, G = S::G, COLS = S::COLS;
  constexpr unsigned RMASK = ROWS ? ROWS : (MA >= 32 ? ~0u : (1u << MA) - 1u);
  extern __shared__ float2 lds[];
  __shared__ float red_v[kBlock / 64];
  __shared__ int32_t red_i[kBlock / 64];

  const int N = a.n_if, R = a.n_rate, P = a.sbd_pad;
  const int PJ = P * J;
  const int NJ = N * J;
  const int t = threadIdx.x;

  // ---- which segment: spread consecutive segments over the 8 XCDs in
  // contiguous ranges so that overlapping segments share an L2.
  int dl, seg;
  int lb = 0, ld = 0;
  if constexpr (LIST) {
    lb = a.seg_list[3 * blockIdx.x];
    ld = a.seg_list[3 * blockIdx.x + 1];
    seg = a.seg_list[3 * blockIdx.x + 2];
    dl = lb * a.n_dm + ld;   // cube row
  } else {
    block_segment(a, DUMP, dl, seg);
  }
  int wi = 0;
  while (wi + 1 < a.n_win && a.win_off[wi + 1] <= seg) ++wi;
  const int l = a.win_len[wi];
  const int q = seg - a.win_off[wi];
  const int64_t k0 = a.win_k0[wi] + int64_t(q) * a.win_hop[wi];
  const float2 *wd = LIST ? nullptr : a.w + int64_t(dl) * a.w_dm_stride + k0 * NJ;
  const float2 *rph = a.rate_ph + a.rate_off[wi];

  int x_off, s_off, t_off, total;
  fringe_lds_plan<J, M, CL>(N, P, x_off, s_off, t_off, total);
  float2 *X = lds + x_off;
  float2 *Sc = lds + s_off;
  float2 *TW = lds + t_off;
  constexpr int XS = J + 1;

  for (int i = t; i < PJ; i += kBlock) TW[i] = a.tw_sbd[i];
  if constexpr (CL) {
    // rows of lattice positions without an IF stay zero
    for (int i = t; i < MB * XS; i += kBlock) X[i] = make_float2(0.f, 0.f);
  } else {
    // the zero row read for empty lattice points
    for (int i = t; i < XS; i += kBlock) X[N * XS + i] = make_float2(0.f, 0.f);
  }

  // ---- per-lane constants of the MBD transform
  const int grp = t / G, gl = t - grp * G;
  const bool m_p1 = gl < MB;  // pass-1 lane: lattice residue i2 = gl
  const bool m_p2 = gl < MA;  // pass-2 lane: output residue k1 = gl
  constexpr int NT = CL ? MB : MA;
  float2 twm[NT];   // general: w_M^(i2 k1) for k1 < MA; compact: w_M^(i2 k1) for i2 < MB
  int rowoff[CL ? 1 : MA];
  if constexpr (CL) {
    if (m_p2) {
      static_for<0, MB>([&](auto i) {
        constexpr int ii = decltype(i)::value;
        twm[ii] = a.tw_mbd[(gl * ii) & (M - 1)];
      });
    }
  } else if (m_p1) {
    static_for<0, MA>([&](auto k) {
      constexpr int kk = decltype(k)::value;
      twm[kk] = a.tw_mbd[(gl * kk) & (M - 1)];
      if constexpr ((RMASK >> kk) & 1u) rowoff[kk] = a.mbd_row[MB * kk + gl] * XS;
    });
  }
  float2 *Sg = Sc + grp * S::SG;

  // ---- per-lane roles of the SBD transform
  const bool s_p1 = t < N * JB;
  const int n1 = t / JB, i2s = t - (t / JB) * JB;

  float best_v = -1.0f;
  int32_t best_i = 0x7fffffff;
  float2 y[JA];

  auto sums = [&](int r) {
    if constexpr (LIST)
      segment_sum_direct<JA, JB>(y, a, lb, ld, k0, rph, r, N, J, l, R, s_p1, n1, i2s);
    else
      segment_sum<JA, JB>(y, wd, rph, r, N, J, l, R, s_p1, n1, i2s);
  };
  // SBD transform of sub-grid c -> X
  auto sbd = [&](int c) {
    __syncthreads();
    sbd_pass1<JA, JB>(y, a.pre_sbd, TW, Sc, c, P, PJ, s_p1, n1, i2s);
    __syncthreads();
    // SBD pass 2: JB-point DFT over i2 -> X[n][a = k1 + JA k2], the SBD
    // bin s' = c + P a of the standard (unshifted) transform.
    for (int v = t; v < N * JA; v += kBlock) {
      const int n2 = v / JA, k1 = v - (v / JA) * JA;
      float2 z[JB];
      static_for<0, JB>([&](auto i) {
        constexpr int ii = decltype(i)::value;
        z[ii] = Sc[(n2 * JA + k1) * (JB + 1) + ii];
      });
      dft<JB>(z);
      const int xrow = CL ? a.mbd_pos[n2] : n2;
      static_for<0, JB>([&](auto k) {
        constexpr int kk = decltype(k)::value;
        X[xrow * XS + k1 + JA * kk] = z[kk];
      });
    }
    __syncthreads();
  };
  // MBD transform of every SBD column of sub-grid c (rate r); FIND: the
  // cells' keys and the running (value, packed index) of the lane, else
  // only the largest |G|^2 (float bits) into blk
  auto mbd = [&](int r, int c, auto find_tag, unsigned &blk) {
    constexpr bool FIND = decltype(find_tag)::value != 0;
    auto column = [&](const float2 (&z)[MB], int col) {
      if constexpr (FIND)
        mbd_column_peak<M, MA, MB, DUMP>(z, r, c, col, gl, P, PJ, a.dump, best_v, best_i);
      else
        mbd_column_max<MB>(z, blk);
    };
    if constexpr (CL) {
      // compact lattice: z[i2] = X(position i2) w_M^(i2 k1), MB-point DFT
      for (int a0 = 0; a0 < J; a0 += COLS) {
        const int col = a0 + grp;
        if (col < J && m_p2) {
          float2 z[MB];
          z[0] = X[col];
          static_for<1, MB>([&](auto i) {
            constexpr int ii = decltype(i)::value;
            z[ii] = cmul(X[ii * XS + col], twm[ii]);
          });
          dft<MB>(z);
          column(z, col);
        }
      }
    } else {
      // MBD over the IF lattice, one column a of this SBD tile per group.
      // Unrolled by 4: the columns' LDS offsets become immediates.
#pragma unroll 4
      for (int a0 = 0; a0 < J; a0 += COLS) {
        const int col = a0 + grp;
        if (col < J) {
          if (m_p1) {
            float2 x[MA];
            static_for<0, MA>([&](auto i) {
              constexpr int ii = decltype(i)::value;
              if constexpr ((RMASK >> ii) & 1u) x[ii] = X[rowoff[ii] + col];
              else x[ii] = make_float2(0.f, 0.f);
            });
            dft_masked<MA, RMASK>(x);
            static_for<0, MA>([&](auto k) {
              constexpr int kk = decltype(k)::value;
              // w_M^(i2 k1) is 1 at k1 = 0
              Sg[kk * MB + (gl ^ (kk & (MB - 1)))] = kk == 0 ? x[0] : cmul(x[kk], twm[kk]);
            });
          }
          wave_lds_sync();
          if (m_p2) {
            float2 z[MB];
            static_for<0, MB>([&](auto i) {
              constexpr int ii = decltype(i)::value;
              z[ii] = Sg[gl * MB + (ii ^ (gl & (MB - 1)))];
            });
            dft<MB>(z);
            column(z, col);
          }
          wave_lds_sync();
        }
      }
    }
  };

  // ---- the search.  DUMP and LIST key every cell as they go, and so does
  // every search with fewer than 8 (rate, sub-grid) pairs, where searching
  // one of them again would cost more than keying saves.  Otherwise the
  // scan keeps per lane only the largest |G|^2 (float bits) over each
  // (rate, sub-grid) and the first (rate, sub-grid) holding the lane's
  // maximum; the one holding the block's maximum is searched again with
  // keys to find its cell.  A cell that is not a number then makes the
  // segment's power NaN (index -1).
  constexpr bool SCAN = !DUMP && !LIST;
  const bool scan = SCAN && R * P >= 8;
  unsigned scan_v = 0u;
  int scan_rc = 0;
  for (int r = 0; r < R; ++r) {
    sums(r);
    for (int c = 0; c < P; ++c) {
      sbd(c);
      unsigned blk = 0u;
      if (!scan) {
        mbd(r, c, Index<1>{}, blk);
      } else {
        mbd(r, c, Index<0>{}, blk);
        if (blk > scan_v) {
          scan_v = blk;
          scan_rc = r * P + c;
        }
      }
    }
  }
  if (scan) {
    // block maximum and its (rate, sub-grid): larger value, then lower
    // (rate, sub-grid)
    for (int off = 32; off > 0; off >>= 1) {
      const unsigned ov = __shfl_xor(scan_v, off, 64);
      const int orc = __shfl_xor(scan_rc, off, 64);
      if (ov > scan_v || (ov == scan_v && orc < scan_rc)) {
        scan_v = ov;
        scan_rc = orc;
      }
    }
    if ((t & 63) == 0) {
      red_v[t >> 6] = __uint_as_float(scan_v);
      red_i[t >> 6] = scan_rc;
    }
    __syncthreads();
    unsigned vmax = __float_as_uint(red_v[0]);
    int rc = red_i[0];
    for (int w = 1; w < kBlock / 64; ++w) {
      const unsigned v = __float_as_uint(red_v[w]);
      if (v > vmax || (v == vmax && red_i[w] < rc)) {
        vmax = v;
        rc = red_i[w];
      }
    }
    if (vmax > 0x7F800000u) {   // a cell that is not a number (non-finite input)
      if (t == 0) {
        const int64_t o = int64_t(dl) * a.seg_total + seg;
        a.power[o] = __builtin_nanf("");
        a.pidx[o] = -1;
      }
      return;
    }
    const int r = rc / P, c = rc - (rc / P) * P;
    sums(r);
    sbd(c);   // its first barrier also ends the reads of red_* above
    unsigned unused = 0u;
    mbd(r, c, Index<1>{}, unused);
  }

  // ---- block reduction: larger |G|^2 wins, ties -> lower packed index
  for (int off = 32; off > 0; off >>= 1) {
    const float ov = __shfl_xor(best_v, off, 64);
    const int32_t oi = __shfl_xor(best_i, off, 64);
    if (ov > best_v || (ov == best_v && oi < best_i)) {
      best_v = ov;
      best_i = oi;
    }
  }
  if ((t & 63) == 0) {
    red_v[t >> 6] = best_v;
    red_i[t >> 6] = best_i;
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
    a.power[o] = bv >= 0.0f ? sqrtf(bv) : __builtin_nanf("");
    a.pidx[o] = bv >= 0.0f ? bi : -1;
  }
}

}  // namespace frbx
