// Host side of libfrbx: argument validation, the float64 tables of the
// search (AP offsets of Eqs. 1-2, calibration phasors of Eq. 5, rate phasors
// of Eq. 4, transform twiddles, the MBD lattice and its matrix-core
// operands), orchestration of the device kernels (whole runs, streamed
// chunks with the DM-overlap carry, power summation, refinement), the host
// steps of Sec. 2.4.1 / Sec. 5.3 (multi-window filter, best-DM merge,
// cross-baseline matching) and the Appendix A calibration extraction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <numeric>
#include <string>
#include <utility>
#include <vector>

#include "../../include/frbx.h"
#include "frbx_internal.h"

using frbx::DevCrossing;

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kDefaultKdm = 4.149e6;  // ms MHz^2 per pc cm^-3

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

template <typename T>
void dfree(T *&p) {
  if (p) hipFree(const_cast<void *>(reinterpret_cast<const void *>(p)));
  p = nullptr;
}

}  // namespace

struct frbx_ctx {
  // layout
  int B = 0, N = 0, J = 0;
  int64_t K = 0;
  double t_ap = 0, df = 0;
  std::vector<double> f0;
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;

  // parameters
  std::vector<double> tau0, phi0;  // [B*N]
  double dm_lo = 0.0, dm_step = 1.0, k_dm = kDefaultKdm;
  int n_dm = 1;
  int sbd_pad = 4, n_mbd = 256;
  double mbd_step_req = 0.0, f_ref_fit = std::numeric_limits<double>::quiet_NaN();
  int n_rate = 1;
  double rate_step_req = 0.0;
  std::vector<int> windows{2, 4};
  int precision = FRBX_PREC_F32;
  double threshold = 3.0;
  int n_win_min = 3, n_bl_min = 2;

  // derived tables
  bool dirty = true;
  std::vector<int32_t> dk;  // [D][N*J]
  int64_t dk_max = 0, k_eff = 0;
  std::vector<int> hop, nseg, segoff;
  int64_t seg_total = 0;
  double mbd_step = 0, t_amb = 0, rate_step = 0;
  std::vector<int32_t> mbd_row;
  std::vector<int64_t> q_if;  // MBD lattice position of each IF
  std::vector<int32_t> mbd_pos;  // compact lattice: q_if less a common shift (empty: general)
  double recheck_band = 0.0;     // matrix-core forms: re-evaluate |P_norm - threshold| < band
  int64_t n_rechecked = 0;       // segments re-evaluated by the last pass
  int32_t *d_list = nullptr;     // their (DM trial, segment) list
  size_t list_cap = 0;
  int32_t mbd_shift = -1;        // that shift, -1 for the general form
  int specialise = 1;            // float32 general form: kernel compiled for the lattice's rows
  int sbd_mfma = 0;              // float16 form: SBD transform on the matrix cores as well
  unsigned rows_mask = 0;        // rows of the kernel in use (0: the statically built kernel)
  hipFunction_t rows_fn = nullptr;
  std::string rows_note;         // why the specialised kernel is not in use
  std::vector<int> rate_off;
  int dd_group = 1;          // DM trials per staged dedispersion tile

  // device memory
  const void *d_vis = nullptr;
  void *d_vis_own = nullptr;
  int vis_f16 = 0;
  float vis_absmax = 0.f;
  bool loaded = false;
  void *d_mfma_hi = nullptr, *d_mfma_lo = nullptr;
  void *d_sbd_a = nullptr;   // float16 form: SBD DFT matrix as MFMA A operands
  unsigned int *d_absmax = nullptr;
  int32_t *d_dk = nullptr;
  float2 *d_cal = nullptr, *d_rate = nullptr, *d_tw_sbd = nullptr, *d_pre = nullptr,
         *d_tw_mbd = nullptr;
  int32_t *d_row = nullptr, *d_pos = nullptr;
  float2 *d_w = nullptr;
  size_t w_cap = 0;
  int dt = 1;
  float *d_power = nullptr;
  int32_t *d_pidx = nullptr;
  size_t cube_cap = 0, pidx_cap = 0;
  double *d_mean = nullptr, *d_sd = nullptr;
  int64_t *d_cnt = nullptr;
  size_t mean_cap = 0, sd_cap = 0, cnt_cap = 0;
  DevCrossing *d_cross = nullptr;
  unsigned long long *d_ncross = nullptr;
  int64_t cross_cap = 0;
  size_t w_budget = size_t(6) << 30;   // bytes for the dedispersed DM tiles
  bool w_budget_strict = false;        // set by the caller: below one trial -> E_NOMEM
  // this device's copy of the no-alloc workspace (looked up at create)
  void *d_noalloc = nullptr;
  std::string noalloc_err;

  // timing
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  struct Span { int kind; int64_t units; hipEvent_t a, b; int64_t bytes; };
  std::vector<Span> spans;
  frbx_timing last_timing{};

  int64_t cube_len = 0;       // segments per (b, d) of the last pass
  std::vector<int> last_off, last_nq;  // window offsets / counts of the last pass

  // streaming state
  bool streaming = false;
  int64_t chunk = 0, carry = 0, buf_frames = 0, valid = 0, buf_start = 0, frames_in = 0;
  float2 *sbuf[2] = {nullptr, nullptr};
  int cur = 0;
  void *stage = nullptr;
  size_t stage_cap = 0;
  float *d_scale = nullptr;
  std::vector<int64_t> next_q, push_first, push_nq;
  std::vector<frbx_candidate> stream_cross;

  // refinement of coarse peaks
  int64_t rn = 0;
  frbx::RefineSeg *d_rseg = nullptr;
  size_t rseg_cap = 0;
  double *d_rtheta = nullptr;
  size_t rtheta_cap = 0;
  float *d_rpower = nullptr;
  size_t rpower_cap = 0;
  frbx::RefineChan *d_rchan = nullptr;
  size_t rchan_cap = 0;
  double *d_rtb = nullptr, *d_rsb = nullptr, *d_rrad = nullptr;  // ascent state
  size_t rtb_cap = 0, rsb_cap = 0, rrad_cap = 0;
  float *d_rpb = nullptr;
  size_t rpb_cap = 0;
  std::vector<double> rtheta0;   // start points of the begun peaks [n][5]
  double rcells[5] = {0, 0, 0, 0, 0};
  double rxbar = 0.0;
  bool rdone = false, rbegun = false;

  // results
  bool have = false;
  std::vector<double> mean, sd;
  std::vector<int64_t> cnt;
  std::vector<frbx_candidate> cross, dets;
  std::vector<frbx_group> groups;

  frbx_status fail(frbx_status s, const std::string &m) {
    err = m;
    return s;
  }
  frbx_status hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return FRBX_OK;
    err = std::string(what) + ": " + hipGetErrorString(e);
    return FRBX_E_DEVICE;
  }
  hipEvent_t event() {
    if (ev_used == ev_pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      ev_pool.push_back(e);
    }
    return ev_pool[ev_used++];
  }
  // record the start of a timed launch; returns the span index or -1
  int span_begin(int kind, int64_t units) {
    if (!timing) return -1;
    hipEvent_t a = event(), b = event();
    if (!a || !b) return -1;
    hipEventRecord(a, stream);
    spans.push_back(Span{kind, units, a, b, 0});
    return int(spans.size()) - 1;
  }
  void span_end(int i) {
    if (i >= 0) hipEventRecord(spans[i].b, stream);
  }
  void collect_timing() {
    frbx_timing t{};
    for (const Span &sp : spans) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, sp.a, sp.b) != hipSuccess) continue;
      if (sp.kind == 0) t.fringe_ms += ms, t.n_fringe++, t.fringe_units += sp.units;
      if (sp.kind == 1)
        t.dedisperse_ms += ms, t.n_dedisperse++, t.dedisperse_units += sp.units, t.dedisperse_bytes += sp.bytes;
      if (sp.kind == 2) t.stats_ms += ms, t.n_stats++;
      if (sp.kind == 3) t.refine_ms += ms, t.n_refine++, t.refine_units += sp.units;
    }
    last_timing = t;
    spans.clear();
    ev_used = 0;
  }
  ~frbx_ctx() {
    hipSetDevice(device);
    for (hipEvent_t e : ev_pool) hipEventDestroy(e);
    dfree(d_vis_own);
    dfree(sbuf[0]);
    dfree(sbuf[1]);
    dfree(stage);
    dfree(d_scale);
    dfree(d_mfma_hi);
    dfree(d_mfma_lo);
    dfree(d_sbd_a);
    dfree(d_absmax);
    dfree(d_dk);
    dfree(d_cal);
    dfree(d_rate);
    dfree(d_tw_sbd);
    dfree(d_pre);
    dfree(d_tw_mbd);
    dfree(d_row);
    dfree(d_pos);
    dfree(d_list);
    dfree(d_w);
    dfree(d_power);
    dfree(d_pidx);
    dfree(d_mean);
    dfree(d_sd);
    dfree(d_cnt);
    dfree(d_cross);
    dfree(d_ncross);
    dfree(d_rseg);
    dfree(d_rtheta);
    dfree(d_rpower);
    dfree(d_rchan);
    dfree(d_rtb);
    dfree(d_rsb);
    dfree(d_rrad);
    dfree(d_rpb);
  }
};

namespace {

frbx_status check_layout(const frbx_layout *L, std::string &why) {
  if (!L) return why = "layout is NULL", FRBX_E_INVAL;
  if (L->n_baselines < 1 || L->n_if < 1 || L->n_frames < 1)
    return why = "n_baselines, n_if and n_frames must be >= 1", FRBX_E_INVAL;
  if (!(L->n_chan == 8 || L->n_chan == 16 || L->n_chan == 32 || L->n_chan == 64 ||
        L->n_chan == 128 || L->n_chan == 256))
    return why = "n_chan must be 8, 16, 32, 64, 128 or 256", FRBX_E_INVAL;
  if (!(L->t_ap_ms > 0) || !(L->chan_bw_mhz > 0) || !std::isfinite(L->t_ap_ms) ||
      !std::isfinite(L->chan_bw_mhz))
    return why = "t_ap_ms and chan_bw_mhz must be finite and > 0", FRBX_E_INVAL;
  if (!L->if_freq_mhz) return why = "if_freq_mhz is NULL", FRBX_E_INVAL;
  for (int n = 0; n < L->n_if; ++n)
    if (!(L->if_freq_mhz[n] > 0) || !std::isfinite(L->if_freq_mhz[n]))
      return why = "IF frequencies must be finite and > 0", FRBX_E_INVAL;
  if (int64_t(L->n_if) * L->n_chan > (1 << 20)) return why = "too many channels", FRBX_E_INVAL;
  return FRBX_OK;
}

// Eq. 2 with Eq. 1: dk = floor(0.5 + k_dm DM (f^-2 - f_ref^-2) / t_ap); the
// reference is the highest channel frequency (Sec. 2.2).
void ap_offset_table(int N, int J, const double *f0, double df, double t_ap, double dm_lo,
                     double dm_step, int n_dm, double k_dm, int32_t *out) {
  double fr = 0.0;
  for (int n = 0; n < N; ++n)
    for (int j = 0; j < J; ++j) fr = std::max(fr, f0[n] + j * df);
  for (int d = 0; d < n_dm; ++d) {
    const double dm = dm_lo + d * dm_step;
    for (int n = 0; n < N; ++n)
      for (int j = 0; j < J; ++j) {
        const double f = f0[n] + j * df;
        const double dt = k_dm * dm * (1.0 / (f * f) - 1.0 / (fr * fr));
        out[(int64_t(d) * N + n) * J + j] = static_cast<int32_t>(std::floor(0.5 + dt / t_ap));
      }
  }
}

// whole-kHz gcd of the IF offsets from IF 0 (0 when all coincide); -1 when
// an offset is not a whole number of kHz
int64_t offset_gcd_khz(const std::vector<double> &f0) {
  int64_t g = 0;
  for (double f : f0) {
    const double x = std::fabs(f - f0[0]) * 1000.0;
    const double r = std::nearbyint(x);
    if (std::fabs(x - r) > 1e-6) return -1;
    g = std::gcd(g, static_cast<int64_t>(r));
  }
  return g;
}

// MBD lattice of Eq. 5 (grid of M points of step mbd_step over the
// ambiguity t_amb): the lattice position q[n] of every IF, the IF on each
// position (row[q], N if none), and the compact form of the float32 kernel:
// a common shift of the positions that brings them all below the first
// pass's row count (shift -1 when there is none).  Returns an error text,
// or nullptr.
struct MbdLattice {
  double t_amb = 0, mbd_step = 0;
  std::vector<int32_t> row;
  std::vector<int64_t> q;
  std::vector<int32_t> pos;
  int32_t shift = -1;
};

const char *mbd_lattice(const std::vector<double> &f0, int J, double df, int M, double step_req,
                        MbdLattice &L) {
  const int N = int(f0.size());
  const int64_t g = offset_gcd_khz(f0);
  if (g > 0)
    L.t_amb = 1000.0 / double(g);
  else if (g == 0)
    L.t_amb = 1.0 / (J * df);
  else if (!(step_req > 0))
    return "IF offsets are not whole kHz: give an explicit MBD step";
  else
    L.t_amb = step_req * M;
  L.mbd_step = step_req > 0 ? step_req : L.t_amb / M;
  L.row.assign(M, N);
  for (int n = 0; n < N; ++n) {
    const double x = (f0[n] - f0[0]) * L.mbd_step * M;
    const double r = std::nearbyint(x);
    if (std::fabs(x - r) > 1e-6) return "MBD step does not put every IF on the transform lattice";
    int64_t qn = static_cast<int64_t>(r) % M;
    if (qn < 0) qn += M;
    if (L.row[qn] != N) return "two IFs fall on the same MBD lattice point: raise n_mbd";
    L.row[qn] = n;
  }
  L.q.assign(N, 0);
  for (int qq = 0; qq < M; ++qq)
    if (L.row[qq] < N) L.q[L.row[qq]] = qq;
  // Compact lattice: a common shift of the positions (a phase factor on G,
  // |G| unchanged) that brings every IF below the row count of the first MBD
  // pass lets the f32 kernel skip that pass.
  L.pos.clear();
  L.shift = -1;
  const int compact_rows = frbx::fringe_compact_rows(M);
  for (int n0 = 0; n0 < N && L.pos.empty(); ++n0) {
    std::vector<int32_t> pos(N);
    bool fits = true;
    for (int n = 0; n < N; ++n) {
      pos[n] = int32_t(((L.q[n] - L.q[n0]) % M + M) % M);
      fits = fits && pos[n] < compact_rows;
    }
    if (fits) {
      L.pos = pos;
      L.shift = int32_t(L.q[n0]);
    }
  }
  return nullptr;
}

// exp(-i 2 pi x) for x in cycles, reduced to [-1/2, 1/2) first
float2 cis_cycles(double x) {
  const double r = x - std::nearbyint(x);
  return make_float2(static_cast<float>(std::cos(kTwoPi * r)),
                     static_cast<float>(-std::sin(kTwoPi * r)));
}

// The float16 form runs both transforms on the matrix cores when asked to
// (frbx_set_sbd_matrix_cores) and the shape allows it (n_chan <= 64);
// otherwise its SBD stays on the vector ALUs.
bool use_gemm(const frbx_ctx *c) {
  return c->sbd_mfma && c->precision == FRBX_PREC_F16 &&
         frbx::fringe_gemm_supported(c->J, c->n_mbd, c->N, c->sbd_pad);
}

// The matrix-core fringe launch of the current precision (both transforms
// on the matrix cores, or the MBD only).
hipError_t launch_matrix_core(const frbx_ctx *c, frbx::FringeArgs &fa, int grid) {
  if (use_gemm(c)) {
    fa.sbd_a = c->d_sbd_a;
    return frbx::launch_fringe_gemm(c->J, c->N, fa, frbx::fringe_gemm_lds_bytes(c->J, c->N, c->sbd_pad), grid,
                                    c->stream);
  }
  const int n_pass = c->precision == FRBX_PREC_F16X3 ? 3 : 1;
  return frbx::launch_fringe_mfma(c->J, c->N, n_pass, fa, frbx::fringe_mfma_lds_bytes(c->J, c->N, c->sbd_pad, n_pass),
                                  grid, c->stream);
}

frbx_status prepare(frbx_ctx *c) {
  if (!c->dirty) return FRBX_OK;
  c->rbegun = false;  // a refinement's cells and tables follow the grids
  const int N = c->N, J = c->J, NJ = N * J, D = c->n_dm;
  // AP offsets and segment layout (Eqs. 1-3)
  c->dk.assign(size_t(D) * NJ, 0);
  ap_offset_table(N, J, c->f0.data(), c->df, c->t_ap, c->dm_lo, c->dm_step, D, c->k_dm,
                  c->dk.data());
  int64_t mx = 0, mn = 0;
  for (int32_t v : c->dk) mx = std::max<int64_t>(mx, v), mn = std::min<int64_t>(mn, v);
  if (mn < 0) return c->fail(FRBX_E_INVAL, "negative AP offset (negative DM trial?)");
  c->dk_max = mx;
  c->k_eff = c->K - mx;
  // largest group of consecutive DM trials whose offsets differ by less than
  // the staged spread for every channel
  {
    int g = 1;
    auto fits = [&](int gs) {
      for (int d0 = 0; d0 + gs - 1 < D; d0 += 1) {
        const int32_t *a0 = c->dk.data() + size_t(d0) * NJ, *a1 = c->dk.data() + size_t(d0 + gs - 1) * NJ;
        for (int i = 0; i < NJ; ++i)
          if (a1[i] - a0[i] >= frbx::kDedispSpread || a1[i] < a0[i]) return false;
      }
      return true;
    };
    while (g < D && g < frbx::kDedispMaxGroup && fits(g + 1)) ++g;
    c->dd_group = g;
  }
  const int nw = int(c->windows.size());
  c->hop.assign(nw, 0);
  c->nseg.assign(nw, 0);
  c->segoff.assign(nw, 0);
  int64_t tot = 0;
  for (int w = 0; w < nw; ++w) {
    const int l = c->windows[w];
    const int h = std::max(1, l / 2);
    const int64_t span = c->K - mx - l;
    const int64_t q = span >= 0 ? span / h + 1 : 0;
    c->hop[w] = h;
    c->nseg[w] = int(q);
    c->segoff[w] = int(tot);
    tot += q;
  }
  c->seg_total = tot;
  if (tot > (int64_t(1) << 30)) return c->fail(FRBX_E_INVAL, "too many segments per DM trial");
  // MBD lattice (Eq. 5 MBD term on a grid of M points)
  const int M = c->n_mbd;
  {
    MbdLattice L;
    if (const char *why = mbd_lattice(c->f0, J, c->df, M, c->mbd_step_req, L)) return c->fail(FRBX_E_INVAL, why);
    c->t_amb = L.t_amb;
    c->mbd_step = L.mbd_step;
    c->mbd_row = L.row;
    c->q_if = L.q;
    c->mbd_pos = L.pos;
    c->mbd_shift = L.shift;
  }
  // rate grid (Eq. 4)
  int lmax = 1;
  for (int l : c->windows) lmax = std::max(lmax, l);
  double fmax = 0;
  for (int n = 0; n < N; ++n) fmax = std::max(fmax, c->f0[n] + (J - 1) * c->df);
  c->rate_step = c->rate_step_req > 0 ? c->rate_step_req
                                      : 1.0 / (2.0 * fmax * 1e6 * lmax * c->t_ap * 1e-3);
  if (int64_t(c->n_rate) * c->sbd_pad * J * M >= (int64_t(1) << 31))
    return c->fail(FRBX_E_INVAL, "rate x SBD x MBD grid too large");
  if (!frbx::fringe_supported(J, M, N, c->sbd_pad))
    return c->fail(FRBX_E_INVAL, "IF count too large for this channel count / grid");

  hipSetDevice(c->device);
  // device tables
  std::vector<float2> rate;
  c->rate_off.assign(nw, 0);
  const int R = c->n_rate;
  for (int w = 0; w < nw; ++w) {
    const int l = c->windows[w];
    c->rate_off[w] = int(rate.size());
    for (int r = 0; r < R; ++r) {
      const double rho = (r - R / 2) * c->rate_step;
      for (int n = 0; n < N; ++n)
        for (int u = 0; u < l; ++u)
          rate.push_back(cis_cycles(1e3 * rho * c->f0[n] * c->t_ap * (u - (l - 1) / 2.0)));
    }
  }
  const int PJ = c->sbd_pad * J;
  const int JA = J >= 128 ? 16 : (J >= 32 ? 8 : 4);
  std::vector<float2> tw_sbd(PJ), pre(size_t(c->sbd_pad) * JA), tw_mbd(M);
  for (int k = 0; k < PJ; ++k) tw_sbd[k] = cis_cycles(double(k) / PJ);
  for (int cc = 0; cc < c->sbd_pad; ++cc)
    for (int i = 0; i < JA; ++i) pre[cc * JA + i] = cis_cycles(double(i * cc) / (c->sbd_pad * JA));
  for (int k = 0; k < M; ++k) tw_mbd[k] = cis_cycles(double(k) / M);
  // calibration phasors (Eq. 5)
  std::vector<float2> cal(size_t(c->B) * NJ);
  for (int b = 0; b < c->B; ++b)
    for (int n = 0; n < N; ++n)
      for (int j = 0; j < J; ++j) {
        const double cyc = (j * c->df - J * c->df / 2.0) * c->tau0[b * N + n] +
                           c->phi0[b * N + n] / kTwoPi;
        cal[(size_t(b) * N + n) * J + j] = cis_cycles(cyc);
      }
  auto up = [&](auto *&dptr, const auto &vec) -> frbx_status {
    dfree(dptr);
    const size_t bytes = vec.size() * sizeof(vec[0]);
    if (bytes == 0) return FRBX_OK;
    if (hipMalloc(reinterpret_cast<void **>(&dptr), bytes) != hipSuccess)
      return c->fail(FRBX_E_NOMEM, "device allocation of a table failed");
    return c->hip(hipMemcpy(dptr, vec.data(), bytes, hipMemcpyHostToDevice), "table upload");
  };
  frbx_status s;
  if ((s = up(c->d_dk, c->dk)) != FRBX_OK) return s;
  if ((s = up(c->d_rate, rate)) != FRBX_OK) return s;
  if ((s = up(c->d_tw_sbd, tw_sbd)) != FRBX_OK) return s;
  if ((s = up(c->d_pre, pre)) != FRBX_OK) return s;
  if ((s = up(c->d_tw_mbd, tw_mbd)) != FRBX_OK) return s;
  if ((s = up(c->d_row, c->mbd_row)) != FRBX_OK) return s;
  if ((s = up(c->d_pos, c->mbd_pos)) != FRBX_OK) return s;
  if ((s = up(c->d_cal, cal)) != FRBX_OK) return s;
  if (c->precision != FRBX_PREC_F32) {
    const int n_pass = c->precision == FRBX_PREC_F16X3 ? 3 : 1;
    if (!frbx::fringe_mfma_supported(J, M, N, c->sbd_pad, n_pass))
      return c->fail(FRBX_E_INVAL, "matrix-core precision needs n_mbd = 256, n_chan >= 16, n_if <= 32");
    // Real-embedded DFT over the IF lattice as MFMA B operands: column tile
    // t < 16 holds Re G for m in [16 t, 16 t + 16), t >= 16 holds Im G;
    // row 2n multiplies Re X(n), row 2n + 1 multiplies Im X(n).  Stored in
    // the per-lane order of v_mfma_f32_16x16x32_f16: lane l, element e of
    // K-chunk kc is row 32 kc + 8 (l / 16) + e, column 16 t + l % 16.
    const int NK = N <= 16 ? 1 : 2;
    std::vector<_Float16> bh(size_t(32) * NK * 64 * 8), bl(bh.size());
    if (frbx::mfma_three_real(J, N, n_pass)) {
      // Three-real-product form: for tile t < 16 (columns m in [16 t,
      // 16 t + 16)) the matrices c = cos, d = -sin and c + d of the
      // twiddle w_M^(q_n m), K = n < 32 (zero for n >= N), in the same
      // per-lane order: lane ln, element e is row 8 (ln / 16) + e.
      for (int t = 0; t < 16; ++t)
        for (int mat = 0; mat < 3; ++mat)
          for (int ln = 0; ln < 64; ++ln)
            for (int e = 0; e < 8; ++e) {
              const int n = 8 * (ln / 16) + e, m = 16 * t + ln % 16;
              double v = 0.0;
              if (n < N) {
                const double th = kTwoPi * double((c->q_if[n] * m) % M) / M;
                const double cs = std::cos(th), dd = -std::sin(th);
                v = mat == 0 ? cs : mat == 1 ? dd : cs + dd;
              }
              const size_t o = ((size_t(t) * 3 + mat) * 64 + ln) * 8 + e;
              bh[o] = static_cast<_Float16>(v);
              bl[o] = static_cast<_Float16>(v - double(bh[o]));
            }
    } else {
      for (int t = 0; t < 32; ++t)
        for (int kc = 0; kc < NK; ++kc)
          for (int ln = 0; ln < 64; ++ln)
            for (int e = 0; e < 8; ++e) {
              const int k = 32 * kc + 8 * (ln / 16) + e, n = k / 2, comp = k % 2;
              const int m = 16 * (t % 16) + ln % 16;
              double v = 0.0;
              if (n < N) {
                const double th = kTwoPi * double((c->q_if[n] * m) % M) / M;
                const double cs = std::cos(th), sn = std::sin(th);
                v = t < 16 ? (comp == 0 ? cs : sn) : (comp == 0 ? -sn : cs);
              }
              const size_t o = ((size_t(t) * NK + kc) * 64 + ln) * 8 + e;
              bh[o] = static_cast<_Float16>(v);
              bl[o] = static_cast<_Float16>(v - double(bh[o]));
            }
    }
    if ((s = up(c->d_mfma_hi, bh)) != FRBX_OK) return s;
    if ((s = up(c->d_mfma_lo, bl)) != FRBX_OK) return s;
    if (use_gemm(c)) {
      // Real-embedded J-point DFT of the SBD sub-grids as MFMA A operands:
      // row 2a (+1) gives Re (Im) X(a), column 2j (+1) multiplies Re (Im) Y(j),
      // so the 2 x 2 block of (a, j) is [cos, sin; -sin, cos] of 2 pi j a / J.
      // Per-lane order of v_mfma_f32_16x16x32_f16: lane ln, element e of
      // K-chunk kc of row tile rt is row 16 rt + ln % 16, column
      // 32 kc + 8 (ln / 16) + e.
      const int SRT = 2 * J / 16, KC = J / 16;
      std::vector<_Float16> fa(size_t(SRT) * KC * 64 * 8);
      for (int rt = 0; rt < SRT; ++rt)
        for (int kc = 0; kc < KC; ++kc)
          for (int ln = 0; ln < 64; ++ln)
            for (int e = 0; e < 8; ++e) {
              const int row = 16 * rt + ln % 16, col = 32 * kc + 8 * (ln / 16) + e;
              const int aa = row / 2, re_im = row % 2, j = col / 2, comp = col % 2;
              const double th = kTwoPi * double((int64_t(j) * aa) % J) / J;
              const double cs = std::cos(th), sn = std::sin(th);
              const double v = re_im == 0 ? (comp == 0 ? cs : sn) : (comp == 0 ? -sn : cs);
              fa[((size_t(rt) * KC + kc) * 64 + ln) * 8 + e] = static_cast<_Float16>(v);
            }
      if ((s = up(c->d_sbd_a, fa)) != FRBX_OK) return s;
    }
  }
  // Float32 general form: the fringe kernel compiled for the rows of the
  // first MBD pass that hold an IF (the same sums, only those rows read
  // and transformed); the statically built kernel when every row holds an
  // IF or the run-time compiler cannot build it.
  c->rows_fn = nullptr;
  c->rows_mask = 0;
  c->rows_note.clear();
  const int MB = frbx::fringe_compact_rows(M);
  if (c->specialise && c->precision == FRBX_PREC_F32 && c->mbd_pos.empty() && MB > 0) {
    const int MA = M / MB;
    unsigned rows = 0;
    for (int n = 0; n < N; ++n) rows |= 1u << (c->q_if[n] / MB);
    const unsigned all = MA >= 32 ? ~0u : (1u << MA) - 1u;
    if (rows != all) {
      c->rows_fn = frbx::fringe_rows_kernel(c->device, J, M, rows, &c->rows_note);
      if (c->rows_fn) c->rows_mask = rows;
    }
  }
  c->dirty = false;
  return FRBX_OK;
}

// float16 operand scale: a power of two with sqrt(2) J l_max max|component|
// * scale <= 2^15, a bound on every SBD output |X(n, s)|
float mfma_scale(const frbx_ctx *c) {
  int lmax = 1;
  for (int l : c->windows) lmax = std::max(lmax, l);
  const double bound = std::sqrt(2.0) * c->J * lmax * double(c->vis_absmax);
  if (!(bound > 0) || !std::isfinite(bound)) return 1.0f;
  const int e = int(std::floor(std::log2(32768.0 / bound)));
  return std::ldexp(1.0f, std::max(-100, std::min(100, e)));
}

template <typename T>
frbx_status ensure(frbx_ctx *c, T *&p, size_t &cap, size_t need) {
  if (need <= cap && p) return FRBX_OK;
  dfree(p);
  cap = 0;
  if (need == 0) return FRBX_OK;
  if (hipMalloc(reinterpret_cast<void **>(&p), need * sizeof(T)) != hipSuccess)
    return c->fail(FRBX_E_NOMEM, "device allocation failed");
  cap = need;
  return FRBX_OK;
}

// ------------------------------------------------------------ host grouping
struct Iv {
  int64_t lo, hi;
};

// Step b of Sec. 2.4.1: join the lowest-numbered group holding a member whose
// closed AP interval overlaps; otherwise open a new group.
int insert_item(std::vector<std::vector<int>> &mem, std::vector<std::vector<Iv>> &ivs, int item,
                Iv iv) {
  for (size_t g = 0; g < mem.size(); ++g)
    for (const Iv &x : ivs[g])
      if (iv.lo <= x.hi && x.lo <= iv.hi) {
        mem[g].push_back(item);
        ivs[g].push_back(iv);
        return int(g);
      }
  mem.push_back({item});
  ivs.push_back({iv});
  return int(mem.size()) - 1;
}

double floor_mod(double a, double p) { return a - p * std::floor(a / p); }

void detect_impl(const frbx_candidate *cr, int64_t nc, double t_amb, int n_win_min, int n_bl_min,
                 bool use_mbd, std::vector<frbx_candidate> &dets_out,
                 std::vector<frbx_group> &groups_out) {
  // per (baseline, DM trial): steps b-d
  std::vector<int64_t> ord(nc);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int64_t x, int64_t y) {
    if (cr[x].baseline != cr[y].baseline) return cr[x].baseline < cr[y].baseline;
    return cr[x].dm_index < cr[y].dm_index;
  });
  std::vector<std::vector<frbx_candidate>> per_b;
  std::vector<int> per_b_id;
  for (int64_t a = 0; a < nc;) {
    int64_t e = a;
    while (e < nc && cr[ord[e]].baseline == cr[ord[a]].baseline &&
           cr[ord[e]].dm_index == cr[ord[a]].dm_index)
      ++e;
    std::vector<int64_t> ids(ord.begin() + a, ord.begin() + e);
    // insertion order: window length descending, then k0, then input order
    std::vector<int64_t> ins(ids.size());
    std::iota(ins.begin(), ins.end(), 0);
    std::stable_sort(ins.begin(), ins.end(), [&](int64_t x, int64_t y) {
      const frbx_candidate &p = cr[ids[x]], &q = cr[ids[y]];
      if (p.window_len != q.window_len) return p.window_len > q.window_len;
      if (p.k0 != q.k0) return p.k0 < q.k0;
      return ids[x] < ids[y];
    });
    std::vector<std::vector<int>> mem;
    std::vector<std::vector<Iv>> ivs;
    for (int64_t i : ins) {
      const frbx_candidate &p = cr[ids[i]];
      insert_item(mem, ivs, int(i), Iv{p.k0, p.k0 + p.window_len - 1});
    }
    const int b = cr[ord[a]].baseline;
    if (per_b.empty() || per_b_id.back() != b) {
      per_b.emplace_back();
      per_b_id.push_back(b);
    }
    for (auto &g : mem) {
      std::vector<int> surv;
      if (use_mbd) {
        // step c: circular mean of MBD over the ambiguity, keep |diff| < T/4
        double sc = 0, ss = 0;
        for (int i : g) {
          const double ang = kTwoPi * cr[ids[i]].mbd_us / t_amb;
          sc += std::cos(ang);
          ss += std::sin(ang);
        }
        const double mbar = t_amb * std::atan2(ss, sc) / kTwoPi;
        for (int i : g) {
          const double dlt = floor_mod(cr[ids[i]].mbd_us - mbar + t_amb / 2.0, t_amb) - t_amb / 2.0;
          if (std::fabs(dlt) < t_amb / 4.0) surv.push_back(i);
        }
      } else {
        surv = g;
      }
      if (surv.empty()) continue;
      std::vector<int> wl;
      for (int i : surv) wl.push_back(cr[ids[i]].window_len);
      std::sort(wl.begin(), wl.end());
      const int n_win = int(std::unique(wl.begin(), wl.end()) - wl.begin());
      if (n_win < n_win_min) continue;
      int best = surv[0];
      for (size_t k = 1; k < surv.size(); ++k)
        if (cr[ids[surv[k]]].power_norm > cr[ids[best]].power_norm) best = surv[k];
      frbx_candidate det = cr[ids[best]];
      det.n_windows = n_win;
      det.group_id = -1;
      per_b.back().push_back(det);
    }
    a = e;
  }
  // best DM bin per pulse (Sec. 5.3), per baseline
  std::vector<frbx_candidate> dets;
  for (auto &v : per_b) {
    std::vector<int> ins(v.size());
    std::iota(ins.begin(), ins.end(), 0);
    std::stable_sort(ins.begin(), ins.end(), [&](int x, int y) {
      if (v[x].dm_index != v[y].dm_index) return v[x].dm_index < v[y].dm_index;
      if (v[x].k0 != v[y].k0) return v[x].k0 < v[y].k0;
      return x < y;
    });
    std::vector<std::vector<int>> mem;
    std::vector<std::vector<Iv>> ivs;
    for (int i : ins) insert_item(mem, ivs, i, Iv{v[i].k0, v[i].k0 + v[i].window_len - 1});
    for (auto &g : mem) {
      int best = g[0];
      for (size_t k = 1; k < g.size(); ++k)
        if (v[g[k]].power_norm > v[best].power_norm) best = g[k];
      dets.push_back(v[best]);
    }
  }
  // cross-baseline matching (Sec. 2.4.1)
  std::vector<int> ins(dets.size());
  std::iota(ins.begin(), ins.end(), 0);
  std::stable_sort(ins.begin(), ins.end(), [&](int x, int y) {
    if (dets[x].baseline != dets[y].baseline) return dets[x].baseline < dets[y].baseline;
    if (dets[x].k0 != dets[y].k0) return dets[x].k0 < dets[y].k0;
    return x < y;
  });
  std::vector<std::vector<int>> mem;
  std::vector<std::vector<Iv>> ivs;
  for (int i : ins) {
    const int g = insert_item(mem, ivs, i, Iv{dets[i].k0, dets[i].k0 + dets[i].window_len - 1});
    dets[i].group_id = g;
  }
  groups_out.clear();
  for (size_t g = 0; g < mem.size(); ++g) {
    std::vector<int> bl;
    for (int i : mem[g]) bl.push_back(dets[i].baseline);
    std::sort(bl.begin(), bl.end());
    frbx_group G{};
    G.group_id = int(g);
    G.n_baselines = int(std::unique(bl.begin(), bl.end()) - bl.begin());
    G.k_start = ivs[g][0].lo;
    G.k_end = ivs[g][0].hi;
    for (const Iv &x : ivs[g]) G.k_start = std::min(G.k_start, x.lo), G.k_end = std::max(G.k_end, x.hi);
    int best = mem[g][0];
    for (size_t k = 1; k < mem[g].size(); ++k)
      if (dets[mem[g][k]].power_norm > dets[best].power_norm) best = mem[g][k];
    G.best = best;
    G.reported = G.n_baselines >= n_bl_min ? 1 : 0;
    groups_out.push_back(G);
  }
  dets_out.swap(dets);
}

template <typename T>
frbx_status copy_out(const std::vector<T> &v, T *out, int64_t cap, int64_t *n) {
  if (n) *n = int64_t(v.size());
  if (cap < int64_t(v.size())) return FRBX_E_RANGE;
  if (out && !v.empty()) std::memcpy(out, v.data(), v.size() * sizeof(T));
  return FRBX_OK;
}

}  // namespace

// ================================================================== C ABI
extern "C" {

const char *frbx_version(void) { return "frbx 0.1 (gfx950)"; }

frbx_status frbx_create(const frbx_layout *L, int device, void *hip_stream, frbx_ctx **out) {
  if (!out) return FRBX_E_INVAL;
  *out = nullptr;
  std::string why;
  frbx_status s = check_layout(L, why);
  if (s != FRBX_OK) {
    std::fprintf(stderr, "frbx_create: %s\n", why.c_str());
    return s;
  }
  int n_dev = 0;
  if (hipGetDeviceCount(&n_dev) != hipSuccess || device < 0 || device >= n_dev) return FRBX_E_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return FRBX_E_DEVICE;
  frbx_ctx *c = new (std::nothrow) frbx_ctx();
  if (!c) return FRBX_E_NOMEM;
  c->B = L->n_baselines;
  c->N = L->n_if;
  c->J = L->n_chan;
  c->K = L->n_frames;
  c->t_ap = L->t_ap_ms;
  c->df = L->chan_bw_mhz;
  c->f0.assign(L->if_freq_mhz, L->if_freq_mhz + L->n_if);
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->tau0.assign(size_t(c->B) * c->N, 0.0);
  c->phi0.assign(size_t(c->B) * c->N, 0.0);
  if (const char *e = std::getenv("FRBX_W_BUDGET_MB")) c->w_budget = size_t(std::atoll(e)) << 20;
  // the device address of this GPU's no-alloc workspace, looked up once per
  // device with the device current (its failure only disables
  // frbx_run_cube_noalloc)
  const hipError_t we = frbx::noalloc_workspace(device, &c->d_noalloc);
  if (we != hipSuccess) {
    c->d_noalloc = nullptr;
    c->noalloc_err = std::string("no-alloc workspace lookup: ") + hipGetErrorString(we);
  }
  *out = c;
  return FRBX_OK;
}

void frbx_destroy(frbx_ctx *ctx) { delete ctx; }

const char *frbx_last_error(const frbx_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

frbx_status frbx_set_calibration(frbx_ctx *c, const double *tau0_us, const double *phi0_rad) {
  if (!c) return FRBX_E_INVAL;
  const size_t n = size_t(c->B) * c->N;
  for (size_t i = 0; i < n; ++i) {
    const double t = tau0_us ? tau0_us[i] : 0.0, p = phi0_rad ? phi0_rad[i] : 0.0;
    if (!std::isfinite(t) || !std::isfinite(p)) return c->fail(FRBX_E_INVAL, "calibration not finite");
  }
  for (size_t i = 0; i < n; ++i) {
    c->tau0[i] = tau0_us ? tau0_us[i] : 0.0;
    c->phi0[i] = phi0_rad ? phi0_rad[i] : 0.0;
  }
  c->dirty = true;
  c->have = false;
  return FRBX_OK;
}

frbx_status frbx_set_dm_grid(frbx_ctx *c, double dm_lo, double dm_step, int32_t n_dm, double k_dm) {
  if (!c) return FRBX_E_INVAL;
  if (n_dm < 1 || n_dm > 65536 || !std::isfinite(dm_lo) || !std::isfinite(dm_step) || dm_lo < 0 ||
      dm_step < 0 || !std::isfinite(k_dm))
    return c->fail(FRBX_E_INVAL, "DM grid: need 1 <= n_dm <= 65536 and finite dm_lo, dm_step >= 0");
  c->dm_lo = dm_lo;
  c->dm_step = dm_step;
  c->n_dm = n_dm;
  c->k_dm = k_dm > 0 ? k_dm : kDefaultKdm;
  c->dirty = true;
  c->have = false;
  return FRBX_OK;
}

frbx_status frbx_set_delay_grid(frbx_ctx *c, int32_t sbd_pad, int32_t n_mbd, double mbd_step_us,
                                double f_ref_fit_mhz) {
  if (!c) return FRBX_E_INVAL;
  if (!(sbd_pad == 1 || sbd_pad == 2 || sbd_pad == 4 || sbd_pad == 8))
    return c->fail(FRBX_E_INVAL, "sbd_pad must be 1, 2, 4 or 8");
  if (!(n_mbd == 16 || n_mbd == 32 || n_mbd == 64 || n_mbd == 128 || n_mbd == 256))
    return c->fail(FRBX_E_INVAL, "n_mbd must be 16, 32, 64, 128 or 256");
  if (!std::isfinite(mbd_step_us)) return c->fail(FRBX_E_INVAL, "mbd_step_us not finite");
  c->sbd_pad = sbd_pad;
  c->n_mbd = n_mbd;
  c->mbd_step_req = mbd_step_us;
  c->f_ref_fit = f_ref_fit_mhz;
  c->dirty = true;
  c->have = false;
  return FRBX_OK;
}

frbx_status frbx_set_rate_grid(frbx_ctx *c, int32_t n_rate, double rate_step) {
  if (!c) return FRBX_E_INVAL;
  if (n_rate < 1 || n_rate > 64 || !std::isfinite(rate_step))
    return c->fail(FRBX_E_INVAL, "rate grid: need 1 <= n_rate <= 64 and a finite step");
  c->n_rate = n_rate;
  c->rate_step_req = rate_step;
  c->dirty = true;
  c->have = false;
  return FRBX_OK;
}

frbx_status frbx_set_windows(frbx_ctx *c, const int32_t *len, int32_t n) {
  if (!c) return FRBX_E_INVAL;
  if (!len || n < 1 || n > frbx::kMaxWindows)
    return c->fail(FRBX_E_INVAL, "need 1..8 window lengths");
  std::vector<int> w(len, len + n);
  for (int i = 0; i < n; ++i) {
    if (w[i] < 1 || w[i] > 4096) return c->fail(FRBX_E_INVAL, "window length must be 1..4096");
    for (int k = 0; k < i; ++k)
      if (w[k] == w[i]) return c->fail(FRBX_E_INVAL, "window lengths must be distinct");
  }
  c->windows = w;
  c->dirty = true;
  c->have = false;
  return FRBX_OK;
}

frbx_status frbx_set_detection(frbx_ctx *c, double threshold, int32_t n_win_min, int32_t n_bl_min) {
  if (!c) return FRBX_E_INVAL;
  if (!std::isfinite(threshold) || n_win_min < 1 || n_bl_min < 1)
    return c->fail(FRBX_E_INVAL, "detection: finite threshold, n_win_min >= 1, n_bl_min >= 1");
  c->threshold = threshold;
  c->n_win_min = n_win_min;
  c->n_bl_min = n_bl_min;
  c->have = false;
  return FRBX_OK;
}

static frbx_status finish_load(frbx_ctx *c, size_t n_cplx, int f16);

static frbx_status load_impl(frbx_ctx *c, const void *vis, int is_device, int f16) {
  if (!c) return FRBX_E_INVAL;
  if (!vis) return c->fail(FRBX_E_INVAL, "vis is NULL");
  if (hipSetDevice(c->device) != hipSuccess) return c->fail(FRBX_E_DEVICE, "hipSetDevice failed");
  c->have = false;
  c->loaded = false;
  const size_t n_cplx = size_t(c->B) * c->N * c->J * size_t(c->K);
  const size_t bytes = n_cplx * (f16 ? 4 : 8);
  if (is_device) {
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, vis) != hipSuccess || at.type != hipMemoryTypeDevice)
      return c->fail(FRBX_E_INVAL, "vis is not a device pointer");
    if (at.device != c->device) return c->fail(FRBX_E_INVAL, "vis is on another device");
    dfree(c->d_vis_own);
    c->d_vis = vis;
  } else {
    dfree(c->d_vis_own);
    if (hipMalloc(&c->d_vis_own, bytes) != hipSuccess)
      return c->fail(FRBX_E_NOMEM, "device allocation for the cross spectra failed");
    frbx_status s = c->hip(hipMemcpyAsync(c->d_vis_own, vis, bytes, hipMemcpyHostToDevice, c->stream),
                           "upload of cross spectra");
    if (s != FRBX_OK) return s;
    c->d_vis = c->d_vis_own;
  }
  c->vis_f16 = f16;
  return finish_load(c, n_cplx, f16);
}

// largest component, for the float16 operand scale of the matrix-core forms
static frbx_status finish_load(frbx_ctx *c, size_t n_cplx, int f16) {
  if (!c->d_absmax && hipMalloc(reinterpret_cast<void **>(&c->d_absmax), sizeof(unsigned int)) != hipSuccess)
    return c->fail(FRBX_E_NOMEM, "device allocation failed");
  unsigned int am = 0;
  frbx_status s = c->hip(hipMemsetAsync(c->d_absmax, 0, sizeof(unsigned int), c->stream), "memset");
  if (s == FRBX_OK) s = c->hip(frbx::launch_absmax(c->d_vis, int64_t(n_cplx), f16, c->d_absmax, c->stream), "absmax launch");
  if (s == FRBX_OK) s = c->hip(hipMemcpyAsync(&am, c->d_absmax, sizeof(am), hipMemcpyDeviceToHost, c->stream), "absmax");
  if (s == FRBX_OK) s = c->hip(hipStreamSynchronize(c->stream), "load");
  if (s != FRBX_OK) return s;
  std::memcpy(&c->vis_absmax, &am, sizeof(float));
  c->loaded = true;
  return FRBX_OK;
}

frbx_status frbx_load(frbx_ctx *c, const void *vis, int is_device) { return load_impl(c, vis, is_device, 0); }

frbx_status frbx_load_f16(frbx_ctx *c, const void *vis, int is_device) { return load_impl(c, vis, is_device, 1); }

frbx_status frbx_load_e4m3(frbx_ctx *c, const void *codes, const float *scale, int is_device) {
  if (!c) return FRBX_E_INVAL;
  if (!codes || !scale) return c->fail(FRBX_E_INVAL, "codes or scale is NULL");
  if (hipSetDevice(c->device) != hipSuccess) return c->fail(FRBX_E_DEVICE, "hipSetDevice failed");
  c->have = false;
  c->loaded = false;
  const int rows = c->B * c->N * c->J;
  const size_t n_cplx = size_t(rows) * size_t(c->K);
  frbx_status s;
  const void *src = codes;
  const float *sc = scale;
  if (!is_device) {
    if ((s = ensure(c, reinterpret_cast<char *&>(c->stage), c->stage_cap, n_cplx * 2)) != FRBX_OK) return s;
    if ((s = c->hip(hipMemcpyAsync(c->stage, codes, n_cplx * 2, hipMemcpyHostToDevice, c->stream), "code upload")) != FRBX_OK)
      return s;
    src = c->stage;
    dfree(c->d_scale);
    if (hipMalloc(reinterpret_cast<void **>(&c->d_scale), size_t(rows) * sizeof(float)) != hipSuccess)
      return c->fail(FRBX_E_NOMEM, "device allocation failed");
    if ((s = c->hip(hipMemcpyAsync(c->d_scale, scale, size_t(rows) * sizeof(float), hipMemcpyHostToDevice, c->stream),
                    "scale upload")) != FRBX_OK)
      return s;
    sc = c->d_scale;
  }
  // decoded exactly into an owned complex64 copy, searched like frbx_load's input
  dfree(c->d_vis_own);
  if (hipMalloc(&c->d_vis_own, n_cplx * sizeof(float2)) != hipSuccess)
    return c->fail(FRBX_E_NOMEM, "device allocation for the cross spectra failed");
  if ((s = c->hip(frbx::launch_ingest(src, FRBX_IN_E4M3, sc, c->K, rows, static_cast<float2 *>(c->d_vis_own), c->K, 0,
                                      c->stream), "fp8 decode")) != FRBX_OK)
    return s;
  c->d_vis = c->d_vis_own;
  c->vis_f16 = 0;
  return finish_load(c, n_cplx, 0);
}

frbx_status frbx_set_tile_budget(frbx_ctx *c, int64_t bytes) {
  if (!c) return FRBX_E_INVAL;
  if (bytes < 0) return c->fail(FRBX_E_INVAL, "tile budget must be >= 0");
  c->w_budget = bytes > 0 ? size_t(bytes) : (size_t(6) << 30);
  c->w_budget_strict = bytes > 0;
  return FRBX_OK;
}

frbx_status frbx_set_precision(frbx_ctx *c, int32_t precision) {
  if (!c) return FRBX_E_INVAL;
  if (precision != FRBX_PREC_F32 && precision != FRBX_PREC_F16X3 && precision != FRBX_PREC_F16)
    return c->fail(FRBX_E_INVAL, "unknown precision");
  c->precision = precision;
  c->dirty = true;
  c->have = false;
  return FRBX_OK;
}

frbx_status frbx_set_sbd_matrix_cores(frbx_ctx *c, int enable) {
  if (!c) return FRBX_E_INVAL;
  c->sbd_mfma = enable ? 1 : 0;
  c->dirty = true;
  return FRBX_OK;
}

frbx_status frbx_set_specialisation(frbx_ctx *c, int enable) {
  if (!c) return FRBX_E_INVAL;
  c->specialise = enable ? 1 : 0;
  c->dirty = true;
  return FRBX_OK;
}

frbx_status frbx_get_specialisation(const frbx_ctx *c, uint32_t *rows, const char **why) {
  if (!c) return FRBX_E_INVAL;
  if (rows) *rows = c->rows_mask;
  if (why) *why = c->rows_note.c_str();
  return FRBX_OK;
}

frbx_status frbx_set_recheck(frbx_ctx *c, double band) {
  if (!c) return FRBX_E_INVAL;
  if (!(band >= 0.0)) return c->fail(FRBX_E_INVAL, "recheck band must be >= 0");
  c->recheck_band = band;
  c->have = false;
  return FRBX_OK;
}

frbx_status frbx_get_recheck(const frbx_ctx *c, double *band, int64_t *n_last) {
  if (!c) return FRBX_E_INVAL;
  if (band) *band = c->recheck_band;
  if (n_last) *n_last = c->n_rechecked;
  return FRBX_OK;
}

}  // extern "C"

namespace {

// One pass of the device search over APs [0, K) of an input buffer
// (complex64 / complex32, layout [B][N J][K]) with, per window, segments
// k0 = k0_w + q hop_w for q < nq_w: dedispersion and fringe search per
// (baseline, DM tile), Eq. 6 statistics and threshold over each window's
// segments of this pass.  Leaves the cube in d_power / d_pidx ([B][D][S]),
// the statistics in c->mean / sd / cnt and the crossings (local q) in `hc`.
struct PassSpec {
  const void *vis;
  int vis_f16;
  int64_t K;        // APs available per channel
  int64_t stride;   // elements between channel rows
  std::vector<int> k0, nq, off;
  int64_t S;
};

// Eq. 6 statistics of every (baseline, DM trial, window) row and the
// segments whose normalised power exceeds `thr` (unordered) into `hc`.
frbx_status stats_pass(frbx_ctx *c, frbx::StatsArgs &st, size_t rows, int64_t S, double thr,
                       std::vector<DevCrossing> &hc) {
  frbx_status s;
  st.threshold = thr;
  st.out = c->d_cross;
  st.cap = c->cross_cap;
  unsigned long long ncr = 0;
  for (int attempt = 0; attempt < 2; ++attempt) {
    if ((s = c->hip(hipMemsetAsync(c->d_ncross, 0, sizeof(unsigned long long), c->stream), "memset")) != FRBX_OK)
      return s;
    const int sp = S > 0 ? c->span_begin(2, int64_t(rows)) : -1;
    if (S > 0 && (s = c->hip(frbx::launch_stats(st, int(rows), c->stream), "stats launch")) != FRBX_OK) return s;
    c->span_end(sp);
    if ((s = c->hip(hipMemcpyAsync(&ncr, c->d_ncross, sizeof(ncr), hipMemcpyDeviceToHost, c->stream),
                    "crossing count")) != FRBX_OK)
      return s;
    if ((s = c->hip(hipStreamSynchronize(c->stream), "search")) != FRBX_OK) return s;
    if (int64_t(ncr) <= c->cross_cap) break;
    dfree(c->d_cross);
    c->cross_cap = 0;
    if (hipMalloc(reinterpret_cast<void **>(&c->d_cross), size_t(ncr) * sizeof(DevCrossing)) != hipSuccess)
      return c->fail(FRBX_E_NOMEM, "device allocation for crossings failed");
    c->cross_cap = int64_t(ncr);
    st.out = c->d_cross;
    st.cap = c->cross_cap;
  }
  hc.assign(ncr, DevCrossing{});
  if (ncr && (s = c->hip(hipMemcpy(hc.data(), c->d_cross, ncr * sizeof(DevCrossing), hipMemcpyDeviceToHost),
                         "crossings copy")) != FRBX_OK)
    return s;
  return FRBX_OK;
}

// Re-evaluation after a matrix-core pass: the segments whose normalised
// power (with this pass's statistics) exceeds threshold - band, i.e. every
// crossing and every segment near the threshold, are searched again by the
// float32 kernel in one launch (one work-group per segment, the segment
// sums gathered straight from the input); their powers and indices in the
// cube are replaced, so the crossings carry float32 peaks and cells.
frbx_status recheck_pass(frbx_ctx *c, const PassSpec &ps, frbx::StatsArgs &st, size_t rows) {
  frbx_status s;
  const int D = c->n_dm, NJ = c->N * c->J, nw = int(c->windows.size()), J = c->J, M = c->n_mbd;
  const int64_t S = ps.S;
  if (!frbx::fringe_supported(J, M, c->N, c->sbd_pad))
    return c->fail(FRBX_E_INVAL, "recheck needs a shape the float32 search supports");
  std::vector<DevCrossing> near;
  if ((s = stats_pass(c, st, rows, S, c->threshold - c->recheck_band, near)) != FRBX_OK) return s;
  std::vector<int32_t> list;
  for (const DevCrossing &x : near) {
    const int bd = x.row / nw;
    list.push_back(bd / D);
    list.push_back(bd % D);
    list.push_back(int32_t(ps.off[x.row % nw] + x.q));
  }
  const int64_t n = int64_t(list.size() / 3);
  c->n_rechecked = n;
  if (n == 0) return FRBX_OK;
  if (n > 2147483647) return c->fail(FRBX_E_INVAL, "too many segments to re-evaluate");
  if ((s = ensure(c, c->d_list, c->list_cap, list.size())) != FRBX_OK) return s;
  if ((s = c->hip(hipMemcpy(c->d_list, list.data(), list.size() * sizeof(int32_t), hipMemcpyHostToDevice),
                  "list upload")) != FRBX_OK)
    return s;
  frbx::FringeArgs fa{};
  fa.n_if = c->N;
  fa.n_rate = c->n_rate;
  fa.sbd_pad = c->sbd_pad;
  fa.n_win = nw;
  for (int w = 0; w < nw; ++w) {
    fa.win_len[w] = c->windows[w];
    fa.win_hop[w] = c->hop[w];
    fa.win_off[w] = ps.off[w];
    fa.win_k0[w] = ps.k0[w];
    fa.rate_off[w] = c->rate_off[w];
  }
  fa.seg_total = int(S);
  fa.n_dt = D;
  fa.rate_ph = c->d_rate;
  fa.tw_sbd = c->d_tw_sbd;
  fa.pre_sbd = c->d_pre;
  fa.tw_mbd = c->d_tw_mbd;
  fa.mbd_row = c->d_row;
  fa.mbd_pos = c->mbd_pos.empty() ? nullptr : c->d_pos;
  fa.seg_list = c->d_list;
  fa.vis = ps.vis;
  fa.vis_f16 = ps.vis_f16;
  fa.n_dm = D;
  fa.vis_stride = ps.stride;
  fa.vis_frames = ps.K;
  fa.dk = c->d_dk;
  fa.cal = c->d_cal;
  fa.power = c->d_power;
  fa.pidx = c->d_pidx;
  const size_t lds = frbx::fringe_lds_bytes(J, M, c->N, c->sbd_pad);
  return c->hip(frbx::launch_fringe_list(J, M, fa, lds, int(n), c->stream), "recheck launch");
}

// Dedispersion and fringe search of every (baseline, DM tile): the DM
// trials are taken dt at a time through the dedispersed-tile buffer wbuf
// ([dt][k_eff][N J]), and every segment's peak goes into the cube
// power / pidx ([B][D][S]).
frbx_status search_tiles(frbx_ctx *c, const PassSpec &ps, float2 *wbuf, int dt, float *power, int32_t *pidx) {
  const int B = c->B, D = c->n_dm, NJ = c->N * c->J, nw = int(c->windows.size());
  const int64_t S = ps.S;
  const int64_t k_eff = ps.K - c->dk_max;
  const int J = c->J, M = c->n_mbd;
  frbx_status s;
  const bool use_mfma = c->precision != FRBX_PREC_F32;
  const size_t lds = frbx::fringe_lds_bytes(J, M, c->N, c->sbd_pad);
  const float scale = mfma_scale(c);
  const size_t in_bytes = ps.vis_f16 ? 4 : 8;
  if (S > 0 && k_eff > 0) {
    for (int b = 0; b < B; ++b) {
      for (int d0 = 0; d0 < D; d0 += dt) {
        const int ndt = std::min(dt, D - d0);
        frbx::DedisperseArgs da{};
        da.vis = static_cast<const char *>(ps.vis) + size_t(b) * NJ * size_t(ps.stride) * in_bytes;
        da.in_f16 = ps.vis_f16;
        da.n_frames = ps.K;
        da.row_stride = ps.stride;
        da.dk = c->d_dk;
        da.d0 = d0;
        da.n_dt = ndt;
        da.cal = c->d_cal + size_t(b) * NJ;
        da.out = wbuf;
        da.k_eff = k_eff;
        da.nj = NJ;
        da.group = c->dd_group;
        int sp = c->span_begin(1, int64_t(ndt) * k_eff);
        if (sp >= 0) {
          // writes: ndt x k_eff spectra; reads: each channel's span of
          // k_eff + (offset spread of the group) APs once per group
          int64_t bytes = int64_t(ndt) * k_eff * NJ * 8;
          for (int g0 = 0; g0 < ndt; g0 += c->dd_group) {
            const int g1 = std::min(ndt, g0 + c->dd_group) - 1;
            const int32_t *a0 = c->dk.data() + size_t(d0 + g0) * NJ, *a1 = c->dk.data() + size_t(d0 + g1) * NJ;
            for (int i = 0; i < NJ; ++i) bytes += (k_eff + (a1[i] - a0[i])) * int64_t(in_bytes);
          }
          c->spans[sp].bytes = bytes;
        }
        if ((s = c->hip(frbx::launch_dedisperse(da, c->stream), "dedisperse launch")) != FRBX_OK) return s;
        c->span_end(sp);
        frbx::FringeArgs fa{};
        fa.w = wbuf;
        fa.w_dm_stride = k_eff * NJ;
        fa.n_if = c->N;
        fa.n_rate = c->n_rate;
        fa.sbd_pad = c->sbd_pad;
        fa.n_win = nw;
        for (int w = 0; w < nw; ++w) {
          fa.win_len[w] = c->windows[w];
          fa.win_hop[w] = c->hop[w];
          fa.win_off[w] = ps.off[w];
          fa.win_k0[w] = ps.k0[w];
          fa.rate_off[w] = c->rate_off[w];
        }
        fa.seg_total = int(S);
        fa.n_dt = ndt;
        fa.rate_ph = c->d_rate;
        fa.tw_sbd = c->d_tw_sbd;
        fa.pre_sbd = c->d_pre;
        fa.tw_mbd = c->d_tw_mbd;
        fa.mbd_row = c->d_row;
        fa.mbd_pos = c->mbd_pos.empty() ? nullptr : c->d_pos;
        fa.power = power + (size_t(b) * D + d0) * S;
        fa.pidx = pidx + (size_t(b) * D + d0) * S;
        fa.dump = nullptr;
        fa.mfma_b_hi = c->d_mfma_hi;
        fa.mfma_b_lo = c->d_mfma_lo;
        fa.mfma_scale = scale;
        sp = c->span_begin(0, int64_t(ndt) * S);
        const hipError_t le =
            use_mfma    ? launch_matrix_core(c, fa, int(ndt * S))
            : c->rows_fn ? frbx::launch_fringe_rows(c->rows_fn, fa, lds, int(ndt * S), c->stream)
                         : frbx::launch_fringe(J, M, fa, lds, int(ndt * S), c->stream);
        if ((s = c->hip(le, "fringe launch")) != FRBX_OK) return s;
        c->span_end(sp);
      }
    }
  }
  return FRBX_OK;
}

frbx_status device_pass(frbx_ctx *c, const PassSpec &ps, std::vector<DevCrossing> &hc) {
  frbx_status s;
  const int B = c->B, D = c->n_dm, NJ = c->N * c->J, nw = int(c->windows.size());
  const int64_t S = ps.S;
  const int64_t k_eff = ps.K - c->dk_max;
  const size_t per_dm = size_t(std::max<int64_t>(k_eff, 0)) * NJ;
  if (c->w_budget_strict && per_dm * sizeof(float2) > c->w_budget)
    return c->fail(FRBX_E_NOMEM, "tile budget of " + std::to_string(c->w_budget) + " bytes is below one DM trial's " +
                                     "dedispersed tile (" + std::to_string(per_dm * sizeof(float2)) + " bytes)");
  c->dt = per_dm ? int(std::max<size_t>(1, std::min<size_t>(D, c->w_budget / (per_dm * sizeof(float2))))) : 1;
  while (c->dt > 1 && int64_t(c->dt) * S > (int64_t(1) << 31) - 1) c->dt /= 2;
  if ((s = ensure(c, c->d_w, c->w_cap, per_dm * c->dt)) != FRBX_OK) return s;
  const size_t cube = size_t(B) * D * std::max<int64_t>(S, 1);
  if ((s = ensure(c, c->d_power, c->cube_cap, cube)) != FRBX_OK) return s;
  if ((s = ensure(c, c->d_pidx, c->pidx_cap, cube)) != FRBX_OK) return s;
  const size_t rows = size_t(B) * D * nw;
  if ((s = ensure(c, c->d_mean, c->mean_cap, rows)) != FRBX_OK) return s;
  if ((s = ensure(c, c->d_sd, c->sd_cap, rows)) != FRBX_OK) return s;
  if ((s = ensure(c, c->d_cnt, c->cnt_cap, rows)) != FRBX_OK) return s;
  if (!c->d_ncross && hipMalloc(reinterpret_cast<void **>(&c->d_ncross), sizeof(unsigned long long)) != hipSuccess)
    return c->fail(FRBX_E_NOMEM, "device allocation failed");
  const int64_t want_cap = std::max<int64_t>(int64_t(1) << 16, int64_t(cube / 64));
  if (c->cross_cap < want_cap) {
    dfree(c->d_cross);
    c->cross_cap = 0;
    if (hipMalloc(reinterpret_cast<void **>(&c->d_cross), size_t(want_cap) * sizeof(DevCrossing)) != hipSuccess)
      return c->fail(FRBX_E_NOMEM, "device allocation failed");
    c->cross_cap = want_cap;
  }
  const bool use_mfma = c->precision != FRBX_PREC_F32;
  if ((s = search_tiles(c, ps, c->d_w, c->dt, c->d_power, c->d_pidx)) != FRBX_OK) return s;
  // Eq. 6 statistics and threshold crossings
  frbx::StatsArgs st{};
  st.power = c->d_power;
  st.pidx = c->d_pidx;
  st.seg_total = int(S);
  st.n_win = nw;
  for (int w = 0; w < nw; ++w) {
    st.win_off[w] = ps.off[w];
    st.win_q[w] = ps.nq[w];
  }
  st.mean = c->d_mean;
  st.stdev = c->d_sd;
  st.count = c->d_cnt;
  st.n_out = c->d_ncross;
  c->n_rechecked = 0;
  if (use_mfma && c->recheck_band > 0 && S > 0 && k_eff > 0 && (s = recheck_pass(c, ps, st, rows)) != FRBX_OK)
    return s;
  if ((s = stats_pass(c, st, rows, S, c->threshold, hc)) != FRBX_OK) return s;
  if (c->timing) c->collect_timing();
  c->mean.assign(rows, 0.0);
  c->sd.assign(rows, 0.0);
  c->cnt.assign(rows, 0);
  if (rows && S > 0) {
    if ((s = c->hip(hipMemcpy(c->mean.data(), c->d_mean, rows * sizeof(double), hipMemcpyDeviceToHost), "stats")) != FRBX_OK ||
        (s = c->hip(hipMemcpy(c->sd.data(), c->d_sd, rows * sizeof(double), hipMemcpyDeviceToHost), "stats")) != FRBX_OK ||
        (s = c->hip(hipMemcpy(c->cnt.data(), c->d_cnt, rows * sizeof(int64_t), hipMemcpyDeviceToHost), "stats")) != FRBX_OK)
      return s;
  }
  std::sort(hc.begin(), hc.end(), [](const DevCrossing &x, const DevCrossing &y) {
    return x.row != y.row ? x.row < y.row : x.q < y.q;
  });
  c->cube_len = S;
  c->last_off = ps.off;
  c->last_nq = ps.nq;
  return FRBX_OK;
}

// crossing record of segment q_global of window w
frbx_candidate make_crossing(const frbx_ctx *c, const DevCrossing &x, int64_t q_global) {
  const int nw = int(c->windows.size()), D = c->n_dm, M = c->n_mbd, PJ = c->sbd_pad * c->J;
  frbx_candidate k{};
  const int w = x.row % nw, bd = x.row / nw;
  k.baseline = bd / D;
  k.dm_index = bd % D;
  k.window_index = w;
  k.window_len = c->windows[w];
  k.segment = q_global;
  k.k0 = q_global * c->hop[w];
  k.dm = c->dm_lo + k.dm_index * c->dm_step;
  k.power = x.power;
  k.power_norm = x.pnorm;
  const int m = x.idx % M, sb = (x.idx / M) % PJ, r = x.idx / (M * PJ);
  k.rate_idx = r;
  k.sbd_idx = sb;
  k.mbd_idx = m;
  k.rate = (r - c->n_rate / 2) * c->rate_step;
  k.sbd_us = (sb - PJ / 2.0) / (PJ * c->df);
  k.mbd_us = (m - M / 2.0) * c->mbd_step;
  k.n_windows = 0;
  k.group_id = -1;
  return k;
}

}  // namespace

extern "C" {

frbx_status frbx_run(frbx_ctx *c) {
  if (!c) return FRBX_E_INVAL;
  if (!c->loaded) return c->fail(FRBX_E_STATE, "frbx_run before frbx_load");
  if (hipSetDevice(c->device) != hipSuccess) return c->fail(FRBX_E_DEVICE, "hipSetDevice failed");
  c->have = false;
  c->spans.clear();
  c->ev_used = 0;
  frbx_status s = prepare(c);
  if (s != FRBX_OK) return s;
  c->streaming = false;
  const int nw = int(c->windows.size());
  PassSpec ps;
  ps.vis = c->d_vis;
  ps.vis_f16 = c->vis_f16;
  ps.K = c->K;
  ps.stride = c->K;
  ps.k0.assign(nw, 0);
  ps.nq = c->nseg;
  ps.off = c->segoff;
  ps.S = c->seg_total;
  std::vector<DevCrossing> hc;
  if ((s = device_pass(c, ps, hc)) != FRBX_OK) return s;
  c->cross.clear();
  c->cross.reserve(hc.size());
  for (const DevCrossing &x : hc) c->cross.push_back(make_crossing(c, x, x.q));
  detect_impl(c->cross.data(), int64_t(c->cross.size()), c->t_amb, c->n_win_min, c->n_bl_min, true,
              c->dets, c->groups);
  c->have = true;
  return FRBX_OK;
}

frbx_status frbx_run_cube_noalloc(frbx_ctx *c, float *power, int32_t *idx, int64_t cap, int64_t *n) {
  if (!c) return FRBX_E_INVAL;
  if (!c->loaded) return c->fail(FRBX_E_STATE, "frbx_run_cube_noalloc before frbx_load");
  if (c->dirty)
    return c->fail(FRBX_E_STATE, "grid tables not built: call frbx_get_segments (or frbx_run) after the last "
                                 "setter; frbx_run_cube_noalloc builds nothing");
  if (!c->d_noalloc) return c->fail(FRBX_E_DEVICE, c->noalloc_err.empty() ? "no-alloc workspace unavailable" : c->noalloc_err);
  if (hipSetDevice(c->device) != hipSuccess) return c->fail(FRBX_E_DEVICE, "hipSetDevice failed");
  const int D = c->n_dm, NJ = c->N * c->J;
  const int64_t S = c->seg_total;
  const int64_t len = int64_t(c->B) * D * S;
  if (n) *n = len;
  if (cap < len) return c->fail(FRBX_E_RANGE, "output capacity below B x D x segments");
  if (len == 0) return FRBX_OK;
  if (!power || !idx) return c->fail(FRBX_E_INVAL, "null output pointer");
  const int64_t k_eff = c->K - c->dk_max;
  const size_t per_dm = size_t(k_eff) * NJ * sizeof(float2);
  if (per_dm > frbx::kNoAllocBytes)
    return c->fail(FRBX_E_INVAL, "one DM trial's dedispersed tile (" + std::to_string(per_dm) +
                                     " bytes) exceeds the no-alloc workspace (" +
                                     std::to_string(frbx::kNoAllocBytes) + " bytes)");
  int dt = int(std::min<size_t>(size_t(D), frbx::kNoAllocBytes / per_dm));
  while (dt > 1 && int64_t(dt) * S > (int64_t(1) << 31) - 1) dt /= 2;
  if (int64_t(dt) * S > (int64_t(1) << 31) - 1) return c->fail(FRBX_E_INVAL, "too many segments per DM trial");
  const int nw = int(c->windows.size());
  PassSpec ps;
  ps.vis = c->d_vis;
  ps.vis_f16 = c->vis_f16;
  ps.K = c->K;
  ps.stride = c->K;
  ps.k0.assign(nw, 0);
  ps.nq = c->nseg;
  ps.off = c->segoff;
  ps.S = S;
  // no timing events (their pool may grow): launches only
  const bool tm = c->timing;
  c->timing = false;
  const frbx_status s = search_tiles(c, ps, static_cast<float2 *>(c->d_noalloc), dt, power, idx);
  c->timing = tm;
  return s;
}

frbx_status frbx_stream_begin(frbx_ctx *c, int64_t chunk_frames) {
  if (!c) return FRBX_E_INVAL;
  if (chunk_frames < 1) return c->fail(FRBX_E_INVAL, "chunk_frames must be >= 1");
  if (hipSetDevice(c->device) != hipSuccess) return c->fail(FRBX_E_DEVICE, "hipSetDevice failed");
  frbx_status s = prepare(c);
  if (s != FRBX_OK) return s;
  int lmax = 1;
  for (int l : c->windows) lmax = std::max(lmax, l);
  c->chunk = chunk_frames;
  c->carry = c->dk_max + lmax - 1;
  c->buf_frames = c->carry + chunk_frames;
  const size_t n = size_t(c->B) * c->N * c->J * size_t(c->buf_frames);
  for (int i = 0; i < 2; ++i) {
    dfree(c->sbuf[i]);
    if (hipMalloc(reinterpret_cast<void **>(&c->sbuf[i]), n * sizeof(float2)) != hipSuccess)
      return c->fail(FRBX_E_NOMEM, "device allocation for the stream buffers failed");
    if ((s = c->hip(hipMemset(c->sbuf[i], 0, n * sizeof(float2)), "memset")) != FRBX_OK) return s;
  }
  c->cur = 0;
  c->valid = c->buf_start = c->frames_in = 0;
  const int nw = int(c->windows.size());
  c->next_q.assign(nw, 0);
  c->push_first.assign(nw, 0);
  c->push_nq.assign(nw, 0);
  c->stream_cross.clear();
  c->streaming = true;
  c->have = false;
  return FRBX_OK;
}

frbx_status frbx_stream_push(frbx_ctx *c, const void *chunk, int32_t kind, const float *scale, int is_device) {
  if (!c) return FRBX_E_INVAL;
  if (!c->streaming) return c->fail(FRBX_E_STATE, "frbx_stream_push before frbx_stream_begin");
  if (c->dirty) return c->fail(FRBX_E_STATE, "grids changed since frbx_stream_begin");
  if (!chunk || kind < FRBX_IN_C64 || kind > FRBX_IN_E4M3 || (kind == FRBX_IN_E4M3 && !scale))
    return c->fail(FRBX_E_INVAL, "bad chunk, kind or scale");
  if (hipSetDevice(c->device) != hipSuccess) return c->fail(FRBX_E_DEVICE, "hipSetDevice failed");
  c->have = false;
  c->spans.clear();
  c->ev_used = 0;
  frbx_status s;
  const int NJ = c->N * c->J, rows = c->B * NJ, nw = int(c->windows.size());
  const size_t elem = kind == FRBX_IN_C64 ? 8 : kind == FRBX_IN_C32 ? 4 : 2;
  const size_t bytes = size_t(rows) * size_t(c->chunk) * elem;
  const void *src = chunk;
  const float *sc = scale;
  if (!is_device) {
    if ((s = ensure(c, reinterpret_cast<char *&>(c->stage), c->stage_cap, bytes)) != FRBX_OK) return s;
    if ((s = c->hip(hipMemcpyAsync(c->stage, chunk, bytes, hipMemcpyHostToDevice, c->stream), "chunk upload")) != FRBX_OK)
      return s;
    src = c->stage;
    if (kind == FRBX_IN_E4M3) {
      if (!c->d_scale && hipMalloc(reinterpret_cast<void **>(&c->d_scale), size_t(rows) * sizeof(float)) != hipSuccess)
        return c->fail(FRBX_E_NOMEM, "device allocation failed");
      if ((s = c->hip(hipMemcpyAsync(c->d_scale, scale, size_t(rows) * sizeof(float), hipMemcpyHostToDevice, c->stream),
                      "scale upload")) != FRBX_OK)
        return s;
      sc = c->d_scale;
    }
  }
  // carry the last dk_max + l_max - 1 APs into the other buffer, append the chunk
  const int other = 1 - c->cur;
  const int64_t keep = std::min(c->carry, c->valid);
  if ((s = c->hip(frbx::launch_carry(c->sbuf[c->cur], c->sbuf[other], rows, c->buf_frames, c->valid - keep, keep,
                                     c->stream), "carry")) != FRBX_OK)
    return s;
  if ((s = c->hip(frbx::launch_ingest(src, kind, sc, c->chunk, rows, c->sbuf[other], c->buf_frames, keep, c->stream),
                  "ingest")) != FRBX_OK)
    return s;
  c->buf_start = c->frames_in == 0 ? 0 : c->buf_start + c->valid - keep;
  c->valid = keep + c->chunk;
  c->cur = other;
  c->frames_in += c->chunk;
  // float16 operand scale of the matrix-core forms from this buffer
  if (c->precision != FRBX_PREC_F32) {
    if (!c->d_absmax && hipMalloc(reinterpret_cast<void **>(&c->d_absmax), sizeof(unsigned int)) != hipSuccess)
      return c->fail(FRBX_E_NOMEM, "device allocation failed");
    unsigned int am = 0;
    s = c->hip(hipMemsetAsync(c->d_absmax, 0, sizeof(unsigned int), c->stream), "memset");
    if (s == FRBX_OK)
      s = c->hip(frbx::launch_absmax(c->sbuf[c->cur], int64_t(rows) * c->buf_frames, 0, c->d_absmax, c->stream), "absmax");
    if (s == FRBX_OK) s = c->hip(hipMemcpyAsync(&am, c->d_absmax, sizeof(am), hipMemcpyDeviceToHost, c->stream), "absmax");
    if (s == FRBX_OK) s = c->hip(hipStreamSynchronize(c->stream), "absmax");
    if (s != FRBX_OK) return s;
    std::memcpy(&c->vis_absmax, &am, sizeof(float));
  }
  // the segments this push completes
  PassSpec ps;
  ps.vis = c->sbuf[c->cur];
  ps.vis_f16 = 0;
  ps.K = c->valid;
  ps.stride = c->buf_frames;
  ps.k0.assign(nw, 0);
  ps.nq.assign(nw, 0);
  ps.off.assign(nw, 0);
  int64_t tot = 0;
  for (int w = 0; w < nw; ++w) {
    const int l = c->windows[w], h = c->hop[w];
    const int64_t last = c->buf_start + c->valid - c->dk_max - l;  // latest complete start AP
    const int64_t qhi = last >= 0 ? last / h : -1;
    const int64_t nq = std::max<int64_t>(0, qhi - c->next_q[w] + 1);
    const int64_t k0 = c->next_q[w] * h - c->buf_start;
    if (nq > 0 && k0 < 0) return c->fail(FRBX_E_STATE, "stream carry too short");
    ps.k0[w] = int(std::max<int64_t>(k0, 0));
    ps.nq[w] = int(nq);
    ps.off[w] = int(tot);
    tot += nq;
    c->push_first[w] = c->next_q[w];
    c->push_nq[w] = nq;
  }
  ps.S = tot;
  std::vector<DevCrossing> hc;
  if ((s = device_pass(c, ps, hc)) != FRBX_OK) return s;
  c->cross.clear();
  for (const DevCrossing &x : hc) {
    const int w = x.row % nw;
    c->cross.push_back(make_crossing(c, x, c->push_first[w] + x.q));
  }
  for (int w = 0; w < nw; ++w) c->next_q[w] += c->push_nq[w];
  c->stream_cross.insert(c->stream_cross.end(), c->cross.begin(), c->cross.end());
  detect_impl(c->stream_cross.data(), int64_t(c->stream_cross.size()), c->t_amb, c->n_win_min, c->n_bl_min, true,
              c->dets, c->groups);
  c->have = true;
  return FRBX_OK;
}

frbx_status frbx_stream_position(const frbx_ctx *c, int64_t *frames_in, int64_t *first, int64_t *nseg) {
  if (!c) return FRBX_E_INVAL;
  if (!c->streaming) return FRBX_E_STATE;
  if (frames_in) *frames_in = c->frames_in;
  for (size_t w = 0; w < c->windows.size(); ++w) {
    if (first) first[w] = c->push_first[w];
    if (nseg) nseg[w] = c->push_nq[w];
  }
  return FRBX_OK;
}

frbx_status frbx_get_segments(const frbx_ctx *cc, int64_t *dk_max, int32_t *hop, int64_t *n_seg,
                              int64_t *cube_len) {
  frbx_ctx *c = const_cast<frbx_ctx *>(cc);
  if (!c) return FRBX_E_INVAL;
  frbx_status s = prepare(c);
  if (s != FRBX_OK) return s;
  if (dk_max) *dk_max = c->dk_max;
  for (size_t w = 0; w < c->windows.size(); ++w) {
    if (hop) hop[w] = c->hop[w];
    if (n_seg) n_seg[w] = c->nseg[w];
  }
  if (cube_len) *cube_len = c->seg_total;
  return FRBX_OK;
}

frbx_status frbx_get_lattice(const frbx_ctx *cc, int64_t *q, double *mbd_step_us, int32_t *compact_shift) {
  frbx_ctx *c = const_cast<frbx_ctx *>(cc);
  if (!c) return FRBX_E_INVAL;
  frbx_status s = prepare(c);
  if (s != FRBX_OK) return s;
  if (q)
    for (int n = 0; n < c->N; ++n) q[n] = c->q_if[n];
  if (mbd_step_us) *mbd_step_us = c->mbd_step;
  if (compact_shift) *compact_shift = c->mbd_shift;
  return FRBX_OK;
}

frbx_status frbx_get_ap_offsets(const frbx_ctx *cc, int32_t *out, int64_t cap, int64_t *n) {
  frbx_ctx *c = const_cast<frbx_ctx *>(cc);
  if (!c) return FRBX_E_INVAL;
  frbx_status s = prepare(c);
  if (s != FRBX_OK) return s;
  return copy_out(c->dk, out, cap, n);
}

frbx_status frbx_get_power_cube(const frbx_ctx *c, float *power, int32_t *idx, int64_t cap, int64_t *n) {
  if (!c) return FRBX_E_INVAL;
  if (!c->have) return FRBX_E_STATE;
  const int64_t len = int64_t(c->B) * c->n_dm * c->cube_len;
  if (n) *n = len;
  if (cap < len) return FRBX_E_RANGE;
  hipSetDevice(c->device);
  if (power && len && hipMemcpy(power, c->d_power, len * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
    return FRBX_E_DEVICE;
  if (idx && len && hipMemcpy(idx, c->d_pidx, len * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
    return FRBX_E_DEVICE;
  return FRBX_OK;
}

frbx_status frbx_get_power_cube_device(const frbx_ctx *c, const float **power, const int32_t **idx) {
  if (!c) return FRBX_E_INVAL;
  if (!c->have) return FRBX_E_STATE;
  if (power) *power = c->d_power;
  if (idx) *idx = c->d_pidx;
  return FRBX_OK;
}

frbx_status frbx_get_stats(const frbx_ctx *c, double *mean, double *stdev, int64_t *count, int64_t cap,
                           int64_t *n) {
  if (!c) return FRBX_E_INVAL;
  if (!c->have) return FRBX_E_STATE;
  const int64_t len = int64_t(c->mean.size());
  if (n) *n = len;
  if (cap < len) return FRBX_E_RANGE;
  if (mean) std::copy(c->mean.begin(), c->mean.end(), mean);
  if (stdev) std::copy(c->sd.begin(), c->sd.end(), stdev);
  if (count) std::copy(c->cnt.begin(), c->cnt.end(), count);
  return FRBX_OK;
}

frbx_status frbx_get_crossings(const frbx_ctx *c, frbx_candidate *out, int64_t cap, int64_t *n) {
  if (!c) return FRBX_E_INVAL;
  if (!c->have) return FRBX_E_STATE;
  return copy_out(c->cross, out, cap, n);
}

frbx_status frbx_get_candidates(const frbx_ctx *c, frbx_candidate *out, int64_t cap, int64_t *n) {
  if (!c) return FRBX_E_INVAL;
  if (!c->have) return FRBX_E_STATE;
  return copy_out(c->dets, out, cap, n);
}

frbx_status frbx_get_groups(const frbx_ctx *c, frbx_group *out, int64_t cap, int64_t *n) {
  if (!c) return FRBX_E_INVAL;
  if (!c->have) return FRBX_E_STATE;
  return copy_out(c->groups, out, cap, n);
}

frbx_status frbx_dump_segment(frbx_ctx *c, int32_t b, int32_t d, int32_t w, int64_t q, float *dev_out) {
  if (!c) return FRBX_E_INVAL;
  if (!c->loaded) return c->fail(FRBX_E_STATE, "dump before frbx_load");
  if (!dev_out) return c->fail(FRBX_E_INVAL, "dev_out is NULL");
  if (hipSetDevice(c->device) != hipSuccess) return c->fail(FRBX_E_DEVICE, "hipSetDevice failed");
  frbx_status s = prepare(c);
  if (s != FRBX_OK) return s;
  if (b < 0 || b >= c->B || d < 0 || d >= c->n_dm || w < 0 || w >= int(c->windows.size()) || q < 0 ||
      q >= c->nseg[w])
    return c->fail(FRBX_E_INVAL, "segment out of range");
  const int NJ = c->N * c->J;
  const size_t per_dm = size_t(c->k_eff) * NJ;
  if ((s = ensure(c, c->d_w, c->w_cap, std::max(c->w_cap, per_dm))) != FRBX_OK) return s;
  frbx::DedisperseArgs da{};
  da.vis = static_cast<const char *>(c->d_vis) + size_t(b) * NJ * size_t(c->K) * (c->vis_f16 ? 4 : 8);
  da.in_f16 = c->vis_f16;
  da.n_frames = c->K;
  da.row_stride = c->K;
  da.dk = c->d_dk;
  da.d0 = d;
  da.n_dt = 1;
  da.cal = c->d_cal + size_t(b) * NJ;
  da.out = c->d_w;
  da.k_eff = c->k_eff;
  da.nj = NJ;
  da.group = 1;
  if ((s = c->hip(frbx::launch_dedisperse(da, c->stream), "dedisperse launch")) != FRBX_OK) return s;
  frbx::FringeArgs fa{};
  fa.w = c->d_w;
  fa.w_dm_stride = c->k_eff * NJ;
  fa.n_if = c->N;
  fa.n_rate = c->n_rate;
  fa.sbd_pad = c->sbd_pad;
  fa.n_win = int(c->windows.size());
  for (int i = 0; i < fa.n_win; ++i) {
    fa.win_len[i] = c->windows[i];
    fa.win_hop[i] = c->hop[i];
    fa.win_off[i] = c->segoff[i];
    fa.rate_off[i] = c->rate_off[i];
  }
  fa.seg_total = int(c->seg_total);
  fa.n_dt = 1;
  fa.rate_ph = c->d_rate;
  fa.tw_sbd = c->d_tw_sbd;
  fa.pre_sbd = c->d_pre;
  fa.tw_mbd = c->d_tw_mbd;
  fa.mbd_row = c->d_row;
  fa.mbd_pos = c->mbd_pos.empty() ? nullptr : c->d_pos;
  fa.dump = dev_out;
  fa.dump_dl = 0;
  fa.dump_seg = int(c->segoff[w] + q);
  const int n_pass = c->precision == FRBX_PREC_F16X3 ? 3 : 1;
  fa.mfma_b_hi = c->d_mfma_hi;
  fa.mfma_b_lo = c->d_mfma_lo;
  fa.mfma_scale = mfma_scale(c);
  hipError_t le;
  (void)n_pass;
  if (c->precision != FRBX_PREC_F32) {
    le = launch_matrix_core(c, fa, 1);
  } else {
    const size_t lds = frbx::fringe_lds_bytes(c->J, c->n_mbd, c->N, c->sbd_pad);
    le = frbx::launch_fringe(c->J, c->n_mbd, fa, lds, 1, c->stream);
  }
  if ((s = c->hip(le, "fringe launch")) != FRBX_OK) return s;
  return c->hip(hipStreamSynchronize(c->stream), "dump");
}

frbx_status frbx_power_sum(frbx_ctx *c, const int32_t *bl, int32_t n_bl, frbx_candidate *out, int64_t cap,
                           int64_t *n) {
  if (!c) return FRBX_E_INVAL;
  if (!c->have) return c->fail(FRBX_E_STATE, "frbx_power_sum before frbx_run");
  if (!bl || n_bl < 1 || n_bl > c->B) return c->fail(FRBX_E_INVAL, "need 1..B baselines");
  for (int i = 0; i < n_bl; ++i) {
    if (bl[i] < 0 || bl[i] >= c->B) return c->fail(FRBX_E_INVAL, "baseline index out of range");
    for (int k = 0; k < i; ++k)
      if (bl[k] == bl[i]) return c->fail(FRBX_E_INVAL, "baselines must be distinct");
  }
  if (hipSetDevice(c->device) != hipSuccess) return c->fail(FRBX_E_DEVICE, "hipSetDevice failed");
  const int D = c->n_dm, nw = int(c->windows.size());
  const int64_t S = c->cube_len, len = int64_t(D) * S;
  const int rows = D * nw;
  const int64_t bl_stride = int64_t(D) * S;
  std::vector<frbx_candidate> cross;
  if (S > 0) {
    float *d_sum = nullptr;
    int32_t *d_bl = nullptr;
    double *d_m = nullptr, *d_s = nullptr;
    int64_t *d_c = nullptr;
    auto cleanup = [&]() { dfree(d_sum); dfree(d_bl); dfree(d_m); dfree(d_s); dfree(d_c); };
    if (hipMalloc(reinterpret_cast<void **>(&d_sum), size_t(len) * sizeof(float)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&d_bl), size_t(n_bl) * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&d_m), size_t(rows) * sizeof(double)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&d_s), size_t(rows) * sizeof(double)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&d_c), size_t(rows) * sizeof(int64_t)) != hipSuccess) {
      cleanup();
      return c->fail(FRBX_E_NOMEM, "device allocation failed");
    }
    frbx_status s = c->hip(hipMemcpy(d_bl, bl, size_t(n_bl) * sizeof(int32_t), hipMemcpyHostToDevice), "copy");
    if (s == FRBX_OK) s = c->hip(frbx::launch_cube_sum(c->d_power, bl_stride, d_bl, n_bl, d_sum, len, c->stream), "sum launch");
    frbx::StatsArgs st{};
    st.power = d_sum;
    st.pidx = c->d_pidx;
    st.seg_total = int(S);
    st.n_win = nw;
    for (int w = 0; w < nw; ++w) {
      st.win_off[w] = c->last_off[w];
      st.win_q[w] = c->last_nq[w];
    }
    st.threshold = c->threshold;
    st.mean = d_m;
    st.stdev = d_s;
    st.count = d_c;
    st.out = c->d_cross;
    st.n_out = c->d_ncross;
    st.cap = c->cross_cap;
    unsigned long long ncr = 0;
    for (int attempt = 0; attempt < 2 && s == FRBX_OK; ++attempt) {
      s = c->hip(hipMemsetAsync(c->d_ncross, 0, sizeof(unsigned long long), c->stream), "memset");
      if (s == FRBX_OK) s = c->hip(frbx::launch_stats(st, rows, c->stream), "stats launch");
      if (s == FRBX_OK)
        s = c->hip(hipMemcpyAsync(&ncr, c->d_ncross, sizeof(ncr), hipMemcpyDeviceToHost, c->stream), "count");
      if (s == FRBX_OK) s = c->hip(hipStreamSynchronize(c->stream), "power sum");
      if (s != FRBX_OK || int64_t(ncr) <= c->cross_cap) break;
      dfree(c->d_cross);
      c->cross_cap = 0;
      if (hipMalloc(reinterpret_cast<void **>(&c->d_cross), size_t(ncr) * sizeof(DevCrossing)) != hipSuccess) {
        cleanup();
        return c->fail(FRBX_E_NOMEM, "device allocation for crossings failed");
      }
      c->cross_cap = int64_t(ncr);
      st.out = c->d_cross;
      st.cap = c->cross_cap;
    }
    std::vector<DevCrossing> hc(ncr);
    if (s == FRBX_OK && ncr)
      s = c->hip(hipMemcpy(hc.data(), c->d_cross, ncr * sizeof(DevCrossing), hipMemcpyDeviceToHost), "copy");
    cleanup();
    if (s != FRBX_OK) return s;
    std::sort(hc.begin(), hc.end(), [](const DevCrossing &x, const DevCrossing &y) {
      return x.row != y.row ? x.row < y.row : x.q < y.q;
    });
    for (const DevCrossing &x : hc) {
      frbx_candidate k{};
      const int w = x.row % nw;
      k.baseline = -1;
      k.dm_index = x.row / nw;
      k.window_index = w;
      k.window_len = c->windows[w];
      const int64_t qg = (c->streaming ? c->push_first[w] : 0) + x.q;
      k.segment = qg;
      k.k0 = qg * c->hop[w];
      k.dm = c->dm_lo + k.dm_index * c->dm_step;
      k.power = x.power;
      k.power_norm = x.pnorm;
      k.rate_idx = k.sbd_idx = k.mbd_idx = -1;
      k.group_id = -1;
      cross.push_back(k);
    }
  }
  std::vector<frbx_candidate> dets;
  std::vector<frbx_group> groups;
  detect_impl(cross.data(), int64_t(cross.size()), c->t_amb, c->n_win_min, 1, false, dets, groups);
  for (auto &d : dets) d.group_id = -1;
  return copy_out(dets, out, cap, n);
}

frbx_status frbx_calibrate(frbx_ctx *c, int32_t b, int64_t k0, int32_t len, double *tau0, double *phi0) {
  if (!c) return FRBX_E_INVAL;
  if (!c->loaded) return c->fail(FRBX_E_STATE, "frbx_calibrate before frbx_load");
  if (b < 0 || b >= c->B || len < 1 || k0 < 0 || k0 + len > c->K || !tau0 || !phi0)
    return c->fail(FRBX_E_INVAL, "calibrator segment out of range");
  if (hipSetDevice(c->device) != hipSuccess) return c->fail(FRBX_E_DEVICE, "hipSetDevice failed");
  frbx_status s = prepare(c);
  if (s != FRBX_OK) return s;
  const int N = c->N, J = c->J, NJ = N * J;
  float2 *d_y = nullptr;
  if (hipMalloc(reinterpret_cast<void **>(&d_y), size_t(NJ) * sizeof(float2)) != hipSuccess)
    return c->fail(FRBX_E_NOMEM, "device allocation failed");
  const void *vb = static_cast<const char *>(c->d_vis) + size_t(b) * NJ * size_t(c->K) * (c->vis_f16 ? 4 : 8);
  std::vector<float2> hy(NJ);
  s = c->hip(frbx::launch_segment_sum(vb, c->vis_f16, c->K, NJ, k0, len, d_y, c->stream), "segment sum");
  if (s == FRBX_OK) s = c->hip(hipStreamSynchronize(c->stream), "segment sum");
  if (s == FRBX_OK) s = c->hip(hipMemcpy(hy.data(), d_y, size_t(NJ) * sizeof(float2), hipMemcpyDeviceToHost), "copy");
  dfree(d_y);
  if (s != FRBX_OK) return s;
  using cd = std::complex<double>;
  auto cis = [](double cycles) {  // exp(-2 pi i cycles), reduced first
    const double r = cycles - std::nearbyint(cycles);
    return cd(std::cos(kTwoPi * r), -std::sin(kTwoPi * r));
  };
  std::vector<cd> Y(NJ);
  for (int i = 0; i < NJ; ++i) Y[i] = (i % J == 0) ? cd(0, 0) : cd(hy[i].x, hy[i].y);
  // (SBD, MBD) cell of maximum |G| (Eq. 5) on the current grids
  const int PJ = c->sbd_pad * J, M = c->n_mbd;
  const double df = c->df, fbw = J * df;
  const double fref = std::isnan(c->f_ref_fit) ? c->f0[0] : c->f_ref_fit;
  std::vector<cd> X(size_t(N) * PJ);
  for (int n = 0; n < N; ++n)
    for (int sb = 0; sb < PJ; ++sb) {
      cd acc(0, 0);
      for (int j = 1; j < J; ++j)
        acc += Y[size_t(n) * J + j] * cis(double((int64_t(j) * (sb - PJ / 2)) % PJ) / PJ);
      X[size_t(n) * PJ + sb] = acc;
    }
  double best = -1.0;
  int bs = 0, bm = 0;
  std::vector<cd> em(size_t(N) * M);
  for (int n = 0; n < N; ++n)
    for (int m = 0; m < M; ++m) em[size_t(n) * M + m] = cis((c->f0[n] - fref) * (m - M / 2) * c->mbd_step);
  for (int sb = 0; sb < PJ; ++sb)
    for (int m = 0; m < M; ++m) {
      cd acc(0, 0);
      for (int n = 0; n < N; ++n) acc += X[size_t(n) * PJ + sb] * em[size_t(n) * M + m];
      const double a = std::abs(acc);
      if (a > best) best = a, bs = sb, bm = m;
    }
  const double sbd = (bs - PJ / 2.0) / (PJ * df), mbd = (bm - M / 2.0) * c->mbd_step;
  // channel delay per IF, then the initial phase of the delay-corrected sum
  const int NG = 64 * J + 1;
  for (int n = 0; n < N; ++n) {
    std::vector<cd> Z(J);
    for (int j = 0; j < J; ++j) Z[j] = Y[size_t(n) * J + j] * cis(j * df * sbd);
    auto amp = [&](double t) {
      const cd step = cis(df * t);
      cd ph = cis(-fbw / 2.0 * t), acc(0, 0);  // exp(-2 pi i (f_j - f_bw/2) t), j = 0 first
      for (int j = 0; j < J; ++j) {
        acc += Z[j] * ph;
        ph *= step;
      }
      return std::abs(acc);
    };
    const double lo = -0.5 / df, hi = 0.5 / df;
    int bi = 0;
    double bv = -1.0;
    for (int g = 0; g < NG; ++g) {
      const double a = amp(lo + (hi - lo) * g / (NG - 1));
      if (a > bv) bv = a, bi = g;
    }
    double a = lo + (hi - lo) * std::max(bi - 1, 0) / (NG - 1);
    double bb = lo + (hi - lo) * std::min(bi + 1, NG - 1) / (NG - 1);
    const double gr = (std::sqrt(5.0) - 1.0) / 2.0;
    double x1 = bb - gr * (bb - a), x2 = a + gr * (bb - a);
    for (int it = 0; it < 80; ++it) {
      if (amp(x1) > amp(x2)) bb = x2;
      else a = x1;
      x1 = bb - gr * (bb - a);
      x2 = a + gr * (bb - a);
    }
    const double t0 = 0.5 * (a + bb);
    cd acc(0, 0);
    for (int j = 1; j < J; ++j)
      acc += Y[size_t(n) * J + j] * cis(j * df * sbd + (c->f0[n] - fref) * mbd + (j * df - fbw / 2.0) * t0);
    tau0[n] = t0;
    phi0[n] = std::atan2(acc.imag(), acc.real());
  }
  return FRBX_OK;
}

frbx_status frbx_top_peaks(const frbx_ctx *c, int64_t n_max, frbx_candidate *out, int64_t cap, int64_t *n) {
  if (!c || !n || n_max < 0) return FRBX_E_INVAL;
  if (!c->have || c->streaming) return FRBX_E_STATE;
  std::vector<frbx_candidate> v(c->cross);
  std::stable_sort(v.begin(), v.end(), [](const frbx_candidate &x, const frbx_candidate &y) {
    if (x.power_norm != y.power_norm) return x.power_norm > y.power_norm;
    if (x.baseline != y.baseline) return x.baseline < y.baseline;
    if (x.dm_index != y.dm_index) return x.dm_index < y.dm_index;
    if (x.window_index != y.window_index) return x.window_index < y.window_index;
    return x.segment < y.segment;
  });
  if (int64_t(v.size()) > n_max) v.resize(size_t(n_max));
  return copy_out(v, out, cap, n);
}

namespace {
frbx::RefineArgs refine_args(const frbx_ctx *c) {
  frbx::RefineArgs a{};
  a.vis = c->d_vis;
  a.in_f16 = c->vis_f16;
  a.n_frames = c->K;
  a.row_stride = c->K;
  a.nj = c->N * c->J;
  a.J = c->J;
  a.chan = c->d_rchan;
  a.cal = c->d_cal;
  a.seg = c->d_rseg;
  a.n = int32_t(c->rn);
  for (int k = 0; k < 5; ++k) a.cells[k] = c->rcells[k];
  a.dm_t = c->rcells[4] > 0 ? -c->rxbar * c->rcells[3] / c->rcells[4] : 0.0;
  a.max_step = 0.5;
  a.theta_best = c->d_rtb;
  a.step_best = c->d_rsb;
  a.p_best = c->d_rpb;
  a.radius = c->d_rrad;
  return a;
}

frbx_status refine_ready(frbx_ctx *c) {
  if (!c) return FRBX_E_INVAL;
  if (!c->rbegun || !c->d_rseg) return c->fail(FRBX_E_STATE, "no refinement begun");
  if (c->dirty || !c->loaded || c->streaming)
    return c->fail(FRBX_E_STATE, "grids or input changed since frbx_refine_begin");
  if (hipSetDevice(c->device) != hipSuccess) return c->fail(FRBX_E_DEVICE, "hipSetDevice failed");
  return FRBX_OK;
}
}  // namespace

frbx_status frbx_refine_cells(frbx_ctx *c, double *cells, double *xbar) {
  if (!c) return FRBX_E_INVAL;
  frbx_status s = prepare(c);
  if (s != FRBX_OK) return s;
  const int N = c->N, J = c->J;
  double fr = 0.0;
  for (int n = 0; n < N; ++n) fr = std::max(fr, c->f0[n] + (J - 1) * c->df);
  double sx = 0.0;
  for (int n = 0; n < N; ++n)
    for (int j = 1; j < J; ++j) {
      const double f = c->f0[n] + j * c->df;
      sx += c->k_dm * (1.0 / (f * f) - 1.0 / (fr * fr)) / c->t_ap;
    }
  c->rxbar = J > 1 ? sx / double(N * (J - 1)) : 0.0;
  c->rcells[0] = 1.0 / (double(c->sbd_pad) * J * c->df);
  c->rcells[1] = c->mbd_step;
  c->rcells[2] = c->n_rate > 1 ? c->rate_step : 0.0;
  c->rcells[3] = c->dm_step;
  c->rcells[4] = 1.0;
  for (int k = 0; k < 5; ++k)
    if (cells) cells[k] = c->rcells[k];
  if (xbar) *xbar = c->rxbar;
  return FRBX_OK;
}

frbx_status frbx_refine_begin(frbx_ctx *c, const frbx_candidate *peaks, int64_t n, double *theta0) {
  if (!c || n < 0 || (n > 0 && !peaks)) return FRBX_E_INVAL;
  if (!c->loaded || c->streaming) return c->fail(FRBX_E_STATE, "refinement needs input loaded with frbx_load");
  if (n > (int64_t(1) << 31) - 1) return c->fail(FRBX_E_RANGE, "too many peaks");
  if (hipSetDevice(c->device) != hipSuccess) return c->fail(FRBX_E_DEVICE, "hipSetDevice failed");
  frbx_status s = frbx_refine_cells(c, nullptr, nullptr);
  if (s != FRBX_OK) return s;
  const int N = c->N, J = c->J, NJ = N * J, PJ = c->sbd_pad * J, M = c->n_mbd;
  std::vector<frbx::RefineSeg> seg(static_cast<size_t>(n));
  std::vector<double> th(static_cast<size_t>(n) * 5);
  for (int64_t i = 0; i < n; ++i) {
    const frbx_candidate &p = peaks[i];
    if (p.baseline < 0 || p.baseline >= c->B || p.dm_index < 0 || p.dm_index >= c->n_dm || p.window_len < 1 ||
        p.window_len > c->K || p.k0 < 0 || p.k0 >= c->K || p.rate_idx < 0 || p.rate_idx >= c->n_rate ||
        p.sbd_idx < 0 || p.sbd_idx >= PJ || p.mbd_idx < 0 || p.mbd_idx >= M)
      return c->fail(FRBX_E_INVAL, "peak record out of range");
    seg[i] = frbx::RefineSeg{p.baseline, p.window_len, p.k0};
    th[5 * i + 0] = (p.sbd_idx - PJ / 2.0) / (PJ * c->df);
    th[5 * i + 1] = (p.mbd_idx - M / 2.0) * c->mbd_step;
    th[5 * i + 2] = (p.rate_idx - c->n_rate / 2) * c->rate_step;
    th[5 * i + 3] = c->dm_lo + p.dm_index * c->dm_step;
    th[5 * i + 4] = 0.0;
  }
  double fr = 0.0;
  for (int nn = 0; nn < N; ++nn) fr = std::max(fr, c->f0[nn] + (J - 1) * c->df);
  std::vector<frbx::RefineChan> ch(NJ);
  for (int nn = 0; nn < N; ++nn)
    for (int j = 0; j < J; ++j) {
      const double f = c->f0[nn] + j * c->df;
      ch[nn * J + j] = frbx::RefineChan{j * c->df, c->f0[nn] - c->f0[0], 1e3 * c->f0[nn] * c->t_ap,
                                        c->k_dm * (1.0 / (f * f) - 1.0 / (fr * fr)) / c->t_ap};
    }
  const size_t nn_alloc = size_t(std::max<int64_t>(n, 1));
  if ((s = ensure(c, c->d_rseg, c->rseg_cap, nn_alloc)) != FRBX_OK) return s;
  if ((s = ensure(c, c->d_rtheta, c->rtheta_cap, nn_alloc * 5)) != FRBX_OK) return s;
  if ((s = ensure(c, c->d_rpower, c->rpower_cap, nn_alloc)) != FRBX_OK) return s;
  if ((s = ensure(c, c->d_rchan, c->rchan_cap, size_t(NJ))) != FRBX_OK) return s;
  if ((s = ensure(c, c->d_rtb, c->rtb_cap, nn_alloc * 5)) != FRBX_OK) return s;
  if ((s = ensure(c, c->d_rsb, c->rsb_cap, nn_alloc * 5)) != FRBX_OK) return s;
  if ((s = ensure(c, c->d_rrad, c->rrad_cap, nn_alloc)) != FRBX_OK) return s;
  if ((s = ensure(c, c->d_rpb, c->rpb_cap, nn_alloc)) != FRBX_OK) return s;
  if (n > 0) {
    if ((s = c->hip(hipMemcpyAsync(c->d_rseg, seg.data(), seg.size() * sizeof(frbx::RefineSeg),
                                   hipMemcpyHostToDevice, c->stream), "refine upload")) != FRBX_OK)
      return s;
    if ((s = c->hip(hipMemcpyAsync(c->d_rtheta, th.data(), th.size() * sizeof(double), hipMemcpyHostToDevice,
                                   c->stream), "refine upload")) != FRBX_OK)
      return s;
  }
  if ((s = c->hip(hipMemcpyAsync(c->d_rchan, ch.data(), ch.size() * sizeof(frbx::RefineChan),
                                 hipMemcpyHostToDevice, c->stream), "refine upload")) != FRBX_OK)
    return s;
  if ((s = c->hip(hipStreamSynchronize(c->stream), "refine upload")) != FRBX_OK) return s;
  c->rn = n;
  c->rdone = false;
  c->rbegun = true;
  c->rtheta0 = th;
  if (theta0) std::copy(th.begin(), th.end(), theta0);
  return FRBX_OK;
}

frbx_status frbx_refine_run(frbx_ctx *c, int32_t n_steps) {
  frbx_status s = refine_ready(c);
  if (s != FRBX_OK) return s;
  if (n_steps < 0) return c->fail(FRBX_E_INVAL, "n_steps < 0");
  c->spans.clear();
  c->ev_used = 0;
  // every run starts from the begun grid points with a fresh ascent state
  const size_t n = size_t(c->rn);
  if (n > 0) {
    const std::vector<double> zeros(n * 5, 0.0), rad(n, 0.5);
    const std::vector<float> none(n, -1.0f);
    const std::pair<void *, const void *> ups[] = {{c->d_rtheta, c->rtheta0.data()}, {c->d_rtb, c->rtheta0.data()},
                                                   {c->d_rsb, zeros.data()}};
    for (const auto &u : ups)
      if ((s = c->hip(hipMemcpyAsync(u.first, u.second, n * 5 * sizeof(double), hipMemcpyHostToDevice, c->stream),
                      "refine state")) != FRBX_OK)
        return s;
    if ((s = c->hip(hipMemcpyAsync(c->d_rrad, rad.data(), n * sizeof(double), hipMemcpyHostToDevice, c->stream),
                    "refine state")) != FRBX_OK)
      return s;
    if ((s = c->hip(hipMemcpyAsync(c->d_rpb, none.data(), n * sizeof(float), hipMemcpyHostToDevice, c->stream),
                    "refine state")) != FRBX_OK)
      return s;
    if ((s = c->hip(hipStreamSynchronize(c->stream), "refine state")) != FRBX_OK) return s;
  }
  frbx::RefineArgs a = refine_args(c);
  a.theta = c->d_rtheta;
  a.power = c->d_rpower;
  for (int k = 0; k <= n_steps; ++k) {
    const int mode = k < n_steps ? frbx::kRefineStep : frbx::kRefineFinal;
    const int sp = c->span_begin(3, c->rn);
    if ((s = c->hip(frbx::launch_refine(mode, a, c->stream), "refine launch")) != FRBX_OK) return s;
    c->span_end(sp);
  }
  if ((s = c->hip(hipStreamSynchronize(c->stream), "refine")) != FRBX_OK) return s;
  if (c->timing) c->collect_timing();
  c->rdone = true;
  return FRBX_OK;
}

frbx_status frbx_refine_results(const frbx_ctx *cc, double *theta, float *power, int64_t cap, int64_t *n) {
  frbx_ctx *c = const_cast<frbx_ctx *>(cc);
  if (!c || !n) return FRBX_E_INVAL;
  if (!c->rdone) return FRBX_E_STATE;
  *n = c->rn;
  if (cap < c->rn) return FRBX_E_RANGE;
  if (hipSetDevice(c->device) != hipSuccess) return c->fail(FRBX_E_DEVICE, "hipSetDevice failed");
  frbx_status s;
  if (theta && c->rn > 0 &&
      (s = c->hip(hipMemcpy(theta, c->d_rtheta, size_t(c->rn) * 5 * sizeof(double), hipMemcpyDeviceToHost),
                  "refine results")) != FRBX_OK)
    return s;
  if (power && c->rn > 0 &&
      (s = c->hip(hipMemcpy(power, c->d_rpower, size_t(c->rn) * sizeof(float), hipMemcpyDeviceToHost),
                  "refine results")) != FRBX_OK)
    return s;
  return FRBX_OK;
}

frbx_status frbx_refine_forward(frbx_ctx *c, const double *theta, float *power) {
  frbx_status s = refine_ready(c);
  if (s != FRBX_OK) return s;
  if (!theta || !power) return c->fail(FRBX_E_INVAL, "null device pointer");
  frbx::RefineArgs a = refine_args(c);
  a.theta = const_cast<double *>(theta);
  a.power = power;
  return c->hip(frbx::launch_refine(frbx::kRefineForward, a, c->stream), "refine forward");
}

frbx_status frbx_refine_backward(frbx_ctx *c, const double *theta, const float *grad_power, double *grad_theta) {
  frbx_status s = refine_ready(c);
  if (s != FRBX_OK) return s;
  if (!theta || !grad_power || !grad_theta) return c->fail(FRBX_E_INVAL, "null device pointer");
  frbx::RefineArgs a = refine_args(c);
  a.theta = const_cast<double *>(theta);
  a.grad_power = grad_power;
  a.grad_theta = grad_theta;
  return c->hip(frbx::launch_refine(frbx::kRefineBackward, a, c->stream), "refine backward");
}

frbx_status frbx_refine_curvature(frbx_ctx *c, const double *theta, double *curv) {
  frbx_status s = refine_ready(c);
  if (s != FRBX_OK) return s;
  if (!theta || !curv) return c->fail(FRBX_E_INVAL, "null device pointer");
  frbx::RefineArgs a = refine_args(c);
  a.theta = const_cast<double *>(theta);
  a.curv = curv;
  return c->hip(frbx::launch_refine(frbx::kRefineCurvature, a, c->stream), "refine curvature");
}

frbx_status frbx_set_timing(frbx_ctx *c, int enable) {
  if (!c) return FRBX_E_INVAL;
  c->timing = enable != 0;
  return FRBX_OK;
}

frbx_status frbx_get_timing(const frbx_ctx *c, frbx_timing *out) {
  if (!c || !out) return FRBX_E_INVAL;
  if (!c->have) return FRBX_E_STATE;
  *out = c->last_timing;
  return FRBX_OK;
}

frbx_status frbx_ap_offsets(const frbx_layout *L, double dm_lo, double dm_step, int32_t n_dm, double k_dm,
                            int32_t *out) {
  std::string why;
  if (check_layout(L, why) != FRBX_OK || !out || n_dm < 1 || !std::isfinite(dm_lo) || !std::isfinite(dm_step))
    return FRBX_E_INVAL;
  ap_offset_table(L->n_if, L->n_chan, L->if_freq_mhz, L->chan_bw_mhz, L->t_ap_ms, dm_lo, dm_step, n_dm,
                  k_dm > 0 ? k_dm : kDefaultKdm, out);
  return FRBX_OK;
}

frbx_status frbx_mbd_lattice(const frbx_layout *Lay, int32_t n_mbd, double mbd_step_us, int64_t *q,
                             double *mbd_step_out, int32_t *compact_shift) {
  std::string why;
  if (check_layout(Lay, why) != FRBX_OK || frbx::fringe_compact_rows(n_mbd) == 0) return FRBX_E_INVAL;
  std::vector<double> f0(Lay->if_freq_mhz, Lay->if_freq_mhz + Lay->n_if);
  MbdLattice L;
  if (mbd_lattice(f0, Lay->n_chan, Lay->chan_bw_mhz, n_mbd, mbd_step_us, L)) return FRBX_E_INVAL;
  if (q)
    for (int n = 0; n < Lay->n_if; ++n) q[n] = L.q[n];
  if (mbd_step_out) *mbd_step_out = L.mbd_step;
  if (compact_shift) *compact_shift = L.shift;
  return FRBX_OK;
}

frbx_status frbx_detect(const frbx_candidate *crossings, int64_t n_cross, double t_amb_us, int32_t n_win_min,
                        int32_t n_bl_min, int32_t use_mbd, frbx_candidate *dets, int64_t det_cap,
                        int64_t *n_dets, frbx_group *groups, int64_t group_cap, int64_t *n_groups) {
  if (n_cross < 0 || (n_cross > 0 && !crossings) || !(t_amb_us > 0) || n_win_min < 1 || n_bl_min < 1)
    return FRBX_E_INVAL;
  std::vector<frbx_candidate> d;
  std::vector<frbx_group> g;
  detect_impl(crossings, n_cross, t_amb_us, n_win_min, n_bl_min, use_mbd != 0, d, g);
  frbx_status s1 = copy_out(d, dets, det_cap, n_dets);
  frbx_status s2 = copy_out(g, groups, group_cap, n_groups);
  return s1 != FRBX_OK ? s1 : s2;
}

}  // extern "C"
