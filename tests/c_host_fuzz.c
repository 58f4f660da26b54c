/* Randomised use of the host-only entry points of libfrbx (no device): the
 * Sec. 2.4.1 grouping over random crossing tables with the size-query and
 * short-capacity protocol, the Eq. 2 AP-offset table and the MBD lattice
 * over random (valid and invalid) layouts.  Built with AddressSanitizer and
 * UndefinedBehaviorSanitizer by the calling test; prints one summary line.
 * Exit status 0 when every call behaved as its declaration states. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "frbx.h"

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint32_t rnd(void) { /* xorshift64* */
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return (uint32_t)((rng_state * 0x2545F4914F6CDD1Dull) >> 32);
}
static double unif(double a, double b) { return a + (b - a) * (rnd() / 4294967296.0); }

static int check_detect(int round) {
  const int n = (int)(rnd() % 1500);
  frbx_candidate *cr = calloc((size_t)(n > 0 ? n : 1), sizeof *cr);
  static const int wl[4] = {2, 4, 8, 16};
  for (int i = 0; i < n; ++i) {
    cr[i].baseline = (int32_t)(rnd() % 6);
    cr[i].dm_index = (int32_t)(rnd() % 8);
    cr[i].window_index = (int32_t)(rnd() % 4);
    cr[i].window_len = wl[cr[i].window_index];
    cr[i].k0 = (int64_t)(rnd() % 400);
    cr[i].power_norm = unif(3.0, 9.0);
    cr[i].mbd_us = unif(-0.02, 0.02);
    cr[i].group_id = -1;
  }
  const double t_amb = unif(0.005, 0.05);
  const int nwin = 1 + (int)(rnd() % 3), nbl = 1 + (int)(rnd() % 3), use_mbd = (int)(rnd() % 2);
  int64_t nd = -1, ng = -1;
  frbx_status s = frbx_detect(cr, n, t_amb, nwin, nbl, use_mbd, NULL, 0, &nd, NULL, 0, &ng);
  if (s != FRBX_OK && s != FRBX_E_RANGE) return 10;
  if (nd < 0 || ng < 0 || nd > n || (nd == 0 && ng != 0)) return 11;
  frbx_candidate *det = calloc((size_t)(nd + 1), sizeof *det);
  frbx_group *grp = calloc((size_t)(ng + 1), sizeof *grp);
  if (frbx_detect(cr, n, t_amb, nwin, nbl, use_mbd, det, nd, &nd, grp, ng, &ng) != FRBX_OK) return 12;
  /* a capacity one short is refused with the size needed */
  if (nd > 0) {
    int64_t nd2 = -1, ng2 = -1;
    if (frbx_detect(cr, n, t_amb, nwin, nbl, use_mbd, det, nd - 1, &nd2, grp, ng, &ng2) != FRBX_E_RANGE)
      return 13;
    if (nd2 != nd || ng2 != ng) return 14;
  }
  /* every detection is one of the crossings, its group exists and holds it */
  for (int64_t i = 0; i < nd; ++i) {
    if (det[i].n_windows < nwin) return 15;
    if (det[i].group_id < 0 || det[i].group_id >= ng) return 16;
    const frbx_group *g = &grp[det[i].group_id];
    if (det[i].k0 < g->k_start || det[i].k0 + det[i].window_len - 1 > g->k_end) return 17;
  }
  for (int64_t i = 0; i < ng; ++i)
    if (grp[i].best < 0 || grp[i].best >= nd || (grp[i].reported != 0) != (grp[i].n_baselines >= nbl)) return 18;
  free(det);
  free(grp);
  free(cr);
  (void)round;
  return 0;
}

static int check_tables(void) {
  static const int chans[6] = {8, 16, 32, 64, 128, 256};
  const int N = 1 + (int)(rnd() % 12), J = chans[rnd() % 6], D = 1 + (int)(rnd() % 16);
  double f0[12];
  /* IFs on a 4 MHz lattice (valid for the MBD grid) unless broken below */
  for (int n = 0; n < N; ++n) f0[n] = 2000.0 + 4.0 * (double)(rnd() % 512);
  const int broken = (int)(rnd() % 4) == 0;
  if (broken && N > 1) f0[N - 1] += 0.0003;  /* off the whole-kHz lattice */
  frbx_layout lay;
  memset(&lay, 0, sizeof lay);
  lay.n_baselines = 1;
  lay.n_if = N;
  lay.n_chan = J;
  lay.n_frames = 1000;
  lay.t_ap_ms = unif(0.1, 2.0);
  lay.chan_bw_mhz = unif(0.1, 2.0);
  lay.if_freq_mhz = f0;
  int32_t *tab = malloc(sizeof(int32_t) * (size_t)(D * N * J));
  if (frbx_ap_offsets(&lay, 0.0, unif(0.5, 50.0), D, 0.0, tab) != FRBX_OK) return 20;
  for (int i = 0; i < D * N * J; ++i)
    if (tab[i] < 0) return 21;
  if (frbx_ap_offsets(&lay, NAN, 1.0, D, 0.0, tab) != FRBX_E_INVAL) return 22;
  if (frbx_ap_offsets(&lay, 0.0, 1.0, 0, 0.0, tab) != FRBX_E_INVAL) return 23;
  free(tab);
  int64_t q[12];
  double step = 0.0;
  int32_t shift = 0;
  const frbx_status s = frbx_mbd_lattice(&lay, 256, 0.0, q, &step, &shift);
  if (s == FRBX_OK) {
    for (int n = 0; n < N; ++n)
      if (q[n] < 0 || q[n] >= 256) return 24;
    if (!(step > 0.0) || shift < -1 || shift >= 256) return 25;
  } else if (s != FRBX_E_INVAL) {
    return 26;
  }
  if (frbx_mbd_lattice(&lay, 100, 0.0, q, &step, &shift) != FRBX_E_INVAL) return 27;
  lay.n_chan = 12; /* not a supported channel count */
  if (frbx_ap_offsets(&lay, 0.0, 1.0, D, 0.0, (int32_t *)q) != FRBX_E_INVAL) return 28;
  return 0;
}

int main(void) {
  for (int r = 0; r < 200; ++r) {
    int e = check_detect(r);
    if (e) {
      printf("detect round %d failed %d\n", r, e);
      return e;
    }
    e = check_tables();
    if (e) {
      printf("tables round %d failed %d\n", r, e);
      return e;
    }
  }
  if (frbx_detect(NULL, 1, 0.03, 1, 1, 1, NULL, 0, NULL, NULL, 0, NULL) != FRBX_E_INVAL) return 30;
  if (frbx_ap_offsets(NULL, 0.0, 1.0, 1, 0.0, NULL) != FRBX_E_INVAL) return 31;
  printf("fuzz ok %s\n", frbx_last_error(NULL));
  return 0;
}
