/* Plain C11 use of the libfrbx C ABI through include/frbx.h, without a
 * device: the host-only entry points (version, the Eq. 2 AP-offset table,
 * the Sec. 2.4.1 grouping), NULL-context handling, and the size-query
 * protocol.  Prints what the calling test compares with the oracle. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "frbx.h"

int main(void) {
  const double f0[4] = {3000.0, 3032.0, 3096.0, 3192.0};
  frbx_layout lay;
  memset(&lay, 0, sizeof lay);
  lay.n_baselines = 1;
  lay.n_if = 4;
  lay.n_chan = 16;
  lay.n_frames = 500;
  lay.t_ap_ms = 1.0;
  lay.chan_bw_mhz = 1.0;
  lay.if_freq_mhz = f0;
  printf("version %s\n", frbx_version());
  int32_t tab[3 * 4 * 16];
  if (frbx_ap_offsets(&lay, 0.0, 150.0, 3, 4.149e6, tab) != FRBX_OK) return 1;
  printf("dk");
  for (int i = 0; i < 3 * 4 * 16; ++i) printf(" %d", tab[i]);
  printf("\n");
  /* MBD lattice: offsets 0, 32, 96, 192 MHz on a 32 MHz lattice */
  int64_t q[4];
  double mbd_step = 0.0;
  int32_t shift = 0;
  if (frbx_mbd_lattice(&lay, 256, 0.0, q, &mbd_step, &shift) != FRBX_OK) return 1;
  printf("lattice %d %.17g %lld %lld %lld %lld\n", (int)shift, mbd_step, (long long)q[0], (long long)q[1],
         (long long)q[2], (long long)q[3]);
  if (frbx_mbd_lattice(&lay, 100, 0.0, q, &mbd_step, &shift) != FRBX_E_INVAL) return 1;
  /* two baselines crossing at overlapping APs -> one reported group */
  frbx_candidate cr[3];
  memset(cr, 0, sizeof cr);
  for (int i = 0; i < 3; ++i) {
    cr[i].baseline = i < 2 ? 0 : 1;
    cr[i].window_len = i == 1 ? 8 : 4;
    cr[i].k0 = 100 + 2 * i;
    cr[i].power_norm = 4.0 + i;
    cr[i].mbd_us = 0.001 * i;
    cr[i].group_id = -1;
  }
  int64_t nd = -1, ng = -1;
  if (frbx_detect(cr, 3, 0.03125, 1, 2, 1, NULL, 0, &nd, NULL, 0, &ng) != FRBX_E_RANGE) return 2;
  frbx_candidate *det = calloc((size_t)nd, sizeof *det);
  frbx_group *grp = calloc((size_t)ng, sizeof *grp);
  if (frbx_detect(cr, 3, 0.03125, 1, 2, 1, det, nd, &nd, grp, ng, &ng) != FRBX_OK) return 3;
  printf("detections %lld groups %lld reported %d\n", (long long)nd, (long long)ng, (int)grp[0].reported);
  for (int64_t i = 0; i < nd; ++i)
    printf("det %d %lld %d %.3f\n", det[i].baseline, (long long)det[i].k0, det[i].window_len, det[i].power_norm);
  if (frbx_run(NULL) != FRBX_E_INVAL) return 4;
  printf("null %s\n", frbx_last_error(NULL));
  free(det);
  free(grp);
  return 0;
}
