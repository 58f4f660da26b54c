/* A whole search through the libfrbx C ABI from plain C (no Python, no
 * PyTorch): cross spectra read from a file are copied in with frbx_load
 * (host pointer), searched on device 0 with the default stream, and the
 * power cube, the packed indices and the candidate count written out.
 * Usage: c_search_check <in.bin> <out.bin> B N J K n_dm dm_step n_rate n_mbd f0...
 * in.bin: complex64 [B][N][J][K]; out.bin: float32 power then int32 index. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "frbx.h"

static int check(frbx_status s, frbx_ctx *c, const char *what) {
  if (s == FRBX_OK) return 0;
  fprintf(stderr, "%s: status %d: %s\n", what, (int)s, frbx_last_error(c));
  return 1;
}

int main(int argc, char **argv) {
  if (argc < 12) return 2;
  const int B = atoi(argv[3]), N = atoi(argv[4]), J = atoi(argv[5]);
  const long long K = atoll(argv[6]);
  const int n_dm = atoi(argv[7]);
  const double dm_step = atof(argv[8]);
  const int n_rate = atoi(argv[9]), n_mbd = atoi(argv[10]);
  if (argc != 11 + N) return 2;
  double *f0 = malloc(sizeof(double) * (size_t)N);
  for (int n = 0; n < N; ++n) f0[n] = atof(argv[11 + n]);
  const size_t n_vis = (size_t)B * N * J * (size_t)K;
  float *vis = malloc(n_vis * 2 * sizeof(float));
  FILE *fi = fopen(argv[1], "rb");
  if (!fi || fread(vis, 2 * sizeof(float), n_vis, fi) != n_vis) return 3;
  fclose(fi);
  frbx_layout lay;
  memset(&lay, 0, sizeof lay);
  lay.n_baselines = B;
  lay.n_if = N;
  lay.n_chan = J;
  lay.n_frames = K;
  lay.t_ap_ms = 1.0;
  lay.chan_bw_mhz = 1.0;
  lay.if_freq_mhz = f0;
  frbx_ctx *c = NULL;
  if (check(frbx_create(&lay, 0, NULL, &c), c, "create")) return 4;
  const int32_t windows[3] = {2, 4, 8};
  if (check(frbx_set_dm_grid(c, 0.0, dm_step, n_dm, 4.149e6), c, "dm grid") ||
      check(frbx_set_delay_grid(c, 4, n_mbd, 0.0, NAN), c, "delay grid") ||
      check(frbx_set_rate_grid(c, n_rate, 0.0), c, "rate grid") ||
      check(frbx_set_windows(c, windows, 3), c, "windows") ||
      check(frbx_set_detection(c, 3.0, 2, 1), c, "detection") ||
      check(frbx_load(c, vis, 0), c, "load") || check(frbx_run(c), c, "run"))
    return 5;
  int64_t n = 0;
  frbx_get_power_cube(c, NULL, NULL, 0, &n);
  float *p = malloc(sizeof(float) * (size_t)n);
  int32_t *idx = malloc(sizeof(int32_t) * (size_t)n);
  if (check(frbx_get_power_cube(c, p, idx, n, &n), c, "power cube")) return 6;
  int64_t nc = 0;
  frbx_get_candidates(c, NULL, 0, &nc);
  int64_t *q = malloc(sizeof(int64_t) * (size_t)N);
  double mbd_step = 0.0;
  int32_t shift = 0;
  if (check(frbx_get_lattice(c, q, &mbd_step, &shift), c, "lattice")) return 8;
  FILE *fo = fopen(argv[2], "wb");
  if (!fo) return 7;
  fwrite(p, sizeof(float), (size_t)n, fo);
  fwrite(idx, sizeof(int32_t), (size_t)n, fo);
  fclose(fo);
  printf("cube %lld candidates %lld\n", (long long)n, (long long)nc);
  printf("lattice %d %.17g", (int)shift, mbd_step);
  for (int i = 0; i < N; ++i) printf(" %lld", (long long)q[i]);
  printf("\n");
  free(q);
  frbx_destroy(c);
  free(p);
  free(idx);
  free(vis);
  free(f0);
  return 0;
}
