/* Drives the oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (test infrastructure; built and run by tests/test_oracle_sanitized.py).
 *
 * Input file (little-endian): int32 H, W, nseq, nf, key_index; float32
 * az0, eps; int32 th, tw; float32 elev[H]; then per frame int64 n,
 * float32 xyz[3 n], float32 M[16].  Writes the frame sizes, one per line,
 * then the finite point count, to stdout. */
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/oracle.h"

static void need(int ok, const char *what) {
  if (!ok) {
    fprintf(stderr, "bad input: %s\n", what);
    exit(2);
  }
}

int main(int argc, char **argv) {
  need(argc == 2, "usage: oracle_driver INPUT");
  FILE *f = fopen(argv[1], "rb");
  need(f != NULL, "open");
  int32_t hdr[5];
  float az0, eps;
  int32_t tile[2];
  need(fread(hdr, sizeof hdr, 1, f) == 1, "header");
  need(fread(&az0, 4, 1, f) == 1 && fread(&eps, 4, 1, f) == 1 && fread(tile, sizeof tile, 1, f) == 1, "params");
  const int H = hdr[0], W = hdr[1], nseq = hdr[2], nf = hdr[3], key = hdr[4], nfr = nseq * nf;
  need(H > 0 && W > 0 && nfr > 0 && key >= 0 && key < nf, "sizes");
  float *elev = malloc(sizeof(float) * H);
  need(fread(elev, sizeof(float), H, f) == (size_t)H, "elevations");
  float *cut = malloc(sizeof(float) * (H + 1)), *ebx = malloc(sizeof(float) * W), *eby = malloc(sizeof(float) * W);
  float *ce = malloc(sizeof(float) * H), *se = malloc(sizeof(float) * H);
  float *ca = malloc(sizeof(float) * W), *sa = malloc(sizeof(float) * W);
  orc_tables(H, W, elev, az0, cut, ebx, eby, ce, se, ca, sa);
  orc_sensor s = {H, W, cut, ebx, eby, ce, se, ca, sa};
  orc_params prm = {eps, tile[0], tile[1], 5, 4, 0.5f};
  float **xyz = malloc(sizeof(float *) * nfr);
  int64_t *count = malloc(sizeof(int64_t) * nfr);
  float *M = malloc(sizeof(float) * 16 * nfr);
  for (int i = 0; i < nfr; i++) {
    need(fread(&count[i], 8, 1, f) == 1 && count[i] >= 0, "point count");
    xyz[i] = malloc(sizeof(float) * 3 * (count[i] ? count[i] : 1));
    need(fread(xyz[i], sizeof(float), 3 * count[i], f) == (size_t)(3 * count[i]), "points");
    need(fread(M + 16 * i, sizeof(float), 16, f) == 16, "transform");
  }
  fclose(f);
  uint64_t *sizes = malloc(sizeof(uint64_t) * nfr);
  int64_t fin = 0;
  orc_encode_sequences(nseq, nf, key, (const float *const *)xyz, count, M, &s, &prm, sizes, &fin);
  for (int i = 0; i < nfr; i++) printf("%llu\n", (unsigned long long)sizes[i]);
  printf("%lld\n", (long long)fin);
  for (int i = 0; i < nfr; i++) free(xyz[i]);
  free(xyz); free(count); free(M); free(sizes);
  free(elev); free(cut); free(ebx); free(eby); free(ce); free(se); free(ca); free(sa);
  return 0;
}
