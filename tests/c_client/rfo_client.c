/* A plain C99 client of the library's C ABI (include/rfo.h), used by the GPU tests to
 * show that the boundary works without the Python binding.
 *
 * Usage: rfo_client IN OUT
 * IN (little-endian): int64 nb, int64 bd, int64 s, int64 p; double T, mu, e_min, e_max;
 *   int64 row_ptr[nb + 1]; int32 col_idx[nnzb]; double values[nnzb][bd][bd];
 *   double R[n][s] (n = nb * bd rows, s probes, row-major).
 * OUT: double NEF[3] and moments[s][p] of rfo_fermi_moments with the density,
 *   density[nnzb][bd][bd]; then NEF[3] and dFdH[nnzb][bd][bd] of rfo_energy_and_dEdH.
 * Exit status 0 on success; otherwise the failing call and rfo_last_error go to stderr. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "rfo.h"

static void *read_or_die(FILE *f, size_t count, size_t size, const char *what) {
  void *p = malloc(count * size + 1);
  if (!p || fread(p, size, count, f) != count) {
    fprintf(stderr, "rfo_client: cannot read %s\n", what);
    exit(2);
  }
  return p;
}

static void write_or_die(FILE *f, const void *p, size_t count, size_t size) {
  if (fwrite(p, size, count, f) != count) {
    fprintf(stderr, "rfo_client: write failed\n");
    exit(2);
  }
}

#define CHECK(call)                                                                 \
  do {                                                                              \
    int rc_ = (call);                                                               \
    if (rc_ != RFO_OK) {                                                            \
      fprintf(stderr, "rfo_client: %s returned %d: %s\n", #call, rc_,              \
              rfo_last_error(ctx));                                                 \
      return 1;                                                                     \
    }                                                                               \
  } while (0)

int main(int argc, char **argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: rfo_client IN OUT\n");
    return 2;
  }
  FILE *in = fopen(argv[1], "rb");
  if (!in) {
    fprintf(stderr, "rfo_client: cannot open %s\n", argv[1]);
    return 2;
  }
  int64_t hdr[4];
  double par[4];
  if (fread(hdr, sizeof(int64_t), 4, in) != 4 || fread(par, sizeof(double), 4, in) != 4) {
    fprintf(stderr, "rfo_client: short header\n");
    return 2;
  }
  const int64_t nb = hdr[0], bd = hdr[1], s = hdr[2], p = hdr[3];
  if (nb < 1 || (bd != 1 && bd != 9) || s < 1 || p < 1) {
    fprintf(stderr, "rfo_client: bad header\n");
    return 2;
  }
  int64_t *row_ptr = read_or_die(in, (size_t)nb + 1, sizeof(int64_t), "row_ptr");
  const int64_t nnzb = row_ptr[nb], n = nb * bd;
  int32_t *col = read_or_die(in, (size_t)nnzb, sizeof(int32_t), "col_idx");
  double *values = read_or_die(in, (size_t)(nnzb * bd * bd), sizeof(double), "values");
  double *R = read_or_die(in, (size_t)(n * s), sizeof(double), "R");
  fclose(in);

  double *moments = malloc((size_t)(s * p) * sizeof(double));
  double *blocks = malloc((size_t)(nnzb * bd * bd) * sizeof(double));
  double nef[3];
  if (!moments || !blocks) return 2;
  FILE *out = fopen(argv[2], "wb");
  if (!out) return 2;

  rfo_ctx *ctx = NULL;
  if (rfo_create(&ctx, 0, NULL) != RFO_OK) {
    fprintf(stderr, "rfo_client: rfo_create: %s\n", rfo_last_error(NULL));
    return 1;
  }
  CHECK(rfo_set_hamiltonian(ctx, nb, (int)bd, row_ptr, col, values, par[2], par[3], RFO_FP64));
  CHECK(rfo_set_probes(ctx, s, R, NULL));
  CHECK(rfo_fermi_moments(ctx, par[0], par[1], p, moments, nef, blocks));
  write_or_die(out, nef, 3, sizeof(double));
  write_or_die(out, moments, (size_t)(s * p), sizeof(double));
  write_or_die(out, blocks, (size_t)(nnzb * bd * bd), sizeof(double));
  CHECK(rfo_energy_and_dEdH(ctx, par[0], par[1], p, nef, blocks));
  write_or_die(out, nef, 3, sizeof(double));
  write_or_die(out, blocks, (size_t)(nnzb * bd * bd), sizeof(double));
  rfo_destroy(ctx);
  fclose(out);
  free(row_ptr);
  free(col);
  free(values);
  free(R);
  free(moments);
  free(blocks);
  return 0;
}
