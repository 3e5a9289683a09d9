/* Brute-force topology check of the oracle on tiny fields (test driver).
 *
 * Every 3x3 field over a 5-value alphabet, at several error bounds, plus
 * random 4x4, 3x3x3 and 4x4x4 fields, goes through compress + decompress; the
 * result is recounted with a classifier written here (independently of the
 * oracle's) and checked against the paper's guarantees: no false positives,
 * no false types (Section III-B, Table II), every lost extremum restored
 * unless the error budget forbade the move, and |a - a^| <= 2e (Section V).
 * Usage: bf_tiny [stride]   (stride > 1 samples the 3x3 enumeration)
 * Exit status 0 when every case passes. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/toposzp_oracle.h"

static int cls_of(const float *v, int nz, int ny, int nx, int z, int y, int x) {
  int ext[3] = {nx, ny, nz}, c[3] = {x, y, z};
  int stride[3] = {1, nx, nx * ny};
  int i = (z * ny + y) * nx + x;
  int higher = 0, lower = 0, total = 0, up_pairs = 0, dn_pairs = 0, bad_pair = 0;
  for (int ax = 0; ax < 3; ax++) {
    if (ext[ax] == 1) continue;
    int n_here = 0, h = 0, l = 0;
    for (int s = -1; s <= 1; s += 2) {
      int cc = c[ax] + s;
      if (cc < 0 || cc >= ext[ax]) continue;
      float b = v[i + s * stride[ax]];
      n_here++;
      total++;
      if (b > v[i]) { higher++; h++; }
      if (b < v[i]) { lower++; l++; }
    }
    if (n_here == 2 && h == 2) up_pairs++;
    else if (n_here == 2 && l == 2) dn_pairs++;
    else bad_pair = 1;
  }
  if (total == 0) return ORA_R;
  if (higher == total) return ORA_MIN;
  if (lower == total) return ORA_MAX;
  if (!bad_pair && up_pairs && dn_pairs) return ORA_SAD;
  return ORA_R;
}

static long n_cases, n_fail, n_fn, n_fn_ext, n_skips;

static void check(const float *f, int nz, int ny, int nx, double eb) {
  uint64_t dims[3];
  int ndim = nz > 1 ? 3 : 2;
  if (ndim == 3) { dims[0] = nz; dims[1] = ny; dims[2] = nx; }
  else { dims[0] = ny; dims[1] = nx; dims[2] = 1; }
  static uint8_t buf[1 << 16];
  size_t sz = 0;
  ora_params p = {1, 0, 0, 16};
  int rc = ora_compress(f, ndim, dims, 0, eb, &p, buf, sizeof(buf), &sz);
  n_cases++;
  if (rc != ORA_OK) { n_fail++; return; }
  int n = nz * ny * nx;
  float rec[64];
  ora_stats st;
  rc = ora_decompress(buf, sz, rec, (size_t)n, &st);
  if (rc != ORA_OK) { n_fail++; return; }
  float e = ora_eps_float(eb);
  long fn_ext = 0;
  for (int z = 0; z < nz; z++)
    for (int y = 0; y < ny; y++)
      for (int x = 0; x < nx; x++) {
        int i = (z * ny + y) * nx + x;
        int a = cls_of(f, nz, ny, nx, z, y, x), b = cls_of(rec, nz, ny, nx, z, y, x);
        int bad = 0;
        if (a == ORA_R && b != ORA_R) bad = 1;               /* FP */
        if (a != ORA_R && b != ORA_R && a != b) bad = 1;     /* FT */
        if (fabs((double)rec[i] - (double)f[i]) > 2.0 * (double)e) bad = 1;
        if (a != ORA_R && b == ORA_R) {
          n_fn++;
          if (a != ORA_SAD) fn_ext++;
        }
        if (bad) {
          if (n_fail < 10) fprintf(stderr, "FAIL eb=%g point %d orig %d recon %d\n", eb, i, a, b);
          n_fail++;
        }
      }
  if (fn_ext != st.budget_skips) {
    if (n_fail < 10) fprintf(stderr, "FAIL eb=%g extrema FN %ld skips %ld\n", eb, fn_ext, (long)st.budget_skips);
    n_fail++;
  }
  n_fn_ext += fn_ext;
  n_skips += st.budget_skips;
}

static unsigned long long rng_state = 88172645463325252ULL;
static double urand(void) {
  rng_state ^= rng_state << 13;
  rng_state ^= rng_state >> 7;
  rng_state ^= rng_state << 17;
  return (double)(rng_state >> 11) / 9007199254740992.0;
}

int main(int argc, char **argv) {
  long stride = argc > 1 ? atol(argv[1]) : 1;
  const double ebs[] = {0.1, 0.125, 0.3, 0.6, 10.0};
  float f[64];
  long total = 1953125; /* 5^9 */
  for (long code = 0; code < total; code += stride) {
    long c = code;
    for (int i = 0; i < 9; i++) {
      f[i] = (float)(c % 5) * 0.25f;
      c /= 5;
    }
    for (int k = 0; k < 5; k++) check(f, 1, 3, 3, ebs[k]);
  }
  long rand_cases = 200000 / (stride > 1 ? stride : 1) + 2000;
  for (long t = 0; t < rand_cases; t++) {
    int shape = (int)(t % 3);
    int nz = shape == 0 ? 1 : (shape == 1 ? 3 : 4), ny = shape == 1 ? 3 : 4, nx = ny;
    int n = nz * ny * nx;
    for (int i = 0; i < n; i++) f[i] = (float)floor(urand() * 7.0) * 0.25f;
    check(f, nz, ny, nx, ebs[t % 5]);
  }
  printf("cases %ld failures %ld FN %ld extremaFN %ld budget_skips %ld\n", n_cases, n_fail, n_fn,
         n_fn_ext, n_skips);
  return n_fail == 0 ? 0 : 1;
}
