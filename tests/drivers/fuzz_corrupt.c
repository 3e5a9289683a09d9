/* Corrupted-stream fuzzing of the oracle decoder (test driver, built with
 * AddressSanitizer and UndefinedBehaviorSanitizer).  Random fields are
 * compressed, then bytes are flipped anywhere in the stream or the stream is
 * truncated; the decoder must return a status (OK or an error code) without
 * any out-of-bounds access or undefined behaviour.  Header corruption must be
 * reported as corrupt.  Exit status 0 when every case behaves. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/toposzp_oracle.h"

static unsigned long long s = 0x9E3779B97F4A7C15ULL;
static unsigned long long next(void) {
  s ^= s << 13;
  s ^= s >> 7;
  s ^= s << 17;
  return s;
}

int main(int argc, char **argv) {
  int iters = argc > 1 ? atoi(argv[1]) : 2000;
  long bad = 0, corrupt = 0, ok = 0;
  for (int it = 0; it < iters; it++) {
    int ndim = (it % 3 == 0) ? 3 : 2;
    uint64_t dims[3] = {1 + next() % 12, 1 + next() % 40, ndim == 3 ? 1 + next() % 9 : 1};
    size_t n = dims[0] * dims[1] * dims[2];
    float *f = malloc(n * sizeof(float));
    for (size_t i = 0; i < n; i++) f[i] = (float)((long)(next() % 2001) - 1000) * 0.01f;
    size_t cap = ora_compress_bound(ndim, dims, it & 1);
    uint8_t *buf = malloc(cap);
    size_t sz = 0;
    ora_params p = {1, it & 1, (it >> 1) & 1, 16};
    if (ora_compress(f, ndim, dims, 0, 0.02 + (double)(next() % 100) * 0.01, &p, buf, cap, &sz) != ORA_OK) {
      bad++;
      continue;
    }
    float *out = malloc(n * sizeof(float));
    int mode = (int)(next() % 3);
    size_t len = sz;
    uint8_t *t = malloc(sz);
    memcpy(t, buf, sz);
    size_t hdr_hit = 0;
    if (mode == 0) {
      size_t nflip = 1 + next() % 4;
      for (size_t k = 0; k < nflip; k++) {
        size_t pos = (size_t)(next() % sz);
        if (pos < 384) hdr_hit = 1;
        t[pos] ^= (uint8_t)(1u << (next() % 8));
      }
    } else if (mode == 1) {
      len = (size_t)(next() % sz);
    } else {
      size_t pos = (size_t)(next() % sz);
      t[pos] = (uint8_t)next();
      if (pos < 384 && t[pos] != buf[pos]) hdr_hit = 1;
    }
    /* decode from an exact-size heap copy so ASan sees any overread */
    uint8_t *exact = malloc(len ? len : 1);
    memcpy(exact, t, len);
    ora_stats st;
    int rc = ora_decompress(exact, len, out, n, &st);
    if (rc == ORA_OK) ok++;
    else if (rc == ORA_E_CORRUPT) corrupt++;
    else bad++;
    if ((hdr_hit || len < sz) && rc != ORA_E_CORRUPT) {
      fprintf(stderr, "header corruption or truncation not detected (iter %d)\n", it);
      bad++;
    }
    free(exact);
    free(t);
    free(out);
    free(buf);
    free(f);
  }
  printf("ok %ld corrupt %ld bad %ld\n", ok, corrupt, bad);
  return bad == 0 ? 0 : 1;
}
