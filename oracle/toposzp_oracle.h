/*
 * TopoSZp CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded C implementation of the TopoSZp compressor
 * and decompressor (Sections II-C, III and IV of the paper), written from the
 * paper's description so that the GPU library can be checked against it.
 * Only the test suite, the smoke check and the CPU leg of the benchmark load
 * this library; the product path never does.  It shares no code, header,
 * table or constant generator with the GPU library.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared  (no fast-math, so
 * IEEE single/double arithmetic, denormals kept, no fused multiply-add).
 *
 * Parity status of each part (what pins it) is listed in toposzp_oracle.c.
 */
#ifndef TOPOSZP_ORACLE_H
#define TOPOSZP_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes (the values are part of the stream/API contract). */
#define ORA_OK 0
#define ORA_E_INVALID_ARG (-1)
#define ORA_E_NONFINITE (-2)
#define ORA_E_RANGE (-3)
#define ORA_E_CAPACITY (-4)
#define ORA_E_CORRUPT (-5)
#define ORA_E_UNSUPPORTED (-7)

/* Point classes, 2-bit codes of Section IV-A (1): r=00, m=01, s=10, M=11. */
#define ORA_R 0
#define ORA_MIN 1
#define ORA_SAD 2
#define ORA_MAX 3

typedef struct {
  int topo;        /* 1: TopoSZp (labels, ranks, stencil, RBF); 0: plain SZp */
  int rank_scope;  /* 0: ranks within a 64-point block; 1: whole field */
  int rbf_policy;  /* 0: adaptive k_size/sigma; 1: always k_size = 3 */
  int max_rounds;  /* RBF rounds cap (1..65535) */
} ora_params;

typedef struct {
  int64_t rounds;         /* RBF rounds executed */
  int64_t commits;        /* RBF updates committed, all rounds */
  int64_t worklist0;      /* saddles the stream marks lost (delta > 0) */
  int64_t stencil_moves;  /* extrema moved by the stencil */
  int64_t budget_skips;   /* lost extrema left unmoved by the error budget */
} ora_stats;

/* Whole pipeline --------------------------------------------------------- */
size_t ora_compress_bound(int ndim, const uint64_t dims[3], int rank_scope);
int ora_compress(const float *f, int ndim, const uint64_t dims[3], int eb_mode,
                 double eb, const ora_params *p, uint8_t *out, size_t out_cap,
                 size_t *out_size);
int ora_decompress(const uint8_t *in, size_t in_size, float *out,
                   size_t out_cap, ora_stats *st);

/* Counts topological errors of `recon` against `orig` (Section III-B):
 * counts[0]=FN, [1]=FP, [2]=FT, [3..6]=critical points of orig by class
 * r,m,s,M, [7..10]=FN by original class r,m,s,M. */
void ora_eval(const float *orig, const float *recon, int ndim,
              const uint64_t dims[3], int64_t counts[11], double *max_abs_err);

/* Pieces exposed for unit tests ------------------------------------------ */
float ora_eps_float(double eps_d);
int ora_quantize(float a, float e, int32_t *q);
float ora_recon(int32_t q, float e);
void ora_classify(const float *g, int ndim, const uint64_t dims[3],
                  uint8_t *cls);
int ora_quantize_field(const float *f, size_t n, float e, int32_t *q);
/* CD + RP of Section IV-A on field f with bin index field q: labels and the
 * rank metadata delta. */
void ora_labels_ranks(const float *f, const int32_t *q, int ndim,
                      const uint64_t dims[3], int rank_scope, uint8_t *label,
                      int32_t *delta);
void ora_rbf_weights(double sigma, float w[10]);
/* One 64-value block of the B+LZ+BE codec: returns the bit width and fills
 * first value, sign word and planes[0..w-1]. */
int ora_encode_block(const int32_t v[64], int32_t *first, uint64_t *sign,
                     uint64_t planes[32]);
void ora_decode_block(int w, int32_t first, uint64_t sign,
                      const uint64_t *planes, int32_t v[64]);
/* Header fields as the oracle wrote them (for tests): returns 0 or error. */
int ora_inspect(const uint8_t *in, size_t in_size, int64_t out[16],
                double dout[4], uint64_t seg_off[13], uint64_t seg_len[13]);

#ifdef __cplusplus
}
#endif
#endif
