/*
 * TopoSZp CPU oracle -- TEST INFRASTRUCTURE ONLY (see toposzp_oracle.h).
 *
 * Plain loops in the paper's order.  Compression (Section IV-A): critical
 * point detection (CD) and relative positions (RP) on the original values,
 * quantization (QZ), blocking + decorrelation (B+LZ) and fixed-length
 * encoding (BE) of the bin indices, then a second B+LZ+BE pass over the rank
 * metadata.  Decompression (Section IV-B): inverse BE/LZ/B/QZ, metadata
 * extraction (MD), the extrema stencil (CP+RP) and the RBF refinement of lost
 * saddles (RS) with the guard against new or changed critical points.
 *
 * Readings of points the paper leaves open:
 *  - QZ: bin q is the unique integer with (2q-1)e <= a < (2q+1)e, i.e.
 *    floor((a+e)/(2e)) in exact arithmetic (Section II-C formula); the
 *    reconstruction is the bin centre, float(2q) * e, rounded once
 *    (the printed "q*2e - e" is the bin edge, contradicting the stated
 *    centre and the |a - a^| <= e bound).  e is the requested bound rounded
 *    down to float32.
 *  - CD: 2D rule of Section IV-A extended to 3D with one axis pair per
 *    dimension; extrema use the available face neighbours (2 at corners,
 *    3 on edges); a saddle needs both neighbours on every axis of extent > 1,
 *    each pair both-higher or both-lower, with both kinds present.
 *  - RP: the rank metadata is stored for the critical points that the plain
 *    SZp reconstruction flattens (a face neighbour falls in the same bin):
 *    for such a maximum, 1 + the number of such maxima in the same bin (and
 *    the same 64-point block, or the whole field) with a smaller value; for a
 *    minimum, 1 + the number with a larger value; for a flattened saddle, 1.
 *    Every other point stores 0.  The decompressor only moves flattened
 *    extrema, so these ranks carry exactly the order it has to restore.
 *  - Lost points: the decoder takes them from the stream, an extremum or
 *    saddle label with delta > 0.  On streams the compressor writes these are
 *    exactly the labelled points that read as regular in the decoded field
 *    (the paper's test), and a lost extremum's neighbour maximum (minimum) of
 *    pre-stencil values is its own bin centre; every stream, canonical or
 *    not, is decoded by this one rule.
 *  - Stencil: eta is one float step (nextafterf), applied delta times from
 *    the bin centre (the pre-stencil neighbour extreme); a move is kept only
 *    if it stays within e of the bin centre.
 *  - RS: the candidate is the Gaussian-weighted mean of the window
 *    {q != p : |q - p|_2 <= floor(k/2)} (convex weights, Eq. (2)); it is kept
 *    only if it stays within e of the bin centre, makes p a saddle again and
 *    changes no neighbour's class other than r -> its own label.  Rounds of
 *    colour phases ((x+2y) mod 5 in 2D, (x+2y+3z) mod 7 in 3D; Jacobi within
 *    a phase) repeat until a round commits nothing or max_rounds is reached.
 *    k_size and sigma are chosen from the mean block bit width.
 *
 * What pins each part (tests/test_oracle_*.py, tests/test_stream_format.py):
 *  - QZ: exact-rational recomputation of the defining inequality, the
 *    worked example of Section III-A (Fig. 2), bin edges and power-of-two e.
 *  - CD: an independently written numpy classifier, closed-form critical point
 *    densities of i.i.d. noise (2D: 1/5, 1/5, 1/15; 3D: 1/7, 1/7, 2/35).
 *  - RP: the Fig. 5 example (M1 < M2 in bin 1 get ranks 1 and 2); the sign
 *    of every same-bin pair of restored minima and maxima against the
 *    original values; a kept and two lost maxima in one bin and block.
 *  - Codec and layout: lossless round trip, widths and signs against direct
 *    definitions, every header field and segment against the format table.
 *  - Stencil/RS: no false positives or false types (Section III-B argument,
 *    Table II), lost extrema all restored when the budget allows (Section V),
 *    |a - a^| <= 2e (Section V), single-bin and wide-gap special cases
 *    (Section IV-B), brute force over every 3x3 field on a 5-value alphabet;
 *    isolated refined saddles against the exact-rational Gaussian mean over
 *    the Euclidean ball (k = 5, 7 in 2D and 3D); one-round pairs against the
 *    Jacobi-within-phase, colour-ordered schedule.
 *  - Evaluation: a recount with the numpy classifier.
 *  - Byte layout of the stream: the paper gives only the list of parts, so
 *    it is pinned by the format table, not by the paper.
 */
#include "toposzp_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define BLK 64
#define QMAX 4194303 /* largest |q|: 2^22 - 1 */
#define HDR_BYTES 512
#define NSEG 13
#define MAXW_DATA 23
#define MAXW_RANK 31

enum {
  SEG_S1, SEG_S2, SEG_S3, SEG_S4, SEG_S6, SEG_R1, SEG_R2,
  SEG_R3, SEG_R4, SEG_X1, SEG_X2, SEG_S5, SEG_R5
};

typedef struct {
  int64_t nx, ny, nz, n;
} grid;

static int make_grid(int ndim, const uint64_t d[3], grid *g) {
  if (ndim == 2) {
    g->nz = 1;
    g->ny = (int64_t)d[0];
    g->nx = (int64_t)d[1];
  } else if (ndim == 3) {
    g->nz = (int64_t)d[0];
    g->ny = (int64_t)d[1];
    g->nx = (int64_t)d[2];
  } else {
    return ORA_E_INVALID_ARG;
  }
  if (g->nx < 1 || g->ny < 1 || g->nz < 1) return ORA_E_INVALID_ARG;
  if (g->nx > (1LL << 31) || g->ny > (1LL << 31) || g->nz > (1LL << 31))
    return ORA_E_UNSUPPORTED;
  g->n = g->nx * g->ny * g->nz;
  if (g->n >= (1LL << 31)) return ORA_E_UNSUPPORTED;
  return ORA_OK;
}

static void coords(const grid *g, int64_t i, int64_t c[3]) {
  c[0] = i % g->nx;
  c[1] = (i / g->nx) % g->ny;
  c[2] = i / (g->nx * g->ny);
}

/* Face neighbours of i that lie in the grid, x axis first, lower side first. */
static int face_neighbours(const grid *g, int64_t i, int64_t nb[6]) {
  int64_t c[3], ext[3] = {g->nx, g->ny, g->nz};
  int64_t stride[3] = {1, g->nx, g->nx * g->ny};
  int k = 0;
  coords(g, i, c);
  for (int ax = 0; ax < 3; ax++) {
    if (c[ax] > 0) nb[k++] = i - stride[ax];
    if (c[ax] < ext[ax] - 1) nb[k++] = i + stride[ax];
  }
  return k;
}

/* Class of point i in field v, where point `pi` (if >= 0) reads as `pv`. */
static int classify_at(const float *v, const grid *g, int64_t i, int64_t pi,
                       float pv) {
#define VAL(j) ((j) == pi ? pv : v[(j)])
  int64_t c[3], ext[3] = {g->nx, g->ny, g->nz};
  int64_t stride[3] = {1, g->nx, g->nx * g->ny};
  float a = VAL(i);
  int navail = 0, all_gt = 1, all_lt = 1;
  int up = 0, down = 0, pairs_ok = 1;
  coords(g, i, c);
  for (int ax = 0; ax < 3; ax++) {
    if (ext[ax] < 2) continue; /* an axis of extent 1 has no neighbours */
    int has_lo = c[ax] > 0, has_hi = c[ax] < ext[ax] - 1;
    int lo_gt = 0, lo_lt = 0, hi_gt = 0, hi_lt = 0;
    if (has_lo) {
      float b = VAL(i - stride[ax]);
      navail++;
      lo_gt = b > a;
      lo_lt = b < a;
      if (!lo_gt) all_gt = 0;
      if (!lo_lt) all_lt = 0;
    }
    if (has_hi) {
      float b = VAL(i + stride[ax]);
      navail++;
      hi_gt = b > a;
      hi_lt = b < a;
      if (!hi_gt) all_gt = 0;
      if (!hi_lt) all_lt = 0;
    }
    if (!(has_lo && has_hi))
      pairs_ok = 0;
    else if (lo_gt && hi_gt)
      up++;
    else if (lo_lt && hi_lt)
      down++;
    else
      pairs_ok = 0;
  }
#undef VAL
  if (navail == 0) return ORA_R;
  if (all_gt) return ORA_MIN;
  if (all_lt) return ORA_MAX;
  if (pairs_ok && up > 0 && down > 0) return ORA_SAD;
  return ORA_R;
}

void ora_classify(const float *g_, int ndim, const uint64_t dims[3],
                  uint8_t *cls) {
  grid g;
  if (make_grid(ndim, dims, &g) != ORA_OK) return;
  for (int64_t i = 0; i < g.n; i++) cls[i] = (uint8_t)classify_at(g_, &g, i, -1, 0.0f);
}

/* Quantization (Section II-C) ------------------------------------------- */

float ora_eps_float(double eps_d) {
  float f = (float)eps_d;
  if ((double)f > eps_d) f = nextafterf(f, 0.0f);
  return f;
}

int ora_quantize(float a, float e, int32_t *q) {
  if (!isfinite(a)) return ORA_E_NONFINITE;
  double ad = (double)a, ed = (double)e;
  double est = floor(ad / (2.0 * ed) + 0.5); /* a first guess only */
  if (est > QMAX + 2.0 || est < -(QMAX + 2.0)) return ORA_E_RANGE;
  int64_t k = (int64_t)est;
  /* (2k+-1) has at most 24 bits and e 24 significant bits, so both products
   * are exact in double: these are exact comparisons with the bin edges. */
  while ((double)(2 * k + 1) * ed <= ad) k++;
  while ((double)(2 * k - 1) * ed > ad) k--;
  if (k > QMAX || k < -QMAX) return ORA_E_RANGE;
  *q = (int32_t)k;
  return ORA_OK;
}

float ora_recon(int32_t q, float e) {
  float twoq = (float)(2 * q); /* exact: |2q| < 2^23 */
  return twoq * e;             /* one correctly rounded float product */
}

int ora_quantize_field(const float *f, size_t n, float e, int32_t *q) {
  for (size_t i = 0; i < n; i++) {
    int rc = ora_quantize(f[i], e, &q[i]);
    if (rc != ORA_OK) return rc;
  }
  return ORA_OK;
}

/* CD + RP (Section IV-A (1), (2)) --------------------------------------- */

static const float *g_sort_f;
static const int32_t *g_sort_q;
static const uint8_t *g_sort_l;

/* Order for field-wide ranks: by class, then bin, then from least to most
 * extreme value (ascending for maxima, descending for minima). */
static int cmp_field_rank(const void *pa, const void *pb) {
  int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
  if (g_sort_l[a] != g_sort_l[b]) return g_sort_l[a] < g_sort_l[b] ? -1 : 1;
  if (g_sort_q[a] != g_sort_q[b]) return g_sort_q[a] < g_sort_q[b] ? -1 : 1;
  float fa = g_sort_f[a], fb = g_sort_f[b];
  if (g_sort_l[a] == ORA_MIN) {
    float t = fa;
    fa = fb;
    fb = t;
  }
  if (fa < fb) return -1;
  if (fa > fb) return 1;
  return a < b ? -1 : (a > b ? 1 : 0);
}

void ora_labels_ranks(const float *f, const int32_t *q, int ndim,
                      const uint64_t dims[3], int rank_scope, uint8_t *label,
                      int32_t *delta) {
  grid g;
  if (make_grid(ndim, dims, &g) != ORA_OK) return;
  int64_t n = g.n;
  uint8_t *lost = (uint8_t *)calloc((size_t)n, 1);
  for (int64_t i = 0; i < n; i++) label[i] = (uint8_t)classify_at(f, &g, i, -1, 0.0f);
  /* A critical point is flattened when some face neighbour shares its bin:
   * then the plain SZp reconstruction ties them and the point turns regular. */
  for (int64_t i = 0; i < n; i++) {
    int64_t nb[6];
    int k = face_neighbours(&g, i, nb);
    if (label[i] == ORA_R) continue;
    for (int j = 0; j < k; j++)
      if (q[nb[j]] == q[i]) lost[i] = 1;
  }
  for (int64_t i = 0; i < n; i++) delta[i] = (lost[i] && label[i] == ORA_SAD) ? 1 : 0;
  if (rank_scope == 0) {
    for (int64_t b0 = 0; b0 < n; b0 += BLK) {
      int64_t b1 = b0 + BLK < n ? b0 + BLK : n;
      for (int64_t p = b0; p < b1; p++) {
        if (!lost[p] || (label[p] != ORA_MIN && label[p] != ORA_MAX)) continue;
        int32_t r = 1;
        for (int64_t j = b0; j < b1; j++) {
          if (!lost[j] || label[j] != label[p] || q[j] != q[p]) continue;
          if (label[p] == ORA_MAX ? (f[j] < f[p]) : (f[j] > f[p])) r++;
        }
        delta[p] = r;
      }
    }
  } else {
    int64_t m = 0;
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; i++)
      if (lost[i] && (label[i] == ORA_MIN || label[i] == ORA_MAX)) idx[m++] = i;
    g_sort_f = f;
    g_sort_q = q;
    g_sort_l = label;
    qsort(idx, (size_t)m, sizeof(int64_t), cmp_field_rank);
    /* rank = 1 + number of group members strictly less extreme */
    int64_t grp = 0, tie = 0;
    for (int64_t t = 0; t < m; t++) {
      int64_t i = idx[t];
      if (t == 0 || label[i] != label[idx[t - 1]] || q[i] != q[idx[t - 1]]) {
        grp = t;
        tie = t;
      } else if (f[i] != f[idx[t - 1]]) {
        tie = t;
      }
      delta[i] = (int32_t)(1 + (tie - grp));
    }
    free(idx);
  }
  free(lost);
}

/* B + LZ + BE (Section II-C, IV-A) -------------------------------------- */

int ora_encode_block(const int32_t v[64], int32_t *first, uint64_t *sign,
                     uint64_t planes[32]) {
  uint32_t mag[BLK];
  uint32_t mx = 0;
  *first = v[0];
  *sign = 0;
  mag[0] = 0; /* slot 0 holds no residual: the first value is stored raw */
  for (int i = 1; i < BLK; i++) {
    int64_t r = (int64_t)v[i] - (int64_t)v[i - 1];
    if (r < 0) {
      *sign |= 1ULL << i;
      mag[i] = (uint32_t)(-r);
    } else {
      mag[i] = (uint32_t)r;
    }
    if (mag[i] > mx) mx = mag[i];
  }
  int w = 0;
  while (w < 32 && (mx >> w) != 0) w++;
  for (int j = 0; j < w; j++) {
    uint64_t pl = 0;
    for (int i = 0; i < BLK; i++) pl |= (uint64_t)((mag[i] >> j) & 1u) << i;
    planes[j] = pl;
  }
  return w;
}

void ora_decode_block(int w, int32_t first, uint64_t sign,
                      const uint64_t *planes, int32_t v[64]) {
  uint32_t acc = (uint32_t)first;
  v[0] = first;
  for (int i = 1; i < BLK; i++) {
    uint32_t m = 0;
    for (int j = 0; j < w; j++) m |= (uint32_t)((planes[j] >> i) & 1u) << j;
    acc = ((sign >> i) & 1u) ? acc - m : acc + m;
    v[i] = (int32_t)acc;
  }
}

/* RBF parameters (Section IV-B (3)) --------------------------------------- */

void ora_rbf_weights(double sigma, float w[10]) {
  for (int d2 = 0; d2 < 10; d2++) w[d2] = (float)exp(-(double)d2 / (2.0 * sigma * sigma));
}

static void rbf_choice(int policy, uint64_t wsum, uint64_t nb, int *k, double *sigma) {
  if (policy == 1) {
    *k = 3;
    *sigma = 0.5;
  } else if (wsum <= nb) {
    *k = 7;
    *sigma = 1.0;
  } else if (wsum <= 3 * nb) {
    *k = 5;
    *sigma = 0.75;
  } else {
    *k = 3;
    *sigma = 0.5;
  }
}

/* Stream layout ----------------------------------------------------------- */

static void put_u16(uint8_t *b, size_t off, uint16_t v) { memcpy(b + off, &v, 2); }
static void put_u32(uint8_t *b, size_t off, uint32_t v) { memcpy(b + off, &v, 4); }
static void put_u64(uint8_t *b, size_t off, uint64_t v) { memcpy(b + off, &v, 8); }
static void put_f32(uint8_t *b, size_t off, float v) { memcpy(b + off, &v, 4); }
static void put_f64(uint8_t *b, size_t off, double v) { memcpy(b + off, &v, 8); }
static uint16_t get_u16(const uint8_t *b, size_t off) { uint16_t v; memcpy(&v, b + off, 2); return v; }
static uint32_t get_u32(const uint8_t *b, size_t off) { uint32_t v; memcpy(&v, b + off, 4); return v; }
static uint64_t get_u64(const uint8_t *b, size_t off) { uint64_t v; memcpy(&v, b + off, 8); return v; }
static float get_f32(const uint8_t *b, size_t off) { float v; memcpy(&v, b + off, 4); return v; }
static double get_f64(const uint8_t *b, size_t off) { double v; memcpy(&v, b + off, 8); return v; }

static uint64_t align8(uint64_t x) { return (x + 7) & ~(uint64_t)7; }

/* Adler-32 (RFC 1950) over the header fields, stored after them so that any
 * corrupted header byte is detected. */
#define HDR_SUMMED 376
static uint32_t adler32(const uint8_t *b, size_t n) {
  uint32_t a = 1, s = 0;
  for (size_t i = 0; i < n; i++) {
    a = (a + b[i]) % 65521u;
    s = (s + a) % 65521u;
  }
  return (s << 16) | a;
}

/* Lengths and offsets of the 13 segments: the fixed-size parts first (their
 * offsets depend on N only), the two variable-size payloads last. */
static uint64_t layout(uint64_t nb, int topo, uint64_t wdata, uint64_t wrank,
                       uint64_t off[NSEG], uint64_t len[NSEG]) {
  uint64_t nch = (nb + BLK - 1) / BLK;
  len[SEG_S1] = 8 * nch;
  len[SEG_S2] = nb;
  len[SEG_S3] = 8 * nb;
  len[SEG_S4] = 4 * nb;
  len[SEG_S6] = topo ? 16 * nb : 0;
  len[SEG_R1] = topo ? 8 * nch : 0;
  len[SEG_R2] = topo ? nb : 0;
  len[SEG_R3] = topo ? 8 * nb : 0;
  len[SEG_R4] = topo ? 4 * nb : 0;
  len[SEG_X1] = 8 * nch;
  len[SEG_X2] = topo ? 8 * nch : 0;
  len[SEG_S5] = 8 * wdata;
  len[SEG_R5] = topo ? 8 * wrank : 0;
  off[0] = HDR_BYTES;
  for (int s = 1; s < NSEG; s++) off[s] = align8(off[s - 1] + len[s - 1]);
  return off[NSEG - 1] + len[NSEG - 1];
}

size_t ora_compress_bound(int ndim, const uint64_t dims[3], int rank_scope) {
  grid g;
  uint64_t off[NSEG], len[NSEG];
  if (make_grid(ndim, dims, &g) != ORA_OK) return 0;
  uint64_t nb = ((uint64_t)g.n + BLK - 1) / BLK;
  return (size_t)layout(nb, 1, nb * MAXW_DATA, nb * (rank_scope ? MAXW_RANK : 7), off, len);
}

/* Encodes the 64-point blocks of v (padded with its last value) into the
 * five parts (1)-(5); returns the total number of planes. */
static uint64_t encode_stream(const int32_t *v, int64_t n, uint8_t *out,
                              const uint64_t off[NSEG], int s1, int s2, int s3,
                              int s4, int sx, int s5) {
  uint64_t nb = ((uint64_t)n + BLK - 1) / BLK;
  uint64_t planes_done = 0;
  for (uint64_t b = 0; b < nb; b++) {
    int32_t blk[BLK], first;
    uint64_t sign, planes[32];
    for (int i = 0; i < BLK; i++) {
      int64_t j = (int64_t)(b * BLK) + i;
      blk[i] = v[j < n ? j : n - 1];
    }
    if (b % BLK == 0) put_u64(out, off[sx] + 8 * (b / BLK), 8 * planes_done);
    int w = ora_encode_block(blk, &first, &sign, planes);
    if (w == 0) out[off[s1] + b / 8] |= (uint8_t)(1u << (b % 8));
    out[off[s2] + b] = (uint8_t)w;
    put_u64(out, off[s3] + 8 * b, sign);
    put_u32(out, off[s4] + 4 * b, (uint32_t)first);
    for (int j = 0; j < w; j++) put_u64(out, off[s5] + 8 * (planes_done + (uint64_t)j), planes[j]);
    planes_done += (uint64_t)w;
  }
  return planes_done;
}

static uint64_t count_planes(const int32_t *v, int64_t n) {
  uint64_t nb = ((uint64_t)n + BLK - 1) / BLK, tot = 0;
  for (uint64_t b = 0; b < nb; b++) {
    int32_t blk[BLK], first;
    uint64_t sign, planes[32];
    for (int i = 0; i < BLK; i++) {
      int64_t j = (int64_t)(b * BLK) + i;
      blk[i] = v[j < n ? j : n - 1];
    }
    tot += (uint64_t)ora_encode_block(blk, &first, &sign, planes);
  }
  return tot;
}

int ora_compress(const float *f, int ndim, const uint64_t dims[3], int eb_mode,
                 double eb, const ora_params *p, uint8_t *out, size_t out_cap,
                 size_t *out_size) {
  grid g;
  ora_params dp = {1, 0, 0, 16};
  if (!p) p = &dp;
  if (!f || !dims || !out || !out_size) return ORA_E_INVALID_ARG;
  int rc = make_grid(ndim, dims, &g);
  if (rc != ORA_OK) return rc;
  if (!(eb > 0.0) || !isfinite(eb) || (eb_mode != 0 && eb_mode != 1)) return ORA_E_INVALID_ARG;
  if ((p->topo != 0 && p->topo != 1) || (p->rank_scope != 0 && p->rank_scope != 1) ||
      (p->rbf_policy != 0 && p->rbf_policy != 1) || p->max_rounds < 1 || p->max_rounds > 65535)
    return ORA_E_INVALID_ARG;
  int64_t n = g.n;
  for (int64_t i = 0; i < n; i++)
    if (!isfinite(f[i])) return ORA_E_NONFINITE;
  float vmin = 0.0f, vmax = 0.0f;
  double eps_d = eb;
  if (eb_mode == 1) {
    vmin = f[0];
    vmax = f[0];
    for (int64_t i = 1; i < n; i++) {
      if (f[i] < vmin) vmin = f[i];
      if (f[i] > vmax) vmax = f[i];
    }
    /* a zero extreme is stored as +0 whichever signed zero came first */
    if (vmin == 0.0f) vmin = 0.0f;
    if (vmax == 0.0f) vmax = 0.0f;
    if (vmax > vmin) eps_d = eb * ((double)vmax - (double)vmin);
  }
  float e = ora_eps_float(eps_d);
  if (!(e >= ldexpf(1.0f, -100)) || !(e <= ldexpf(1.0f, 100))) return ORA_E_RANGE;

  int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  uint8_t *label = (uint8_t *)calloc((size_t)n, 1);
  int32_t *delta = (int32_t *)calloc((size_t)n, sizeof(int32_t));
  rc = ora_quantize_field(f, (size_t)n, e, q);
  if (rc != ORA_OK) goto done;
  if (p->topo) ora_labels_ranks(f, q, ndim, dims, p->rank_scope, label, delta);

  uint64_t nb = ((uint64_t)n + BLK - 1) / BLK;
  uint64_t nch = (nb + BLK - 1) / BLK;
  uint64_t wdata = count_planes(q, n);
  uint64_t wrank = p->topo ? count_planes(delta, n) : 0;
  uint64_t off[NSEG], len[NSEG];
  uint64_t total = layout(nb, p->topo, wdata, wrank, off, len);
  if (total > out_cap) {
    rc = ORA_E_CAPACITY;
    goto done;
  }
  memset(out, 0, (size_t)total);

  int k;
  double sigma;
  float w[10];
  rbf_choice(p->rbf_policy, wdata, nb, &k, &sigma);
  ora_rbf_weights(sigma, w);

  /* header */
  memcpy(out, "TSZ1", 4);
  put_u16(out, 4, 1);
  out[6] = (uint8_t)ndim;
  out[7] = (uint8_t)((p->topo ? 1 : 0) | (p->rank_scope ? 2 : 0));
  for (int d = 0; d < 3; d++) put_u64(out, 8 + 8 * (size_t)d, d < ndim ? dims[d] : 1);
  put_u64(out, 32, (uint64_t)n);
  put_u64(out, 40, nb);
  put_u32(out, 48, BLK);
  out[52] = (uint8_t)eb_mode;
  out[53] = (uint8_t)k;
  put_u16(out, 54, (uint16_t)p->max_rounds);
  put_f64(out, 56, eb);
  put_f64(out, 64, eps_d);
  put_f32(out, 72, e);
  put_f32(out, 76, vmin);
  put_f32(out, 80, vmax);
  put_f32(out, 84, (float)sigma);
  for (int d2 = 0; d2 < 10; d2++) put_f32(out, 88 + 4 * (size_t)d2, w[d2]);
  put_u64(out, 128, total);
  put_u64(out, 136, wdata);
  put_u64(out, 144, wrank);
  put_u64(out, 152, nch);
  for (int s = 0; s < NSEG; s++) {
    put_u64(out, 160 + 8 * (size_t)s, off[s]);
    put_u64(out, 264 + 8 * (size_t)s, len[s]);
  }

  put_u32(out, HDR_SUMMED, adler32(out, HDR_SUMMED));

  /* parts (1)-(5) of the bin indices */
  encode_stream(q, n, out, off, SEG_S1, SEG_S2, SEG_S3, SEG_S4, SEG_X1, SEG_S5);
  if (p->topo) {
    /* part (6): 2-bit labels, point i at byte i/4, bits 2(i%4) and up */
    for (int64_t i = 0; i < n; i++)
      out[off[SEG_S6] + (uint64_t)(i >> 2)] |= (uint8_t)(label[i] << (2 * (i & 3)));
    /* part (7): the rank metadata through B+LZ+BE again, without QZ */
    encode_stream(delta, n, out, off, SEG_R1, SEG_R2, SEG_R3, SEG_R4, SEG_X2, SEG_R5);
  }
  *out_size = (size_t)total;
  rc = ORA_OK;
done:
  free(q);
  free(label);
  free(delta);
  return rc;
}

/* Header validation and decoding ------------------------------------------ */

typedef struct {
  int ndim, topo, scope, eb_mode, k, max_rounds;
  uint64_t dims[3], n, nb, nch, total, wdata, wrank;
  float e, sigma, w[10];
  double eb, eps_d;
  uint64_t off[NSEG], len[NSEG];
} hdr_t;

static int parse_header(const uint8_t *in, size_t in_size, hdr_t *h) {
  if (!in || in_size < HDR_BYTES) return ORA_E_CORRUPT;
  if (memcmp(in, "TSZ1", 4) != 0 || get_u16(in, 4) != 1) return ORA_E_CORRUPT;
  if (get_u32(in, HDR_SUMMED) != adler32(in, HDR_SUMMED) || get_u32(in, HDR_SUMMED + 4) != 0)
    return ORA_E_CORRUPT;
  h->ndim = in[6];
  if (h->ndim != 2 && h->ndim != 3) return ORA_E_CORRUPT;
  if (in[7] & ~3u) return ORA_E_CORRUPT;
  h->topo = in[7] & 1;
  h->scope = (in[7] >> 1) & 1;
  uint64_t prod = 1;
  for (int d = 0; d < 3; d++) {
    h->dims[d] = get_u64(in, 8 + 8 * (size_t)d);
    if (h->dims[d] < 1 || h->dims[d] > (1ULL << 31)) return ORA_E_CORRUPT;
    if (d >= h->ndim && h->dims[d] != 1) return ORA_E_CORRUPT;
    prod *= h->dims[d];
    if (prod >= (1ULL << 31)) return ORA_E_CORRUPT;
  }
  h->n = get_u64(in, 32);
  h->nb = get_u64(in, 40);
  h->nch = get_u64(in, 152);
  if (h->n != prod || h->nb != (h->n + BLK - 1) / BLK || h->nch != (h->nb + BLK - 1) / BLK)
    return ORA_E_CORRUPT;
  if (get_u32(in, 48) != BLK) return ORA_E_CORRUPT;
  h->eb_mode = in[52];
  h->k = in[53];
  h->max_rounds = get_u16(in, 54);
  if (h->eb_mode > 1 || (h->k != 3 && h->k != 5 && h->k != 7) || h->max_rounds < 1)
    return ORA_E_CORRUPT;
  h->eb = get_f64(in, 56);
  h->eps_d = get_f64(in, 64);
  h->e = get_f32(in, 72);
  if (!(h->e >= ldexpf(1.0f, -100)) || !(h->e <= ldexpf(1.0f, 100))) return ORA_E_CORRUPT;
  h->sigma = get_f32(in, 84);
  for (int d2 = 0; d2 < 10; d2++) {
    h->w[d2] = get_f32(in, 88 + 4 * (size_t)d2);
    if (!(h->w[d2] > 0.0f) || !(h->w[d2] <= 1.0f)) return ORA_E_CORRUPT;
  }
  h->total = get_u64(in, 128);
  h->wdata = get_u64(in, 136);
  h->wrank = get_u64(in, 144);
  if (h->wdata > h->nb * MAXW_DATA || h->wrank > h->nb * MAXW_RANK) return ORA_E_CORRUPT;
  uint64_t off[NSEG], len[NSEG];
  uint64_t total = layout(h->nb, h->topo, h->wdata, h->wrank, off, len);
  if (total != h->total || total > in_size) return ORA_E_CORRUPT;
  for (int s = 0; s < NSEG; s++) {
    h->off[s] = get_u64(in, 160 + 8 * (size_t)s);
    h->len[s] = get_u64(in, 264 + 8 * (size_t)s);
    if (h->off[s] != off[s] || h->len[s] != len[s]) return ORA_E_CORRUPT;
  }
  return ORA_OK;
}

int ora_inspect(const uint8_t *in, size_t in_size, int64_t out[16],
                double dout[4], uint64_t seg_off[13], uint64_t seg_len[13]) {
  hdr_t h;
  int rc = parse_header(in, in_size, &h);
  if (rc != ORA_OK) return rc;
  int64_t v[16] = {h.ndim, h.topo, h.scope, h.eb_mode, h.k, h.max_rounds,
                   (int64_t)h.dims[0], (int64_t)h.dims[1], (int64_t)h.dims[2],
                   (int64_t)h.n, (int64_t)h.nb, (int64_t)h.nch, (int64_t)h.total,
                   (int64_t)h.wdata, (int64_t)h.wrank, 0};
  memcpy(out, v, sizeof(v));
  dout[0] = h.eb;
  dout[1] = h.eps_d;
  dout[2] = h.e;
  dout[3] = h.sigma;
  memcpy(seg_off, h.off, sizeof(h.off));
  memcpy(seg_len, h.len, sizeof(h.len));
  return ORA_OK;
}

/* Decodes the blocks of parts (1)-(5) into v[0..n); checks each width and
 * the chunk index against the widths. */
static int decode_stream(const uint8_t *in, const hdr_t *h, int s1, int s2,
                         int s3, int s4, int sx, int s5, int maxw, int64_t vmin,
                         int64_t vmax, int32_t *v) {
  uint64_t planes_done = 0;
  for (uint64_t b = 0; b < h->nb; b++) {
    int w = in[h->off[s2] + b];
    int cbit = (in[h->off[s1] + b / 8] >> (b % 8)) & 1;
    if (w > maxw || cbit != (w == 0)) return ORA_E_CORRUPT;
    if (b % BLK == 0 && get_u64(in, h->off[sx] + 8 * (b / BLK)) != 8 * planes_done)
      return ORA_E_CORRUPT;
    if (8 * (planes_done + (uint64_t)w) > h->len[s5]) return ORA_E_CORRUPT;
    uint64_t planes[32];
    for (int j = 0; j < w; j++) planes[j] = get_u64(in, h->off[s5] + 8 * (planes_done + (uint64_t)j));
    int32_t blk[BLK];
    ora_decode_block(w, (int32_t)get_u32(in, h->off[s4] + 4 * b), get_u64(in, h->off[s3] + 8 * b),
                     planes, blk);
    for (int i = 0; i < BLK; i++) {
      uint64_t j = b * BLK + (uint64_t)i;
      if (j >= h->n) continue;
      if (blk[i] < vmin || blk[i] > vmax) return ORA_E_CORRUPT;
      v[j] = blk[i];
    }
    planes_done += (uint64_t)w;
  }
  if (8 * planes_done != h->len[s5]) return ORA_E_CORRUPT;
  /* the bitmap's bits past the last block are 0 */
  for (uint64_t b = h->nb; b < 64 * h->nch; b++)
    if ((in[h->off[s1] + b / 8] >> (b % 8)) & 1) return ORA_E_CORRUPT;
  return ORA_OK;
}

/* delta float steps from v: up (+) or down (-); a zero result is +0. */
static float float_steps(float v, int32_t delta, int up) {
  for (int32_t t = 0; t < delta; t++) {
    v = nextafterf(v, up ? INFINITY : -INFINITY);
    if (v == 0.0f) v = 0.0f;
  }
  return v;
}

int ora_decompress(const uint8_t *in, size_t in_size, float *out,
                   size_t out_cap, ora_stats *st) {
  hdr_t h;
  ora_stats local = {0, 0, 0, 0, 0};
  if (!st) st = &local;
  memset(st, 0, sizeof(*st));
  if (!out) return ORA_E_INVALID_ARG;
  int rc = parse_header(in, in_size, &h);
  if (rc != ORA_OK) return rc;
  if (h.n > out_cap) return ORA_E_CAPACITY;
  grid g;
  if (make_grid(h.ndim, h.dims, &g) != ORA_OK) return ORA_E_CORRUPT;
  int64_t n = g.n;
  int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *delta = NULL;
  uint8_t *label = NULL;
  int64_t *work = NULL, *acc_i = NULL;
  float *acc_v = NULL;

  /* inverse BE, LZ + B, QZ: the plain SZp reconstruction */
  rc = decode_stream(in, &h, SEG_S1, SEG_S2, SEG_S3, SEG_S4, SEG_X1, SEG_S5, MAXW_DATA, -QMAX,
                     QMAX, q);
  if (rc != ORA_OK) goto done;
  for (int64_t i = 0; i < n; i++) out[i] = ora_recon(q[i], h.e);
  if (!h.topo) goto done;

  /* MD: labels and ranks */
  delta = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  label = (uint8_t *)malloc((size_t)n);
  /* ranks lie in [0, 64] within a block and in [0, N] field-wide */
  rc = decode_stream(in, &h, SEG_R1, SEG_R2, SEG_R3, SEG_R4, SEG_X2, SEG_R5, MAXW_RANK, 0,
                     h.scope ? (int64_t)h.n : BLK, delta);
  if (rc != ORA_OK) goto done;
  for (int64_t i = 0; i < n; i++)
    label[i] = (uint8_t)((in[h.off[SEG_S6] + (uint64_t)(i >> 2)] >> (2 * (i & 3))) & 3u);

  /* CP + RP: the extrema stencil.  The lost critical points are the ones
   * the stream marks with delta > 0 (an extremum or saddle label); the
   * compressor marks exactly those with a face neighbour in their own bin,
   * which are exactly the critical points that read as regular in the
   * decoded field (R is strictly increasing, so every strict neighbour order
   * across bins survives and every tie within a bin breaks the point).  For
   * a lost maximum every neighbour's decoded value is at most its own bin
   * centre and one equals it, so the neighbour maximum of the paper's
   * stencil is the point's own centre R(q); likewise the neighbour minimum
   * of a lost minimum.  The decoder therefore reads both from the stream
   * instead of reclassifying: delta float steps up (maximum) or down
   * (minimum) from R(q), kept only within e of R(q).  A stream that marks
   * other points (the compressor never writes one) is decoded by the same
   * rule. */
  for (int64_t i = 0; i < n; i++) {
    if ((label[i] != ORA_MIN && label[i] != ORA_MAX) || delta[i] == 0) continue;
    float rq = ora_recon(q[i], h.e);
    float v = float_steps(rq, delta[i], label[i] == ORA_MAX);
    if (fabs((double)v - (double)rq) <= (double)h.e) {
      out[i] = v;
      st->stencil_moves++;
    } else {
      st->budget_skips++;
    }
  }

  /* RS: RBF refinement of saddles that are still lost */
  {
    int r = h.k / 2;
    int64_t ncol = (h.ndim == 3) ? 7 : 5;
    int offs[400][4];
    int noff = 0;
    int rz = (h.ndim == 3) ? r : 0;
    for (int dz = -rz; dz <= rz; dz++)
      for (int dy = -r; dy <= r; dy++)
        for (int dx = -r; dx <= r; dx++) {
          int d2 = dz * dz + dy * dy + dx * dx;
          if (d2 == 0 || d2 > r * r) continue;
          offs[noff][0] = dz;
          offs[noff][1] = dy;
          offs[noff][2] = dx;
          offs[noff][3] = d2;
          noff++;
        }
    int64_t nw = 0;
    work = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    acc_i = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    acc_v = (float *)malloc(sizeof(float) * (size_t)(n > 0 ? n : 1));
    /* the lost saddles, as the stream marks them; one that the stencil has
     * already made a saddle again is skipped by every round below */
    for (int64_t i = 0; i < n; i++)
      if (label[i] == ORA_SAD && delta[i] > 0) work[nw++] = i;
    st->worklist0 = nw;
    for (int round = 1; round <= h.max_rounds; round++) {
      int64_t commits = 0;
      st->rounds = round;
      for (int64_t col = 0; col < ncol; col++) {
        int64_t nacc = 0;
        for (int64_t t = 0; t < nw; t++) {
          int64_t p = work[t], c[3];
          coords(&g, p, c);
          int64_t colour = (h.ndim == 3) ? (c[0] + 2 * c[1] + 3 * c[2]) % 7 : (c[0] + 2 * c[1]) % 5;
          if (colour != col) continue;
          if (classify_at(out, &g, p, -1, 0.0f) == ORA_SAD) continue;
          /* candidate: normalized Gaussian average over the window */
          double num = 0.0, den = 0.0;
          for (int o = 0; o < noff; o++) {
            int64_t z = c[2] + offs[o][0], y = c[1] + offs[o][1], x = c[0] + offs[o][2];
            if (z < 0 || z >= g.nz || y < 0 || y >= g.ny || x < 0 || x >= g.nx) continue;
            double wt = (double)h.w[offs[o][3]];
            num = num + wt * (double)out[(z * g.ny + y) * g.nx + x];
            den = den + wt;
          }
          if (den == 0.0) continue;
          float v = (float)(num / den);
          /* (i) stays within e of the bin centre */
          if (!(fabs((double)v - (double)ora_recon(q[p], h.e)) <= (double)h.e)) continue;
          /* (ii) p becomes a saddle again */
          if (classify_at(out, &g, p, p, v) != ORA_SAD) continue;
          /* (iii) no neighbour changes class, except r -> its own label */
          int64_t nb[6];
          int k = face_neighbours(&g, p, nb), ok = 1;
          for (int j = 0; j < k && ok; j++) {
            int before = classify_at(out, &g, nb[j], -1, 0.0f);
            int after = classify_at(out, &g, nb[j], p, v);
            if (after != before && !(before == ORA_R && after == label[nb[j]])) ok = 0;
          }
          if (!ok) continue;
          acc_i[nacc] = p;
          acc_v[nacc] = v;
          nacc++;
        }
        for (int64_t t = 0; t < nacc; t++) out[acc_i[t]] = acc_v[t];
        commits += nacc;
      }
      st->commits += commits;
      if (commits == 0) break;
    }
  }
  rc = ORA_OK;
done:
  free(q);
  free(delta);
  free(label);
  free(work);
  free(acc_i);
  free(acc_v);
  return rc;
}

void ora_eval(const float *orig, const float *recon, int ndim,
              const uint64_t dims[3], int64_t counts[11], double *max_abs_err) {
  grid g;
  for (int k = 0; k < 11; k++) counts[k] = 0;
  *max_abs_err = 0.0;
  if (make_grid(ndim, dims, &g) != ORA_OK) return;
  for (int64_t i = 0; i < g.n; i++) {
    int lo = classify_at(orig, &g, i, -1, 0.0f);
    int lr = classify_at(recon, &g, i, -1, 0.0f);
    counts[3 + lo]++;
    if (lo != ORA_R && lr == ORA_R) {
      counts[0]++;
      counts[7 + lo]++;
    }
    if (lo == ORA_R && lr != ORA_R) counts[1]++;
    if (lo != ORA_R && lr != ORA_R && lo != lr) counts[2]++;
    double d = fabs((double)orig[i] - (double)recon[i]);
    if (d > *max_abs_err) *max_abs_err = d;
  }
}
