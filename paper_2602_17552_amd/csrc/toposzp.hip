// libtoposzp: TopoSZp compression and decompression on MI355X (gfx950).
//
// One wave of 64 lanes handles one 64-point block (lane = point); a
// workgroup handles a chunk of 64 blocks (4096 points).
//
// Compression (Section IV-A):
//   range_kernel     relative bound only: per-workgroup min/max partials.
//   encode_kernel    per chunk: critical point detection and ranks on the
//                    original values, exact quantization, 1-D differences,
//                    per-block bit widths, sign and bit-plane ballots, 2-bit
//                    labels; fixed-size parts written in place, the chunk's
//                    bit planes staged compactly; chunk plane totals.
//   scan_kernel      one workgroup: exclusive scan of the chunk totals.
//   finalize_kernel  per chunk: staged planes to their final offsets, chunk
//                    index; workgroup 0 writes the header and status.
// Decompression (Section IV-B):
//   decode_kernel    per chunk: planes -> residuals -> in-wave prefix sum ->
//                    bin centres; labels and ranks; the extrema stencil (a
//                    flattened extremum moves delta float steps off its bin
//                    centre); flattened saddles queued per chunk.
//   refine_kernel    per chunk: the RBF refinement of queued saddles.
//                    Queued saddles that cannot influence each other's
//                    evaluation evolve independently under the colour-phased
//                    schedule, so an isolated saddle is settled by a single
//                    evaluation and a small cluster by one thread replaying
//                    the schedule on its members.
//   tail_kernel      one workgroup: the same schedule with workgroup
//                    barriers for the rare clusters too large for one
//                    thread; status and counters.
//
// No kernel contends on a single global address; every device wait is
// bounded.  Readings of points the paper leaves open are stated where used.
#include <hip/hip_runtime.h>

#include <cmath>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "toposzp.h"

namespace {

constexpr int kB = 64;                 // points per block (one wave)
constexpr int kQMax = 4194303;         // |q| <= 2^22 - 1
constexpr int kHdr = 512;              // header bytes
constexpr int kSummed = 376;           // header bytes covered by Adler-32
constexpr int kMaxWData = 23;          // widest value residual: 2 * kQMax < 2^23
constexpr int kMaxWRankBlk = 7;        // block-scope ranks lie in [0, 64]
constexpr int kMaxWRankAny = 31;       // field-scope ranks lie in [0, N]
constexpr int kNSeg = 13;
constexpr int kMaxRounds = 65535;
constexpr int kChunk = kB * kB;        // points per chunk
constexpr int kRangeWG = 512;          // max range-pass workgroups
constexpr int kClusterMax = 32;        // cluster members one thread replays
constexpr int kRefineThreads = 128;
constexpr int kSpreadLines = 64;       // counters spread over cache lines
enum { S1, S2, S3, S4, S6, R1, R2, R3, R4, X1, X2, S5, R5 };
enum { CLS_R = 0, CLS_MIN = 1, CLS_SAD = 2, CLS_MAX = 3 };

// ---------------------------------------------------------------------------
// Workspace layout: control block, spread counters, range partials, then a
// region whose layout depends on the call's field size (each call writes
// what it reads there).

struct Div {
  unsigned m;
  int l;
};
struct GeomD {
  int n, nx, ny, nz, nxy;
  Div dx, dy;
};

struct Plan {                 // decode -> refine/tail hand-off
  int valid, topo, ndim, k, ncol, max_rounds, nch;
  GeomD g;
  float e;
  float w[10];
  uint64_t s6_off;
};

struct Ctrl {
  // compression: written by scan_kernel, read by finalize_kernel
  unsigned long long tot_data, tot_rank;
  unsigned cflags;            // 1 non-finite, 2 bound out of range, 4 |q| too big
  float e, vmin, vmax;
  double eps;
  // decompression
  unsigned hflags;            // header check of this call: 0 good, 1 corrupt, 2 capacity
  unsigned big_count;         // saddles in clusters left to the tail kernel
  unsigned long long stats[5];// rounds, commits, queued, stencil moves, budget skips
  Plan plan;
};
static_assert(sizeof(Ctrl) <= 1024 - 16, "control block");

struct Spread {               // one cache line each
  unsigned commits, rounds, queued, pad[13];
};

constexpr size_t kSpreadOff = 1024;
constexpr size_t kPartOff = (kSpreadOff + sizeof(Spread) * kSpreadLines + 255) & ~size_t(255);
constexpr size_t kRegionOff = (kPartOff + 16 * kRangeWG + 255) & ~size_t(255);

__host__ __device__ constexpr uint64_t al256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

struct CompLayout {
  uint64_t tot_d, tot_r, cflag, stage_d, stage_r, end;
};
__host__ __device__ inline CompLayout comp_layout(uint64_t nch) {
  CompLayout L;
  L.tot_d = kRegionOff;
  L.tot_r = L.tot_d + 4 * nch;
  L.cflag = L.tot_r + 4 * nch;
  L.stage_d = al256(L.cflag + 4 * nch);
  L.stage_r = al256(L.stage_d + 8ull * kB * kMaxWData * nch);
  L.end = al256(L.stage_r + 8ull * kB * kMaxWRankBlk * nch);
  return L;
}

struct DecLayout {
  uint64_t cnt, moves, skips, dflag, bitmap, idx, col, state, pend, big, end;
};
__host__ __device__ inline DecLayout dec_layout(uint64_t nb, uint64_t nch) {
  DecLayout L;
  const uint64_t slots = nch * kChunk;
  L.cnt = kRegionOff;
  L.moves = L.cnt + 4 * nch;
  L.skips = L.moves + 4 * nch;
  L.dflag = L.skips + 4 * nch;
  L.bitmap = al256(L.dflag + 4 * nch);
  L.idx = al256(L.bitmap + 8 * nb);
  L.col = al256(L.idx + 4 * slots);
  L.state = al256(L.col + slots);
  L.pend = al256(L.state + slots);
  L.big = al256(L.pend + 4 * slots);
  L.end = al256(L.big + 4 * slots);
  return L;
}

// ---------------------------------------------------------------------------
// Device helpers.

__device__ __forceinline__ int fkey(float x) {
  // order-preserving integer key of a float; -0 and +0 share key 0
  int b = __float_as_int(x);
  return b >= 0 ? b : (int)(0x80000000u - (unsigned)b);
}
__device__ __forceinline__ float key2f(long long k) {
  if (k > 0x7F800000LL) k = 0x7F800001LL;  // past +inf: not a finite value
  if (k < -0x7F800000LL) k = -0x7F800001LL;
  unsigned b = k >= 0 ? (unsigned)k : 0x80000000u + (unsigned)(-k);
  return __int_as_float((int)b);
}
__device__ __forceinline__ unsigned ukey(float x) { return (unsigned)fkey(x) ^ 0x80000000u; }
__device__ __forceinline__ float ukey2f(unsigned u) { return key2f((int)(u ^ 0x80000000u)); }

__device__ __forceinline__ float round_down_f(double d) {
  float f = (float)d;
  if ((double)f > d) f = __int_as_float(__float_as_int(f) - 1);  // d > 0 here
  return f;
}

// Bin index of a: the unique q with (2q-1)e <= a < (2q+1)e.  A float estimate
// is corrected once by an exact test: with |q| < 2^23 the product q*2e is
// exact in double and a - q*2e is exact near the bin edges, so the two
// comparisons with +-e decide the edges exactly.
__device__ __forceinline__ int quantize(float a, float inv2e, double ed) {
  float t = rintf(a * inv2e);
  t = fminf(fmaxf(t, -4194305.0f), 4194305.0f);
  int q = (int)t;
  double d = (double)a - (double)q * (2.0 * ed);
  q += (d >= ed) ? 1 : ((d < -ed) ? -1 : 0);
  return q;
}

// Class from the six face neighbours [x-, x+, y-, y+, z-, z+]; axes of
// extent 1 carry no neighbours and take no part in the saddle test.
__device__ __forceinline__ int classify6(float a, const float nb[6], const bool av[6],
                                         const bool deg[3]) {
  int navail = 0, up = 0, dn = 0;
  bool all_gt = true, all_lt = true, pairs_ok = true;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    if (deg[ax]) continue;
    const bool hl = av[2 * ax], hh = av[2 * ax + 1];
    const bool lg = hl && nb[2 * ax] > a, ll = hl && nb[2 * ax] < a;
    const bool hg = hh && nb[2 * ax + 1] > a, hs = hh && nb[2 * ax + 1] < a;
    navail += (int)hl + (int)hh;
    if (hl && !lg) all_gt = false;
    if (hl && !ll) all_lt = false;
    if (hh && !hg) all_gt = false;
    if (hh && !hs) all_lt = false;
    if (!(hl && hh)) pairs_ok = false;
    else if (lg && hg) ++up;
    else if (ll && hs) ++dn;
    else pairs_ok = false;
  }
  if (navail == 0) return CLS_R;
  if (all_gt) return CLS_MIN;
  if (all_lt) return CLS_MAX;
  if (pairs_ok && up > 0 && dn > 0) return CLS_SAD;
  return CLS_R;
}

// Division by an invariant 31-bit divisor d (Granlund-Montgomery): with
// l = ceil(log2 d) and m = ceil(2^(31+l) / d) < 2^32, floor(n / d) =
// floor(n * m / 2^(31+l)) for every 0 <= n < 2^31.
__host__ __device__ inline Div make_div(unsigned d) {
  int l = 0;
  while ((1ull << l) < d) ++l;
  const unsigned long long m = ((1ull << (31 + l)) + d - 1) / d;
  return {(unsigned)m, l};
}
__device__ __forceinline__ int fdiv(int n, Div v) {
  return v.l == 0 ? n : (int)(__umulhi((unsigned)n, v.m) >> (v.l - 1));
}

// Grid coordinates of flat index i (x fastest).
struct Pt {
  int x, y, z;
};
__device__ __forceinline__ Pt coords_of(int i, const GeomD& g) {
  const int t = fdiv(i, g.dx);
  const int z = fdiv(t, g.dy);
  return {i - t * g.nx, t - z * g.ny, z};
}

// Cross-lane moves on the data-parallel-primitives path (all 64 lanes active):
// wave_shr:1 (lane i reads lane i-1, lane 0 reads `edge`), wave_shl:1 (lane i
// reads lane i+1, lane 63 reads `edge`), and row-level patterns.
__device__ __forceinline__ int dpp_from_prev(int v, int edge) {
  return __builtin_amdgcn_update_dpp(edge, v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ int dpp_from_next(int v, int edge) {
  return __builtin_amdgcn_update_dpp(edge, v, 0x130, 0xf, 0xf, false);
}
__device__ __forceinline__ unsigned wave_max_u(unsigned v) {
  // within each row of 16: xor 1, xor 2 (quad permutes), rotate 4, rotate 8
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xf, 0xf, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xf, 0xf, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x124, 0xf, 0xf, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xf, 0xf, false));
  const unsigned a = (unsigned)__builtin_amdgcn_readlane((int)v, 0);
  const unsigned b = (unsigned)__builtin_amdgcn_readlane((int)v, 16);
  const unsigned c = (unsigned)__builtin_amdgcn_readlane((int)v, 32);
  const unsigned d = (unsigned)__builtin_amdgcn_readlane((int)v, 48);
  return max(max(a, b), max(c, d));
}
// Inclusive prefix sum over the wave: shifts by 1, 2, 4, 8 within rows of
// 16, then row 0's total into row 1 (and 2's into 3), then rows 0-1 into 2-3.
__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
  (void)lane;
  unsigned u = (unsigned)v;
  u += (unsigned)__builtin_amdgcn_update_dpp(0, (int)u, 0x111, 0xf, 0xf, false);
  u += (unsigned)__builtin_amdgcn_update_dpp(0, (int)u, 0x112, 0xf, 0xf, false);
  u += (unsigned)__builtin_amdgcn_update_dpp(0, (int)u, 0x114, 0xf, 0xf, false);
  u += (unsigned)__builtin_amdgcn_update_dpp(0, (int)u, 0x118, 0xf, 0xf, false);
  u += (unsigned)__builtin_amdgcn_update_dpp(0, (int)u, 0x142, 0xa, 0xf, false);
  u += (unsigned)__builtin_amdgcn_update_dpp(0, (int)u, 0x143, 0xc, 0xf, false);
  return (int)u;
}
// Lane `l` (uniform) takes the uniform value `v`; other lanes keep `old`.
__device__ __forceinline__ unsigned write_lane(unsigned old, unsigned v, int l) {
  return (int)(threadIdx.x & 63) == l ? v : old;
}
// OR over each row of 16 lanes, complete in the row's last lane.
__device__ __forceinline__ unsigned row_or_last(unsigned v) {
  v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);
  v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);
  v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);
  v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);
  return v;
}
__device__ __forceinline__ unsigned mbcnt(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// B + LZ + BE of one 64-value block held one value per lane: residuals
// r_0 = 0, r_i = v_i - v_{i-1}; width = bit length of max |r_i|; the sign and
// each bit plane are one 64-bit ballot.  Planes go to dst[0..w) (LDS).
template <int MAXW>
__device__ __forceinline__ int encode_block(int v, int lane, unsigned* dst,
                                            unsigned long long& sign, int& first, bool& over) {
  const int prev = dpp_from_prev(v, v);  // lane 0 sees itself: residual 0
  const long long r = (long long)v - (long long)prev;
  sign = __ballot(r < 0);
  const unsigned mag = (unsigned)(r < 0 ? -r : r);
  const unsigned mx = wave_max_u(mag);
  int w = mx ? 32 - __builtin_clz(mx) : 0;
  if (w > MAXW) {
    over = true;
    w = MAXW;
  }
  // plane j = ballot of bit j; its two halves go to lanes 2j, 2j+1
  unsigned mine = 0;
  for (int j = 0; j < w; ++j) {
    const unsigned long long pl = __ballot((mag >> j) & 1u);
    mine = write_lane(mine, (unsigned)pl, 2 * j);
    mine = write_lane(mine, (unsigned)(pl >> 32), 2 * j + 1);
  }
  if (lane < 2 * w) dst[lane] = mine;
  first = __builtin_amdgcn_readlane(v, 0);
  return w;
}

// Inverse: planes (uniform addresses) -> magnitudes -> signed residuals ->
// in-wave inclusive prefix sum.
__device__ __forceinline__ int decode_block(const uint8_t* planes, int w, int first,
                                            unsigned long long sign, int lane) {
  unsigned mag = 0;
  const unsigned sh = (unsigned)lane & 31u, hi = (unsigned)lane >> 5;
  for (int j = 0; j < w; ++j) {
    const unsigned long long pl = *(const unsigned long long*)(planes + 8 * (size_t)j);
    const unsigned half = hi ? (unsigned)(pl >> 32) : (unsigned)pl;
    mag |= ((half >> sh) & 1u) << j;
  }
  int r = ((sign >> lane) & 1ull) ? (int)(0u - mag) : (int)mag;
  if (lane == 0) r = first;
  return wave_incl_scan(r, lane);
}

// ---------------------------------------------------------------------------
// Kernel arguments.

struct Geom {
  int n, nx, ny, nz, ndim;
};

struct EncArgs {
  const float* f;
  uint8_t* out;
  uint8_t* ws;
  GeomD gd;
  int nb, nch, topo, eb_mode, nrange;
  double eb;
  float e_abs;
  uint64_t off[kNSeg], len[kNSeg];
};

struct ScanArgs {
  uint8_t* ws;
  int nch, eb_mode, nrange;
  double eb;
  float e_abs;
};

struct FinArgs {
  uint8_t* out;
  uint8_t* ws;
  uint64_t* out_size;
  int32_t* status;
  Geom g;
  uint64_t dims[3];
  int nb, nch, topo, eb_mode, rbf_policy, max_rounds;
  double eb;
  uint64_t off[kNSeg], len[kNSeg];
  float wtab[3][10];
};

struct DecArgs {
  const uint8_t* in;
  uint64_t in_size;
  float* out;
  uint64_t out_cap;
  uint8_t* ws;
  uint64_t ws_bytes;
};

struct RefArgs {
  const uint8_t* in;
  float* out;
  uint8_t* ws;
  int32_t* status;
};

__device__ __forceinline__ Ctrl* ctrl_of(uint8_t* ws) { return reinterpret_cast<Ctrl*>(ws); }
__device__ __forceinline__ Spread* spread_of(uint8_t* ws) {
  return reinterpret_cast<Spread*>(ws + kSpreadOff);
}

// Segment lengths and offsets: fixed-size parts first (offsets depend on the
// block count only), the two variable-size payloads last.
__host__ __device__ inline uint64_t seg_layout(uint64_t nb, int topo, uint64_t wdata,
                                               uint64_t wrank, uint64_t* off, uint64_t* len) {
  const uint64_t nch = (nb + kB - 1) / kB;
  const uint64_t t = topo ? 1 : 0;
  len[S1] = 8 * nch;
  len[S2] = nb;
  len[S3] = 8 * nb;
  len[S4] = 4 * nb;
  len[S6] = t * 16 * nb;
  len[R1] = t * 8 * nch;
  len[R2] = t * nb;
  len[R3] = t * 8 * nb;
  len[R4] = t * 4 * nb;
  len[X1] = 8 * nch;
  len[X2] = t * 8 * nch;
  len[S5] = 8 * wdata;
  len[R5] = t * 8 * wrank;
  off[0] = kHdr;
  for (int s = 1; s < kNSeg; ++s) off[s] = (off[s - 1] + len[s - 1] + 7) & ~uint64_t(7);
  return off[kNSeg - 1] + len[kNSeg - 1];
}

// ---------------------------------------------------------------------------
// Workspace initialisation.

__global__ void ws_init_kernel(uint8_t* ws, uint64_t nbytes) {
  const uint64_t n8 = nbytes / 8;
  unsigned long long* p = reinterpret_cast<unsigned long long*>(ws);
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n8;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// ---------------------------------------------------------------------------
// Relative-bound range pass: one partial (min key, max key, non-finite) per
// workgroup; consumers reduce the partials.

__global__ __launch_bounds__(256) void range_kernel(const float* __restrict__ f, int n, uint8_t* ws) {
  __shared__ unsigned s_lo[4], s_hi[4], s_bad[4];
  float lo = INFINITY, hi = -INFINITY;
  bool bad = false;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int stride = gridDim.x * blockDim.x;
  const int n4 = n / 4;
  const float4* f4 = reinterpret_cast<const float4*>(f);
  for (int i = blockIdx.x * blockDim.x + tid; i < n4; i += stride) {
    const float4 v = f4[i];
    bad |= !isfinite(v.x) || !isfinite(v.y) || !isfinite(v.z) || !isfinite(v.w);
    lo = fminf(lo, fminf(fminf(v.x, v.y), fminf(v.z, v.w)));
    hi = fmaxf(hi, fmaxf(fmaxf(v.x, v.y), fmaxf(v.z, v.w)));
  }
  for (int i = 4 * n4 + blockIdx.x * blockDim.x + tid; i < n; i += stride) {
    const float v = f[i];
    bad |= !isfinite(v);
    lo = fminf(lo, v);
    hi = fmaxf(hi, v);
  }
  unsigned ulo = ukey(lo), uhi = ukey(hi);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    ulo = min(ulo, (unsigned)__shfl_xor((int)ulo, o));
    uhi = max(uhi, (unsigned)__shfl_xor((int)uhi, o));
  }
  const bool anybad = __ballot(bad) != 0;
  if (lane == 0) {
    s_lo[wv] = ulo;
    s_hi[wv] = uhi;
    s_bad[wv] = anybad;
  }
  __syncthreads();
  if (tid == 0) {
    unsigned a = s_lo[0], b = s_hi[0], c = s_bad[0];
    for (int k = 1; k < (int)(blockDim.x / 64); ++k) {
      a = min(a, s_lo[k]);
      b = max(b, s_hi[k]);
      c |= s_bad[k];
    }
    unsigned* p = reinterpret_cast<unsigned*>(ws + kPartOff + 16 * (size_t)blockIdx.x);
    p[0] = a;
    p[1] = b;
    p[2] = c;
  }
}

// Bound of the call (one wave): relative mode reduces the range partials.
__device__ void call_bound(const uint8_t* ws, int eb_mode, double eb, float e_abs, int nrange,
                           int lane, float* e, float* vmin, float* vmax, double* eps, bool* bad) {
  unsigned lo = 0xFFFFFFFFu, hi = 0u, nf = 0u;
  if (eb_mode == TOPOSZP_EB_REL) {
    for (int k = lane; k < nrange; k += 64) {
      const unsigned* p = reinterpret_cast<const unsigned*>(ws + kPartOff + 16 * (size_t)k);
      lo = min(lo, p[0]);
      hi = max(hi, p[1]);
      nf |= p[2];
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      lo = min(lo, (unsigned)__shfl_xor((int)lo, o));
      hi = max(hi, (unsigned)__shfl_xor((int)hi, o));
      nf |= (unsigned)__shfl_xor((int)nf, o);
    }
  }
  if (eb_mode == TOPOSZP_EB_REL) {
    const float a = ukey2f(lo), b = ukey2f(hi);
    *vmin = a;
    *vmax = b;
    *eps = (b > a) ? eb * ((double)b - (double)a) : eb;
    *e = round_down_f(*eps);
  } else {
    *vmin = 0.0f;
    *vmax = 0.0f;
    *eps = eb;
    *e = e_abs;
  }
  *bad = nf != 0;
}

// ---------------------------------------------------------------------------
// Compression.

template <int WAVES>
__global__ __launch_bounds__(WAVES * 64) void encode_kernel(EncArgs a) {
  constexpr int BPW = kB / WAVES;  // blocks per wave
  __shared__ unsigned s_pd[kB][2 * kMaxWData];
  __shared__ unsigned s_pr[kB][2 * kMaxWRankBlk];
  __shared__ int s_wd[kB], s_wr[kB];
  __shared__ int s_pfd[kB + 1], s_pfr[kB + 1];
  __shared__ float s_e;
  __shared__ unsigned s_flags;

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int c = blockIdx.x;
  if (wv == 0) {
    float e, vmin, vmax;
    double eps;
    bool nf;
    call_bound(a.ws, a.eb_mode, a.eb, a.e_abs, a.nrange, lane, &e, &vmin, &vmax, &eps, &nf);
    if (lane == 0) {
      s_e = e;
      s_flags = (e >= 0x1p-100f && e <= 0x1p100f) ? 0u : 2u;
    }
  }
  __syncthreads();
  const float e = s_e;
  const double ed = (double)e;
  const float inv2e = 1.0f / (2.0f * e);
  const GeomD& g = a.gd;
  const int n = g.n;
  const bool deg[3] = {g.nx < 2, g.ny < 2, g.nz < 2};
  const float* __restrict__ f = a.f;
  bool nonfinite = false, qover = false, wover = false;

  for (int k = 0; k < BPW; ++k) {
    const int lb = wv * BPW + k;
    const int b = c * kB + lb;
    if (b >= a.nb) {
      if (lane == 0) {
        s_wd[lb] = 0;
        s_wr[lb] = 0;
      }
      continue;
    }
    const int b0 = b * kB;
    const int i = b0 + lane;
    const bool valid = i < n;
    const float av = valid ? f[i] : 0.0f;
    nonfinite |= valid && !isfinite(av);

    int lab = CLS_R, q = quantize(av, inv2e, ed);
    bool lost = false;
    if (a.topo) {
      // x neighbours come from the wave itself; the block's two outer
      // neighbours are broadcast loads
      const float el = b0 > 0 ? f[b0 - 1] : 0.0f;
      const float er = b0 + kB < n ? f[b0 + kB] : 0.0f;
      const float xl = __int_as_float(dpp_from_prev(__float_as_int(av), __float_as_int(el)));
      const float xr = __int_as_float(dpp_from_next(__float_as_int(av), __float_as_int(er)));
      if (valid) {
        const Pt pc = coords_of(i, g);
        float nb[6];
        bool avl[6];
        avl[0] = pc.x > 0;
        avl[1] = pc.x < g.nx - 1;
        avl[2] = pc.y > 0;
        avl[3] = pc.y < g.ny - 1;
        avl[4] = pc.z > 0;
        avl[5] = pc.z < g.nz - 1;
        nb[0] = xl;
        nb[1] = xr;
        nb[2] = avl[2] ? f[i - g.nx] : 0.0f;
        nb[3] = avl[3] ? f[i + g.nx] : 0.0f;
        nb[4] = avl[4] ? f[i - g.nxy] : 0.0f;
        nb[5] = avl[5] ? f[i + g.nxy] : 0.0f;
        lab = classify6(av, nb, avl, deg);
        if (lab != CLS_R) {
          // flattened by plain SZp iff some face neighbour shares the bin:
          // -e <= a_n - 2qe < e, exact in double (see quantize); a higher
          // neighbour can only share it from above, a lower one from below
          const double c2 = (double)q * (2.0 * ed);
#pragma unroll
          for (int j = 0; j < 6; ++j) {
            const double d = (double)nb[j] - c2;
            lost |= avl[j] && (nb[j] > av ? (d < ed) : (d >= -ed));
          }
        }
      }
    }
    qover |= valid && (q > kQMax || q < -kQMax);

    // ranks of flattened extrema among the flattened extrema of the same
    // class and bin in this block: 1 + number less extreme
    int delta = 0;
    if (a.topo) {
      const bool isext = lost && (lab == CLS_MIN || lab == CLS_MAX);
      unsigned long long m = __ballot(isext);
      const int ck = (q << 1) | (lab == CLS_MAX ? 1 : 0);
      const int ok = (lab == CLS_MAX) ? fkey(av) : -fkey(av);
      int cnt = 0;
      while (m) {
        const int j = __ffsll((long long)m) - 1;
        m &= m - 1;
        const int ckj = __builtin_amdgcn_readlane(ck, j);
        const int okj = __builtin_amdgcn_readlane(ok, j);
        cnt += (ck == ckj && okj < ok) ? 1 : 0;
      }
      delta = lost ? (lab == CLS_SAD ? 1 : 1 + cnt) : 0;
    }

    // the last block is padded with its last value (residual 0)
    if (b == a.nb - 1 && (n & (kB - 1))) {
      const int last = (n - 1) - b0;
      const int ql = __builtin_amdgcn_readlane(q, last);
      const int dl = __builtin_amdgcn_readlane(delta, last);
      if (!valid) {
        q = ql;
        delta = dl;
      }
    }

    unsigned long long sign;
    int first;
    const int w = encode_block<kMaxWData>(q, lane, s_pd[lb], sign, first, wover);
    uint8_t* out = a.out;
    if (lane == 0) {
      s_wd[lb] = w;
      out[a.off[S2] + b] = (uint8_t)w;
      *reinterpret_cast<unsigned long long*>(out + a.off[S3] + 8 * (size_t)b) = sign;
      *reinterpret_cast<int*>(out + a.off[S4] + 4 * (size_t)b) = first;
    }
    if (a.topo) {
      // 2-bit labels: point i at byte i/4, bits 2(i%4); 16 points per dword
      const unsigned lv = row_or_last((unsigned)lab << (2 * (lane & 15)));
      if ((lane & 15) == 15)
        *reinterpret_cast<unsigned*>(out + a.off[S6] + 16 * (size_t)b + 4 * (lane >> 4)) = lv;
      unsigned long long rsign;
      int rfirst;
      bool rover = false;
      const int wr = encode_block<kMaxWRankBlk>(delta, lane, s_pr[lb], rsign, rfirst, rover);
      if (lane == 0) {
        s_wr[lb] = wr;
        out[a.off[R2] + b] = (uint8_t)wr;
        *reinterpret_cast<unsigned long long*>(out + a.off[R3] + 8 * (size_t)b) = rsign;
        *reinterpret_cast<int*>(out + a.off[R4] + 4 * (size_t)b) = rfirst;
      }
    } else if (lane == 0) {
      s_wr[lb] = 0;
    }
  }
  {
    const bool nf = __ballot(nonfinite) != 0, qo = __ballot(qover || wover) != 0;
    if (lane == 0 && (nf || qo)) atomicOr(&s_flags, (nf ? 1u : 0u) | (qo ? 4u : 0u));
  }
  __syncthreads();

  // chunk: constant-block bitmaps, local prefix of widths, chunk totals
  const CompLayout L = comp_layout((uint64_t)a.nch);
  if (wv == 0) {
    const int b = c * kB + lane;
    const bool bv = b < a.nb;
    const int wd = s_wd[lane], wr = s_wr[lane];
    const unsigned long long cb = __ballot(bv && wd == 0), cr = __ballot(bv && wr == 0);
    const int sd = wave_incl_scan(wd, lane), sr = wave_incl_scan(wr, lane);
    s_pfd[lane + 1] = sd;
    s_pfr[lane + 1] = sr;
    if (lane == 0) {
      s_pfd[0] = 0;
      s_pfr[0] = 0;
      *reinterpret_cast<unsigned long long*>(a.out + a.off[S1] + 8 * (size_t)c) = cb;
      if (a.topo) *reinterpret_cast<unsigned long long*>(a.out + a.off[R1] + 8 * (size_t)c) = cr;
    }
    if (lane == 63) {
      reinterpret_cast<unsigned*>(a.ws + L.tot_d)[c] = (unsigned)sd;
      reinterpret_cast<unsigned*>(a.ws + L.tot_r)[c] = (unsigned)sr;
      reinterpret_cast<unsigned*>(a.ws + L.cflag)[c] = s_flags;
    }
  }
  __syncthreads();

  // this chunk's planes, compact, to its staging slot (coalesced from LDS)
  {
    const int totd = 2 * s_pfd[kB];
    unsigned* dst = reinterpret_cast<unsigned*>(a.ws + L.stage_d) + (size_t)c * kB * 2 * kMaxWData;
    for (int o = tid; o < totd; o += WAVES * 64) {
      int lo = 0, hi = kB;  // find lb with 2 s_pfd[lb] <= o < 2 s_pfd[lb+1]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (2 * s_pfd[mid] <= o) lo = mid; else hi = mid;
      }
      dst[o] = s_pd[lo][o - 2 * s_pfd[lo]];
    }
    if (a.topo) {
      const int totr = 2 * s_pfr[kB];
      unsigned* rdst = reinterpret_cast<unsigned*>(a.ws + L.stage_r) + (size_t)c * kB * 2 * kMaxWRankBlk;
      for (int o = tid; o < totr; o += WAVES * 64) {
        int lo = 0, hi = kB;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (2 * s_pfr[mid] <= o) lo = mid; else hi = mid;
        }
        rdst[o] = s_pr[lo][o - 2 * s_pfr[lo]];
      }
    }
  }
  // the last chunk zeroes the alignment gaps between the fixed-size parts
  if (c == a.nch - 1 && tid < 8 * (X2 + 1)) {
    const int s = tid >> 3, k = tid & 7;
    const uint64_t end = a.off[s] + a.len[s];
    if (end + k < a.off[s + 1]) a.out[end + k] = 0;
  }
}

// Exclusive scan of the chunk plane totals (in place), flags, and the bound.
__global__ __launch_bounds__(1024) void scan_kernel(ScanArgs a) {
  __shared__ unsigned long long s_w[2][16];
  __shared__ unsigned long long s_carry[2];
  __shared__ unsigned s_fl;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const CompLayout L = comp_layout((uint64_t)a.nch);
  unsigned* td = reinterpret_cast<unsigned*>(a.ws + L.tot_d);
  unsigned* tr = reinterpret_cast<unsigned*>(a.ws + L.tot_r);
  const unsigned* cf = reinterpret_cast<const unsigned*>(a.ws + L.cflag);
  Ctrl* ct = ctrl_of(a.ws);
  if (tid == 0) {
    s_carry[0] = 0;
    s_carry[1] = 0;
    s_fl = 0;
  }
  __syncthreads();
  unsigned fl = 0;
  for (int base = 0; base < a.nch; base += 1024) {
    const int c = base + tid;
    const bool v = c < a.nch;
    const unsigned long long xd = v ? td[c] : 0, xr = v ? tr[c] : 0;
    if (v) fl |= cf[c];
    unsigned long long sd = xd, sr = xr;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const unsigned long long t1 = __shfl_up(sd, o), t2 = __shfl_up(sr, o);
      if (lane >= o) {
        sd += t1;
        sr += t2;
      }
    }
    if (lane == 63) {
      s_w[0][wv] = sd;
      s_w[1][wv] = sr;
    }
    __syncthreads();
    unsigned long long od = s_carry[0], orr = s_carry[1];
    for (int k = 0; k < wv; ++k) {
      od += s_w[0][k];
      orr += s_w[1][k];
    }
    if (v) {
      td[c] = (unsigned)(od + sd - xd);
      tr[c] = (unsigned)(orr + sr - xr);
    }
    __syncthreads();
    if (tid == 1023) {
      s_carry[0] = od + sd;
      s_carry[1] = orr + sr;
    }
    __syncthreads();
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) fl |= (unsigned)__shfl_xor((int)fl, o);
  if (lane == 0 && fl) atomicOr(&s_fl, fl);
  __syncthreads();
  if (wv == 0) {
    float e, vmin, vmax;
    double eps;
    bool nf;
    call_bound(a.ws, a.eb_mode, a.eb, a.e_abs, a.nrange, lane, &e, &vmin, &vmax, &eps, &nf);
    if (lane == 0) {
      unsigned flags = s_fl | (nf ? 1u : 0u);
      if (!(e >= 0x1p-100f && e <= 0x1p100f)) flags |= 2u;
      ct->tot_data = s_carry[0];
      ct->tot_rank = s_carry[1];
      ct->cflags = flags;
      ct->e = e;
      ct->vmin = vmin;
      ct->vmax = vmax;
      ct->eps = eps;
    }
  }
}

// ---------------------------------------------------------------------------
// Finalize: payload placement, chunk index, header, status.

__device__ void put8(uint8_t* h, int off, uint64_t v) { memcpy(h + off, &v, 8); }
__device__ void put4(uint8_t* h, int off, uint32_t v) { memcpy(h + off, &v, 4); }
__device__ void put2(uint8_t* h, int off, uint16_t v) { memcpy(h + off, &v, 2); }

__global__ __launch_bounds__(256) void finalize_kernel(FinArgs a) {
  __shared__ uint8_t hdr[kHdr];
  __shared__ unsigned s_sa[4], s_sb[4];
  const Ctrl* ct = ctrl_of(a.ws);
  const int tid = threadIdx.x;
  const int c = blockIdx.x;
  const CompLayout L = comp_layout((uint64_t)a.nch);
  const uint64_t totd = ct->tot_data, totr = a.topo ? ct->tot_rank : 0;
  const unsigned* pd = reinterpret_cast<const unsigned*>(a.ws + L.tot_d);
  const unsigned* pr = reinterpret_cast<const unsigned*>(a.ws + L.tot_r);
  {
    const uint64_t b0 = pd[c], b1 = c + 1 < a.nch ? pd[c + 1] : totd;
    const uint64_t* src = reinterpret_cast<const uint64_t*>(a.ws + L.stage_d) + (size_t)c * kB * kMaxWData;
    uint64_t* dst = reinterpret_cast<uint64_t*>(a.out + a.off[S5]) + b0;
    for (uint64_t o = tid; o < b1 - b0; o += blockDim.x) dst[o] = src[o];
    if (tid == 0) *reinterpret_cast<uint64_t*>(a.out + a.off[X1] + 8 * (size_t)c) = 8 * b0;
    if (a.topo) {
      const uint64_t r0 = pr[c], r1 = c + 1 < a.nch ? pr[c + 1] : totr;
      const uint64_t* rsrc =
          reinterpret_cast<const uint64_t*>(a.ws + L.stage_r) + (size_t)c * kB * kMaxWRankBlk;
      uint64_t* rdst = reinterpret_cast<uint64_t*>(a.out + a.off[S5] + 8 * totd) + r0;
      for (uint64_t o = tid; o < r1 - r0; o += blockDim.x) rdst[o] = rsrc[o];
      if (tid == 0) *reinterpret_cast<uint64_t*>(a.out + a.off[X2] + 8 * (size_t)c) = 8 * r0;
    }
  }
  if (c != 0) return;

  const unsigned flags = ct->cflags;
  int status = TOPOSZP_OK;
  if (flags & 1u) status = TOPOSZP_E_NONFINITE;
  else if (flags & 6u) status = TOPOSZP_E_RANGE;
  for (int k = tid; k < kHdr; k += blockDim.x) hdr[k] = 0;
  __syncthreads();
  if (tid == 0) {
    int k = 3;
    float sigma = 0.5f;
    int si = 0;
    if (a.rbf_policy == 0 && totd <= (uint64_t)a.nb) { k = 7; sigma = 1.0f; si = 2; }
    else if (a.rbf_policy == 0 && totd <= 3 * (uint64_t)a.nb) { k = 5; sigma = 0.75f; si = 1; }
    uint64_t off[kNSeg], len[kNSeg];
    const uint64_t total = seg_layout((uint64_t)a.nb, a.topo, totd, totr, off, len);
    hdr[0] = 'T'; hdr[1] = 'S'; hdr[2] = 'Z'; hdr[3] = '1';
    put2(hdr, 4, 1);
    hdr[6] = (uint8_t)a.g.ndim;
    hdr[7] = (uint8_t)(a.topo ? 1 : 0);
    for (int d = 0; d < 3; ++d) put8(hdr, 8 + 8 * d, a.dims[d]);
    put8(hdr, 32, (uint64_t)a.g.n);
    put8(hdr, 40, (uint64_t)a.nb);
    put4(hdr, 48, kB);
    hdr[52] = (uint8_t)a.eb_mode;
    hdr[53] = (uint8_t)k;
    put2(hdr, 54, (uint16_t)a.max_rounds);
    uint64_t u;
    memcpy(&u, &a.eb, 8); put8(hdr, 56, u);
    memcpy(&u, &ct->eps, 8); put8(hdr, 64, u);
    uint32_t v;
    memcpy(&v, &ct->e, 4); put4(hdr, 72, v);
    memcpy(&v, &ct->vmin, 4); put4(hdr, 76, v);
    memcpy(&v, &ct->vmax, 4); put4(hdr, 80, v);
    memcpy(&v, &sigma, 4); put4(hdr, 84, v);
    for (int d2 = 0; d2 < 10; ++d2) { memcpy(&v, &a.wtab[si][d2], 4); put4(hdr, 88 + 4 * d2, v); }
    put8(hdr, 128, total);
    put8(hdr, 136, totd);
    put8(hdr, 144, totr);
    put8(hdr, 152, (uint64_t)a.nch);
    for (int s = 0; s < kNSeg; ++s) {
      put8(hdr, 160 + 8 * s, off[s]);
      put8(hdr, 264 + 8 * s, len[s]);
    }
    *a.status = status;
    *a.out_size = status == TOPOSZP_OK ? total : 0;
  }
  __syncthreads();
  // Adler-32 of bytes [0, 376): A = 1 + sum b_i, B = n + sum (n - i) b_i (mod 65521)
  unsigned sa = 0, sb = 0;
  for (int i = tid; i < kSummed; i += blockDim.x) {
    sa += hdr[i];
    sb += (unsigned)(kSummed - i) * hdr[i];
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    sa += (unsigned)__shfl_xor((int)sa, o);
    sb += (unsigned)__shfl_xor((int)sb, o);
  }
  if ((tid & 63) == 0) {
    s_sa[tid >> 6] = sa;
    s_sb[tid >> 6] = sb;
  }
  __syncthreads();
  if (tid == 0) {
    uint64_t A = 1, B = kSummed;
    for (int k = 0; k < (int)(blockDim.x / 64); ++k) {
      A += s_sa[k];
      B += s_sb[k];
    }
    A %= 65521u;
    B %= 65521u;
    put4(hdr, kSummed, (uint32_t)((B << 16) | A));
  }
  __syncthreads();
  for (int k = tid; k < kHdr; k += blockDim.x) a.out[k] = hdr[k];
}

// ---------------------------------------------------------------------------
// Decompression.

struct Hdr {
  int ok, ndim, topo, scope, k, max_rounds;
  uint64_t dims[3], n, nb, nch, total, wdata, wrank;
  float e, w[10];
  uint64_t off[kNSeg], len[kNSeg];
};

template <typename T>
__device__ __forceinline__ T rd(const uint8_t* p, int off) {
  T v;
  memcpy(&v, p + off, sizeof(T));
  return v;
}

// Header checks (one wave): the header is copied to LDS in parallel, then
// lane 0 checks the checksum, field ranges and the segment table against the
// layout rule.  Result in *h: ok = 0 corrupt, -1 capacity, 1 good.
__device__ void parse_header(const uint8_t* in, uint64_t in_size, uint64_t out_cap, Hdr* h,
                             uint8_t* hb, int lane) {
  const bool good = in_size >= (uint64_t)kHdr;
  unsigned sa = 0, sb = 0;
  if (good) {
    // 512 header bytes: 8 per lane
    const uint64_t w = *reinterpret_cast<const uint64_t*>(in + 8 * lane);
    *reinterpret_cast<uint64_t*>(hb + 8 * lane) = w;
    for (int j = 0; j < 8; ++j) {
      const int i = 8 * lane + j;
      const unsigned b = (unsigned)((w >> (8 * j)) & 0xFFu);
      if (i < kSummed) {
        sa += b;
        sb += (unsigned)(kSummed - i) * b;
      }
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    sa += (unsigned)__shfl_xor((int)sa, o);
    sb += (unsigned)__shfl_xor((int)sb, o);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (lane != 0) return;
  h->ok = 0;
  if (!good) return;
  const uint32_t adler = (uint32_t)((((uint64_t)kSummed + sb) % 65521u) << 16 | ((1ull + sa) % 65521u));
  if (hb[0] != 'T' || hb[1] != 'S' || hb[2] != 'Z' || hb[3] != '1') return;
  if (rd<uint16_t>(hb, 4) != 1) return;
  if (rd<uint32_t>(hb, kSummed) != adler || rd<uint32_t>(hb, kSummed + 4) != 0) return;
  h->ndim = hb[6];
  if (h->ndim != 2 && h->ndim != 3) return;
  if (hb[7] & ~3u) return;
  h->topo = hb[7] & 1;
  h->scope = (hb[7] >> 1) & 1;
  uint64_t prod = 1;
  for (int d = 0; d < 3; ++d) {
    h->dims[d] = rd<uint64_t>(hb, 8 + 8 * d);
    if (h->dims[d] < 1 || h->dims[d] > (1ull << 31)) return;
    if (d >= h->ndim && h->dims[d] != 1) return;
    prod *= h->dims[d];
    if (prod >= (1ull << 31)) return;
  }
  h->n = rd<uint64_t>(hb, 32);
  h->nb = rd<uint64_t>(hb, 40);
  h->nch = rd<uint64_t>(hb, 152);
  if (h->n != prod || h->nb != (h->n + kB - 1) / kB || h->nch != (h->nb + kB - 1) / kB) return;
  if (rd<uint32_t>(hb, 48) != (uint32_t)kB) return;
  h->k = hb[53];
  h->max_rounds = rd<uint16_t>(hb, 54);
  if (hb[52] > 1 || (h->k != 3 && h->k != 5 && h->k != 7) || h->max_rounds < 1) return;
  h->e = rd<float>(hb, 72);
  if (!(h->e >= 0x1p-100f) || !(h->e <= 0x1p100f)) return;
  for (int d2 = 0; d2 < 10; ++d2) {
    h->w[d2] = rd<float>(hb, 88 + 4 * d2);
    if (!(h->w[d2] > 0.0f) || !(h->w[d2] <= 1.0f)) return;
  }
  h->total = rd<uint64_t>(hb, 128);
  h->wdata = rd<uint64_t>(hb, 136);
  h->wrank = rd<uint64_t>(hb, 144);
  if (h->wdata > h->nb * kMaxWData || h->wrank > h->nb * kMaxWRankAny) return;
  uint64_t off[kNSeg], len[kNSeg];
  const uint64_t total = seg_layout(h->nb, h->topo, h->wdata, h->wrank, off, len);
  if (total != h->total || total > in_size) return;
  for (int s = 0; s < kNSeg; ++s) {
    h->off[s] = rd<uint64_t>(hb, 160 + 8 * s);
    h->len[s] = rd<uint64_t>(hb, 264 + 8 * s);
    if (h->off[s] != off[s] || h->len[s] != len[s]) return;
  }
  h->ok = (h->n <= out_cap) ? 1 : -1;
}

template <int WAVES>
__global__ __launch_bounds__(WAVES * 64) void decode_kernel(DecArgs a) {
  constexpr int BPW = kB / WAVES;
  __shared__ Hdr s_h;
  __shared__ uint64_t s_hb[kHdr / 8];
  __shared__ int s_pfd[kB + 1], s_pfr[kB + 1], s_wd[kB], s_wr[kB];
  __shared__ unsigned long long s_xd, s_xr;
  __shared__ int s_bad;
  __shared__ unsigned s_qn, s_moves, s_skips, s_corrupt;
  __shared__ unsigned s_qi[kChunk];
  __shared__ uint8_t s_qc[kChunk];
  Ctrl* ct = ctrl_of(a.ws);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int c = blockIdx.x;
  if (wv == 0) parse_header(a.in, a.in_size, a.out_cap, &s_h, reinterpret_cast<uint8_t*>(s_hb), lane);
  if (tid == 0) {
    s_bad = 0;
    s_qn = 0;
    s_moves = 0;
    s_skips = 0;
    s_corrupt = 0;
  }
  __syncthreads();
  const Hdr& h = s_h;
  const uint64_t nb = h.ok == 1 ? h.nb : 0, nch = h.ok == 1 ? h.nch : 0;
  const DecLayout L = dec_layout(nb, nch);
  const bool room = h.ok == 1 && L.end <= a.ws_bytes;
  if (c == 0 && tid == 0) {
    // this call's header verdict and counters for refine/tail
    ct->hflags = h.ok == 1 ? (room ? 0u : 2u) : (h.ok == -1 ? 2u : 1u);
    ct->big_count = 0;
    Plan& p = ct->plan;
    p.valid = room ? 1 : 0;
    if (room) {
      p.topo = h.topo;
      p.ndim = h.ndim;
      p.k = h.k;
      p.ncol = h.ndim == 3 ? 7 : 5;
      p.max_rounds = h.max_rounds;
      p.nch = (int)h.nch;
      p.g.n = (int)h.n;
      p.g.nx = h.ndim == 3 ? (int)h.dims[2] : (int)h.dims[1];
      p.g.ny = h.ndim == 3 ? (int)h.dims[1] : (int)h.dims[0];
      p.g.nz = h.ndim == 3 ? (int)h.dims[0] : 1;
      p.g.nxy = p.g.nx * p.g.ny;
      p.g.dx = make_div((unsigned)p.g.nx);
      p.g.dy = make_div((unsigned)p.g.ny);
      p.e = h.e;
      for (int d2 = 0; d2 < 10; ++d2) p.w[d2] = h.w[d2];
      p.s6_off = h.off[S6];
    }
  }
  if (c == 0 && tid < kSpreadLines) {
    Spread* sp = spread_of(a.ws);
    sp[tid].commits = 0;
    sp[tid].rounds = 0;
    sp[tid].queued = 0;
  }
  if (!room || (uint64_t)c >= h.nch) return;
  const int n = (int)h.n;
  const int nx = h.ndim == 3 ? (int)h.dims[2] : (int)h.dims[1];
  const int ny = h.ndim == 3 ? (int)h.dims[1] : (int)h.dims[0];

  // this chunk's widths, constant flags and payload offsets
  if (wv == 0) {
    const uint64_t b = (uint64_t)c * kB + lane;
    const bool bv = b < h.nb;
    const int wd = bv ? a.in[h.off[S2] + b] : 0;
    const int wr = (bv && h.topo) ? a.in[h.off[R2] + b] : 0;
    const unsigned long long cb = *reinterpret_cast<const unsigned long long*>(a.in + h.off[S1] + 8 * (uint64_t)c);
    bool bad = bv && (wd > kMaxWData || (int)((cb >> lane) & 1) != (wd == 0));
    if (h.topo) {
      const unsigned long long cr = *reinterpret_cast<const unsigned long long*>(a.in + h.off[R1] + 8 * (uint64_t)c);
      bad |= bv && (wr > kMaxWRankAny || (int)((cr >> lane) & 1) != (wr == 0));
      bad |= !bv && (((cr >> lane) & 1) != 0);
    }
    bad |= !bv && (((cb >> lane) & 1) != 0);
    const int sd = wave_incl_scan(wd, lane), sr = wave_incl_scan(wr, lane);
    s_pfd[lane + 1] = sd;
    s_pfr[lane + 1] = sr;
    s_wd[lane] = wd;
    s_wr[lane] = wr;
    const bool anybad = __ballot(bad) != 0;
    if (lane == 0) {
      s_pfd[0] = 0;
      s_pfr[0] = 0;
      const uint64_t totd = 8ull * (unsigned)__builtin_amdgcn_readlane(sd, 63);
      const uint64_t totr = 8ull * (unsigned)__builtin_amdgcn_readlane(sr, 63);
      const uint64_t xd = *reinterpret_cast<const uint64_t*>(a.in + h.off[X1] + 8 * (uint64_t)c);
      const uint64_t nxd = (uint64_t)c + 1 < h.nch
                               ? *reinterpret_cast<const uint64_t*>(a.in + h.off[X1] + 8 * ((uint64_t)c + 1))
                               : h.len[S5];
      bool b2 = anybad || (c == 0 && xd != 0) || xd > h.len[S5] || totd > h.len[S5] - xd || xd + totd != nxd;
      uint64_t xr = 0;
      if (h.topo) {
        xr = *reinterpret_cast<const uint64_t*>(a.in + h.off[X2] + 8 * (uint64_t)c);
        const uint64_t nxr = (uint64_t)c + 1 < h.nch
                                 ? *reinterpret_cast<const uint64_t*>(a.in + h.off[X2] + 8 * ((uint64_t)c + 1))
                                 : h.len[R5];
        b2 = b2 || (c == 0 && xr != 0) || xr > h.len[R5] || totr > h.len[R5] - xr || xr + totr != nxr;
      }
      s_xd = xd;
      s_xr = xr;
      s_bad = b2 ? 1 : 0;
    }
  }
  __syncthreads();
  unsigned* dflag = reinterpret_cast<unsigned*>(a.ws + L.dflag);
  unsigned long long* bitmap = reinterpret_cast<unsigned long long*>(a.ws + L.bitmap);
  if (s_bad) {
    if (tid == 0) {
      dflag[c] = 1;
      reinterpret_cast<unsigned*>(a.ws + L.cnt)[c] = 0;
      reinterpret_cast<unsigned*>(a.ws + L.moves)[c] = 0;
      reinterpret_cast<unsigned*>(a.ws + L.skips)[c] = 0;
    }
    if (tid < kB && (uint64_t)c * kB + tid < h.nb) bitmap[(uint64_t)c * kB + tid] = 0;
    return;
  }
  const double ed = (double)h.e;
  const float two_e = 2.0f * h.e;
  const int dmax = h.scope ? n : kB;
  bool corrupt = false;
  unsigned moves = 0, skips = 0;
  for (int k = 0; k < BPW; ++k) {
    const int lb = wv * BPW + k;
    const uint64_t b = (uint64_t)c * kB + lb;
    if (b >= h.nb) continue;
    const int i = (int)(b * kB) + lane;
    const bool valid = i < n;
    const int first = *reinterpret_cast<const int*>(a.in + h.off[S4] + 4 * b);
    const unsigned long long sign = *reinterpret_cast<const unsigned long long*>(a.in + h.off[S3] + 8 * b);
    const int q = decode_block(a.in + h.off[S5] + s_xd + 8ull * s_pfd[lb], s_wd[lb], first, sign, lane);
    corrupt |= valid && (q > kQMax || q < -kQMax);
    const float rq = (float)q * two_e;  // float(2q) * e: the same exact product
    float v = rq;
    bool queue = false;
    if (h.topo) {
      const int rfirst = *reinterpret_cast<const int*>(a.in + h.off[R4] + 4 * b);
      const unsigned long long rsign = *reinterpret_cast<const unsigned long long*>(a.in + h.off[R3] + 8 * b);
      const int dl = decode_block(a.in + h.off[R5] + s_xr + 8ull * s_pfr[lb], s_wr[lb], rfirst, rsign, lane);
      corrupt |= valid && (dl < 0 || dl > dmax);
      const unsigned lw = valid ? *reinterpret_cast<const unsigned*>(a.in + h.off[S6] + 16 * b + 4 * (lane >> 4)) : 0u;
      const int lab = (int)((lw >> (2 * (lane & 15))) & 3u);
      if (valid && dl > 0 && (lab == CLS_MIN || lab == CLS_MAX)) {
        // flattened extremum: its neighbour maximum (minimum) is its own bin
        // centre, so the stencil value is delta float steps beyond it
        const long long kk = (long long)fkey(rq) + (lab == CLS_MAX ? (long long)dl : -(long long)dl);
        const float cand = key2f(kk);
        if (fabs((double)cand - (double)rq) <= ed) {
          v = cand;
          ++moves;
        } else {
          ++skips;
        }
      }
      queue = valid && dl > 0 && lab == CLS_SAD;
    }
    if (valid) a.out[i] = v;
    if (h.topo) {
      const unsigned long long qm = __ballot(queue);
      if (lane == 0) bitmap[b] = qm;
      if (qm) {
        unsigned base = 0;
        if (lane == 0) base = atomicAdd(&s_qn, (unsigned)__popcll(qm));
        base = (unsigned)__builtin_amdgcn_readlane((int)base, 0);
        if (queue) {
          const unsigned pos = base + mbcnt(qm);
          const long long x = i % nx, t = i / nx, y = t % ny, z = t / ny;
          s_qi[pos] = (unsigned)i;
          s_qc[pos] = (uint8_t)(h.ndim == 3 ? (x + 2 * y + 3 * z) % 7 : (x + 2 * y) % 5);
        }
      }
    }
  }
  const bool cb = __ballot(corrupt) != 0;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    moves += (unsigned)__shfl_xor((int)moves, o);
    skips += (unsigned)__shfl_xor((int)skips, o);
  }
  if (lane == 0) {
    if (moves) atomicAdd(&s_moves, moves);
    if (skips) atomicAdd(&s_skips, skips);
    if (cb) atomicOr(&s_corrupt, 1u);
  }
  __syncthreads();
  // the chunk's queue to its slot range, and its counters
  const unsigned qn = s_qn;
  unsigned* qi = reinterpret_cast<unsigned*>(a.ws + L.idx) + (size_t)c * kChunk;
  uint8_t* qc = a.ws + L.col + (size_t)c * kChunk;
  for (unsigned t = tid; t < qn; t += WAVES * 64) {
    qi[t] = s_qi[t];
    qc[t] = s_qc[t];
  }
  if (tid == 0) {
    reinterpret_cast<unsigned*>(a.ws + L.cnt)[c] = qn;
    reinterpret_cast<unsigned*>(a.ws + L.moves)[c] = s_moves;
    reinterpret_cast<unsigned*>(a.ws + L.skips)[c] = s_skips;
    dflag[c] = s_corrupt;
  }
}

// ---------------------------------------------------------------------------
// Saddle refinement (specialised on the dimension and kernel size, so the
// neighbourhoods below are compile-time).

template <int ND>
__device__ __forceinline__ int classify_at(const float* fld, int i, Pt c, int pi, float pv, const GeomD& g) {
  float nb[6];
  bool av[6];
  av[0] = c.x > 0;
  av[1] = c.x < g.nx - 1;
  av[2] = c.y > 0;
  av[3] = c.y < g.ny - 1;
  av[4] = ND == 3 && c.z > 0;
  av[5] = ND == 3 && c.z < g.nz - 1;
  const int nbi[6] = {i - 1, i + 1, i - g.nx, i + g.nx, i - g.nxy, i + g.nxy};
#pragma unroll
  for (int j = 0; j < 6; ++j) nb[j] = av[j] ? (nbi[j] == pi ? pv : fld[nbi[j]]) : 0.0f;
  const bool deg[3] = {g.nx < 2, g.ny < 2, ND != 3 || g.nz < 2};
  const float a = (i == pi) ? pv : fld[i];
  return classify6(a, nb, av, deg);
}

// Candidate for a flattened saddle p and the acceptance tests:
// 0 reject, 1 already a saddle, 2 accept (value in *vout).
template <int ND, int K>
__device__ int evaluate(const float* fld, const uint8_t* labels, int p, const Plan& pl, float* vout) {
  const GeomD& g = pl.g;
  const Pt c = coords_of(p, g);
  if (classify_at<ND>(fld, p, c, -1, 0.0f, g) == CLS_SAD) return 1;
  constexpr int r = K / 2, rz = ND == 3 ? r : 0;
  double num = 0.0, den = 0.0;
#pragma unroll
  for (int dz = -rz; dz <= rz; ++dz)
#pragma unroll
    for (int dy = -r; dy <= r; ++dy)
#pragma unroll
      for (int dx = -r; dx <= r; ++dx) {
        const int d2 = dz * dz + dy * dy + dx * dx;
        if (d2 == 0 || d2 > r * r) continue;
        const int zz = c.z + dz, yy = c.y + dy, xx = c.x + dx;
        if (zz < 0 || zz >= g.nz || yy < 0 || yy >= g.ny || xx < 0 || xx >= g.nx) continue;
        const double wt = (double)pl.w[d2];
        num = num + wt * (double)fld[p + dz * g.nxy + dy * g.nx + dx];
        den = den + wt;
      }
  if (den == 0.0) return 0;
  const float v = (float)(num / den);
  if (!(fabs((double)v - (double)fld[p]) <= (double)pl.e)) return 0;
  if (classify_at<ND>(fld, p, c, p, v, g) != CLS_SAD) return 0;
  const int nbi[6] = {p - 1, p + 1, p - g.nx, p + g.nx, p - g.nxy, p + g.nxy};
  const Pt nbc[6] = {{c.x - 1, c.y, c.z}, {c.x + 1, c.y, c.z}, {c.x, c.y - 1, c.z},
                     {c.x, c.y + 1, c.z}, {c.x, c.y, c.z - 1}, {c.x, c.y, c.z + 1}};
  const bool av[6] = {c.x > 0, c.x < g.nx - 1, c.y > 0, c.y < g.ny - 1,
                      ND == 3 && c.z > 0, ND == 3 && c.z < g.nz - 1};
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    if (!av[j]) continue;
    const int q = nbi[j];
    const int before = classify_at<ND>(fld, q, nbc[j], -1, 0.0f, g);
    const int after = classify_at<ND>(fld, q, nbc[j], p, v, g);
    const int lab = (labels[q >> 2] >> (2 * (q & 3))) & 3;
    if (after != before && !(before == CLS_R && after == lab)) return 0;
  }
  *vout = v;
  return 2;
}

__device__ __forceinline__ int colour_of(int i, const GeomD& g, int ndim) {
  const Pt c = coords_of(i, g);
  return ndim == 3 ? (int)(((unsigned)c.x + 2u * (unsigned)c.y + 3u * (unsigned)c.z) % 7u)
                   : (int)(((unsigned)c.x + 2u * (unsigned)c.y) % 5u);
}

// Offsets through which two queued saddles can influence each other's
// evaluation: the candidate window (Euclidean radius floor(k/2)) and the
// cells the acceptance tests classify (L1 distance <= 2).
__host__ __device__ constexpr bool in_reach(int dx, int dy, int dz, int r) {
  return (dx * dx + dy * dy + dz * dz) > 0 &&
         ((dx * dx + dy * dy + dz * dz) <= r * r ||
          (dx < 0 ? -dx : dx) + (dy < 0 ? -dy : dy) + (dz < 0 ? -dz : dz) <= 2);
}

// Queued saddles within reach of cur, appended to mem[m..] if new; returns
// false when the list would exceed kClusterMax.
template <int ND, int K>
__device__ __forceinline__ bool gather(const unsigned long long* bm, int cur, const GeomD& g, unsigned* mem,
                                       int& m) {
  constexpr int r = K / 2, R = r > 2 ? r : 2, RZ = ND == 3 ? R : 0;
  const Pt c = coords_of(cur, g);
#pragma unroll
  for (int dz = -RZ; dz <= RZ; ++dz)
#pragma unroll
    for (int dy = -R; dy <= R; ++dy)
#pragma unroll
      for (int dx = -R; dx <= R; ++dx) {
        if (!in_reach(dx, dy, dz, r)) continue;
        const int xx = c.x + dx, yy = c.y + dy, zz = c.z + dz;
        const bool in = xx >= 0 && xx < g.nx && yy >= 0 && yy < g.ny && zz >= 0 && zz < g.nz;
        const int q = cur + dz * g.nxy + dy * g.nx + dx;
        const unsigned long long word = in ? bm[q >> 6] : 0ull;
        if (!((word >> (q & 63)) & 1ull)) continue;
        bool seen = false;
        for (int j = 0; j < m; ++j) seen |= mem[j] == (unsigned)q;
        if (seen) continue;
        if (m == kClusterMax) return false;
        mem[m++] = (unsigned)q;
      }
  return true;
}

template <int ND, int K>
__device__ void refine_chunk(const RefArgs& a, const Plan& pl, unsigned* mem, float* val, uint8_t* st,
                             unsigned& my_commits, unsigned& my_rounds) {
  const int c = blockIdx.x;
  const int tid = threadIdx.x;
  const uint64_t nb = ((uint64_t)pl.g.n + kB - 1) / kB;
  const DecLayout L = dec_layout(nb, (uint64_t)pl.nch);
  const unsigned cnt0 = reinterpret_cast<const unsigned*>(a.ws + L.cnt)[c];
  const unsigned cnt = cnt0 < (unsigned)kChunk ? cnt0 : (unsigned)kChunk;
  const unsigned* idx = reinterpret_cast<const unsigned*>(a.ws + L.idx);
  const unsigned long long* bm = reinterpret_cast<const unsigned long long*>(a.ws + L.bitmap);
  unsigned* big = reinterpret_cast<unsigned*>(a.ws + L.big);
  const uint8_t* labels = a.in + pl.s6_off;
  for (unsigned t = tid; t < cnt; t += kRefineThreads) {
    const unsigned slot = (unsigned)c * kChunk + t;
    const int p = (int)idx[slot];
    // the connected set of queued saddles around p (bounded)
    mem[0] = (unsigned)p;
    int m = 1, head = 0;
    bool fits = true;
    while (head < m && fits) fits = gather<ND, K>(bm, (int)mem[head++], pl.g, mem, m);
    if (!fits) {
      // left to the tail kernel (every member's search overflows the same way)
      const unsigned pos = atomicAdd(&ctrl_of(a.ws)->big_count, 1u);
      if (pos < (unsigned)pl.nch * kChunk) big[pos] = slot;
      continue;
    }
    unsigned owner = mem[0];
    for (int j = 1; j < m; ++j) owner = min(owner, mem[j]);
    if (owner != (unsigned)p) continue;  // another thread replays this cluster
    // replay the colour-phased rounds on the cluster (Jacobi within a phase)
    for (int j = 0; j < m; ++j) st[j] = (uint8_t)(colour_of((int)mem[j], pl.g, ND) << 2);
    int round = 1;
    for (; round <= pl.max_rounds; ++round) {
      unsigned commits = 0;
      for (int cc = 0; cc < pl.ncol; ++cc) {
        bool any = false;
        for (int j = 0; j < m; ++j) {
          if ((st[j] & 3) == 1 || (st[j] >> 2) != cc) continue;
          float v;
          const int res = evaluate<ND, K>(a.out, labels, (int)mem[j], pl, &v);
          if (res == 1) {
            st[j] = (uint8_t)((st[j] & ~3) | 1);
          } else if (res == 2) {
            st[j] = (uint8_t)((st[j] & ~3) | 2);
            val[j] = v;
            any = true;
          }
        }
        if (!any) continue;
        for (int j = 0; j < m; ++j)
          if ((st[j] & 3) == 2) {
            a.out[mem[j]] = val[j];
            st[j] = (uint8_t)((st[j] & ~3) | 1);
            ++commits;
          }
      }
      my_commits += commits;
      if (commits == 0) break;
    }
    my_rounds = max(my_rounds, (unsigned)(round <= pl.max_rounds ? round : pl.max_rounds));
  }
}

__global__ __launch_bounds__(kRefineThreads) void refine_kernel(RefArgs a) {
  __shared__ Plan s_p;
  __shared__ unsigned s_mem[kRefineThreads][kClusterMax];
  __shared__ float s_val[kRefineThreads][kClusterMax];
  __shared__ uint8_t s_st[kRefineThreads][kClusterMax];
  __shared__ unsigned s_commits, s_rounds, s_ok;
  Ctrl* ct = ctrl_of(a.ws);
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_p = ct->plan;
    s_ok = ct->hflags == 0 && s_p.valid && s_p.topo;
    s_commits = 0;
    s_rounds = 0;
  }
  __syncthreads();
  const Plan& pl = s_p;
  const int c = blockIdx.x;
  if (!s_ok || c >= pl.nch) return;
  unsigned my_commits = 0, my_rounds = 0;
  unsigned* mem = s_mem[tid];
  float* val = s_val[tid];
  uint8_t* st = s_st[tid];
  switch (pl.ndim * 8 + pl.k) {
    case 2 * 8 + 3: refine_chunk<2, 3>(a, pl, mem, val, st, my_commits, my_rounds); break;
    case 2 * 8 + 5: refine_chunk<2, 5>(a, pl, mem, val, st, my_commits, my_rounds); break;
    case 2 * 8 + 7: refine_chunk<2, 7>(a, pl, mem, val, st, my_commits, my_rounds); break;
    case 3 * 8 + 3: refine_chunk<3, 3>(a, pl, mem, val, st, my_commits, my_rounds); break;
    case 3 * 8 + 5: refine_chunk<3, 5>(a, pl, mem, val, st, my_commits, my_rounds); break;
    default: refine_chunk<3, 7>(a, pl, mem, val, st, my_commits, my_rounds); break;
  }
  if (my_commits) atomicAdd(&s_commits, my_commits);
  if (my_rounds) atomicMax(&s_rounds, my_rounds);
  __syncthreads();
  if (tid == 0 && (s_commits || s_rounds)) {
    Spread* sp = spread_of(a.ws) + (c % kSpreadLines);
    if (s_commits) atomicAdd(&sp->commits, s_commits);
    atomicMax(&sp->rounds, s_rounds);
  }
}

// Clusters too large for one thread: the colour-phased rounds by one
// workgroup with workgroup barriers (rare).  Then status and counters.
template <int ND, int K>
__device__ unsigned tail_rounds(const RefArgs& a, const Plan& pl, const DecLayout& L, unsigned nbig) {
  __shared__ unsigned s_commits;
  const unsigned* bigl = reinterpret_cast<const unsigned*>(a.ws + L.big);
  const unsigned* idx = reinterpret_cast<const unsigned*>(a.ws + L.idx);
  const uint8_t* col = a.ws + L.col;
  uint8_t* state = a.ws + L.state;
  float* pend = reinterpret_cast<float*>(a.ws + L.pend);
  const uint8_t* labels = a.in + pl.s6_off;
  const unsigned tid = threadIdx.x, nthr = blockDim.x;
  for (unsigned t = tid; t < nbig; t += nthr) state[bigl[t]] = 0;
  __syncthreads();
  int round = 1;
  unsigned total = 0;
  for (; round <= pl.max_rounds; ++round) {
    if (tid == 0) s_commits = 0;
    __syncthreads();
    for (int cc = 0; cc < pl.ncol; ++cc) {
      // Jacobi within the phase: evaluate every candidate, then commit
      for (unsigned t = tid; t < nbig; t += nthr) {
        const unsigned s = bigl[t];
        if (state[s] || col[s] != cc) continue;
        float v;
        const int res = evaluate<ND, K>(a.out, labels, (int)idx[s], pl, &v);
        if (res == 1) {
          state[s] = 1;
        } else if (res == 2) {
          pend[s] = v;
          state[s] = 2;
          atomicAdd(&s_commits, 1u);
        }
      }
      __threadfence_block();
      __syncthreads();
      for (unsigned t = tid; t < nbig; t += nthr) {
        const unsigned s = bigl[t];
        if (state[s] == 2) {
          a.out[idx[s]] = pend[s];
          state[s] = 1;
        }
      }
      __threadfence_block();
      __syncthreads();
    }
    const unsigned commits = s_commits;
    __syncthreads();
    total += commits;
    if (commits == 0) break;
  }
  if (tid == 0) ctrl_of(a.ws)->stats[1] = total;
  return (unsigned)(round <= pl.max_rounds ? round : pl.max_rounds);
}

__global__ __launch_bounds__(1024) void tail_kernel(RefArgs a) {
  __shared__ Plan s_p;
  __shared__ unsigned s_big, s_ok, s_hf;
  __shared__ unsigned long long s_sum[3];
  __shared__ unsigned s_fl;
  Ctrl* ct = ctrl_of(a.ws);
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_p = ct->plan;
    s_hf = ct->hflags;
    s_ok = s_hf == 0 && s_p.valid;
    s_big = ct->big_count;
    s_sum[0] = s_sum[1] = s_sum[2] = 0;
    s_fl = 0;
    ct->stats[1] = 0;
  }
  __syncthreads();
  const Plan& pl = s_p;
  const bool ok = s_ok != 0;
  const uint64_t nb = ok ? ((uint64_t)pl.g.n + kB - 1) / kB : 0;
  const DecLayout L = dec_layout(nb, ok ? (uint64_t)pl.nch : 0);
  const unsigned cap = ok ? (unsigned)pl.nch * kChunk : 0;
  const unsigned nbig = ok && pl.topo ? (s_big < cap ? s_big : cap) : 0;
  unsigned trounds = 0;
  if (nbig > 0) {
    switch (pl.ndim * 8 + pl.k) {
      case 2 * 8 + 3: trounds = tail_rounds<2, 3>(a, pl, L, nbig); break;
      case 2 * 8 + 5: trounds = tail_rounds<2, 5>(a, pl, L, nbig); break;
      case 2 * 8 + 7: trounds = tail_rounds<2, 7>(a, pl, L, nbig); break;
      case 3 * 8 + 3: trounds = tail_rounds<3, 3>(a, pl, L, nbig); break;
      case 3 * 8 + 5: trounds = tail_rounds<3, 5>(a, pl, L, nbig); break;
      default: trounds = tail_rounds<3, 7>(a, pl, L, nbig); break;
    }
  }
  __syncthreads();
  unsigned long long q = 0, mv = 0, sk = 0;
  unsigned fl = 0;
  if (ok) {
    const unsigned* cnt = reinterpret_cast<const unsigned*>(a.ws + L.cnt);
    const unsigned* mo = reinterpret_cast<const unsigned*>(a.ws + L.moves);
    const unsigned* skp = reinterpret_cast<const unsigned*>(a.ws + L.skips);
    const unsigned* df = reinterpret_cast<const unsigned*>(a.ws + L.dflag);
    for (int k = tid; k < pl.nch; k += blockDim.x) {
      q += cnt[k];
      mv += mo[k];
      sk += skp[k];
      fl |= df[k];
    }
  }
  atomicAdd(&s_sum[0], q);
  atomicAdd(&s_sum[1], mv);
  atomicAdd(&s_sum[2], sk);
  if (fl) atomicOr(&s_fl, fl);
  __syncthreads();
  if (tid == 0) {
    const Spread* sp = spread_of(a.ws);
    unsigned long long commits = ct->stats[1];
    unsigned rounds = trounds;
    for (int k = 0; k < kSpreadLines; ++k) {
      commits += sp[k].commits;
      rounds = max(rounds, sp[k].rounds);
    }
    if (ok && pl.topo && rounds == 0) rounds = 1;  // a round that found nothing to do
    ct->stats[0] = ok && pl.topo ? rounds : 0;
    ct->stats[1] = commits;
    ct->stats[2] = s_sum[0];
    ct->stats[3] = s_sum[1];
    ct->stats[4] = s_sum[2];
    int status = TOPOSZP_OK;
    if (s_hf == 2u) status = TOPOSZP_E_CAPACITY;
    else if (s_hf != 0u || s_fl) status = TOPOSZP_E_CORRUPT;
    *a.status = status;
  }
}

// ---------------------------------------------------------------------------
// Host side.

struct HostGeom {
  Geom g;
  uint64_t dims[3];
  uint64_t nb, nch;
};

int host_geom(uint32_t ndim, const uint64_t* dims, HostGeom* hg) {
  if (!dims || (ndim != 2 && ndim != 3)) return TOPOSZP_E_INVALID_ARG;
  uint64_t n = 1;
  for (uint32_t d = 0; d < ndim; ++d) {
    if (dims[d] < 1) return TOPOSZP_E_INVALID_ARG;
    if (dims[d] > (1ull << 31)) return TOPOSZP_E_UNSUPPORTED;
    n *= dims[d];
    if (n >= (1ull << 31)) return TOPOSZP_E_UNSUPPORTED;
  }
  hg->dims[0] = dims[0];
  hg->dims[1] = dims[1];
  hg->dims[2] = ndim == 3 ? dims[2] : 1;
  hg->g.ndim = (int)ndim;
  hg->g.n = (int)n;
  hg->g.nx = (int)(ndim == 3 ? dims[2] : dims[1]);
  hg->g.ny = (int)(ndim == 3 ? dims[1] : dims[0]);
  hg->g.nz = (int)(ndim == 3 ? dims[0] : 1);
  hg->nb = (n + kB - 1) / kB;
  hg->nch = (hg->nb + kB - 1) / kB;
  return TOPOSZP_OK;
}

size_t ws_need(const HostGeom& hg) {
  const uint64_t c = comp_layout(hg.nch).end, d = dec_layout(hg.nb, hg.nch).end;
  return (size_t)al256(c > d ? c : d);
}

float host_round_down(double d) {
  float f = (float)d;
  if ((double)f > d) f = nextafterf(f, 0.0f);
  return f;
}

// timing
bool g_timing = false;
hipEvent_t g_ev[6][2];
bool g_ev_used[6];
bool g_ev_init = false;

void ev_begin(int k, hipStream_t s) {
  if (!g_timing) return;
  if (!g_ev_init) {
    for (int i = 0; i < 6; ++i) {
      (void)hipEventCreate(&g_ev[i][0]);
      (void)hipEventCreate(&g_ev[i][1]);
    }
    g_ev_init = true;
  }
  (void)hipEventRecord(g_ev[k][0], s);
}
void ev_end(int k, hipStream_t s) {
  if (!g_timing) return;
  (void)hipEventRecord(g_ev[k][1], s);
  g_ev_used[k] = true;
}

constexpr int kEncWaves = 4;
constexpr int kDecWaves = 4;

}  // namespace

extern "C" {

int toposzp_version(void) { return 1; }

const char* toposzp_strerror(int status) {
  switch (status) {
    case TOPOSZP_OK: return "ok";
    case TOPOSZP_E_INVALID_ARG: return "invalid argument";
    case TOPOSZP_E_NONFINITE: return "non-finite value in the input field";
    case TOPOSZP_E_RANGE: return "error bound or values outside the quantizer range";
    case TOPOSZP_E_CAPACITY: return "output or workspace buffer too small";
    case TOPOSZP_E_CORRUPT: return "corrupt compressed stream";
    case TOPOSZP_E_DEVICE: return "HIP runtime error";
    case TOPOSZP_E_UNSUPPORTED: return "unsupported request";
    default: return "unknown status";
  }
}

size_t toposzp_compress_bound(uint32_t ndim, const uint64_t* dims) {
  HostGeom hg;
  if (host_geom(ndim, dims, &hg) != TOPOSZP_OK) return 0;
  uint64_t off[kNSeg], len[kNSeg];
  return (size_t)seg_layout(hg.nb, 1, hg.nb * kMaxWData, hg.nb * kMaxWRankBlk, off, len);
}

size_t toposzp_workspace_size(uint32_t ndim, const uint64_t* dims) {
  HostGeom hg;
  if (host_geom(ndim, dims, &hg) != TOPOSZP_OK) return 0;
  return ws_need(hg);
}

int toposzp_workspace_init(void* d_ws, size_t ws_bytes, void* stream) {
  if (!d_ws || ws_bytes < kRegionOff || ((uintptr_t)d_ws & 255)) return TOPOSZP_E_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  const uint64_t n8 = ws_bytes / 8;
  unsigned grid = (unsigned)((n8 + 255) / 256);
  if (grid > 4096) grid = 4096;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(ws_init_kernel, dim3(grid), dim3(256), 0, s, (uint8_t*)d_ws, (uint64_t)ws_bytes);
  return hipGetLastError() == hipSuccess ? TOPOSZP_OK : TOPOSZP_E_DEVICE;
}

int toposzp_compress(const float* d_field, uint32_t ndim, const uint64_t* dims, int eb_mode,
                     double eb, const toposzp_params* params, void* d_ws, size_t ws_bytes,
                     uint8_t* d_out, size_t out_cap, uint64_t* d_out_size, int32_t* d_status,
                     void* stream) {
  toposzp_params p = {64, 0, 0, 16, 1};
  if (params) p = *params;
  HostGeom hg;
  int rc = host_geom(ndim, dims, &hg);
  if (rc != TOPOSZP_OK) return rc;
  if (!d_field || !d_ws || !d_out || !d_out_size || !d_status) return TOPOSZP_E_INVALID_ARG;
  if (((uintptr_t)d_field & 15) || ((uintptr_t)d_ws & 255) || ((uintptr_t)d_out & 7) ||
      ((uintptr_t)d_out_size & 7) || ((uintptr_t)d_status & 3))
    return TOPOSZP_E_INVALID_ARG;
  if (!(eb > 0.0) || !std::isfinite(eb) || (eb_mode != TOPOSZP_EB_ABS && eb_mode != TOPOSZP_EB_REL))
    return TOPOSZP_E_INVALID_ARG;
  if (p.block != (uint32_t)kB || (p.topo != 0 && p.topo != 1) || (p.rank_scope != 0 && p.rank_scope != 1) ||
      (p.rbf_policy != 0 && p.rbf_policy != 1) || p.max_rounds < 1 || p.max_rounds > kMaxRounds)
    return TOPOSZP_E_INVALID_ARG;
  if (p.rank_scope == 1 && p.topo) return TOPOSZP_E_UNSUPPORTED;
  if (out_cap < toposzp_compress_bound(ndim, dims)) return TOPOSZP_E_CAPACITY;
  if (ws_bytes < ws_need(hg)) return TOPOSZP_E_CAPACITY;
  hipStream_t s = (hipStream_t)stream;

  int nrange = (int)((hg.g.n / 4 + 4095) / 4096);
  if (nrange > kRangeWG) nrange = kRangeWG;
  if (nrange < 1) nrange = 1;
  const float e_abs = host_round_down(eb);

  EncArgs ea;
  ea.f = d_field;
  ea.out = d_out;
  ea.ws = (uint8_t*)d_ws;
  ea.gd.n = hg.g.n;
  ea.gd.nx = hg.g.nx;
  ea.gd.ny = hg.g.ny;
  ea.gd.nz = hg.g.nz;
  ea.gd.nxy = hg.g.nx * hg.g.ny;
  ea.gd.dx = make_div((unsigned)hg.g.nx);
  ea.gd.dy = make_div((unsigned)hg.g.ny);
  ea.nb = (int)hg.nb;
  ea.nch = (int)hg.nch;
  ea.topo = p.topo;
  ea.eb_mode = eb_mode;
  ea.nrange = nrange;
  ea.eb = eb;
  ea.e_abs = e_abs;
  seg_layout(hg.nb, p.topo, 0, 0, ea.off, ea.len);

  ScanArgs sa;
  sa.ws = (uint8_t*)d_ws;
  sa.nch = ea.nch;
  sa.eb_mode = eb_mode;
  sa.nrange = nrange;
  sa.eb = eb;
  sa.e_abs = e_abs;

  FinArgs fa;
  fa.out = d_out;
  fa.ws = (uint8_t*)d_ws;
  fa.out_size = d_out_size;
  fa.status = d_status;
  fa.g = hg.g;
  for (int d = 0; d < 3; ++d) fa.dims[d] = hg.dims[d];
  fa.nb = ea.nb;
  fa.nch = ea.nch;
  fa.topo = p.topo;
  fa.eb_mode = eb_mode;
  fa.rbf_policy = p.rbf_policy;
  fa.max_rounds = p.max_rounds;
  fa.eb = eb;
  memcpy(fa.off, ea.off, sizeof(ea.off));
  memcpy(fa.len, ea.len, sizeof(ea.len));
  const double sig[3] = {0.5, 0.75, 1.0};
  for (int t = 0; t < 3; ++t)
    for (int d2 = 0; d2 < 10; ++d2) fa.wtab[t][d2] = (float)exp(-(double)d2 / (2.0 * sig[t] * sig[t]));

  for (int k = 0; k < 3; ++k) g_ev_used[k] = false;
  if (eb_mode == TOPOSZP_EB_REL) {
    ev_begin(0, s);
    hipLaunchKernelGGL(range_kernel, dim3(nrange), dim3(256), 0, s, d_field, hg.g.n, (uint8_t*)d_ws);
    ev_end(0, s);
  }
  ev_begin(1, s);
  hipLaunchKernelGGL(encode_kernel<kEncWaves>, dim3(ea.nch), dim3(kEncWaves * 64), 0, s, ea);
  ev_end(1, s);
  ev_begin(2, s);
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, sa);
  hipLaunchKernelGGL(finalize_kernel, dim3(ea.nch), dim3(256), 0, s, fa);
  ev_end(2, s);
  return hipGetLastError() == hipSuccess ? TOPOSZP_OK : TOPOSZP_E_DEVICE;
}

int toposzp_decompress(const uint8_t* d_in, size_t in_size, float* d_out, size_t out_cap_elems,
                       void* d_ws, size_t ws_bytes, int32_t* d_status, void* stream) {
  if (!d_in || !d_out || !d_ws || !d_status || out_cap_elems < 1) return TOPOSZP_E_INVALID_ARG;
  if (((uintptr_t)d_in & 7) || ((uintptr_t)d_out & 3) || ((uintptr_t)d_ws & 255) || ((uintptr_t)d_status & 3))
    return TOPOSZP_E_INVALID_ARG;
  if (ws_bytes < kRegionOff + 4096) return TOPOSZP_E_CAPACITY;
  hipStream_t s = (hipStream_t)stream;
  uint64_t cap = out_cap_elems;
  if (cap > (1ull << 31)) cap = (1ull << 31);
  const uint64_t nch = ((cap + kB - 1) / kB + kB - 1) / kB;
  DecArgs da;
  da.in = d_in;
  da.in_size = in_size;
  da.out = d_out;
  da.out_cap = out_cap_elems;
  da.ws = (uint8_t*)d_ws;
  da.ws_bytes = ws_bytes;
  for (int k = 3; k < 5; ++k) g_ev_used[k] = false;
  ev_begin(3, s);
  hipLaunchKernelGGL(decode_kernel<kDecWaves>, dim3((unsigned)nch), dim3(kDecWaves * 64), 0, s, da);
  ev_end(3, s);
  RefArgs ra;
  ra.in = d_in;
  ra.out = d_out;
  ra.ws = (uint8_t*)d_ws;
  ra.status = d_status;
  ev_begin(4, s);
  hipLaunchKernelGGL(refine_kernel, dim3((unsigned)nch), dim3(kRefineThreads), 0, s, ra);
  hipLaunchKernelGGL(tail_kernel, dim3(1), dim3(1024), 0, s, ra);
  ev_end(4, s);
  return hipGetLastError() == hipSuccess ? TOPOSZP_OK : TOPOSZP_E_DEVICE;
}

int toposzp_compress_sync(const float* d_field, uint32_t ndim, const uint64_t* dims, int eb_mode,
                          double eb, const toposzp_params* params, void* d_ws, size_t ws_bytes,
                          uint8_t* d_out, size_t out_cap, uint64_t* h_out_size, void* stream) {
  // status and size travel through the tail of the workspace's control area
  uint8_t* ws = (uint8_t*)d_ws;
  if (!ws || ws_bytes < kRegionOff) return TOPOSZP_E_INVALID_ARG;
  uint64_t* d_size = reinterpret_cast<uint64_t*>(ws + kSpreadOff - 16);
  int32_t* d_stat = reinterpret_cast<int32_t*>(ws + kSpreadOff - 8);
  int rc = toposzp_compress(d_field, ndim, dims, eb_mode, eb, params, d_ws, ws_bytes, d_out, out_cap,
                            d_size, d_stat, stream);
  if (rc != TOPOSZP_OK) return rc;
  uint64_t sz = 0;
  int32_t st = 0;
  if (hipMemcpyAsync(&sz, d_size, 8, hipMemcpyDeviceToHost, (hipStream_t)stream) != hipSuccess ||
      hipMemcpyAsync(&st, d_stat, 4, hipMemcpyDeviceToHost, (hipStream_t)stream) != hipSuccess ||
      hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
    return TOPOSZP_E_DEVICE;
  if (h_out_size) *h_out_size = sz;
  return st;
}

int toposzp_decompress_sync(const uint8_t* d_in, size_t in_size, float* d_out, size_t out_cap_elems,
                            void* d_ws, size_t ws_bytes, void* stream) {
  uint8_t* ws = (uint8_t*)d_ws;
  if (!ws || ws_bytes < kRegionOff) return TOPOSZP_E_INVALID_ARG;
  int32_t* d_stat = reinterpret_cast<int32_t*>(ws + kSpreadOff - 8);
  int rc = toposzp_decompress(d_in, in_size, d_out, out_cap_elems, d_ws, ws_bytes, d_stat, stream);
  if (rc != TOPOSZP_OK) return rc;
  int32_t st = 0;
  if (hipMemcpyAsync(&st, d_stat, 4, hipMemcpyDeviceToHost, (hipStream_t)stream) != hipSuccess ||
      hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
    return TOPOSZP_E_DEVICE;
  return st;
}

int toposzp_inspect(const uint8_t* h, size_t n, toposzp_info* out) {
  if (!h || !out) return TOPOSZP_E_INVALID_ARG;
  if (n < (size_t)kHdr) return TOPOSZP_E_CORRUPT;
  uint32_t A = 1, B = 0;
  for (int i = 0; i < kSummed; ++i) {
    A = (A + h[i]) % 65521u;
    B = (B + A) % 65521u;
  }
  uint32_t stored, pad;
  memcpy(&stored, h + kSummed, 4);
  memcpy(&pad, h + kSummed + 4, 4);
  if (memcmp(h, "TSZ1", 4) != 0 || stored != ((B << 16) | A) || pad != 0) return TOPOSZP_E_CORRUPT;
  uint16_t ver, mr;
  memcpy(&ver, h + 4, 2);
  if (ver != 1) return TOPOSZP_E_CORRUPT;
  memset(out, 0, sizeof(*out));
  out->ndim = h[6];
  out->topo = h[7] & 1;
  out->rank_scope = (h[7] >> 1) & 1;
  out->eb_mode = h[52];
  out->k_size = h[53];
  memcpy(&mr, h + 54, 2);
  out->max_rounds = mr;
  memcpy(out->dims, h + 8, 24);
  memcpy(&out->n, h + 32, 8);
  memcpy(&out->nblocks, h + 40, 8);
  memcpy(&out->eb, h + 56, 8);
  memcpy(&out->eps, h + 64, 8);
  memcpy(&out->e, h + 72, 4);
  memcpy(&out->vmin, h + 76, 4);
  memcpy(&out->vmax, h + 80, 4);
  memcpy(&out->sigma, h + 84, 4);
  memcpy(&out->total_bytes, h + 128, 8);
  memcpy(&out->data_planes, h + 136, 8);
  memcpy(&out->rank_planes, h + 144, 8);
  if (out->ndim != 2 && out->ndim != 3) return TOPOSZP_E_CORRUPT;
  return TOPOSZP_OK;
}

int toposzp_decompress_stats(const void* d_ws, int64_t out[5], void* stream) {
  if (!d_ws || !out) return TOPOSZP_E_INVALID_ARG;
  const Ctrl* ct = (const Ctrl*)d_ws;
  unsigned long long st[5];
  if (hipMemcpyAsync(st, (const void*)ct->stats, sizeof(st), hipMemcpyDeviceToHost, (hipStream_t)stream) !=
          hipSuccess ||
      hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
    return TOPOSZP_E_DEVICE;
  for (int k = 0; k < 5; ++k) out[k] = (int64_t)st[k];
  return TOPOSZP_OK;
}

int toposzp_set_timing(int enable) {
  g_timing = enable != 0;
  return TOPOSZP_OK;
}

int toposzp_kernel_times(float* ms, int max) {
  if (!ms) return 0;
  int k = 0;
  for (; k < 5 && k < max; ++k) {
    ms[k] = -1.0f;
    if (g_ev_init && g_ev_used[k]) {
      float t = -1.0f;
      if (hipEventElapsedTime(&t, g_ev[k][0], g_ev[k][1]) == hipSuccess) ms[k] = t;
    }
  }
  return k;
}

}  // extern "C"
