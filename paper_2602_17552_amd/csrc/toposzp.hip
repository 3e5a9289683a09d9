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
//                    evaluation, and a cluster (gathered by one lane) is
//                    replayed by the workgroup, one member per lane.  The
//                    first workgroup also writes the call's status.  For a
//                    small field, refine_split_kernel divides each chunk's
//                    queue over up to 8 workgroups.
//   tail_kernel      one workgroup: the same schedule for the rare clusters
//                    of more than 64 members, gathered and replayed from
//                    LDS (the whole field's queue when they do not fit).
//   stats_kernel     one workgroup, on request: the decompression's counters.
//
// No kernel contends on a single global address; every device wait is
// bounded.  Readings of points the paper leaves open are stated where used.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <type_traits>
#include <vector>


#include "toposzp.h"

// The compiler's lane-write intrinsic (v_writelane_b32): lane `l` (uniform)
// of `old` takes the uniform value `v`.
__device__ int llvm_writelane(int v, int l, int old) __asm("llvm.amdgcn.writelane.i32");

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
constexpr int kRangeWG = 1024;         // max range-pass workgroups
constexpr int kRangeVec = 8;           // float4 loads per thread per pass
constexpr int kFuseMax = 4096;         // chunk counts whose scan finalize does itself
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
  double wsum;  // the window's weight sum when every cell lies in the grid
  uint64_t s6_off;
};

constexpr int kOverMax = 128;  // owner candidates of over-size clusters kept for the tail

struct Ctrl {
  // compression: written by scan_kernel, read by finalize_kernel
  unsigned long long tot_data, tot_rank;
  unsigned cflags;            // 1 non-finite, 2 bound out of range, 4 |q| too big
  float e, vmin, vmax;
  double eps;
  // decompression
  unsigned hflags;            // header check of this call: 0 good, 1 corrupt, 2 capacity
  unsigned big;               // owner candidates whose cluster was too large for a workgroup
  unsigned long long stats[5];// rounds, commits, queued, stencil moves, budget skips
  unsigned long long rp_commits;  // commits of the tail's replay of over-size clusters
  unsigned rp_rounds;             // and its rounds
  Plan plan;
  unsigned fs_count;          // field-scope compression: flattened extrema marked
  unsigned over[kOverMax];    // the first kOverMax of those candidates
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
// Rank planes per block the staging holds: 7 for block-scope ranks (at most
// 64), 31 for field-scope ranks.
__host__ __device__ constexpr int rank_w(int field) { return field ? kMaxWRankAny : kMaxWRankBlk; }
__host__ __device__ constexpr CompLayout comp_layout(uint64_t nch, int field = 0) {
  CompLayout L{};
  // three per-chunk arrays of u32, each padded to 16 bytes (read as uint4)
  const uint64_t arr = (4 * nch + 15) & ~uint64_t(15);
  L.tot_d = kRegionOff;
  L.tot_r = L.tot_d + arr;
  L.cflag = L.tot_r + arr;
  // staged planes: one slot per block (its planes at the slot's start)
  L.stage_d = al256(L.cflag + arr);
  L.stage_r = al256(L.stage_d + 8ull * kB * kMaxWData * nch);
  L.end = al256(L.stage_r + 8ull * kB * rank_w(field) * nch);
  return L;
}

struct DecLayout {
  uint64_t cnt, moves, skips, dflag, bitmap, capped, idx, state, pend, end;
};
__host__ __device__ inline DecLayout dec_layout(uint64_t nb, uint64_t nch) {
  DecLayout L;
  const uint64_t slots = nch * kChunk;
  L.cnt = kRegionOff;
  L.moves = L.cnt + 4 * nch;
  L.skips = L.moves + 4 * nch;
  L.dflag = L.skips + 4 * nch;
  L.bitmap = al256(L.dflag + 4 * nch);
  L.capped = al256(L.bitmap + 8 * nb);  // members of clusters stopped by the round cap
  L.idx = al256(L.capped + 8 * nb);
  L.state = al256(L.idx + 4 * slots);
  L.pend = al256(L.state + slots);
  L.end = al256(L.pend + 4 * slots);
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
__device__ __forceinline__ float key2f32(int k) {
  if (k > 0x7F800000) k = 0x7F800001;
  if (k < -0x7F800000) k = -0x7F800001;
  const unsigned b = k >= 0 ? (unsigned)k : 0x80000000u + (0u - (unsigned)k);
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

// Class from the six face neighbours [x-, x+, y-, y+, z-, z+] (Section
// III-A).  avm: bit j set if neighbour j exists; ndeg: bit 2*axis set for
// each axis of extent >= 2 (an axis of extent 1 has no neighbours and takes
// no part in the saddle test).  Minimum: every neighbour higher; maximum:
// every neighbour lower; saddle: along every axis both neighbours higher or
// both lower, with at least one axis of each kind.
__device__ __forceinline__ int classify_bits(float a, const float nb[6], unsigned avm, unsigned ndeg) {
  unsigned gt = 0, lt = 0;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    gt |= (nb[j] > a ? 1u : 0u) << j;
    lt |= (nb[j] < a ? 1u : 0u) << j;
  }
  gt &= avm;
  lt &= avm;
  const unsigned bg = gt & (gt >> 1) & 0x15u, bl = lt & (lt >> 1) & 0x15u;
  int cls = CLS_R;
  if (((bg | bl) & ndeg) == ndeg && bg != 0 && bl != 0) cls = CLS_SAD;
  if (avm != 0 && lt == avm) cls = CLS_MAX;
  if (avm != 0 && gt == avm) cls = CLS_MIN;
  return cls;
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
// Sum and OR over the wave (uniform results).
__device__ __forceinline__ unsigned wave_sum(unsigned v) {
  return (unsigned)__builtin_amdgcn_readlane((int)(unsigned)wave_incl_scan((int)v, 0), 63);
}
__device__ __forceinline__ unsigned wave_or(unsigned v) {
  v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);
  v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);
  v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);
  v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);
  v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);
  v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
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
// This lane's bit of a uniform lane mask, as a per-lane condition.
__device__ __forceinline__ bool lane_in(unsigned long long m) { return __builtin_amdgcn_inverse_ballot_w64(m); }
__device__ __forceinline__ unsigned mbcnt(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// Bit length of the largest of the lanes' values: the highest set bit of
// their OR is the largest value's (an OR over the wave, then one scalar
// find-last-bit).
__device__ __forceinline__ int wave_bitlen(unsigned v) {
  const unsigned o = wave_or(v);
  return o ? 32 - __builtin_clz(o) : 0;
}

// B + LZ + BE of one 64-value block held one value per lane: residuals
// r_0 = 0, r_i = v_i - v_{i-1}; width = bit length of max |r_i|; the sign and
// each bit plane are one 64-bit lane mask; plane j goes to dst[2j], dst[2j+1]
// (LDS) through lanes 2j, 2j+1.
template <int MAXW>
__device__ __forceinline__ int encode_block(int v, int lane, unsigned* dst,
                                            unsigned long long& sign, int& first, bool& over) {
  const int prev = dpp_from_prev(v, v);  // lane 0 sees itself: residual 0
  const int r = v - prev;                // |v| < 2^23: no overflow
  sign = __ballot(r < 0);
  const unsigned mag = (unsigned)(r < 0 ? -r : r);
  int w = wave_bitlen(mag);
  if (w > MAXW) {
    over = true;
    w = MAXW;
  }
  int mine = 0;
  for (int j = 0; j < w; ++j) {
    const unsigned long long pl = __ballot((mag >> j) & 1u);
    mine = llvm_writelane((int)(unsigned)pl, 2 * j, mine);
    mine = llvm_writelane((int)(unsigned)(pl >> 32), 2 * j + 1, mine);
  }
  if (lane < 2 * w) dst[lane] = (unsigned)mine;
  first = __builtin_amdgcn_readfirstlane(v);
  return w;
}

// The float32 products pm*e and pp*e rounded toward +infinity (the smallest
// floats >= the exact products).  The two multiplies run with the f32
// rounding mode set to round-up and the mode is restored at once; nothing
// else runs in between.
__device__ __forceinline__ void mul_round_up2(float pm, float pp, float e, float& lo, float& hi) {
  asm volatile(
      "s_setreg_imm32_b32 hwreg(HW_REG_MODE, 0, 2), 1\n\t"
      "s_nop 1\n\t"
      "v_mul_f32 %0, %2, %4\n\t"
      "v_mul_f32 %1, %3, %4\n\t"
      "s_setreg_imm32_b32 hwreg(HW_REG_MODE, 0, 2), 0\n\t"
      "s_nop 1"
      : "=&v"(lo), "=&v"(hi)
      : "v"(pm), "v"(pp), "v"(e));
}

// Bit planes of a block (BE), the lanes' magnitudes `mag` of width w <=
// MAXW: plane j is the ballot of bit j, kept in lanes 2j (low word) and
// 2j+1 (high word) and written to dst[0, 2w).  Each plane is nested in the
// previous one's test, so that a block of width w tests w + 1 conditions.
template <int J, int MAXW>
__device__ __forceinline__ void plane_run(unsigned mag, int w, int& mine) {
  if constexpr (J < MAXW) {
    if (J < w) {
      const unsigned long long pl = __ballot((mag >> J) & 1u);
      mine = llvm_writelane((int)(unsigned)pl, 2 * J, mine);
      mine = llvm_writelane((int)(unsigned)(pl >> 32), 2 * J + 1, mine);
      plane_run<J + 1, MAXW>(mag, w, mine);
    }
  }
}
template <int MAXW>
__device__ __forceinline__ void put_planes(unsigned mag, int w, unsigned* dst, int lane) {
  int mine = 0;
  plane_run<0, MAXW>(mag, w, mine);
  if (lane < 2 * w) dst[lane] = (unsigned)mine;
}

// |x - y| of unsigned values (v_sad_u32).
__device__ __forceinline__ unsigned absdiff_u32(unsigned x, unsigned y) {
  unsigned d;
  asm("v_sad_u32 %0, %1, %2, 0" : "=v"(d) : "v"(x), "v"(y));
  return d;
}

// Inverse: each lane reads its own 32-bit half of every plane (lanes 0-31
// the low word, 32-63 the high word) and takes its bit; signed residuals;
// in-wave inclusive prefix sum.
template <typename PlanePtr>
__device__ __forceinline__ int decode_block(PlanePtr planes, int w, int first, unsigned long long sign,
                                            int lane) {
  const auto pw = reinterpret_cast<const unsigned*>(planes) + (lane >> 5);
  const unsigned sh = (unsigned)lane & 31u;
  unsigned mag = 0;
#pragma unroll 4
  for (int j = 0; j < w; ++j) mag |= ((pw[2 * j] >> sh) & 1u) << j;
  int r = ((sign >> lane) & 1ull) ? (int)(0u - mag) : (int)mag;
  if (lane == 0) r = first;
  return wave_incl_scan(r, lane);
}

// Two blocks at once (as decode_block each): their plane reads and prefix
// sums are independent chains that the scheduler interleaves.
template <typename PlanePtr>
__device__ __forceinline__ void decode_pair(PlanePtr pa, int wa, int fa, unsigned long long sa, PlanePtr pb, int wb,
                                            int fb, unsigned long long sb, int lane, int& qa, int& qb) {
  const auto ua = reinterpret_cast<const unsigned*>(pa) + (lane >> 5);
  const auto ub = reinterpret_cast<const unsigned*>(pb) + (lane >> 5);
  const unsigned sh = (unsigned)lane & 31u;
  unsigned ma = 0, mb = 0;
  const int wc = wa < wb ? wa : wb;
  int j = 0;
#pragma unroll 2
  for (; j < wc; ++j) {
    ma |= ((ua[2 * j] >> sh) & 1u) << j;
    mb |= ((ub[2 * j] >> sh) & 1u) << j;
  }
  for (int t = j; t < wa; ++t) ma |= ((ua[2 * t] >> sh) & 1u) << t;
  for (int t = j; t < wb; ++t) mb |= ((ub[2 * t] >> sh) & 1u) << t;
  int ra = ((sa >> lane) & 1ull) ? (int)(0u - ma) : (int)ma;
  int rb = ((sb >> lane) & 1ull) ? (int)(0u - mb) : (int)mb;
  if (lane == 0) {
    ra = fa;
    rb = fb;
  }
  unsigned x = (unsigned)ra, y = (unsigned)rb;
  x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);
  y += (unsigned)__builtin_amdgcn_update_dpp(0, (int)y, 0x111, 0xf, 0xf, false);
  x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);
  y += (unsigned)__builtin_amdgcn_update_dpp(0, (int)y, 0x112, 0xf, 0xf, false);
  x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);
  y += (unsigned)__builtin_amdgcn_update_dpp(0, (int)y, 0x114, 0xf, 0xf, false);
  x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);
  y += (unsigned)__builtin_amdgcn_update_dpp(0, (int)y, 0x118, 0xf, 0xf, false);
  x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);
  y += (unsigned)__builtin_amdgcn_update_dpp(0, (int)y, 0x142, 0xa, 0xf, false);
  x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);
  y += (unsigned)__builtin_amdgcn_update_dpp(0, (int)y, 0x143, 0xc, 0xf, false);
  qa = (int)x;
  qb = (int)y;
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
  int nb, nch, topo, eb_mode, nrange, field;
  double eb;
  float e_abs;
  uint64_t off[kNSeg], len[kNSeg];
  unsigned long long* keys;  // field scope: compacted sort keys of the mark pass
  unsigned* vals;            // and their point indices
  unsigned long long* skeys; // each wave's staging slice of keys (indexed like points)
  unsigned* svals;           // and of indices
  unsigned* ccnt;            // field scope: flattened extrema per chunk
  const int* delta;          // field scope: ranks per point for the encode pass
};

struct ScanArgs {
  uint8_t* ws;
  int nch, eb_mode, nrange, field;
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
  int nb, nch, topo, eb_mode, rbf_policy, max_rounds, nrange, fused, field;
  double eb;
  float e_abs;
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
  int slots;  // workgroups per sub-slice (chunk slots of the launch)
  int split;  // sub-slices each chunk's queue is divided into
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

__device__ __forceinline__ void range_body(const float* __restrict__ f, int n, uint8_t* ws, int blk, int nblk) {
  __shared__ unsigned s_lo[4], s_hi[4], s_bad[4];
  float lo = INFINITY, hi = -INFINITY;
  bool bad = false;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n4 = n / 4;
  const float4* f4 = reinterpret_cast<const float4*>(f);
  // kRangeVec float4 per thread in flight at once; clamped indices repeat
  // the last vector, which changes neither extreme
  for (int base = blk * 256 * kRangeVec; base < n4; base += nblk * 256 * kRangeVec) {
    float4 v[kRangeVec];
#pragma unroll
    for (int t = 0; t < kRangeVec; ++t) v[t] = f4[min(base + t * 256 + tid, n4 - 1)];
#pragma unroll
    for (int t = 0; t < kRangeVec; ++t) {
      bad |= !(fabsf(v[t].x) <= FLT_MAX) || !(fabsf(v[t].y) <= FLT_MAX) || !(fabsf(v[t].z) <= FLT_MAX) ||
             !(fabsf(v[t].w) <= FLT_MAX);
      lo = fminf(lo, fminf(fminf(v[t].x, v[t].y), fminf(v[t].z, v[t].w)));
      hi = fmaxf(hi, fmaxf(fmaxf(v[t].x, v[t].y), fmaxf(v[t].z, v[t].w)));
    }
  }
  if (blk == 0 && tid < n - 4 * n4) {
    const float v = f[4 * n4 + tid];
    bad |= !(fabsf(v) <= FLT_MAX);
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
    const uint4 part = {min(min(s_lo[0], s_lo[1]), min(s_lo[2], s_lo[3])),
                        max(max(s_hi[0], s_hi[1]), max(s_hi[2], s_hi[3])), s_bad[0] | s_bad[1] | s_bad[2] | s_bad[3],
                        0u};
    reinterpret_cast<uint4*>(ws + kPartOff)[blk] = part;
  }
}

__global__ __launch_bounds__(256) void range_kernel(const float* __restrict__ f, int n, uint8_t* ws) {
  range_body(f, n, ws, blockIdx.x, gridDim.x);
}

// Bound of the call (one wave): relative mode reduces the range partials.
// LDS for the range reduction below (one slot per wave, up to 16 waves).
struct RangeSh {
  unsigned lo[16], hi[16], nf[16];
};

// The bound of this call (Section II-C).  A relative bound takes the field's
// range from the range kernel's partials, reduced by the whole workgroup:
// each thread loads up to four partials (blockDim.x >= kRangeWG / 4), the
// waves combine through LDS.  Every thread gets the result.  It contains a
// barrier: call it from workgroup-uniform control flow.
__device__ __forceinline__ void call_bound(const uint8_t* ws, int eb_mode, double eb, float e_abs, int nrange,
                                           RangeSh& rs, float* e, float* vmin, float* vmax, double* eps, bool* bad) {
  unsigned lo = 0xFFFFFFFFu, hi = 0u, nf = 0u;
  if (eb_mode == TOPOSZP_EB_REL) {
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wv = tid >> 6;
    const uint4* part = reinterpret_cast<const uint4*>(ws + kPartOff);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int j = tid + t * nt;
      if (j < nrange) {
        const uint4 p = part[j];
        lo = min(lo, p.x);
        hi = max(hi, p.y);
        nf |= p.z;
      }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      lo = min(lo, (unsigned)__shfl_xor((int)lo, o));
      hi = max(hi, (unsigned)__shfl_xor((int)hi, o));
      nf |= (unsigned)__shfl_xor((int)nf, o);
    }
    if (lane == 0) {
      rs.lo[wv] = lo;
      rs.hi[wv] = hi;
      rs.nf[wv] = nf;
    }
    __syncthreads();
    for (int w = 0; w < (nt >> 6); ++w) {
      lo = min(lo, rs.lo[w]);
      hi = max(hi, rs.hi[w]);
      nf |= rs.nf[w];
    }
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

// The dispatcher deals workgroups to the eight XCDs in turn (workgroup w
// runs on XCD w % 8).  Giving each XCD a contiguous range of chunks keeps the
// rows above and below a chunk in that XCD's L2.  The grid has 8 * per
// workgroups; those past the last chunk return at once.
__host__ __device__ inline int xcd_grid(int nch) { return 8 * ((nch + 7) >> 3); }
__device__ __forceinline__ int xcd_chunk(int w, int nch) { return (w & 7) * ((nch + 7) >> 3) + (w >> 3); }

// Values one block needs: the lane's own, its y/z face neighbours, and in
// xe the value just before the block (lane 0) or just after it (other
// lanes; lane 63 uses it), the x neighbours the wave itself lacks.  Every
// address is clamped into the field, so each load is in bounds and none is
// conditional (unused values are masked later); keeping the loads
// unconditional lets the compiler wait for exactly the block in use.
struct EncIn {
  float c, ym, yp, zm, zp, xe;
};

template <int ND>
__device__ __forceinline__ EncIn enc_fetch(const float* __restrict__ f, int b, int lane, const GeomD& g) {
  EncIn r;
  const int n1 = g.n - 1;
  const int b0 = min(b * kB, n1);
  const int i = min(b0 + lane, n1);
  r.c = f[i];
  r.ym = f[max(i - g.nx, 0)];
  r.yp = f[min(i + g.nx, n1)];
  if (ND == 3) {
    r.zm = f[max(i - g.nxy, 0)];
    r.zp = f[min(i + g.nxy, n1)];
  } else {
    r.zm = r.zp = 0.0f;
  }
  r.xe = f[lane == 0 ? max(b0 - 1, 0) : min(b0 + kB, n1)];
  return r;
}

// f(std::integral_constant<int, K>) for K = K0 .. N-1: a loop whose index is
// a compile-time constant in every iteration.
template <int K, int N, typename F>
__device__ __forceinline__ void unroll(F&& f) {
  if constexpr (K < N) {
    f(std::integral_constant<int, K>{});
    unroll<K + 1, N>(f);
  }
}

// The values of enc_fetch for block k of a wave whose first block starts at
// p, when every read of the wave lies inside the field: uniform base
// addresses plus the lane's offset, the block's offset a constant of the
// load instructions.  xoff is 0 for lane 0 (the value before the block) and
// 65 for the others (the value after it, seen from one before the block).
template <int ND>
__device__ __forceinline__ EncIn enc_fetch_wave(const float* __restrict__ p, int k, unsigned lane, unsigned xoff,
                                                const GeomD& g) {
  EncIn r;
  const unsigned o = lane + (unsigned)(k * kB);
  r.c = p[o];
  r.ym = (p - g.nx)[o];
  r.yp = (p + g.nx)[o];
  if (ND == 3) {
    r.zm = (p - g.nxy)[o];
    r.zp = (p + g.nxy)[o];
  } else {
    r.zm = r.zp = 0.0f;
  }
  r.xe = (p - 1)[xoff + (unsigned)(k * kB)];
  return r;
}

// Whether every read of block b lies inside the field.
template <int ND>
__device__ __forceinline__ bool reads_inside(int b, const GeomD& g) {
  const int b0 = b * kB, st = ND == 3 ? g.nxy : g.nx;
  return b0 - st >= 0 && b0 >= 1 && b0 + (kB - 1) + st <= g.n - 1 && b0 + kB <= g.n - 1;
}

// LDS of the encode kernel (one per workgroup, whatever the dimension);
// MAXWR = widest rank planes (block or field scope).
template <int MAXWR>
struct EncSharedT {
  unsigned long long sign[kB], rsign[kB];
  int first[kB], rfirst[kB];
  unsigned lab[kB * 4];
  int wd[kB], wr[kB];
  int pfd[kB + 1], pfr[kB + 1];
  RangeSh rs;
  unsigned wfl[16];  // each wave's error flags
  unsigned hs[16 * 64];  // each wave's 64 slots for the shared-key test
};

using EncShared = EncSharedT<kMaxWRankBlk>;
using EncSharedField = EncSharedT<kMaxWRankAny>;

// Encode modes: ranks within the block; the field-scope mark pass (sort keys
// of the flattened extrema, nothing encoded); encoding with field-scope ranks;
// plain SZp streams (no topology parts: a kernel of its own, so the others
// carry none of its code).
enum { kModeBlock = 0, kModeMark = 1, kModeField = 2, kModePlain = 3 };

// Encodes chunk c of the field of `a` (all WAVES waves of the workgroup).
template <int ND, int WAVES, int MODE = kModeBlock>
__device__ __forceinline__ void encode_body(const EncArgs& a, int c,
                                            EncSharedT<MODE == kModeField ? kMaxWRankAny : kMaxWRankBlk>& sh) {
  constexpr int BPW = kB / WAVES;  // blocks per wave
  constexpr int MAXWR = MODE == kModeField ? kMaxWRankAny : kMaxWRankBlk;
  static_assert(BPW % 4 == 0, "four blocks in flight per wave");
  static_assert(BPW <= 32, "per-wave block masks are 32-bit");
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const GeomD& g = a.gd;
  const float* __restrict__ f = a.f;
  const bool topo = a.topo != 0;
  const int bw = c * kB + wv * BPW;  // this wave's first block
  // each block's planes go to its own staging slot (finalize gathers them)
  const CompLayout L = comp_layout((uint64_t)a.nch, a.field);
  unsigned* stg_d = reinterpret_cast<unsigned*>(a.ws + L.stage_d);
  unsigned* stg_r = reinterpret_cast<unsigned*>(a.ws + L.stage_r);

  // interior blocks of a topology stream in block scope take block_fast
  // (below) when the field is at least 64 wide
  const bool fast_mode = (MODE == kModePlain || topo) && g.nx >= kB;
  // a wave whose blocks read only inside the field loads without clamping
  const bool inner = fast_mode && reads_inside<ND>(bw, g) && reads_inside<ND>(bw + BPW - 1, g);
  const unsigned xoff = lane == 0 ? 0u : 65u;
  const float* __restrict__ pw = f + (size_t)bw * kB;
  // (two versions of the wave loop below, one per kind of load)
  auto fetch_inner = [&](int k) -> EncIn { return enc_fetch_wave<ND>(pw, k, (unsigned)lane, xoff, g); };
  auto fetch_clamped = [&](int k) -> EncIn { return enc_fetch<ND>(f, bw + k, lane, g); };
  // Block k of the wave (lane k computes it) is interior when every point
  // has both y (and z) neighbours; it then lies in one row, or in two
  // consecutive rows of one plane (nx >= 64).  xbm marks interior blocks
  // with a point at x = 0 or x = nx - 1; l0, l1 are the lanes of those
  // points in block k.
  unsigned fastm = 0, xbm = 0;  // bits [0, BPW): at most 16 blocks per wave
  int l0v = 0, l1v = 0;
  if (fast_mode) {
    const int b = bw + (lane < BPW ? lane : 0);
    const int b0 = b * kB, t = fdiv(b0, g.dx), x = b0 - t * g.nx;
    int y = t;
    bool ok = lane < BPW && b < a.nb;
    if (ND == 3) {
      const int z = fdiv(t, g.dy);
      y = t - z * g.ny;
      ok = ok && z >= 1 && z <= g.nz - 2;
    }
    const int xe = x + kB - 1;
    ok = ok && y >= 1 && y + (xe >= g.nx ? 1 : 0) <= g.ny - 2;
    const bool xb = x == 0 || xe >= g.nx - 1;
    if constexpr (MODE == kModePlain) {
      // plain SZp has no x neighbours to mask: its boundary blocks are fast too
      fastm = (unsigned)__ballot(ok);  // lanes >= BPW never set ok
    } else {
      fastm = (unsigned)__ballot(ok && !xb);
      xbm = (unsigned)__ballot(ok && xb);
    }
    l0v = x == 0 ? 0 : g.nx - x;
    l1v = g.nx - 1 - x;
  }

  // The bound of this call, from the whole workgroup (call_bound; every
  // wave calls this exactly once, after its first loads are out).
  float e = 0.0f, inv2e = 0.0f;
  double ed = 0.0;
  unsigned wflag = 0;  // this wave's error flags
  auto get_bound = [&]() {
    float vmin, vmax;
    double eps;
    bool nf;
    call_bound(a.ws, a.eb_mode, a.eb, a.e_abs, a.nrange, sh.rs, &e, &vmin, &vmax, &eps, &nf);
    ed = (double)e;
    inv2e = 1.0f / (2.0f * e);
    wflag = (e >= 0x1p-100f && e <= 0x1p100f) ? 0u : 2u;
  };
  const int n = g.n;
  const unsigned ndeg = (g.nx > 1 ? 1u : 0u) | (g.ny > 1 ? 4u : 0u) | (ND == 3 && g.nz > 1 ? 16u : 0u);
  bool nfm = false, qom = false;  // some lane had a non-finite value, |q| too large
  bool wover = false;

  const unsigned lab_shift = 2u * (unsigned)(lane & 15);
  const unsigned lab_b0 = 1u << lab_shift, lab_b1 = 2u << lab_shift;
  // this wave's slots in the per-block LDS arrays (block k of the wave at
  // index k; the label dword of lanes 16j..16j+15 at 4k + j)
  const int lb0 = wv * BPW;
  int* const wd_w = sh.wd + lb0;
  int* const wr_w = sh.wr + lb0;
  int* const first_w = sh.first + lb0;
  int* const rfirst_w = sh.rfirst + lb0;
  unsigned long long* const sign_w = sh.sign + lb0;
  unsigned long long* const rsign_w = sh.rsign + lb0;
  unsigned* const lab_w = sh.lab + 4 * lb0 + (lane >> 4);
  int wcnt = 0;  // mark pass: entries in this wave's slice
  auto block = [&](const EncIn& in, int b) {
    const int lb = b - c * kB;
    if (b >= a.nb) {  // past the end (last chunk only)
      if (lane == 0) {
        sh.wd[lb] = 0;
        sh.wr[lb] = 0;
      }
      if (lane < 4) sh.lab[4 * lb + lane] = 0;
      return;
    }
    const int b0 = b * kB;
    const int i = b0 + lane;
    // lane masks (bit L = lane L): classification, bins and ranks are
    // decided with one compare per lane and scalar mask algebra
    const unsigned long long vm = n - b0 >= kB ? ~0ull : ((1ull << (n - b0)) - 1ull);
    const float av = in.c;
    nfm |= (__ballot(!isfinite(av)) & vm) != 0;
    int q = quantize(av, inv2e, ed);
    qom |= (__ballot((unsigned)(q + kQMax) > 2u * kQMax) & vm) != 0;
    unsigned long long m_min = 0, m_max = 0, m_sad = 0, lostm = 0;
    if (topo) {
      const float xl = __int_as_float(dpp_from_prev(__float_as_int(av), __float_as_int(in.xe)));
      const float xr = __int_as_float(dpp_from_next(__float_as_int(av), __float_as_int(in.xe)));
      const float nb[6] = {xl, xr, in.ym, in.yp, in.zm, in.zp};
      const Pt pc = coords_of(i, g);
      unsigned long long am[6];  // neighbour j exists
      am[0] = __ballot(pc.x > 0) & vm;
      am[1] = __ballot(pc.x < g.nx - 1) & vm;
      am[2] = __ballot(pc.y > 0) & vm;
      am[3] = __ballot(pc.y < g.ny - 1) & vm;
      am[4] = ND == 3 ? __ballot(pc.z > 0) & vm : 0ull;
      am[5] = ND == 3 ? __ballot(pc.z < g.nz - 1) & vm : 0ull;
      unsigned long long gt[6], lt[6];
#pragma unroll
      for (int j = 0; j < 2 * ND; ++j) {
        gt[j] = __ballot(nb[j] > av) & am[j];
        lt[j] = __ballot(nb[j] < av) & am[j];
      }
      unsigned long long anyn = 0, notgt = 0, notlt = 0, pairs = vm, anybg = 0, anybl = 0;
#pragma unroll
      for (int j = 0; j < 2 * ND; ++j) {
        anyn |= am[j];
        notgt |= am[j] & ~gt[j];
        notlt |= am[j] & ~lt[j];
      }
#pragma unroll
      for (int ax = 0; ax < ND; ++ax) {
        const unsigned long long bg = gt[2 * ax] & gt[2 * ax + 1], bl = lt[2 * ax] & lt[2 * ax + 1];
        anybg |= bg;
        anybl |= bl;
        if ((ndeg >> (2 * ax)) & 1u) pairs &= bg | bl;
      }
      m_min = anyn & ~notgt;
      m_max = anyn & ~notlt;
      m_sad = pairs & anybg & anybl;
      // flattened by plain SZp iff some face neighbour shares the bin:
      // -e <= a_n - 2qe < e, exact in double (see quantize)
      const double c2 = (double)q * (2.0 * ed);
      unsigned long long same = 0;
#pragma unroll
      for (int j = 0; j < 2 * ND; ++j) {
        const double d = (double)nb[j] - c2;
        same |= am[j] & __ballot(d < ed) & __ballot(d >= -ed);
      }
      lostm = (m_min | m_max | m_sad) & same;
    }

    // ranks of flattened extrema among the flattened extrema of the same
    // class and bin in this block: 1 + number less extreme; a flattened
    // saddle gets 1
    int delta = 0;
    if (MODE == kModeMark) {
      // sort key of each flattened extremum: class, bin, then the order in
      // which less extreme values come first; packed into the wave's slice
      const unsigned long long ext = lostm & (m_min | m_max);
      if (ext) {
        const bool ismax = lane_in(m_max);
        const unsigned ord = (unsigned)(ismax ? fkey(av) : -fkey(av)) ^ 0x80000000u;
        const unsigned long long key = ((unsigned long long)(ismax ? 1u : 0u) << 55) |
                                       ((unsigned long long)(unsigned)(q + (1 << 22)) << 32) | ord;
        if (lane_in(ext)) {
          const int pos = wcnt + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(ext >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((unsigned)ext, 0u));
          a.skeys[(size_t)bw * kB + pos] = key;
          a.svals[(size_t)bw * kB + pos] = (unsigned)i;
        }
        wcnt += __popcll(ext);
      }
      return;
    }
    if (MODE == kModeField && topo) {
      // field-scope ranks come from the sorted pass; a flattened saddle gets 1
      const unsigned long long ext = lostm & (m_min | m_max);
      delta = lane_in(ext) ? a.delta[i] : (lane_in(lostm) ? 1 : 0);
    } else if (topo) {
      const unsigned long long ext = lostm & (m_min | m_max);
      int cnt = 0;
      if (ext) {
        const bool ismax = lane_in(m_max);
        const int ck = (q << 1) | (ismax ? 1 : 0);
        const int ok = ismax ? fkey(av) : -fkey(av);
        unsigned long long m = ext;
        while (m) {
          const int j = __ffsll((long long)m) - 1;
          m &= m - 1;
          const int ckj = __builtin_amdgcn_readlane(ck, j);
          const int okj = __builtin_amdgcn_readlane(ok, j);
          cnt += (ck == ckj && okj < ok) ? 1 : 0;
        }
      }
      delta = (lane_in(lostm) ? 1 : 0) + (lane_in(ext) ? cnt : 0);
    }

    // the last block is padded with its last value (residual 0)
    if (vm != ~0ull) {
      const int last = (n - 1) - b0;
      const int ql = __builtin_amdgcn_readlane(q, last);
      const int dl = __builtin_amdgcn_readlane(delta, last);
      if (!lane_in(vm)) {
        q = ql;
        delta = dl;
      }
    }

    unsigned long long sign;
    int first;
    const int w = encode_block<kMaxWData>(q, lane, stg_d + (size_t)b * 2 * kMaxWData, sign, first, wover);
    if (lane == 0) {
      sh.wd[lb] = w;
      sh.sign[lb] = sign;
      sh.first[lb] = first;
    }
    if (topo) {
      // 2-bit labels: point i at byte i/4, bits 2(i%4); 16 points per dword
      int lab = lane_in(m_min) ? CLS_MIN : CLS_R;
      lab = lane_in(m_sad) ? CLS_SAD : lab;
      lab = lane_in(m_max) ? CLS_MAX : lab;
      const unsigned lv = row_or_last((unsigned)lab << lab_shift);
      if ((lane & 15) == 15) sh.lab[4 * lb + (lane >> 4)] = lv;
      unsigned long long rsign;
      int rfirst;
      bool rover = false;
      const int wr = encode_block<MAXWR>(delta, lane, stg_r + (size_t)b * 2 * MAXWR, rsign, rfirst, rover);
      if (lane == 0) {
        sh.wr[lb] = wr;
        sh.rsign[lb] = rsign;
        sh.rfirst[lb] = rfirst;
      }
    } else if (lane == 0) {
      sh.wr[lb] = 0;
    }
  };

  // An interior block (see fast_mode below), in any mode: the same parts
  // (or, in the mark pass, the same sort keys) as `block` with fewer
  // instructions.  The bin index comes from a float
  // estimate t whose exact float edges lo = (2t-1)e and hi = (2t+1)e,
  // rounded up, decide both the point's own bin (t is its bin iff
  // lo <= a < hi) and its neighbours' (a neighbour shares the bin iff it
  // lies in [lo, hi)): for a float x and a real L, x >= L iff x >= the
  // smallest float >= L.  Returns false, having written nothing, when some
  // lane's estimate is off, out of the bin index range or not finite; the
  // caller then runs `block`.
  auto block_fast = [&](const EncIn& in, auto kc, auto xbc, unsigned long long xm0, unsigned long long xm1) -> bool {
    constexpr bool xb = decltype(xbc)::value;
    const int k = kc;  // a compile-time constant in the unrolled loop
    const int b = bw + k;
    const float av = in.c;
    const float t = rintf(av * inv2e);
    float lo, hi;
    mul_round_up2(fmaf(t, 2.0f, -1.0f), fmaf(t, 2.0f, 1.0f), e, lo, hi);
    if (~(__ballot(av >= lo) & __ballot(av < hi) & __ballot(fabsf(t) <= (float)kQMax)) != 0ull) return false;
    const int q = (int)t;
    if constexpr (MODE == kModePlain) {
      // plain SZp: the bin indices' residuals, width and planes only
      const unsigned qb = (unsigned)q ^ 0x80000000u;
      const unsigned pb = (unsigned)dpp_from_prev((int)qb, (int)qb);
      const unsigned md = absdiff_u32(qb, pb);
      const unsigned long long sign = __ballot(qb < pb);
      const unsigned od = wave_or(md);
      const int w = od ? 32 - __builtin_clz(od) : 0;
      if (lane == 0) {
        wd_w[k] = w;
        sign_w[k] = sign;
        first_w[k] = q;
        wr_w[k] = 0;
      }
      put_planes<kMaxWData>(md, w, stg_d + (size_t)b * 2 * kMaxWData, lane);
      return true;
    }
    // classification (Section III-A): strict compares with the face
    // neighbours; the x neighbours come from the adjacent lanes
    const float xl = __int_as_float(dpp_from_prev(__float_as_int(av), __float_as_int(in.xe)));
    const float xr = __int_as_float(dpp_from_next(__float_as_int(av), __float_as_int(in.xe)));
    unsigned long long g0 = __ballot(xl > av), l0 = __ballot(xl < av);
    unsigned long long g1 = __ballot(xr > av), l1 = __ballot(xr < av);
    const unsigned long long g2 = __ballot(in.ym > av), l2 = __ballot(in.ym < av);
    const unsigned long long g3 = __ballot(in.yp > av), l3 = __ballot(in.yp < av);
    // flattened by plain SZp iff some face neighbour lies in [lo, hi)
    unsigned long long sx = (__ballot(xl >= lo) & __ballot(xl < hi)), sx1 = (__ballot(xr >= lo) & __ballot(xr < hi));
    unsigned long long same = (__ballot(in.ym >= lo) & __ballot(in.ym < hi)) |
                              (__ballot(in.yp >= lo) & __ballot(in.yp < hi));
    unsigned long long m_min, m_max;
    if constexpr (xb) {
      // a lane at x = 0 has no x- neighbour, one at x = nx - 1 no x+
      // neighbour: extrema ignore it, a saddle needs the pair complete
      g0 &= xm0;
      l0 &= xm0;
      g1 &= xm1;
      l1 &= xm1;
      sx &= xm0;
      sx1 &= xm1;
      m_min = (g0 | ~xm0) & (g1 | ~xm1);
      m_max = (l0 | ~xm0) & (l1 | ~xm1);
    } else {
      m_min = g0 & g1;
      m_max = l0 & l1;
    }
    same |= sx | sx1;
    const unsigned long long bgx = g0 & g1, blx = l0 & l1, bgy = g2 & g3, bly = l2 & l3;
    m_min &= bgy;
    m_max &= bly;
    unsigned long long m_sad;
    if (ND == 3) {
      const unsigned long long g4 = __ballot(in.zm > av), l4 = __ballot(in.zm < av);
      const unsigned long long g5 = __ballot(in.zp > av), l5 = __ballot(in.zp < av);
      const unsigned long long bgz = g4 & g5, blz = l4 & l5;
      m_min &= bgz;
      m_max &= blz;
      m_sad = (bgx | blx) & (bgy | bly) & (bgz | blz) & (bgx | bgy | bgz) & (blx | bly | blz);
      same |= (__ballot(in.zm >= lo) & __ballot(in.zm < hi)) | (__ballot(in.zp >= lo) & __ballot(in.zp < hi));
    } else {
      m_sad = (bgx & bly) | (blx & bgy);
    }
    const unsigned long long lostm = (m_min | m_max | m_sad) & same;
    const unsigned long long ext = lostm & (m_min | m_max);
    if constexpr (MODE == kModeMark) {
      // the sort keys of the flattened extrema, as in `block`
      if (ext) {
        const bool ismax = lane_in(m_max);
        const unsigned ord = (unsigned)(ismax ? fkey(av) : -fkey(av)) ^ 0x80000000u;
        const unsigned long long key = ((unsigned long long)(ismax ? 1u : 0u) << 55) |
                                       ((unsigned long long)(unsigned)(q + (1 << 22)) << 32) | ord;
        if (lane_in(ext)) {
          const int pos = wcnt + (int)mbcnt(ext);
          a.skeys[(size_t)bw * kB + pos] = key;
          a.svals[(size_t)bw * kB + pos] = (unsigned)(b * kB + lane);
        }
        wcnt += __popcll(ext);
      }
      return true;
    }
    // ranks (Section IV-A (2)): in field scope from the sorted pass (a
    // flattened saddle gets 1); in block scope as in `block`, where with at
    // most one flattened extremum per (class, bin) every rank is 1, the
    // common case, so the pairwise count runs only when two of them share a
    // bin and class
    int cnt = 0;
    if (MODE == kModeBlock && ND == 3 && (ext & (ext - 1))) {
      // (3D: the pairwise count over all of them once any two share a bin
      // and class; the kernel is at its register limit, and the 2D form
      // below costs it more than it saves)
      const int ck = (q << 1) | (lane_in(m_max) ? 1 : 0);
      unsigned shared = 0;
      unsigned long long m = ext;
      while (m) {
        const unsigned long long grp = __ballot(ck == __builtin_amdgcn_readlane(ck, __ffsll((long long)m) - 1)) & ext;
        m &= ~grp;
        shared |= __popcll(grp) - 1;
      }
      if (shared) {
        const int ok = lane_in(m_max) ? fkey(av) : -fkey(av);
        unsigned long long mm = ext;
        while (mm) {
          const int j = __ffsll((long long)mm) - 1;
          mm &= mm - 1;
          const int ckj = __builtin_amdgcn_readlane(ck, j);
          const int okj = __builtin_amdgcn_readlane(ok, j);
          cnt += (ck == ckj && okj < ok) ? 1 : 0;
        }
      }
    }
    if (MODE == kModeBlock && ND == 2 && (ext & (ext - 1))) {
      // the (class, bin) groups one at a time; only the members of a group
      // of two or more compare their order keys, and only with each other
      const int ck = (q << 1) | (lane_in(m_max) ? 1 : 0);
      // two flattened extrema of one (class, bin) land on one of the wave's
      // 64 LDS slots (the key's low bits): each writes its lane there, and
      // one of them then reads back another lane; without such a clash the
      // keys are distinct and every count is 0
      volatile __attribute__((address_space(3))) unsigned* const hs =
          (volatile __attribute__((address_space(3))) unsigned*)(sh.hs + wv * 64 + (ck & 63));
      bool clash = false;
      if (lane_in(ext)) {
        *hs = (unsigned)lane;
        clash = *hs != (unsigned)lane;
      }
      const int ok = lane_in(m_max) ? fkey(av) : -fkey(av);
      unsigned long long m = __ballot(clash) ? ext : 0ull;
      while (m) {
        const unsigned long long grp = __ballot(ck == __builtin_amdgcn_readlane(ck, __ffsll((long long)m) - 1)) & ext;
        m &= ~grp;
        if ((grp & (grp - 1)) && lane_in(grp)) {
          unsigned long long mm = grp;
          while (mm) {
            const int j = __ffsll((long long)mm) - 1;
            mm &= ~(1ull << j);
            cnt += __builtin_amdgcn_readlane(ok, j) < ok ? 1 : 0;
          }
        }
      }
    }
    const int delta = MODE == kModeField ? (lane_in(ext) ? a.delta[b * kB + lane] : (lane_in(lostm) ? 1 : 0))
                                         : (lane_in(lostm) ? 1 : 0) + (lane_in(ext) ? cnt : 0);
    // B + LZ (residual i = v_i - v_{i-1}, residual 0 = 0) and BE of the bin
    // indices (offset by 2^31 so that unsigned order is signed order) and of
    // the ranks; one OR over the wave gives both widths (data below bit 24,
    // ranks of at most 7 bits above)
    const unsigned qb = (unsigned)q ^ 0x80000000u;
    const unsigned pb = (unsigned)dpp_from_prev((int)qb, (int)qb);
    const unsigned md = absdiff_u32(qb, pb);
    const unsigned long long sign = __ballot(qb < pb);
    const unsigned ud = (unsigned)delta;
    const unsigned pr = (unsigned)dpp_from_prev((int)ud, (int)ud);
    const unsigned mr = absdiff_u32(ud, pr);
    const unsigned long long rsign = __ballot(ud < pr);
    // (field-scope ranks may take all 31 bits: two ORs there)
    const unsigned o = MODE == kModeField ? 0u : wave_or(md | (mr << 24));
    const unsigned od = MODE == kModeField ? wave_or(md) : o & 0xFFFFFFu;
    const unsigned orr = MODE == kModeField ? wave_or(mr) : o >> 24;
    const int w = od ? 32 - __builtin_clz(od) : 0;
    const int wr = orr ? 32 - __builtin_clz(orr) : 0;
    // 2-bit labels (Section IV-A (1)), 16 points per dword: bit 0 marks an
    // extremum, bit 1 a saddle or maximum (m=01, s=10, M=11).  The labels
    // and the block's fixed-size parts go out before the planes, so that no
    // classification mask stays live across the plane runs.
    const unsigned lv = row_or_last((lane_in(m_min | m_max) ? lab_b0 : 0u) | (lane_in(m_sad | m_max) ? lab_b1 : 0u));
    if ((lane & 15) == 15) lab_w[4 * k] = lv;
    // lane 0 holds the block's first value and first rank
    if (lane == 0) {
      wd_w[k] = w;
      sign_w[k] = sign;
      first_w[k] = q;
      wr_w[k] = wr;
      rsign_w[k] = rsign;
      rfirst_w[k] = delta;
    }
    put_planes<kMaxWData>(md, w, stg_d + (size_t)b * 2 * kMaxWData, lane);
    put_planes<MAXWR>(mr, wr, stg_r + (size_t)b * 2 * MAXWR, lane);
    return true;
  };

  if (fast_mode) {
    // the wave's blocks with four in flight; blocks that are not interior,
    // those at an x boundary and those whose fast attempt fails are left in
    // `todo` for a second pass (inlining the x-boundary case here measures
    // slower: it costs registers and so occupancy)
    constexpr int kDepth = 4;  // blocks in flight
    unsigned todo = (1u << BPW) - 1u;
    auto wave_loop = [&](auto fetch) {
      EncIn P[kDepth];
      unroll<0, kDepth>([&](auto kc) { P[kc.value] = fetch(kc.value); });
      // (a barrier: each wave of the workgroup reaches it once, whichever
      // version of this loop it runs)
      get_bound();
      unroll<0, BPW>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        const EncIn& in = P[k % kDepth];
        if ((fastm >> k) & 1u) {
          if (block_fast(in, kc, std::false_type{}, ~0ull, ~0ull)) todo &= ~(1u << k);
        }
        if constexpr (k + kDepth < BPW) P[k % kDepth] = fetch(k + kDepth);
      });
    };
    if (inner)
      wave_loop(fetch_inner);
    else
      wave_loop(fetch_clamped);
    while (todo) {
      const int k = __ffs((int)todo) - 1;
      todo &= todo - 1;
      const EncIn in = enc_fetch<ND>(f, bw + k, lane, g);
      if ((xbm >> k) & 1u) {
        const int l0 = __builtin_amdgcn_readlane(l0v, k), l1 = __builtin_amdgcn_readlane(l1v, k);
        const unsigned long long xm0 = l0 < kB ? ~(1ull << l0) : ~0ull, xm1 = l1 < kB ? ~(1ull << l1) : ~0ull;
        if (block_fast(in, k, std::true_type{}, xm0, xm1)) continue;
      }
      block(in, bw + k);
    }
  } else {
    // four blocks in flight per wave: each buffer is refilled as soon as its
    // block has been encoded (the last refills repeat the wave's last block)
    const int blast = bw + BPW - 1;
    EncIn P0 = fetch_clamped(0), P1 = fetch_clamped(1), P2 = fetch_clamped(2), P3 = fetch_clamped(3);
    get_bound();
    for (int k = 0; k < BPW; k += 4) {
      block(P0, bw + k);
      P0 = enc_fetch<ND>(f, min(bw + k + 4, blast), lane, g);
      block(P1, bw + k + 1);
      P1 = enc_fetch<ND>(f, min(bw + k + 5, blast), lane, g);
      block(P2, bw + k + 2);
      P2 = enc_fetch<ND>(f, min(bw + k + 6, blast), lane, g);
      block(P3, bw + k + 3);
      P3 = enc_fetch<ND>(f, min(bw + k + 7, blast), lane, g);
    }
  }
  if (MODE == kModeMark) {
    // the chunk's keys, compacted at the start of its own region of the
    // arrays (its first point's index): each wave copies its slice after the
    // slices of the waves before it, and the chunk's count goes out for the
    // scan.  Errors are the encode pass's.
    if (lane == 0) sh.pfd[wv] = wcnt;
    __syncthreads();
    if (tid == 0) {
      int tot = 0;
      for (int w = 0; w < WAVES; ++w) tot += sh.pfd[w];
      a.ccnt[c] = (unsigned)tot;
    }
    int off = c * kChunk;
    for (int w = 0; w < wv; ++w) off += sh.pfd[w];
    const size_t sb = (size_t)bw * kB;
    for (int j = lane; j < wcnt; j += 64) {
      a.keys[off + j] = a.skeys[sb + j];
      a.vals[off + j] = a.svals[sb + j];
    }
    return;
  }
  {
    const bool nf = nfm, qo = qom || wover;
    if (lane == 0) sh.wfl[wv] = wflag | (nf ? 1u : 0u) | (qo ? 4u : 0u);
  }
  // this wave's blocks' fixed-size parts, from its own LDS slots (written
  // by lane 0 and by the label lanes above; the fences keep the reads after
  // those writes): widths, signs and first values by lanes [0, BPW) for the
  // data and [BPW, 2 BPW) for the ranks, then the labels, 4 dwords per block
  uint8_t* out = a.out;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  {
    const int k = lane % BPW, b = bw + k;
    if (b < a.nb) {
      if (lane < BPW) {
        out[a.off[S2] + b] = (uint8_t)wd_w[k];
        *reinterpret_cast<unsigned long long*>(out + a.off[S3] + 8 * (size_t)b) = sign_w[k];
        *reinterpret_cast<int*>(out + a.off[S4] + 4 * (size_t)b) = first_w[k];
      } else if (lane < 2 * BPW && topo) {
        out[a.off[R2] + b] = (uint8_t)wr_w[k];
        *reinterpret_cast<unsigned long long*>(out + a.off[R3] + 8 * (size_t)b) = rsign_w[k];
        *reinterpret_cast<int*>(out + a.off[R4] + 4 * (size_t)b) = rfirst_w[k];
      }
    }
    static_assert(4 * BPW <= 64, "one label dword per lane");
    if (topo && lane < 4 * BPW && bw + (lane >> 2) < a.nb)
      *reinterpret_cast<unsigned*>(out + a.off[S6] + 16 * (size_t)bw + 4 * (size_t)lane) = sh.lab[4 * lb0 + lane];
  }
  __syncthreads();

  // chunk: constant-block bitmaps and plane totals
  if (wv == 0) {
    const int b = c * kB + lane;
    const bool bv = b < a.nb;
    const int wd = sh.wd[lane], wr = sh.wr[lane];
    const unsigned long long cb = __ballot(bv && wd == 0), cr = __ballot(bv && wr == 0);
    const int sd = wave_incl_scan(wd, lane), sr = wave_incl_scan(wr, lane);
    if (lane == 0) {
      *reinterpret_cast<unsigned long long*>(out + a.off[S1] + 8 * (size_t)c) = cb;
      if (topo) *reinterpret_cast<unsigned long long*>(out + a.off[R1] + 8 * (size_t)c) = cr;
    }
    if (lane == 63) {
      reinterpret_cast<unsigned*>(a.ws + L.tot_d)[c] = (unsigned)sd;
      reinterpret_cast<unsigned*>(a.ws + L.tot_r)[c] = (unsigned)sr;
      unsigned fl = 0;
      for (int w = 0; w < WAVES; ++w) fl |= sh.wfl[w];
      reinterpret_cast<unsigned*>(a.ws + L.cflag)[c] = fl;
    }
  }

  // the last chunk zeroes the alignment gaps between the fixed-size parts
  if (c == a.nch - 1 && tid < 8 * (X2 + 1)) {
    const int s = tid >> 3, k = tid & 7;
    const uint64_t end = a.off[s] + a.len[s];
    if (end + k < a.off[s + 1]) a.out[end + k] = 0;
  }
}

// At most 80 SGPRs and 64 VGPRs: eight waves per SIMD, so a CU holds four
// eight-wave workgroups (measured: with 94 SGPRs it holds three, and the 3D
// instance at 84 VGPRs two), at the cost of a few values kept in VGPR lanes.
template <int ND, int WAVES, int MODE = kModeBlock>
__global__ __launch_bounds__(WAVES * 64) __attribute__((amdgpu_num_sgpr(80), amdgpu_waves_per_eu(8, 8))) void
encode_kernel(EncArgs a) {
  __shared__ EncSharedT<MODE == kModeField ? kMaxWRankAny : kMaxWRankBlk> sh;
  const int c = xcd_chunk(blockIdx.x, a.nch);
  if (c < a.nch) encode_body<ND, WAVES, MODE>(a, c, sh);
}

// Clears the field-scope mark counter ahead of the mark pass.
// Field-scope ranks (Section IV-A (2) read field-wide): the flattened extrema
// of the whole field are put in the order of their sort keys (class, bin,
// then less extreme first) by a merge sort whose every size is read on the
// device, so the call never waits for the host.  Each chunk's keys are sorted
// in LDS into a run; runs of 2^L chunks are then merged pairwise, each key
// finding its place in the merged run by one binary search in the other
// run.

// One workgroup per chunk: its m keys (at most one per point) into LDS, each
// placed by the count of keys before it (smaller, or equal with a smaller
// index), and written as the chunk's sorted run at coff[c], the keys of the
// chunks before it, which the workgroup sums itself (coff[nch] = all keys,
// from the last chunk).
constexpr int kFsThreads = 256;
__global__ __launch_bounds__(kFsThreads) void fs_sort_kernel(const unsigned long long* __restrict__ keys,
                                                             const unsigned* __restrict__ vals,
                                                             const unsigned* __restrict__ ccnt, unsigned* coff,
                                                             int nch, uint8_t* ws, unsigned long long* okeys,
                                                             unsigned* ovals) {
  __shared__ unsigned long long s_k[kChunk];
  __shared__ unsigned s_part[kFsThreads / 64];
  const int c = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  const int m = (int)ccnt[c];
  const size_t src = (size_t)c * kChunk;
  for (int e = tid; e < m; e += kFsThreads) s_k[e] = keys[src + e];
  unsigned part = 0;
  for (int j = tid; j < c; j += kFsThreads) part += ccnt[j];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) part += (unsigned)__shfl_xor((int)part, o);
  if (lane == 0) s_part[tid >> 6] = part;
  __syncthreads();
  unsigned base = 0;
#pragma unroll
  for (int w = 0; w < kFsThreads / 64; ++w) base += s_part[w];
  if (tid == 0) {
    coff[c] = base;
    if (c == nch - 1) {
      coff[nch] = base + (unsigned)m;
      ctrl_of(ws)->fs_count = base + (unsigned)m;
    }
  }
  for (int e = tid; e < m; e += kFsThreads) {
    const unsigned long long k = s_k[e];
    int pos = 0;
    for (int j = 0; j < m; ++j) {
      const unsigned long long kj = s_k[j];
      pos += (kj < k || (kj == k && j < e)) ? 1 : 0;
    }
    okeys[base + pos] = k;
    ovals[base + pos] = vals[src + e];
  }
}

// First index in [lo, hi) whose key is >= k (UPPER: > k).
template <bool UPPER>
__device__ __forceinline__ unsigned fs_bound(const unsigned long long* __restrict__ keys, unsigned lo, unsigned hi,
                                             unsigned long long k) {
  while (lo < hi) {
    const unsigned mid = (lo + hi) >> 1;
    const unsigned long long km = keys[mid];
    if (UPPER ? km <= k : km < k) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Merge pass L: the four runs of chunks [b0 + r 4^L, b0 + (r+1) 4^L),
// r = 0..3, b0 a multiple of 4^(L+1), become one run.  A key of run r goes
// after the smaller or equal keys of the runs before it and the smaller keys
// of the runs after it, so equal keys keep their order; its three searches
// are independent.  A key's run follows from the chunk it came from, its
// point index / kChunk: merging only moves keys within their run.
__global__ __launch_bounds__(256) void fs_merge_kernel(const unsigned long long* __restrict__ keys,
                                                       const unsigned* __restrict__ vals,
                                                       const unsigned* __restrict__ coff, int nch, int L,
                                                       unsigned long long* okeys, unsigned* ovals) {
  const unsigned total = coff[nch];
  for (unsigned i = blockIdx.x * 256u + threadIdx.x; i < total; i += gridDim.x * 256u) {
    const unsigned v = vals[i];
    const int c = (int)(v / (unsigned)kChunk);
    const int b0 = (c >> (2 * L + 2)) << (2 * L + 2);
    unsigned S[5];
#pragma unroll
    for (int r = 0; r <= 4; ++r) S[r] = coff[min(b0 + (r << (2 * L)), nch)];
    const int own = (c - b0) >> (2 * L);  // 0..3
    const unsigned long long k = keys[i];
    unsigned pos = i - S[own];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (r < own) pos += fs_bound<true>(keys, S[r], S[r + 1], k) - S[r];
      else if (r > own) pos += fs_bound<false>(keys, S[r], S[r + 1], k) - S[r];
    }
    okeys[S[0] + pos] = k;
    ovals[S[0] + pos] = v;
  }
}

// Merge pass L as fs_merge_kernel, with one workgroup per group of four
// runs and the group's keys staged in LDS, so the searches read LDS.  For
// the low levels, where groups are many and small; a group larger than the
// staging area searches its keys in global memory.
constexpr int kFsMergeCap = 8192;
__global__ __launch_bounds__(1024) void fs_merge_lds_kernel(const unsigned long long* __restrict__ keys,
                                                            const unsigned* __restrict__ vals,
                                                            const unsigned* __restrict__ coff, int nch, int L,
                                                            unsigned long long* okeys, unsigned* ovals) {
  __shared__ unsigned long long s_k[kFsMergeCap];
  const long long b0l = (long long)blockIdx.x << (2 * L + 2);
  if (b0l >= nch) return;
  const int b0 = (int)b0l;
  unsigned S[5];
#pragma unroll
  for (int r = 0; r <= 4; ++r) S[r] = coff[(int)min((long long)b0 + ((long long)r << (2 * L)), (long long)nch)];
  const unsigned m = S[4] - S[0];
  unsigned R[5];
#pragma unroll
  for (int r = 0; r <= 4; ++r) R[r] = S[r] - S[0];
  const unsigned long long* gk = keys + S[0];
  // the position of key e (run own) in the merged group, searching in `src`
  auto place = [&](const unsigned long long* src, unsigned e, unsigned long long k) {
    const int own = (e >= R[1] ? 1 : 0) + (e >= R[2] ? 1 : 0) + (e >= R[3] ? 1 : 0);
    unsigned pos = e - R[own];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (r < own) pos += fs_bound<true>(src, R[r], R[r + 1], k) - R[r];
      else if (r > own) pos += fs_bound<false>(src, R[r], R[r + 1], k) - R[r];
    }
    return pos;
  };
  if (m <= (unsigned)kFsMergeCap) {
    for (unsigned e = threadIdx.x; e < m; e += blockDim.x) s_k[e] = gk[e];
    __syncthreads();
    for (unsigned e = threadIdx.x; e < m; e += blockDim.x) {
      const unsigned long long k = s_k[e];
      const unsigned pos = place(s_k, e, k);
      okeys[S[0] + pos] = k;
      ovals[S[0] + pos] = vals[S[0] + e];
    }
  } else {
    for (unsigned e = threadIdx.x; e < m; e += blockDim.x) {
      const unsigned long long k = gk[e];
      const unsigned pos = place(gk, e, k);
      okeys[S[0] + pos] = k;
      ovals[S[0] + pos] = vals[S[0] + e];
    }
  }
}

// The first index j <= i whose key is >= k (keys sorted, keys[i] >= k), by
// galloping back from i: steps of 1, 2, 4, ... until a key below k (or
// index 0), then a binary search in the last step.  The cost follows the
// distance to the answer (a group or a tie run), not the array's size.
__device__ __forceinline__ unsigned fs_back(const unsigned long long* __restrict__ keys, unsigned i,
                                            unsigned long long k) {
  unsigned hi = i, step = 1;  // keys[hi] >= k
  unsigned lo = 0;            // lower bound of the search, once a key below k is found
  while (hi > 0) {
    const unsigned j = hi > step ? hi - step : 0;
    if (keys[j] < k) {
      lo = j + 1;
      break;
    }
    hi = j;
    step <<= 1;
  }
  return fs_bound<false>(keys, lo, hi, k);
}

// Field-scope ranks from the sorted keys: a flattened extremum's rank is 1 +
// the number of entries of its (class, bin) group sorted before its value
// (ties share a rank).  Both starts are lower bounds in the sorted prefix.
__global__ __launch_bounds__(256) void fs_rank_kernel(const unsigned long long* __restrict__ keys,
                                                      const unsigned* __restrict__ vals,
                                                      const unsigned* __restrict__ coff, int nch, int* delta) {
  const unsigned n = coff[nch];
  for (unsigned i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) {
    const unsigned long long k = keys[i];
    const unsigned long long gk = k & ~0xFFFFFFFFull;
    const unsigned g0 = fs_back(keys, i, gk);
    const unsigned t0 = fs_back(keys, i, k);
    delta[vals[i]] = (int)(1 + t0 - g0);
  }
}

// Exclusive scan of the chunk plane totals (in place), flags, and the bound.
__device__ __forceinline__ void scan_body(const ScanArgs& a) {
  __shared__ unsigned long long s_w[2][16];
  __shared__ unsigned long long s_carry[2];
  __shared__ unsigned s_fl;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const CompLayout L = comp_layout((uint64_t)a.nch, a.field);
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
  {
    __shared__ RangeSh s_rs;
    float e, vmin, vmax;
    double eps;
    bool nf;
    call_bound(a.ws, a.eb_mode, a.eb, a.e_abs, a.nrange, s_rs, &e, &vmin, &vmax, &eps, &nf);
    if (tid == 0) {
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

__global__ __launch_bounds__(1024) void scan_kernel(ScanArgs a) { scan_body(a); }

// ---------------------------------------------------------------------------
// Finalize: payload placement, chunk index, header, status.

__device__ void put8(uint8_t* h, int off, uint64_t v) { memcpy(h + off, &v, 8); }
__device__ void put4(uint8_t* h, int off, uint32_t v) { memcpy(h + off, &v, 4); }
__device__ void put2(uint8_t* h, int off, uint16_t v) { memcpy(h + off, &v, 2); }

// Places chunk c's staged planes; chunk 0 also writes the header.
__device__ __forceinline__ void finalize_body(const FinArgs& a, int c) {
  __shared__ uint8_t hdr[kHdr];
  __shared__ uint64_t s_seg[2 * kNSeg];
  __shared__ unsigned s_sa[4], s_sb[4];
  __shared__ unsigned s_red[5][4];
  __shared__ unsigned s_flags;
  __shared__ float s_e, s_vmin, s_vmax;
  __shared__ double s_eps;
  Ctrl* ct = ctrl_of(a.ws);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // the first chunk's workgroup (dispatched first) also writes the header,
  // so that its longer chain overlaps the other chunks' copies
  const bool head = c == 0;
  const CompLayout L = comp_layout((uint64_t)a.nch, a.field);
  const unsigned* td = reinterpret_cast<const unsigned*>(a.ws + L.tot_d);
  const unsigned* tr = reinterpret_cast<const unsigned*>(a.ws + L.tot_r);
  const unsigned* cf = reinterpret_cast<const unsigned*>(a.ws + L.cflag);
  uint64_t b0, r0, nd, nr, totd, totr;
  if (a.fused) {
    // td/tr hold per-chunk plane counts: every workgroup sums its
    // predecessors' (its offsets) and everybody's (the rank planes follow
    // all data planes); the header's workgroup also gathers the flags
    // (four chunks per 16-byte load; the arrays are padded to 16 bytes)
    unsigned pd = 0, pr = 0, ad = 0, ar = 0, fl = 0;
    const uint4* td4 = reinterpret_cast<const uint4*>(td);
    const uint4* tr4 = reinterpret_cast<const uint4*>(tr);
    const uint4* cf4 = reinterpret_cast<const uint4*>(cf);
    const int n4 = (a.nch + 3) >> 2;
    for (int j4 = tid; j4 < n4; j4 += 256) {
      const uint4 vd = td4[j4], vr = tr4[j4];
      const uint4 vf = head ? cf4[j4] : make_uint4(0u, 0u, 0u, 0u);
      const unsigned d[4] = {vd.x, vd.y, vd.z, vd.w}, r[4] = {vr.x, vr.y, vr.z, vr.w};
      const unsigned f[4] = {vf.x, vf.y, vf.z, vf.w};
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int j = 4 * j4 + t;
        if (j < a.nch) {
          ad += d[t];
          ar += r[t];
          fl |= f[t];
          if (j < c) {
            pd += d[t];
            pr += r[t];
          }
        }
      }
    }
    pd = wave_sum(pd);
    pr = wave_sum(pr);
    ad = wave_sum(ad);
    ar = wave_sum(ar);
    fl = wave_or(fl);
    if (lane == 0) {
      s_red[0][wv] = pd;
      s_red[1][wv] = pr;
      s_red[2][wv] = ad;
      s_red[3][wv] = ar;
      s_red[4][wv] = fl;
    }
    if (head) {
      __shared__ RangeSh s_rs;
      float e, vmin, vmax;
      double eps;
      bool nf;
      call_bound(a.ws, a.eb_mode, a.eb, a.e_abs, a.nrange, s_rs, &e, &vmin, &vmax, &eps, &nf);
      if (tid == 0) {
        s_e = e;
        s_vmin = vmin;
        s_vmax = vmax;
        s_eps = eps;
        s_flags = (nf ? 1u : 0u) | ((e >= 0x1p-100f && e <= 0x1p100f) ? 0u : 2u);
      }
    }
    __syncthreads();
    b0 = (uint64_t)s_red[0][0] + s_red[0][1] + s_red[0][2] + s_red[0][3];
    r0 = (uint64_t)s_red[1][0] + s_red[1][1] + s_red[1][2] + s_red[1][3];
    totd = (uint64_t)s_red[2][0] + s_red[2][1] + s_red[2][2] + s_red[2][3];
    totr = (uint64_t)s_red[3][0] + s_red[3][1] + s_red[3][2] + s_red[3][3];
    nd = td[c];
    nr = tr[c];
    if (head && tid == 0) s_flags |= s_red[4][0] | s_red[4][1] | s_red[4][2] | s_red[4][3];
  } else {
    // td/tr hold exclusive prefixes, the control block the totals
    totd = ct->tot_data;
    totr = ct->tot_rank;
    b0 = td[c];
    nd = (c + 1 < a.nch ? (uint64_t)td[c + 1] : totd) - b0;
    r0 = tr[c];
    nr = (c + 1 < a.nch ? (uint64_t)tr[c + 1] : totr) - r0;
    if (head && tid == 0) {
      s_flags = ct->cflags;
      s_e = ct->e;
      s_vmin = ct->vmin;
      s_vmax = ct->vmax;
      s_eps = ct->eps;
    }
  }
  if (!a.topo) totr = 0;
  {
    // each block's planes sit at the start of its staging slot: the chunk's
    // widths (S2, R2, written by encode) give every block's position in the
    // chunk's run; four threads copy each block
    __shared__ int s_bd[kB + 1], s_br[kB + 1];
    if (wv == 0) {
      const uint64_t bb = (uint64_t)c * kB + lane;
      const bool bv = bb < (uint64_t)a.nb;
      const int wd = bv ? a.out[a.off[S2] + bb] : 0;
      const int wr = (bv && a.topo) ? a.out[a.off[R2] + bb] : 0;
      s_bd[lane + 1] = wave_incl_scan(wd, lane);
      s_br[lane + 1] = wave_incl_scan(wr, lane);
      if (lane == 0) {
        s_bd[0] = 0;
        s_br[0] = 0;
      }
    }
    __syncthreads();
    const int lb = tid >> 2, q4 = tid & 3;
    const int rw = rank_w(a.field);
    const uint64_t* src = reinterpret_cast<const uint64_t*>(a.ws + L.stage_d) + ((size_t)c * kB + lb) * kMaxWData;
    uint64_t* dst = reinterpret_cast<uint64_t*>(a.out + a.off[S5]) + b0 + s_bd[lb];
    for (int j = q4; j < s_bd[lb + 1] - s_bd[lb]; j += 4) dst[j] = src[j];
    if (tid == 0) *reinterpret_cast<uint64_t*>(a.out + a.off[X1] + 8 * (size_t)c) = 8 * b0;
    if (a.topo) {
      const uint64_t* rsrc = reinterpret_cast<const uint64_t*>(a.ws + L.stage_r) + ((size_t)c * kB + lb) * rw;
      uint64_t* rdst = reinterpret_cast<uint64_t*>(a.out + a.off[S5] + 8 * totd) + r0 + s_br[lb];
      for (int j = q4; j < s_br[lb + 1] - s_br[lb]; j += 4) rdst[j] = rsrc[j];
      if (tid == 0) *reinterpret_cast<uint64_t*>(a.out + a.off[X2] + 8 * (size_t)c) = 8 * r0;
    }
    (void)nd;
    (void)nr;
  }
  if (!head) return;
  __syncthreads();

  const unsigned flags = s_flags;
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
    // the segment table goes through LDS (registers would hold 26 words)
    uint64_t* off = s_seg;
    uint64_t* len = s_seg + kNSeg;
    const uint64_t total = seg_layout((uint64_t)a.nb, a.topo, totd, totr, off, len);
    hdr[0] = 'T'; hdr[1] = 'S'; hdr[2] = 'Z'; hdr[3] = '1';
    put2(hdr, 4, 1);
    hdr[6] = (uint8_t)a.g.ndim;
    hdr[7] = (uint8_t)((a.topo ? 1 : 0) | (a.field ? 2 : 0));
    for (int d = 0; d < 3; ++d) put8(hdr, 8 + 8 * d, a.dims[d]);
    put8(hdr, 32, (uint64_t)a.g.n);
    put8(hdr, 40, (uint64_t)a.nb);
    put4(hdr, 48, kB);
    hdr[52] = (uint8_t)a.eb_mode;
    hdr[53] = (uint8_t)k;
    put2(hdr, 54, (uint16_t)a.max_rounds);
    uint64_t u;
    memcpy(&u, &a.eb, 8); put8(hdr, 56, u);
    memcpy(&u, &s_eps, 8); put8(hdr, 64, u);
    uint32_t v;
    memcpy(&v, &s_e, 4); put4(hdr, 72, v);
    memcpy(&v, &s_vmin, 4); put4(hdr, 76, v);
    memcpy(&v, &s_vmax, 4); put4(hdr, 80, v);
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

__global__ __launch_bounds__(256) void finalize_kernel(FinArgs a) {
  const int c = xcd_chunk(blockIdx.x, a.nch);  // same XCD as the chunk's encode
  if (c < a.nch) finalize_body(a, c);
}

// ---------------------------------------------------------------------------
// Decompression.

struct Hdr {
  int ok, ndim, topo, scope, k, max_rounds;
  uint64_t dims[3], n, nb, nch, total, wdata, wrank;
  float e, w[10];
  uint64_t off[kNSeg], len[kNSeg];
};


// Header checks (one wave): the header is copied to LDS in parallel, then
// lane 0 checks the checksum, field ranges and the segment table against the
// layout rule.  Result in *h: ok = 0 corrupt, -1 capacity, 1 good.
// Lane l's 8 header bytes [8l, 8l + 8), read from any lane.
__device__ __forceinline__ uint64_t hdr_word(uint64_t w, int l) {
  return (uint64_t)(unsigned)__builtin_amdgcn_readlane((int)(unsigned)w, l) |
         (uint64_t)(unsigned)__builtin_amdgcn_readlane((int)(unsigned)(w >> 32), l) << 32;
}

// Parses and checks the 512-byte header (one wave; lane 0 writes *h).  Each
// lane loads 8 bytes; every field is then read from the lanes' registers, so
// the checks wait on no memory.
__device__ __forceinline__ void parse_header(const uint8_t* in, uint64_t in_size, uint64_t out_cap, Hdr* h,
                                             int lane) {
  const bool good = in_size >= (uint64_t)kHdr;
  unsigned sa = 0, sb = 0;
  uint64_t w = 0;
  if (good) {
    w = *reinterpret_cast<const uint64_t*>(in + 8 * lane);
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
  if (lane != 0) return;
  h->ok = 0;
  if (!good) return;
  // Adler-32 of bytes [0, kSummed): sa <= 376 * 255 and sb < 2^25, so 32 bits hold both sums
  const uint32_t adler = (((unsigned)kSummed + sb) % 65521u) << 16 | ((1u + sa) % 65521u);
  const uint64_t w0 = hdr_word(w, 0);
  if ((uint32_t)w0 != 0x315A5354u) return;  // "TSZ1"
  if (((w0 >> 32) & 0xFFFFu) != 1) return;
  const uint64_t w47 = hdr_word(w, kSummed / 8);
  if ((uint32_t)w47 != adler || (uint32_t)(w47 >> 32) != 0) return;
  h->ndim = (int)((w0 >> 48) & 0xFFu);
  if (h->ndim != 2 && h->ndim != 3) return;
  const unsigned flags = (unsigned)(w0 >> 56);
  if (flags & ~3u) return;
  h->topo = flags & 1;
  h->scope = (flags >> 1) & 1;
  uint64_t prod = 1;
  for (int d = 0; d < 3; ++d) {
    h->dims[d] = hdr_word(w, 1 + d);
    if (h->dims[d] < 1 || h->dims[d] > (1ull << 31)) return;
    if (d >= h->ndim && h->dims[d] != 1) return;
    prod *= h->dims[d];
    if (prod >= (1ull << 31)) return;
  }
  h->n = hdr_word(w, 4);
  h->nb = hdr_word(w, 5);
  h->nch = hdr_word(w, 19);
  if (h->n != prod || h->nb != (h->n + kB - 1) / kB || h->nch != (h->nb + kB - 1) / kB) return;
  const uint64_t w6 = hdr_word(w, 6);  // block (48), eb mode (52), k (53), rounds (54)
  if ((uint32_t)w6 != (uint32_t)kB) return;
  h->k = (int)((w6 >> 40) & 0xFFu);
  h->max_rounds = (int)(w6 >> 48);
  if (((w6 >> 32) & 0xFFu) > 1 || (h->k != 3 && h->k != 5 && h->k != 7) || h->max_rounds < 1) return;
  h->e = __uint_as_float((unsigned)hdr_word(w, 9));  // byte 72
  if (!(h->e >= 0x1p-100f) || !(h->e <= 0x1p100f)) return;
  for (int d2 = 0; d2 < 10; d2 += 2) {
    const uint64_t wk = hdr_word(w, 11 + d2 / 2);  // bytes 88 + 4 d2
    h->w[d2] = __uint_as_float((unsigned)wk);
    h->w[d2 + 1] = __uint_as_float((unsigned)(wk >> 32));
    if (!(h->w[d2] > 0.0f) || !(h->w[d2] <= 1.0f) || !(h->w[d2 + 1] > 0.0f) || !(h->w[d2 + 1] <= 1.0f)) return;
  }
  h->total = hdr_word(w, 16);
  h->wdata = hdr_word(w, 17);
  h->wrank = hdr_word(w, 18);
  if (h->wdata > h->nb * kMaxWData || h->wrank > h->nb * kMaxWRankAny) return;
  uint64_t off[kNSeg], len[kNSeg];
  const uint64_t total = seg_layout(h->nb, h->topo, h->wdata, h->wrank, off, len);
  if (total != h->total || total > in_size) return;
  for (int sg = 0; sg < kNSeg; ++sg) {
    h->off[sg] = hdr_word(w, 20 + sg);  // bytes 160 + 8 s
    h->len[sg] = hdr_word(w, 33 + sg);  // bytes 264 + 8 s
    if (h->off[sg] != off[sg] || h->len[sg] != len[sg]) return;
  }
  h->ok = (h->n <= out_cap) ? 1 : -1;
}

// Decodes the chunk behind workgroup slot w_id (slots cover xcd_grid of the
// capacity's chunk count; slot 0 also publishes the header verdict).
template <int WAVES>
__device__ __forceinline__ void decode_body(const DecArgs& a, int w_id) {
  constexpr int BPW = kB / WAVES;
  constexpr int kRankLds = kB * kMaxWRankBlk;  // rank planes staged when they fit
  __shared__ Hdr s_h;
  __shared__ unsigned long long s_pl[kB * kMaxWData], s_rpl[kRankLds];
  __shared__ unsigned long long s_sign[kB], s_rsign[kB], s_bm[kB];
  __shared__ int s_first[kB], s_rfirst[kB];
  __shared__ unsigned s_lab[kB * 4];
  __shared__ int s_pfd[kB + 1], s_pfr[kB + 1], s_wd[kB], s_wr[kB];
  __shared__ int s_bad;
  __shared__ unsigned s_moves, s_skips, s_corrupt;
  Ctrl* ct = ctrl_of(a.ws);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (wv == 0) parse_header(a.in, a.in_size, a.out_cap, &s_h, lane);
  if (tid == 0) {
    s_bad = 0;
    s_moves = 0;
    s_skips = 0;
    s_corrupt = 0;
  }
  __syncthreads();
  const Hdr& h = s_h;
  const uint64_t nb = h.ok == 1 ? h.nb : 0, nch = h.ok == 1 ? h.nch : 0;
  const DecLayout L = dec_layout(nb, nch);
  const bool room = h.ok == 1 && L.end <= a.ws_bytes;
  if (w_id == 0 && tid == 0) {
    // this call's header verdict and counters for refine/tail
    ct->hflags = h.ok == 1 ? (room ? 0u : 2u) : (h.ok == -1 ? 2u : 1u);
    ct->big = 0;
    ct->rp_commits = 0;
    ct->rp_rounds = 0;
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
      // the candidate's weight sum for a window wholly inside the grid, added
      // in the candidate's own (dz, dy, dx) order
      {
        const int r = p.k / 2, rz = p.ndim == 3 ? r : 0;
        double ws = 0.0;
        for (int dz = -rz; dz <= rz; ++dz)
          for (int dy = -r; dy <= r; ++dy)
            for (int dx = -r; dx <= r; ++dx) {
              const int d2 = dz * dz + dy * dy + dx * dx;
              if (d2 == 0 || d2 > r * r) continue;
              ws = ws + (double)p.w[d2];
            }
        p.wsum = ws;
      }
      p.s6_off = h.off[S6];
    }
  }
  if (w_id == 0 && tid < kSpreadLines) {
    Spread* sp = spread_of(a.ws);
    sp[tid].commits = 0;
    sp[tid].rounds = 0;
    sp[tid].queued = 0;
  }
  // the grid is sized for the output capacity; the chunk mapping covers
  // exactly the stream's own xcd_grid(nch) workgroups
  if (!room || w_id >= xcd_grid((int)h.nch)) return;
  const int c = xcd_chunk(w_id, (int)h.nch);
  if ((uint64_t)c >= h.nch) return;
  const int n = (int)h.n;
  const bool topo = h.topo != 0;

  // The chunk's payload ranges (X1, X2), read by every wave: each wave starts
  // its share of the plane copy to LDS at once, bounds-checked against the
  // segment, while wave 0 checks the ranges against the widths below.
  const uint64_t* x1 = reinterpret_cast<const uint64_t*>(a.in + h.off[X1]);
  const uint64_t xd = x1[c], nxd = (uint64_t)c + 1 < h.nch ? x1[c + 1] : h.len[S5];
  uint64_t xr = 0, nxr = 0;
  if (topo) {
    const uint64_t* x2 = reinterpret_cast<const uint64_t*>(a.in + h.off[X2]);
    xr = x2[c];
    nxr = (uint64_t)c + 1 < h.nch ? x2[c + 1] : h.len[R5];
  }
  const bool dfit = xd <= nxd && nxd <= h.len[S5] && nxd - xd <= 8ull * kB * kMaxWData;
  const bool rank_lds = topo && xr <= nxr && nxr <= h.len[R5] && nxr - xr <= 8ull * kRankLds;
  {
    if (dfit) {
      const unsigned long long* src = reinterpret_cast<const unsigned long long*>(a.in + h.off[S5] + (xd & ~7ull));
      const int nd = (int)((nxd - xd) >> 3);
      for (int o = tid; o < nd; o += WAVES * 64) s_pl[o] = src[o];
    }
    if (rank_lds) {
      const unsigned long long* rsrc = reinterpret_cast<const unsigned long long*>(a.in + h.off[R5] + (xr & ~7ull));
      const int nr = (int)((nxr - xr) >> 3);
      for (int o = tid; o < nr; o += WAVES * 64) s_rpl[o] = rsrc[o];
    }
  }
  // the chunk's fixed-size parts to LDS (every thread), and its widths and
  // constant flags (wave 0)
  {
    const int lb = tid & 63, part = tid >> 6;
    const uint64_t b = (uint64_t)c * kB + lb;
    if (b < h.nb) {
      if (part == 1) {
        s_sign[lb] = *reinterpret_cast<const unsigned long long*>(a.in + h.off[S3] + 8 * b);
        s_first[lb] = *reinterpret_cast<const int*>(a.in + h.off[S4] + 4 * b);
      } else if (part == 2 && topo) {
        s_rsign[lb] = *reinterpret_cast<const unsigned long long*>(a.in + h.off[R3] + 8 * b);
        s_rfirst[lb] = *reinterpret_cast<const int*>(a.in + h.off[R4] + 4 * b);
      }
    }
    // the chunk's labels: 4 dwords per block, one per thread of the first 256
    if (topo && tid < kB * 4 && (uint64_t)c * kB + (tid >> 2) < h.nb)
      s_lab[tid] = *reinterpret_cast<const unsigned*>(a.in + h.off[S6] + 16 * (uint64_t)c * kB + 4 * tid);
  }
  if (wv == 0) {
    const uint64_t b = (uint64_t)c * kB + lane;
    const bool bv = b < h.nb;
    const int wd = bv ? a.in[h.off[S2] + b] : 0;
    const int wr = (bv && topo) ? a.in[h.off[R2] + b] : 0;
    const unsigned long long cb = *reinterpret_cast<const unsigned long long*>(a.in + h.off[S1] + 8 * (uint64_t)c);
    bool bad = bv && (wd > kMaxWData || (int)((cb >> lane) & 1) != (wd == 0));
    if (topo) {
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
      // the payload ranges must be exactly the chunk's planes (the copy
      // above then holds them all)
      const uint64_t totd = 8ull * (unsigned)__builtin_amdgcn_readlane(sd, 63);
      const uint64_t totr = 8ull * (unsigned)__builtin_amdgcn_readlane(sr, 63);
      bool b2 = anybad || (c == 0 && xd != 0) || xd > h.len[S5] || totd > h.len[S5] - xd || xd + totd != nxd;
      if (topo)
        b2 = b2 || (c == 0 && xr != 0) || xr > h.len[R5] || totr > h.len[R5] - xr || xr + totr != nxr;
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
    if (tid < kB && (uint64_t)c * kB + tid < h.nb) {
      bitmap[(uint64_t)c * kB + tid] = 0;
      reinterpret_cast<unsigned long long*>(a.ws + L.capped)[(uint64_t)c * kB + tid] = 0;
    }
    return;
  }

  const double ed = (double)h.e;
  const float two_e = 2.0f * h.e;
  const int dmax = h.scope ? n : kB;
  const unsigned long long* rglob = reinterpret_cast<const unsigned long long*>(a.in + h.off[R5] + xr);
  unsigned* qi = reinterpret_cast<unsigned*>(a.ws + L.idx) + (size_t)c * kChunk;
  // wave-uniform tallies: lanes that read corrupt, stencil moves and skips
  unsigned long long corrupt_m = 0;
  unsigned moves = 0, skips = 0;
  const unsigned lsh = 2u * ((unsigned)lane & 15u);  // this lane's label bits in its dword
  // one block's work once its values (q) and ranks (dl) are decoded; the
  // per-point decisions are wave masks, so no lane branches
  auto finish = [&](int lb, int q, int dl) {
    const int i0 = (c * kB + lb) * kB;  // the block's first point (n < 2^31)
    const int nv = n - i0;              // points of the block inside the field
    const unsigned long long vm = nv >= kB ? ~0ull : ((1ull << nv) - 1ull);
    // |q| <= kQMax, as one unsigned compare
    corrupt_m |= __ballot((unsigned)q + (unsigned)kQMax > 2u * (unsigned)kQMax) & vm;
    const float rq = (float)q * two_e;  // float(2q) * e: the same exact product
    float v = rq;
    if (topo) {
      corrupt_m |= __ballot((unsigned)dl > (unsigned)dmax) & vm;  // dl < 0 reads as large
      const unsigned lw = s_lab[4 * lb + (lane >> 4)];
      // label bit 0 marks an extremum, bit 1 a saddle or a maximum
      const unsigned long long b0 = __ballot((lw >> lsh) & 1u), b1 = __ballot((lw >> lsh) & 2u);
      const unsigned long long pos = __ballot(dl > 0) & vm;
      const unsigned long long mv = pos & b0;  // flattened extrema
      if (mv) {
        // the extremum's neighbour maximum (minimum) is its own bin centre,
        // so its stencil value is delta float steps beyond it
        const unsigned sd = lane_in(b1) ? (unsigned)dl : 0u - (unsigned)dl;
        float cand;
        bool fits;
        if (h.scope == 0) {
          // block scope: delta <= 64, and the key of a finite float lies well
          // inside int32, so the 32-bit sum is exact (a corrupt delta only
          // wraps; the call then reports the stream corrupt).  At most 64
          // steps from a bin centre (0, or at least 2e >= 2^-99 in size) the
          // candidate keeps the centre's sign and lies within a factor 2 of
          // it, so their float difference is exact (Sterbenz) and the budget
          // test needs no double
          cand = key2f32((int)((unsigned)fkey(rq) + sd));
          fits = fabsf(cand - rq) <= h.e;
        } else {
          cand = key2f((long long)fkey(rq) + (long long)(int)sd);
          fits = fabs((double)cand - (double)rq) <= ed;
        }
        const unsigned long long fm = __ballot(fits) & mv;
        v = lane_in(fm) ? cand : rq;
        moves += (unsigned)__popcll(fm);
        skips += (unsigned)__popcll(mv & ~fm);
      }
      // flattened saddles: queued (their indices go out after the barrier)
      if (lane == 0) s_bm[lb] = pos & b1 & ~b0;
    }
    float* const ob = a.out + i0;
    if (lane_in(vm)) ob[lane] = v;
  };
  // blocks two at a time (BPW is even): the pair's plane reads and prefix
  // sums interleave; a pair past the end of the field keeps its first block
  static_assert(BPW % 2 == 0, "blocks in pairs");
  for (int k = 0; k < BPW; k += 2) {
    const int lb = wv * BPW + k;
    const uint64_t b = (uint64_t)c * kB + lb;
    if (b >= h.nb) break;
    const bool two = b + 1 < h.nb;
    int q0, q1, d0 = 0, d1 = 0;
    decode_pair(s_pl + s_pfd[lb], s_wd[lb], s_first[lb], s_sign[lb], s_pl + s_pfd[lb + 1], two ? s_wd[lb + 1] : 0,
                s_first[lb + 1], s_sign[lb + 1], lane, q0, q1);
    if (topo) {
      const int wr1 = two ? s_wr[lb + 1] : 0;
      if (s_wr[lb] == 0 && wr1 == 0) {
        // two constant rank blocks (the common case away from flattened
        // points): every rank is the block's first
        d0 = s_rfirst[lb];
        d1 = s_rfirst[lb + 1];
      } else if (rank_lds)
        decode_pair(s_rpl + s_pfr[lb], s_wr[lb], s_rfirst[lb], s_rsign[lb], s_rpl + s_pfr[lb + 1], wr1,
                    s_rfirst[lb + 1], s_rsign[lb + 1], lane, d0, d1);
      else
        decode_pair(rglob + s_pfr[lb], s_wr[lb], s_rfirst[lb], s_rsign[lb], rglob + s_pfr[lb + 1], wr1,
                    s_rfirst[lb + 1], s_rsign[lb + 1], lane, d0, d1);
    }
    finish(lb, q0, d0);
    if (two) finish(lb + 1, q1, d1);
  }
  if (lane == 0) {
    if (moves) atomicAdd(&s_moves, moves);
    if (skips) atomicAdd(&s_skips, skips);
    if (corrupt_m) atomicOr(&s_corrupt, 1u);
  }
  __syncthreads();
  // the chunk's queue of flattened saddles, in block order: each wave writes
  // its own blocks' entries at offsets scanned from the queued-saddle bitmap
  unsigned qtot = 0;
  if (topo) {
    const unsigned long long mine = (uint64_t)c * kB + lane < h.nb ? s_bm[lane] : 0ull;
    const int pc = __popcll(mine);
    const int incl = wave_incl_scan(pc, lane);
    qtot = (unsigned)__builtin_amdgcn_readlane(incl, 63);
    for (int k = 0; k < BPW; ++k) {
      const int lb = wv * BPW + k;
      const unsigned long long qm =
          (unsigned long long)(unsigned)__builtin_amdgcn_readlane((int)(unsigned)mine, lb) |
          ((unsigned long long)(unsigned)__builtin_amdgcn_readlane((int)(unsigned)(mine >> 32), lb) << 32);
      if (qm) {
        const unsigned off = (unsigned)__builtin_amdgcn_readlane(incl - pc, lb);
        if (lane_in(qm)) qi[off + mbcnt(qm)] = (unsigned)((c * kB + lb) * kB + lane);
      }
    }
  }
  // the chunk's queued-saddle bitmap (and a cleared word of the capped
  // bitmap beside each), and counters
  if (tid < kB && (uint64_t)c * kB + tid < h.nb) {
    bitmap[(uint64_t)c * kB + tid] = topo ? s_bm[tid] : 0ull;
    reinterpret_cast<unsigned long long*>(a.ws + L.capped)[(uint64_t)c * kB + tid] = 0;
  }
  if (tid == 0) {
    reinterpret_cast<unsigned*>(a.ws + L.cnt)[c] = qtot;
    reinterpret_cast<unsigned*>(a.ws + L.moves)[c] = s_moves;
    reinterpret_cast<unsigned*>(a.ws + L.skips)[c] = s_skips;
    dflag[c] = s_corrupt;
  }
}

template <int WAVES>
__global__ __launch_bounds__(WAVES * 64) void decode_kernel(DecArgs a) {
  decode_body<WAVES>(a, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Saddle refinement (Section IV-B), compiled per (dimension, kernel size) so
// that every neighbourhood below is a compile-time set of offsets.
//
// An evaluation of a queued saddle p reads the cells of its read set: the
// candidate window (Euclidean distance <= floor(k/2)) and the cells the
// acceptance tests classify (L1 distance <= 2).  It writes only p.  Queued
// saddles linked through read-set offsets form clusters; distinct clusters
// never see each other's updates, so each evolves under the colour-phased
// schedule exactly as in the whole-field run, and a field-wide round count
// is the largest of the clusters' (a cluster stops at its first round without
// a commit; later rounds would not change it).

template <int ND, int K>
struct Hood {
  static constexpr int r = K / 2;
  static constexpr int R = r > 2 ? r : 2;  // half-width of a box holding the read set
  static constexpr int RZ = ND == 3 ? R : 0;
  static constexpr int S = 2 * R + 1;
  static constexpr int SZ = 2 * RZ + 1;
  static constexpr int BOX = S * S * SZ;
  __host__ __device__ static constexpr int iabs(int v) { return v < 0 ? -v : v; }
  __host__ __device__ static constexpr bool read(int dx, int dy, int dz) {
    return dx * dx + dy * dy + dz * dz <= r * r || iabs(dx) + iabs(dy) + iabs(dz) <= 2;
  }
  // any offset: inside the box and in the read set
  __host__ __device__ static constexpr bool reads(int dx, int dy, int dz) {
    return iabs(dx) <= R && iabs(dy) <= R && iabs(dz) <= RZ && read(dx, dy, dz);
  }
};

// p's coordinates and the in-range flags of its box offsets.
template <int ND, int K>
struct Around {
  bool xin[Hood<ND, K>::S], yin[Hood<ND, K>::S], zin[Hood<ND, K>::SZ];
  __device__ __forceinline__ Around(Pt c, const GeomD& g) {
    using H = Hood<ND, K>;
#pragma unroll
    for (int d = -H::R; d <= H::R; ++d) {
      xin[d + H::R] = (unsigned)(c.x + d) < (unsigned)g.nx;
      yin[d + H::R] = (unsigned)(c.y + d) < (unsigned)g.ny;
    }
#pragma unroll
    for (int d = -H::RZ; d <= H::RZ; ++d) zin[d + H::RZ] = (unsigned)(c.z + d) < (unsigned)g.nz;
  }
  __device__ __forceinline__ bool in(int dx, int dy, int dz) const {
    using H = Hood<ND, K>;
    if (dz < -H::RZ || dz > H::RZ) return false;
    return zin[dz + H::RZ] && yin[dy + H::R] && xin[dx + H::R];
  }
};

// True if every point within two rows/planes (and two columns) of p lies in
// the array: then the row spans below can be loaded whole.  Only points
// near the first or last rows of the field fail this.
template <int ND>
__device__ __forceinline__ bool far_from_ends(int p, const GeomD& g) {
  const int reachf = (ND == 3 ? 3 * g.nxy : 0) + 3 * g.nx + 3;
  return p >= reachf && p < g.n - reachf;
}

// Bits [lo, lo + 31] of the queued-saddle bitmap (lo >= 0), from the two
// words holding bit lo.  The second word may lie past the bitmap's last word
// (still inside the workspace); its bits are then never used.
__device__ __forceinline__ unsigned bm_span(const unsigned long long* bm, int lo) {
  unsigned long long w[2];
  __builtin_memcpy(w, bm + (lo >> 6), sizeof(w));
  const int sh = lo & 63;
  return (unsigned)(sh ? (w[0] >> sh) | (w[1] << (64 - sh)) : w[0]);
}

// The core of an evaluation of p: the values at L1 distance <= 2 (all that
// the classifications read; entries for cells outside the grid hold values
// that are never used) and the labels of p's face neighbours.
template <int ND>
struct Core {
  static constexpr int CZ = ND == 3 ? 2 : 0;
  float v[2 * CZ + 1][5][5];  // [dz + CZ][dy + 2][dx + 2], entries with L1 <= 2
  int lab[6];
};

// The read set of an evaluation lies inside its core when the Gaussian
// window does (radius 1, or radius 2 in 2D): such an evaluation needs no
// memory once the core is known.  The replay keeps cores in registers in 2D
// only (13 values); the 25 of a 3D core would spill.
template <int ND, int K>
constexpr bool kCoreOnly = ND == 2 && K / 2 <= 2;

// Loads the core of p (one batch of loads).
template <int ND, int K>
__device__ __forceinline__ void load_core(const float* fld, const uint8_t* labels, int p, Pt c, const GeomD& g,
                                          Core<ND>& C) {
  constexpr int CZ = Core<ND>::CZ;
  const Around<ND, K> ar(c, g);
  auto& v = C.v;
  if (far_from_ends<ND>(p, g)) {
    // one vector load per row of the core (every span lies inside the
    // array); rows outside the grid read p's own row instead
#pragma unroll
    for (int dz = -CZ; dz <= CZ; ++dz)
#pragma unroll
      for (int dy = -2; dy <= 2; ++dy) {
        const int sp = 2 - Hood<ND, K>::iabs(dy) - Hood<ND, K>::iabs(dz);
        if (sp < 0) continue;
        const int q0 = ar.in(0, dy, dz) ? p + dz * g.nxy + dy * g.nx : p;
        __builtin_memcpy(&v[dz + CZ][dy + 2][2 - sp], fld + (q0 - sp), sizeof(float) * (2 * sp + 1));
      }
  } else {
#pragma unroll
    for (int dz = -CZ; dz <= CZ; ++dz)
#pragma unroll
      for (int dy = -2; dy <= 2; ++dy)
#pragma unroll
        for (int dx = -2; dx <= 2; ++dx) {
          if (Hood<ND, K>::iabs(dx) + Hood<ND, K>::iabs(dy) + Hood<ND, K>::iabs(dz) > 2) continue;
          const int q = ar.in(dx, dy, dz) ? p + dz * g.nxy + dy * g.nx + dx : p;
          v[dz + CZ][dy + 2][dx + 2] = fld[q];
        }
  }
  constexpr int U[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
#pragma unroll
  for (int j = 0; j < 2 * ND; ++j) {
    const bool ex = ar.in(U[j][0], U[j][1], U[j][2]);
    const int q = ex ? p + U[j][2] * g.nxy + U[j][1] * g.nx + U[j][0] : p;
    C.lab[j] = (labels[q >> 2] >> (2 * (q & 3))) & 3;
  }
}

// Sets the core entry at offset (dx, dy, dz) (L1 <= 2) to x: unrolled
// selects, so that the core stays in registers.
template <int ND>
__device__ __forceinline__ void core_set(Core<ND>& C, int dx, int dy, int dz, float x) {
  constexpr int CZ = Core<ND>::CZ;
#pragma unroll
  for (int oz = -CZ; oz <= CZ; ++oz)
#pragma unroll
    for (int oy = -2; oy <= 2; ++oy)
#pragma unroll
      for (int ox = -2; ox <= 2; ++ox) {
        if ((ox < 0 ? -ox : ox) + (oy < 0 ? -oy : oy) + (oz < 0 ? -oz : oz) > 2) continue;
        if (dx == ox && dy == oy && dz == oz) C.v[oz + CZ][oy + 2][ox + 2] = x;
      }
}

// One evaluation of the queued saddle p from its core: 0 reject, 1 already a
// saddle, 2 accept (value in *vout).  Window cells beyond the core are read
// from fld as the sum reaches them.
template <int ND, int K>
__device__ __forceinline__ int eval_core(const float* fld, const Core<ND>& C, int p, Pt c, const Plan& pl,
                                         float* vout) {
  using H = Hood<ND, K>;
  constexpr int r = H::r, CZ = Core<ND>::CZ;
  const GeomD& g = pl.g;
  const Around<ND, K> ar(c, g);
  const auto& v = C.v;
  const int* lab = C.lab;
  constexpr int U[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
  const unsigned ndeg = (g.nx > 1 ? 1u : 0u) | (g.ny > 1 ? 4u : 0u) | (ND == 3 && g.nz > 1 ? 16u : 0u);
  // class of the cell at offset o (L1 <= 1) with p's value taken as pv
  auto cls = [&](int ox, int oy, int oz, float pv) -> int {
    float nb[6];
    unsigned avm = 0;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      nb[j] = 0.0f;
      if (j >= 2 * ND) continue;
      const int x = ox + U[j][0], y = oy + U[j][1], z = oz + U[j][2];
      if (ar.in(x, y, z)) avm |= 1u << j;
      nb[j] = (x == 0 && y == 0 && z == 0) ? pv : v[z + CZ][y + 2][x + 2];
    }
    const float a0 = (ox == 0 && oy == 0 && oz == 0) ? pv : v[oz + CZ][oy + 2][ox + 2];
    return classify_bits(a0, nb, avm, ndeg);
  };
  const float p0 = v[CZ][2][2];
  if (cls(0, 0, 0, p0) == CLS_SAD) return 1;
  // normalised Gaussian window without p, in (dz, dy, dx) order; cells
  // outside the grid carry weight 0, which leaves both sums unchanged.  A
  // window wholly inside the grid skips the range tests, and its weight sum
  // is the plan's (the same additions in the same order).
  constexpr int rz = ND == 3 ? r : 0;
  double num = 0.0, den = 0.0;
  const bool inside = ar.in(-r, -r, -rz) && ar.in(r, r, rz);
  auto sum = [&](auto all_in) {
    constexpr bool AI = decltype(all_in)::value;
    auto cell = [&](int dx, int dy, int dz, float x) {
      const int d2 = dz * dz + dy * dy + dx * dx;
      if (AI) {
        num = num + (double)pl.w[d2] * (double)x;
      } else {
        const double wt = ar.in(dx, dy, dz) ? (double)pl.w[d2] : 0.0;
        num = num + wt * (double)x;
        den = den + wt;
      }
    };
    auto at = [&](int dx, int dy, int dz) {
      return fld[AI || ar.in(dx, dy, dz) ? p + dz * g.nxy + dy * g.nx + dx : p];
    };
    if constexpr (ND == 3 && K == 7) {
      // planes in turn (a runtime loop keeps one plane's loads in
      // registers); every cell of these planes is read from memory
#pragma unroll 1
      for (int dz = -rz; dz <= rz; ++dz) {
#pragma unroll
        for (int dy = -r; dy <= r; ++dy)
#pragma unroll
          for (int dx = -r; dx <= r; ++dx) {
            const int d2 = dz * dz + dy * dy + dx * dx;
            if (d2 == 0 || d2 > r * r) continue;
            cell(dx, dy, dz, at(dx, dy, dz));
          }
      }
    } else {
#pragma unroll
      for (int dz = -rz; dz <= rz; ++dz)
#pragma unroll
        for (int dy = -r; dy <= r; ++dy)
#pragma unroll
          for (int dx = -r; dx <= r; ++dx) {
            const int d2 = dz * dz + dy * dy + dx * dx;
            if (d2 == 0 || d2 > r * r) continue;
            const bool core = Hood<ND, K>::iabs(dx) + Hood<ND, K>::iabs(dy) + Hood<ND, K>::iabs(dz) <= 2;
            cell(dx, dy, dz, core ? v[dz + CZ][dy + 2][dx + 2] : at(dx, dy, dz));
          }
    }
    if (AI) den = pl.wsum;
  };
  if (inside) sum(std::true_type{});
  else sum(std::false_type{});
  if (den == 0.0) return 0;
  const float cand = (float)(num / den);
  if (!(fabs((double)cand - (double)p0) <= (double)pl.e)) return 0;
  if (cls(0, 0, 0, cand) != CLS_SAD) return 0;
#pragma unroll
  for (int j = 0; j < 2 * ND; ++j) {
    if (!ar.in(U[j][0], U[j][1], U[j][2])) continue;
    const int before = cls(U[j][0], U[j][1], U[j][2], p0);
    const int after = cls(U[j][0], U[j][1], U[j][2], cand);
    if (after != before && !(before == CLS_R && after == lab[j])) return 0;
  }
  *vout = cand;
  return 2;
}

// One evaluation of the queued saddle p on the current field (as eval_core,
// after loading the core).
template <int ND, int K>
__device__ __forceinline__ int evaluate(const float* fld, const uint8_t* labels, int p, Pt c,
                                        const Plan& pl, float* vout) {
  Core<ND> C;
  load_core<ND, K>(fld, labels, p, c, pl.g, C);
  return eval_core<ND, K>(fld, C, p, c, pl, vout);
}

__device__ __forceinline__ int colour_of(Pt c, int ndim) {
  return ndim == 3 ? (int)(((unsigned)c.x + 2u * (unsigned)c.y + 3u * (unsigned)c.z) % 7u)
                   : (int)(((unsigned)c.x + 2u * (unsigned)c.y) % 5u);
}

// Queued saddles among p's read set (p excluded): any, and any with a
// smaller flat index.
template <int ND, int K>
__device__ __forceinline__ void reach(const unsigned long long* bm, int p, Pt c, const GeomD& g, bool& any,
                                      bool& smaller) {
  using H = Hood<ND, K>;
  const Around<ND, K> ar(c, g);
  any = smaller = false;
  if (far_from_ends<ND>(p, g) && H::R <= 3) {
    // one two-word load per row of the read set
    auto plane = [&](int dz) {
#pragma unroll
      for (int dy = -H::R; dy <= H::R; ++dy) {
        unsigned rm = 0, lm = 0;  // read-set cells of the row (bit dx + R), those left of p
#pragma unroll
        for (int dx = -H::R; dx <= H::R; ++dx)
          if (H::read(dx, dy, dz) && !(dx == 0 && dy == 0 && dz == 0)) {
            if (ar.in(dx, dy, dz)) rm |= 1u << (dx + H::R);
            if (dx < 0) lm |= 1u << (dx + H::R);
          }
        if (!rm) continue;
        const unsigned bits = bm_span(bm, p + dz * g.nxy + dy * g.nx - H::R) & rm;
        any |= bits != 0;
        if (dz < 0 || (dz == 0 && dy < 0)) smaller |= bits != 0;
        if (dz == 0 && dy == 0) smaller |= (bits & lm) != 0;
      }
    };
    if constexpr (ND == 3 && K == 7) {
#pragma unroll 1
      for (int dz = -H::RZ; dz <= H::RZ; ++dz) plane(dz);
    } else {
#pragma unroll
      for (int dz = -H::RZ; dz <= H::RZ; ++dz) plane(dz);
    }
    return;
  }
  auto plane = [&](int dz) {
#pragma unroll
    for (int dy = -H::R; dy <= H::R; ++dy)
#pragma unroll
      for (int dx = -H::R; dx <= H::R; ++dx) {
        if (!H::read(dx, dy, dz) || (dx == 0 && dy == 0 && dz == 0)) continue;
        const bool in = ar.in(dx, dy, dz);
        const int q = in ? p + dz * g.nxy + dy * g.nx + dx : p;
        const bool hit = in && ((bm[q >> 6] >> (q & 63)) & 1ull);
        any |= hit;
        if (dz < 0 || (dz == 0 && (dy < 0 || (dy == 0 && dx < 0)))) smaller |= hit;
      }
  };
  if constexpr (ND == 3 && K == 7) {
#pragma unroll 1
    for (int dz = -H::RZ; dz <= H::RZ; ++dz) plane(dz);  // a plane's loads at a time
  } else {
#pragma unroll
    for (int dz = -H::RZ; dz <= H::RZ; ++dz) plane(dz);
  }
}

constexpr int kClusterMax = 64;   // members of a cluster replayed in a workgroup
static_assert(kClusterMax % 4 == 0, "member lists are read four at a time");
#ifndef TSZ_REFINE_WAVES
#define TSZ_REFINE_WAVES 2
#endif
constexpr int kRefThreads = 64 * TSZ_REFINE_WAVES;  // refine workgroup
static_assert(kRefThreads <= kChunk, "one queue slot per refine thread");
constexpr int kCandMax = 512;                        // queued saddles per chunk per pass
constexpr int kBatch = 64;                           // owners gathered at once

// LDS of the refine kernel.
struct RefShared {
  unsigned cand[kCandMax];          // owners found in phase A
  unsigned vis[kBatch][8];          // per gathering lane: members in a 256-cell window at its owner
  alignas(16) unsigned memb[kBatch][kClusterMax];  // their clusters
  unsigned msize[kBatch];           // member count; 0 = not an owner or too large
  unsigned off[kBatch + 1];         // first lane of each cluster in the pack
  unsigned cflag[kBatch];           // bit0 still running, bit1 committed this round
  unsigned crounds[kBatch];
  unsigned cpts[kRefThreads];       // ring of committed points (entry k at k mod kRefThreads)
  float cval[kRefThreads];          // and their new values
  unsigned ncp;                     // commits of the pack so far
  unsigned nc, any;
};

// Gathers the cluster of owner candidate p0 (lane-serial): every queued
// saddle reachable through read-set offsets.  Returns the member count, or
// 0 if a smaller member exists (it owns the cluster) or there are more than
// kClusterMax members (*over set).
template <int K>
__device__ unsigned gather2d(const unsigned long long* bm, unsigned p0, const GeomD& g, unsigned* mem,
                             unsigned* vis, bool* over);

// In 3D, membership of a cell within a 4x8x8 window (the owner's plane and
// the 3 after it, 4 rows and columns either side; members lie at larger
// indices) is one bit of `vis` (8 words); cells outside it are looked up in
// the member list.
template <int ND, int K>
__device__ unsigned gather(const unsigned long long* bm, unsigned p0, const GeomD& g, unsigned* mem,
                           unsigned* vis, bool* over) {
  if constexpr (ND == 2) return gather2d<K>(bm, p0, g, mem, vis, over);
  using H = Hood<ND, K>;
  mem[0] = p0;
  unsigned m = 1;
  bool owner = true;
  *over = false;
  const Pt oc = coords_of((int)p0, g);
#pragma unroll
  for (int w = 0; w < 8; ++w) vis[w] = 0u;
  vis[(4 * 8 + 4) >> 5] = 1u << ((4 * 8 + 4) & 31);  // the owner
  for (unsigned head = 0; head < m && owner && !*over; ++head) {
    const int cur = (int)mem[head];
    const Pt cc = coords_of(cur, g);
    const Around<ND, K> ar(cc, g);
    const bool far = far_from_ends<ND>(cur, g);
    // q at offset (dx, dy, dz) from the current member
    auto add = [&](int q, int dx, int dy, int dz) {
      const int rx = cc.x + dx - oc.x + 4, ry = cc.y + dy - oc.y + 4, rz = cc.z + dz - oc.z;
      if ((unsigned)rx < 8u && (unsigned)ry < 8u && (unsigned)rz < 4u) {
        const unsigned bit = (unsigned)((rz * 8 + ry) * 8 + rx), mk = 1u << (bit & 31u);
        const unsigned w = vis[bit >> 5];
        if (w & mk) return;
        vis[bit >> 5] = w | mk;
      } else {
        // already a member? (four members per 16-byte read; mem is 16-byte
        // aligned and holds kClusterMax entries, a multiple of 4)
        bool seen = false;
        const uint4* m4 = reinterpret_cast<const uint4*>(mem);
        for (unsigned j = 0; j < m; j += 4) {
          const uint4 w = m4[j >> 2];
          seen |= w.x == (unsigned)q || (j + 1 < m && w.y == (unsigned)q) || (j + 2 < m && w.z == (unsigned)q) ||
                  (j + 3 < m && w.w == (unsigned)q);
        }
        if (seen) return;
      }
      if ((unsigned)q < p0) owner = false;
      if (m == (unsigned)kClusterMax) *over = true;
      else mem[m++] = (unsigned)q;
    };
    auto plane = [&](int dz) {
#pragma unroll
      for (int dy = -H::R; dy <= H::R; ++dy) {
        if (far) {
          // the row's queued cells from one two-word load
          unsigned rm = 0;
#pragma unroll
          for (int dx = -H::R; dx <= H::R; ++dx)
            if (H::read(dx, dy, dz) && !(dx == 0 && dy == 0 && dz == 0) && ar.in(dx, dy, dz))
              rm |= 1u << (dx + H::R);
          if (!rm) continue;
          const int row = cur + dz * g.nxy + dy * g.nx;
          for (unsigned bits = bm_span(bm, row - H::R) & rm; bits; bits &= bits - 1) {
            const int dx = __builtin_ctz(bits) - H::R;
            add(row + dx, dx, dy, dz);
          }
        } else {
#pragma unroll
          for (int dx = -H::R; dx <= H::R; ++dx) {
            if (!H::read(dx, dy, dz) || (dx == 0 && dy == 0 && dz == 0)) continue;
            const bool in = ar.in(dx, dy, dz);
            const int q = in ? cur + dz * g.nxy + dy * g.nx + dx : cur;
            if (in && ((bm[q >> 6] >> (q & 63)) & 1ull)) add(q, dx, dy, dz);
          }
        }
      }
    };
    if constexpr (ND == 3 && K == 7) {
#pragma unroll 1
      for (int dz = -H::RZ; dz <= H::RZ; ++dz) plane(dz);
    } else {
#pragma unroll
      for (int dz = -H::RZ; dz <= H::RZ; ++dz) plane(dz);
    }
  }
  return owner && !*over ? m : 0u;
}

// The same gather for 2D fields, with the bitmap rows of the next queued
// member requested while the current member's rows are scanned (members
// away from the first and last rows only), so that the queue's steps do not
// each wait a full load round trip.  Membership of a cell within a 16x16
// window (the owner's row and the 15 below it, 8 columns either side) is one
// bit of `vis` (8 words); only cells outside it are looked up in the member
// list.  Members of an owner's cluster all lie at larger indices, so no row
// above the owner's is needed.
template <int K>
__device__ unsigned gather2d(const unsigned long long* bm, unsigned p0, const GeomD& g, unsigned* mem,
                             unsigned* vis, bool* over) {
  using H = Hood<2, K>;
  constexpr int NR = 2 * H::R + 1;
  mem[0] = p0;
  unsigned m = 1;
  bool owner = true;
  *over = false;
  const Pt oc = coords_of((int)p0, g);
#pragma unroll
  for (int w = 0; w < 8; ++w) vis[w] = 0u;
  vis[0] = 1u << 8;  // the owner
  // q at grid coordinates (qx, qy)
  auto add = [&](int q, int qx, int qy) {
    const int rx = qx - oc.x + 8, ry = qy - oc.y;
    if ((unsigned)rx < 16u && (unsigned)ry < 16u) {
      const unsigned bit = (unsigned)(ry * 16 + rx), mk = 1u << (bit & 31u);
      const unsigned w = vis[bit >> 5];
      if (w & mk) return;
      vis[bit >> 5] = w | mk;
    } else {
      // already a member? (four members per 16-byte read; mem is 16-byte
      // aligned and holds kClusterMax entries, a multiple of 4)
      bool seen = false;
      const uint4* m4 = reinterpret_cast<const uint4*>(mem);
      for (unsigned j = 0; j < m; j += 4) {
        const uint4 w = m4[j >> 2];
        seen |= w.x == (unsigned)q || (j + 1 < m && w.y == (unsigned)q) || (j + 2 < m && w.z == (unsigned)q) ||
                (j + 3 < m && w.w == (unsigned)q);
      }
      if (seen) return;
    }
    if ((unsigned)q < p0) owner = false;
    if (m == (unsigned)kClusterMax) *over = true;
    else mem[m++] = (unsigned)q;
  };
  // the two bitmap words holding bits [p + dy nx - R, p + dy nx + R] of
  // each row dy (p away from the first and last rows: every index >= 0)
  auto fetch = [&](int p, unsigned long long (&w)[NR][2]) {
#pragma unroll
    for (int dy = -H::R; dy <= H::R; ++dy) {
      const int lo = p + dy * g.nx - H::R;
      w[dy + H::R][0] = bm[lo >> 6];
      w[dy + H::R][1] = bm[(lo >> 6) + 1];
    }
  };
  unsigned long long cw[NR][2];
  bool have = false;  // cw holds the rows of the member at the head
  for (unsigned head = 0; head < m && owner && !*over; ++head) {
    const int cur = (int)mem[head];
    const Pt cc = coords_of(cur, g);
    const Around<2, K> ar(cc, g);
    const bool far = far_from_ends<2>(cur, g);
    unsigned bits[NR];
    if (far) {
      if (!have) fetch(cur, cw);
#pragma unroll
      for (int dy = -H::R; dy <= H::R; ++dy) {
        unsigned rm = 0;
#pragma unroll
        for (int dx = -H::R; dx <= H::R; ++dx)
          if (H::read(dx, dy, 0) && !(dx == 0 && dy == 0) && ar.in(dx, dy, 0)) rm |= 1u << (dx + H::R);
        const int sh = (cur + dy * g.nx - H::R) & 63;
        const unsigned long long w0 = cw[dy + H::R][0], w1 = cw[dy + H::R][1];
        bits[dy + H::R] = (unsigned)(sh ? (w0 >> sh) | (w1 << (64 - sh)) : w0) & rm;
      }
    }
    // the next member's rows go out before this member's cells are added
    have = false;
    if (head + 1 < m) {
      const int nxt = (int)mem[head + 1];
      if (far_from_ends<2>(nxt, g)) {
        fetch(nxt, cw);
        have = true;
      }
    }
    if (far) {
#pragma unroll
      for (int dy = -H::R; dy <= H::R; ++dy) {
        const int row = cur + dy * g.nx;
        for (unsigned b = bits[dy + H::R]; b; b &= b - 1) {
          const int dx = __builtin_ctz(b) - H::R;
          add(row + dx, cc.x + dx, cc.y + dy);
        }
      }
    } else {
#pragma unroll
      for (int dy = -H::R; dy <= H::R; ++dy)
#pragma unroll
        for (int dx = -H::R; dx <= H::R; ++dx) {
          if (!H::read(dx, dy, 0) || (dx == 0 && dy == 0)) continue;
          const bool in = ar.in(dx, dy, 0);
          const int q = in ? cur + dy * g.nx + dx : cur;
          if (in && ((bm[q >> 6] >> (q & 63)) & 1ull)) add(q, cc.x + dx, cc.y + dy);
        }
    }
  }
  return owner && !*over ? m : 0u;
}

// Inlined into each kernel for every (dimension, kernel size): as calls, the
// larger instantiations paid the call convention's register saves and spills
// (2D k = 7 refinement 15% slower, 3D 5-9%).
template <int ND, int K, bool SPLIT>
__device__ __attribute__((always_inline)) void refine_chunk(const RefArgs& a, const Plan& pl, int c, int sub,
                                                            RefShared& sh, unsigned& commits, unsigned& rounds) {
  using H = Hood<ND, K>;
  const int tid = threadIdx.x;
  const uint64_t nb = ((uint64_t)pl.g.n + kB - 1) / kB;
  const DecLayout L = dec_layout(nb, (uint64_t)pl.nch);
  const unsigned cnt0 = reinterpret_cast<const unsigned*>(a.ws + L.cnt)[c];
  unsigned cnt = cnt0 < (unsigned)kChunk ? cnt0 : (unsigned)kChunk;
  const unsigned* idx = reinterpret_cast<const unsigned*>(a.ws + L.idx) + (size_t)c * kChunk;
  if constexpr (SPLIT) {
    // this workgroup's share of the chunk's queue: a cluster is refined by
    // the workgroup holding its owner's entry, so any division gives the
    // same result
    const unsigned lo = cnt * (unsigned)sub / (unsigned)a.split;  // cnt <= 4096, split <= 8
    cnt = cnt * (unsigned)(sub + 1) / (unsigned)a.split - lo;
    idx += lo;
  }
  const unsigned long long* bm = reinterpret_cast<const unsigned long long*>(a.ws + L.bitmap);
  const uint8_t* labels = a.in + pl.s6_off;
  const GeomD& g = pl.g;
  const int cap = pl.max_rounds;

  // the first entry of this thread, read beside the count (entries past the
  // count, at most 127 past the chunk's slots, lie inside the workspace and
  // are not used)
  const unsigned first = idx[tid];
  for (unsigned base = 0; base < cnt; base += kCandMax) {
    // phase A, one lane per queued saddle: isolated saddles are settled by
    // one evaluation; a saddle with no smaller queued saddle in reach owns
    // its cluster (if it is the cluster's smallest member)
    if (tid == 0) sh.nc = 0;
    __syncthreads();
    const unsigned lim = min(cnt, base + kCandMax);
    for (unsigned t = base + tid; t < lim; t += kRefThreads) {
      const int p = (int)(t == (unsigned)tid ? first : idx[t]);
      const Pt pc = coords_of(p, g);
      // the reach test and the evaluation read disjoint data: both go out
      // at once, and the evaluation counts only for an isolated saddle
      bool any, smaller;
      reach<ND, K>(bm, p, pc, g, any, smaller);
      float v = 0.0f;
      const int res = evaluate<ND, K>(a.out, labels, p, pc, pl, &v);
      if (!any) {
        if (res == 2) {
          a.out[p] = v;
          ++commits;
        }
        rounds = max(rounds, (unsigned)min(res == 2 ? 2 : 1, cap));
      } else if (!smaller) {
        sh.cand[atomicAdd(&sh.nc, 1u)] = (unsigned)p;
      }
    }
    __syncthreads();
    const unsigned nc = sh.nc;

    // phase B, kBatch owners at a time: each gathers its cluster in its own
    // lane; the clusters are then packed one member per lane and replayed
    // together under the colour-phased schedule
    for (unsigned b0 = 0; b0 < nc; b0 += kBatch) {
      const unsigned nbat = min(nc - b0, (unsigned)kBatch);
      if ((unsigned)tid < nbat) {
        bool over;
        sh.msize[tid] = gather<ND, K>(bm, sh.cand[b0 + tid], g, sh.memb[tid], sh.vis[tid], &over);
        if (over) {  // left to the tail, which gathers such clusters from these candidates
          Ctrl* ct = ctrl_of(a.ws);
          const unsigned k = atomicAdd(&ct->big, 1u);
          if (k < (unsigned)kOverMax) ct->over[k] = sh.cand[b0 + tid];
        }
      }
      __syncthreads();
      for (unsigned k0 = 0; k0 < nbat;) {
        // pack clusters k0.. while they fit the workgroup
        unsigned k1 = k0, tot = 0;
        while (k1 < nbat && tot + sh.msize[k1] <= (unsigned)kRefThreads) tot += sh.msize[k1++];
        if ((unsigned)tid <= k1 - k0) {
          unsigned o = 0;
          for (unsigned j = k0; j < k0 + tid; ++j) o += sh.msize[j];
          sh.off[tid] = o;
        }
        if ((unsigned)tid < k1 - k0) {
          sh.cflag[tid] = sh.msize[k0 + tid] ? 1u : 0u;
          sh.crounds[tid] = 0;
        }
        if (tid == 0) sh.ncp = 0;
        __syncthreads();
        const bool act = (unsigned)tid < tot;
        unsigned cl = 0;
        while (act && cl + 1 < k1 - k0 && sh.off[cl + 1] <= (unsigned)tid) ++cl;
        const int my = act ? (int)sh.memb[k0 + cl][tid - sh.off[cl]] : 0;
        const Pt myc = coords_of(my, g);
        const int col = colour_of(myc, ND);
        bool settled = !act;
        // when the read set lies inside the core, each member keeps its core
        // in registers for the whole pack, loaded once and updated from the
        // commit lists: its evaluations then read no memory
        constexpr bool CO = kCoreOnly<ND, K>;
        Core<ND> C;
        if constexpr (CO) {
          if (act) load_core<ND, K>(a.out, labels, my, myc, g, C);
        }
        auto eval = [&](float* vv) {
          if constexpr (CO) return eval_core<ND, K>(a.out, C, my, myc, pl, vv);
          else return evaluate<ND, K>(a.out, labels, my, myc, pl, vv);
        };
        unsigned seen = 0;  // commits of the pack already scanned
        int round = 1;
        for (; round <= cap; ++round) {
          // every unsettled member is evaluated on the field as the round
          // starts; an evaluation depends only on its read set, so it is
          // redone at the member's phase only if a commit earlier in the
          // round landed there (dirty)
          const bool live = act && (sh.cflag[cl] & 1u);
          int res = 0;
          float v = 0.0f;
          if (live && !settled) res = eval(&v);
          bool dirty = false;
          for (int ph = 0; ph < pl.ncol; ++ph) {
            const bool mine = live && !settled && col == ph;
            if constexpr (CO) {
              // the core changes only between phases: no reader to wait for
              if (mine && dirty) res = eval(&v);
            } else if (__syncthreads_or(mine && dirty)) {
              if (mine && dirty) res = eval(&v);
              __syncthreads();  // Jacobi: every evaluation of the phase reads before any commit
            }
            const bool commit = mine && res == 2;
            if (mine && res != 0) settled = true;
            // commits append to a ring and the count only grows, so nothing
            // is reset between phases (with register cores no barrier
            // separates a reset from the next phase's commits); a phase's
            // commits come after the barrier that ends the previous phase's
            // scans, and a phase holds at most kRefThreads of them
            if (commit) {
              a.out[my] = v;
              const unsigned k = atomicAdd(&sh.ncp, 1u) % (unsigned)kRefThreads;
              sh.cpts[k] = (unsigned)my;
              sh.cval[k] = v;
              atomicOr(&sh.cflag[cl], 2u);
              ++commits;
            }
            __threadfence_block();
            __syncthreads();
            const unsigned upto = sh.ncp;  // no commit until every thread has passed the next barrier
            for (; seen != upto; ++seen) {
              const unsigned j = seen % (unsigned)kRefThreads;
              const Pt ck = coords_of((int)sh.cpts[j], g);
              const int dx = ck.x - myc.x, dy = ck.y - myc.y, dz = ck.z - myc.z;
              dirty |= H::reads(dx, dy, dz);
              if constexpr (CO) {
                if (act && (dx < 0 ? -dx : dx) + (dy < 0 ? -dy : dy) + (dz < 0 ? -dz : dz) <= 2)
                  core_set<ND>(C, dx, dy, dz, sh.cval[j]);
              }
            }
            __syncthreads();
          }
          // a cluster stops at its first round without a commit
          __syncthreads();
          if ((unsigned)tid < k1 - k0) {
            const unsigned f = sh.cflag[tid];
            if ((f & 1u) && !(f & 2u)) {
              sh.cflag[tid] = 0;
              sh.crounds[tid] = (unsigned)round;
            } else {
              sh.cflag[tid] = f & 1u;
            }
          }
          if (!__syncthreads_or((unsigned)tid < k1 - k0 && (sh.cflag[tid] & 1u))) break;
        }
        if ((unsigned)tid < k1 - k0 && sh.msize[k0 + tid])
          rounds = max(rounds, (sh.cflag[tid] & 1u) ? (unsigned)cap : sh.crounds[tid]);
        // a cluster still committing when the round cap stopped it is not
        // settled: the whole-field replay must leave its members alone
        if (act && (sh.cflag[cl] & 1u))
          atomicOr(reinterpret_cast<unsigned long long*>(a.ws + L.capped) + (my >> 6), 1ull << (my & 63));
        __syncthreads();
        k0 = k1;
      }
    }
    __syncthreads();
  }
}

// The call's status, from the header check and the flags of the decode
// workgroups (all finished before the refine kernel starts).
__device__ __forceinline__ void status_body(const RefArgs& a, const Plan& pl, unsigned hf) {
  __shared__ unsigned s_fl;
  const int tid = threadIdx.x;
  if (tid == 0) s_fl = 0;
  __syncthreads();
  if (hf == 0 && pl.valid) {
    const DecLayout L = dec_layout(((uint64_t)pl.g.n + kB - 1) / kB, (uint64_t)pl.nch);
    const unsigned* df = reinterpret_cast<const unsigned*>(a.ws + L.dflag);
    unsigned fl = 0;
    for (int k = tid; k < pl.nch; k += (int)blockDim.x) fl |= df[k];
    if (fl) atomicOr(&s_fl, fl);
  }
  __syncthreads();
  if (tid == 0) *a.status = hf == 2u ? TOPOSZP_E_CAPACITY : (hf != 0u || s_fl) ? TOPOSZP_E_CORRUPT : TOPOSZP_OK;
}

// Refines the queued saddles of the chunk behind workgroup slot w_id (with
// SPLIT, its share of them); slot 0 also writes the call's status.
template <bool SPLIT>
__device__ __forceinline__ void refine_body(const RefArgs& a, int w_id, RefShared& sh) {
  __shared__ Plan s_p;
  __shared__ unsigned s_commits, s_rounds, s_ok, s_hf;
  Ctrl* ct = ctrl_of(a.ws);
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_p = ct->plan;
    s_hf = ct->hflags;
    s_ok = s_hf == 0 && s_p.valid && s_p.topo;
    s_commits = 0;
    s_rounds = 0;
  }
  __syncthreads();
  const Plan& pl = s_p;
  if (w_id == 0) status_body(a, pl, s_hf);
  // slot-major sub-slices: workgroups `slots` apart share a chunk (and, the
  // slot count being a multiple of 8, an XCD)
  const int sub = SPLIT ? w_id / a.slots : 0, cs = SPLIT ? w_id - sub * a.slots : w_id;
  if (!s_ok || cs >= xcd_grid(pl.nch)) return;
  const int c = xcd_chunk(cs, pl.nch);
  if (c >= pl.nch) return;
  unsigned commits = 0, rounds = 0;
  switch (pl.ndim * 8 + pl.k) {
    case 2 * 8 + 3: refine_chunk<2, 3, SPLIT>(a, pl, c, sub, sh, commits, rounds); break;
    case 2 * 8 + 5: refine_chunk<2, 5, SPLIT>(a, pl, c, sub, sh, commits, rounds); break;
    case 2 * 8 + 7: refine_chunk<2, 7, SPLIT>(a, pl, c, sub, sh, commits, rounds); break;
    case 3 * 8 + 3: refine_chunk<3, 3, SPLIT>(a, pl, c, sub, sh, commits, rounds); break;
    case 3 * 8 + 5: refine_chunk<3, 5, SPLIT>(a, pl, c, sub, sh, commits, rounds); break;
    default: refine_chunk<3, 7, SPLIT>(a, pl, c, sub, sh, commits, rounds); break;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    commits += (unsigned)__shfl_xor((int)commits, o);
    rounds = max(rounds, (unsigned)__shfl_xor((int)rounds, o));
  }
  if ((tid & 63) == 0) {
    if (commits) atomicAdd(&s_commits, commits);
    if (rounds) atomicMax(&s_rounds, rounds);
  }
  __syncthreads();
  if (tid == 0 && (s_commits || s_rounds)) {
    Spread* sp = spread_of(a.ws) + (c % kSpreadLines);
    if (s_commits) atomicAdd(&sp->commits, s_commits);
    atomicMax(&sp->rounds, s_rounds);
  }
}

__global__ __launch_bounds__(kRefThreads) __attribute__((amdgpu_waves_per_eu(4))) void refine_kernel(RefArgs a) {
  __shared__ RefShared sh;
  refine_body<false>(a, blockIdx.x, sh);
}

// The same with each chunk's queue divided over a.split workgroups (small
// fields: too few chunks to fill the chip).
__global__ __launch_bounds__(kRefThreads) __attribute__((amdgpu_waves_per_eu(4))) void refine_split_kernel(RefArgs a) {
  __shared__ RefShared sh;
  refine_body<true>(a, blockIdx.x, sh);
}

// Whole-field replay of the schedule over every queued saddle, by one
// workgroup with workgroup barriers.  Runs only when the clusters too large
// for the refine kernel do not fit the tail's LDS.  Clusters the refine
// kernel settled neither commit nor change here (their inputs are
// unchanged), and those it stopped at the round cap start settled, so only
// the large ones progress.  Returns the rounds run; the commits go to the
// control block.
template <int ND, int K>
__device__ unsigned replay_all(const RefArgs& a, const Plan& pl, const DecLayout& L) {
  __shared__ unsigned s_commits;
  const unsigned* cnt = reinterpret_cast<const unsigned*>(a.ws + L.cnt);
  const unsigned* idx = reinterpret_cast<const unsigned*>(a.ws + L.idx);
  uint8_t* state = a.ws + L.state;
  float* pend = reinterpret_cast<float*>(a.ws + L.pend);
  const uint8_t* labels = a.in + pl.s6_off;
  const unsigned long long* capped = reinterpret_cast<const unsigned long long*>(a.ws + L.capped);
  const unsigned tid = threadIdx.x, nthr = blockDim.x;
  // members of clusters that the refine kernel replayed up to the round cap
  // start settled: more rounds would take them past the cap
  for (int c = 0; c < pl.nch; ++c)
    for (unsigned t = tid; t < min(cnt[c], (unsigned)kChunk); t += nthr) {
      const unsigned p = idx[(size_t)c * kChunk + t];
      state[(size_t)c * kChunk + t] = (uint8_t)((capped[p >> 6] >> (p & 63)) & 1ull);
    }
  __syncthreads();
  int round = 1;
  unsigned long long total = 0;
  for (; round <= pl.max_rounds; ++round) {
    if (tid == 0) s_commits = 0;
    __syncthreads();
    for (int ph = 0; ph < pl.ncol; ++ph) {
      for (int c = 0; c < pl.nch; ++c) {
        const unsigned n = min(cnt[c], (unsigned)kChunk);
        for (unsigned t = tid; t < n; t += nthr) {
          const size_t sl = (size_t)c * kChunk + t;
          const int p = (int)idx[sl];
          const Pt pc = coords_of(p, pl.g);
          if (state[sl] || colour_of(pc, ND) != ph) continue;
          float v;
          const int res = evaluate<ND, K>(a.out, labels, p, pc, pl, &v);
          if (res == 1) {
            state[sl] = 1;
          } else if (res == 2) {
            pend[sl] = v;
            state[sl] = 2;
            atomicAdd(&s_commits, 1u);
          }
        }
      }
      __threadfence_block();
      __syncthreads();
      for (int c = 0; c < pl.nch; ++c) {
        const unsigned n = min(cnt[c], (unsigned)kChunk);
        for (unsigned t = tid; t < n; t += nthr) {
          const size_t sl = (size_t)c * kChunk + t;
          if (state[sl] == 2) {
            a.out[idx[sl]] = pend[sl];
            state[sl] = 1;
          }
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
  if (tid == 0) ctrl_of(a.ws)->rp_commits = total;
  return (unsigned)min(round, pl.max_rounds);
}

// The over-size clusters, gathered and replayed by the tail workgroup from
// LDS.  Clusters are independent of each other (no member lies in another
// cluster's read set), so replaying only these runs the same schedule on
// them as the whole-field replay, and leaves every other point as the refine
// kernel left it.
constexpr int kTailMax = 4096;             // members the tail holds
constexpr int kTailHash = 2 * kTailMax;    // open-addressing set of those members
constexpr unsigned kTailEmpty = 0xffffffffu;

struct TailShared {
  unsigned mem[kTailMax];
  union {
    unsigned hash[kTailHash];  // while gathering
    struct {
      float pend[kTailMax];
      uint8_t state[kTailMax];  // 0 open, 1 settled, 2 commit pending
    } r;                        // while replaying
  };
  unsigned nm, fail, commits;
};

// Gathers every queued saddle connected to one of the ns seeds, level by
// level.  Returns the member count, or 0 when they do not fit (the field is
// left untouched then).
template <int ND, int K>
__device__ unsigned gather_over(const unsigned long long* bm, const GeomD& g, const unsigned* seeds,
                                unsigned ns, TailShared& t) {
  using H = Hood<ND, K>;
  const unsigned tid = threadIdx.x, nthr = blockDim.x;
  for (unsigned i = tid; i < (unsigned)kTailHash; i += nthr) t.hash[i] = kTailEmpty;
  if (tid == 0) {
    t.nm = 0;
    t.fail = 0;
  }
  __syncthreads();
  // adds q unless present; every probe sequence is bounded by the table size
  auto insert = [&](unsigned q) {
    unsigned h = (q * 2654435761u) & (unsigned)(kTailHash - 1);
    for (int n = 0; n < kTailHash; ++n) {
      const unsigned old = atomicCAS(&t.hash[h], kTailEmpty, q);
      if (old == kTailEmpty) {
        const unsigned sl = atomicAdd(&t.nm, 1u);
        if (sl < (unsigned)kTailMax) t.mem[sl] = q;
        else t.fail = 1;
        return;
      }
      if (old == q) return;
      h = (h + 1) & (unsigned)(kTailHash - 1);
    }
    t.fail = 1;
  };
  for (unsigned i = tid; i < ns; i += nthr) insert(seeds[i]);
  __syncthreads();
  unsigned lo = 0;
  for (;;) {
    // the level's bounds, read by every thread before anyone inserts
    const unsigned hi = min(t.nm, (unsigned)kTailMax);
    const bool fail = t.fail != 0;
    __syncthreads();
    if (fail) return 0;
    if (lo == hi) return hi;
    for (unsigned i = lo + tid; i < hi; i += nthr) {
      const int cur = (int)t.mem[i];
      const Pt cc = coords_of(cur, g);
#pragma unroll 1
      for (int dz = -H::RZ; dz <= H::RZ; ++dz) {
        if ((unsigned)(cc.z + dz) >= (unsigned)g.nz) continue;
#pragma unroll 1
        for (int dy = -H::R; dy <= H::R; ++dy) {
          if ((unsigned)(cc.y + dy) >= (unsigned)g.ny) continue;
          for (int dx = -H::R; dx <= H::R; ++dx) {
            if (!H::read(dx, dy, dz) || (dx == 0 && dy == 0 && dz == 0)) continue;
            if ((unsigned)(cc.x + dx) >= (unsigned)g.nx) continue;
            const int q = cur + dz * g.nxy + dy * g.nx + dx;
            if ((bm[q >> 6] >> (q & 63)) & 1ull) insert((unsigned)q);
          }
        }
      }
    }
    __syncthreads();
    lo = hi;
  }
}

// The colour-phased Jacobi schedule over the nm gathered members.  Returns
// the rounds run; the commits go to the control block.
template <int ND, int K>
__device__ unsigned replay_list(const RefArgs& a, const Plan& pl, TailShared& t, unsigned nm) {
  const uint8_t* labels = a.in + pl.s6_off;
  const unsigned tid = threadIdx.x, nthr = blockDim.x;
  for (unsigned i = tid; i < nm; i += nthr) t.r.state[i] = 0;
  __syncthreads();
  int round = 1;
  unsigned long long total = 0;
  for (; round <= pl.max_rounds; ++round) {
    if (tid == 0) t.commits = 0;
    __syncthreads();
    for (int ph = 0; ph < pl.ncol; ++ph) {
      for (unsigned i = tid; i < nm; i += nthr) {
        if (t.r.state[i]) continue;
        const int p = (int)t.mem[i];
        const Pt pc = coords_of(p, pl.g);
        if (colour_of(pc, ND) != ph) continue;
        float v;
        const int res = evaluate<ND, K>(a.out, labels, p, pc, pl, &v);
        if (res == 1) {
          t.r.state[i] = 1;
        } else if (res == 2) {
          t.r.pend[i] = v;
          t.r.state[i] = 2;
          atomicAdd(&t.commits, 1u);
        }
      }
      __threadfence_block();
      __syncthreads();
      for (unsigned i = tid; i < nm; i += nthr)
        if (t.r.state[i] == 2) {
          a.out[t.mem[i]] = t.r.pend[i];
          t.r.state[i] = 1;
        }
      __threadfence_block();
      __syncthreads();
    }
    const unsigned commits = t.commits;
    __syncthreads();
    total += commits;
    if (commits == 0) break;
  }
  if (tid == 0) ctrl_of(a.ws)->rp_commits = total;
  return (unsigned)min(round, pl.max_rounds);
}

// Replays the over-size clusters from the recorded candidates; false (with
// nothing changed) when there are more candidates or members than the tail
// holds, and the whole-field replay has to run instead.
template <int ND, int K>
__device__ bool replay_over(const RefArgs& a, const Plan& pl, const DecLayout& L, unsigned ncand,
                            TailShared& t, unsigned* rounds) {
  if (ncand > (unsigned)kOverMax) return false;
  const unsigned long long* bm = reinterpret_cast<const unsigned long long*>(a.ws + L.bitmap);
  const unsigned nm = gather_over<ND, K>(bm, pl.g, ctrl_of(a.ws)->over, ncand, t);
  if (!nm) return false;
  *rounds = replay_list<ND, K>(a, pl, t, nm);
  return true;
}

// After the refine kernel (one workgroup of 256 threads): the replay of the
// clusters too large for it, if there are any.
__device__ __forceinline__ void tail_body(const RefArgs& a) {
  __shared__ Plan s_p;
  __shared__ unsigned s_big;
  __shared__ TailShared s_t;
  Ctrl* ct = ctrl_of(a.ws);
  if (threadIdx.x == 0) {
    s_big = 0;
    const unsigned big = ct->big;  // set only by a refine kernel that ran on a valid stream
    if (big) {
      s_p = ct->plan;
      s_big = big;
    }
  }
  __syncthreads();
  if (!s_big) return;
  const Plan& pl = s_p;
  const DecLayout L = dec_layout(((uint64_t)pl.g.n + kB - 1) / kB, (uint64_t)pl.nch);
  const unsigned nc = s_big;
  unsigned trounds = 0;
  switch (pl.ndim * 8 + pl.k) {
    case 2 * 8 + 3:
      if (!replay_over<2, 3>(a, pl, L, nc, s_t, &trounds)) trounds = replay_all<2, 3>(a, pl, L);
      break;
    case 2 * 8 + 5:
      if (!replay_over<2, 5>(a, pl, L, nc, s_t, &trounds)) trounds = replay_all<2, 5>(a, pl, L);
      break;
    case 2 * 8 + 7:
      if (!replay_over<2, 7>(a, pl, L, nc, s_t, &trounds)) trounds = replay_all<2, 7>(a, pl, L);
      break;
    case 3 * 8 + 3:
      if (!replay_over<3, 3>(a, pl, L, nc, s_t, &trounds)) trounds = replay_all<3, 3>(a, pl, L);
      break;
    case 3 * 8 + 5:
      if (!replay_over<3, 5>(a, pl, L, nc, s_t, &trounds)) trounds = replay_all<3, 5>(a, pl, L);
      break;
    default:
      if (!replay_over<3, 7>(a, pl, L, nc, s_t, &trounds)) trounds = replay_all<3, 7>(a, pl, L);
      break;
  }
  if (threadIdx.x == 0) ct->rp_rounds = trounds;
}

// The counters of the last decompression on a workspace, from the per-chunk
// counts of the decode kernel, the refine kernel's spread lines and the
// tail's replay (one workgroup, on request).
__global__ __launch_bounds__(1024) void stats_kernel(uint8_t* ws) {
  __shared__ Plan s_p;
  __shared__ unsigned s_ok, s_rounds;
  __shared__ unsigned long long s_sum[4];
  Ctrl* ct = ctrl_of(ws);
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_p = ct->plan;
    s_ok = ct->hflags == 0 && s_p.valid;
    s_sum[0] = s_sum[1] = s_sum[2] = s_sum[3] = 0;
    s_rounds = 0;
  }
  __syncthreads();
  const Plan& pl = s_p;
  const bool ok = s_ok != 0;
  unsigned long long q = 0, mv = 0, sk = 0, cm = 0;
  unsigned rd = 0;
  if (ok) {
    const DecLayout L = dec_layout(((uint64_t)pl.g.n + kB - 1) / kB, (uint64_t)pl.nch);
    const unsigned* cnt = reinterpret_cast<const unsigned*>(ws + L.cnt);
    const unsigned* mo = reinterpret_cast<const unsigned*>(ws + L.moves);
    const unsigned* skp = reinterpret_cast<const unsigned*>(ws + L.skips);
    for (int k = tid; k < pl.nch; k += blockDim.x) {
      q += cnt[k];
      mv += mo[k];
      sk += skp[k];
    }
  }
  if (tid < kSpreadLines) {
    const Spread* sp = spread_of(ws) + tid;
    cm = sp->commits;
    rd = sp->rounds;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    q += __shfl_xor(q, o);
    mv += __shfl_xor(mv, o);
    sk += __shfl_xor(sk, o);
    cm += __shfl_xor(cm, o);
    rd = max(rd, (unsigned)__shfl_xor((int)rd, o));
  }
  if ((tid & 63) == 0) {
    atomicAdd(&s_sum[0], q);
    atomicAdd(&s_sum[1], mv);
    atomicAdd(&s_sum[2], sk);
    atomicAdd(&s_sum[3], cm);
    if (rd) atomicMax(&s_rounds, rd);
  }
  __syncthreads();
  if (tid == 0) {
    const bool topo = ok && pl.topo;
    unsigned rounds = max(ct->rp_rounds, s_rounds);
    if (topo && rounds == 0) rounds = 1;  // a round that found nothing to do
    ct->stats[0] = topo ? rounds : 0;
    ct->stats[1] = ct->rp_commits + s_sum[3];
    ct->stats[2] = s_sum[0];
    ct->stats[3] = s_sum[1];
    ct->stats[4] = s_sum[2];
  }
}

__global__ __launch_bounds__(256) void tail_kernel(RefArgs a) { tail_body(a); }

// ---------------------------------------------------------------------------
// Topological errors of a reconstruction (Section III-B): per point, the
// class in the original and in the reconstruction; false negatives (a
// critical point that became regular), false positives (a regular point
// that became critical) and false types (critical in both, of another type),
// with the largest absolute difference.

__global__ void eval_clear_kernel(unsigned long long* counts, double* max_err) {
  if (threadIdx.x < 11) counts[threadIdx.x] = 0;
  if (threadIdx.x == 0) *max_err = 0.0;
}

template <int ND>
__global__ __launch_bounds__(256) void eval_kernel(const float* __restrict__ o, const float* __restrict__ r,
                                                   GeomD g, unsigned long long* counts, double* max_err) {
  __shared__ unsigned s_c[11];
  __shared__ unsigned long long s_m;
  const int tid = threadIdx.x;
  if (tid < 11) s_c[tid] = 0;
  if (tid == 0) s_m = 0;
  __syncthreads();
  const unsigned ndeg = (g.nx > 1 ? 1u : 0u) | (g.ny > 1 ? 4u : 0u) | (ND == 3 && g.nz > 1 ? 16u : 0u);
  unsigned c[11] = {0};
  double mx = 0.0;
  for (int i = blockIdx.x * 256 + tid; i < g.n; i += gridDim.x * 256) {
    const Pt pc = coords_of(i, g);
    unsigned avm = (pc.x > 0 ? 1u : 0u) | (pc.x < g.nx - 1 ? 2u : 0u) | (pc.y > 0 ? 4u : 0u) |
                   (pc.y < g.ny - 1 ? 8u : 0u);
    if (ND == 3) avm |= (pc.z > 0 ? 16u : 0u) | (pc.z < g.nz - 1 ? 32u : 0u);
    const int nbi[6] = {i - 1, i + 1, i - g.nx, i + g.nx, i - g.nxy, i + g.nxy};
    float no[6], nr[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const int q = ((avm >> j) & 1u) ? nbi[j] : i;
      no[j] = o[q];
      nr[j] = r[q];
    }
    const int lo = classify_bits(o[i], no, avm, ndeg), lr = classify_bits(r[i], nr, avm, ndeg);
    c[3 + lo]++;
    if (lo != CLS_R && lr == CLS_R) {
      c[0]++;
      c[7 + lo]++;
    }
    if (lo == CLS_R && lr != CLS_R) c[1]++;
    if (lo != CLS_R && lr != CLS_R && lo != lr) c[2]++;
    mx = fmax(mx, fabs((double)o[i] - (double)r[i]));
  }
#pragma unroll
  for (int k = 0; k < 11; ++k) {
    unsigned v = c[k];
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) v += (unsigned)__shfl_xor((int)v, s);
    if ((tid & 63) == 0 && v) atomicAdd(&s_c[k], v);
  }
  unsigned long long mb = (unsigned long long)__double_as_longlong(mx);  // non-negative: ordered as integers
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) mb = max(mb, (unsigned long long)__shfl_xor((long long)mb, s));
  if ((tid & 63) == 0) atomicMax(&s_m, mb);
  __syncthreads();
  if (tid < 11 && s_c[tid]) atomicAdd(&counts[tid], (unsigned long long)s_c[tid]);
  if (tid == 0) atomicMax(reinterpret_cast<unsigned long long*>(max_err), s_m);
}

// ---------------------------------------------------------------------------
// Batched form: many fields (or streams) in one launch per stage.  A table
// of per-field kernel arguments sits at the head of the workspace; a
// persistent grid walks the (field, chunk) items, each XCD taking a
// contiguous range of them, and runs the same bodies as the one-field
// kernels, so every field's bytes are those of a one-field call.

constexpr int kBatchMax = 4096;

struct CompJob {
  EncArgs enc;
  FinArgs fin;
  ScanArgs scan;
  int ndim, nrange;
};
struct DecJob {
  DecArgs dec;
  RefArgs ref;
};
struct BatchHdr {
  int count, n_range, n_chunk, n_slot;
};
// Table: BatchHdr, int pre_a[count + 1], int pre_b[count + 1], then the jobs
// (16-byte aligned).  Compression: pre_a over range items, pre_b over chunks;
// decompression: pre_a over decode/refine slots.
__host__ __device__ inline size_t tab_jobs_off(int count) {
  return (sizeof(BatchHdr) + 2 * sizeof(int) * (size_t)(count + 1) + 15) & ~size_t(15);
}

// Field owning `item`: the largest f with pre[f] <= item (empty fields skipped).
__device__ __forceinline__ int find_job(const int* pre, int count, int item) {
  int lo = 0, hi = count;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= item) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Items [0, T) over a grid of a multiple of 8 workgroups: XCD x (= workgroup
// mod 8) takes the x-th eighth of the items, its workgroups in turn.
template <typename Fn>
__device__ __forceinline__ void for_items(int T, Fn&& fn) {
  const int gx = (int)gridDim.x >> 3, x = (int)blockIdx.x & 7, j = (int)blockIdx.x >> 3;
  const int per = (T + 7) >> 3;
  const int end = min((x + 1) * per, T);
  for (int i = x * per + j; i < end; i += gx) {
    fn(i);
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void range_batch_kernel(const uint8_t* __restrict__ tab) {
  const BatchHdr* h = reinterpret_cast<const BatchHdr*>(tab);
  const int* pre = reinterpret_cast<const int*>(tab + sizeof(BatchHdr));
  const CompJob* jobs = reinterpret_cast<const CompJob*>(tab + tab_jobs_off(h->count));
  for_items(h->n_range, [&](int it) {
    const int f = find_job(pre, h->count, it);
    const CompJob& J = jobs[f];
    range_body(J.enc.f, J.enc.gd.n, J.enc.ws, it - pre[f], J.nrange);
  });
}

// At most 80 VGPRs (six waves per SIMD): both dimensions' bodies in one
// kernel otherwise take 81-213 VGPRs, and the batch measured 8% faster so.
template <int WAVES>
__global__ __launch_bounds__(WAVES * 64) __attribute__((amdgpu_waves_per_eu(6, 6))) void encode_batch_kernel(const uint8_t* __restrict__ tab) {
  __shared__ EncShared sh;
  const BatchHdr* h = reinterpret_cast<const BatchHdr*>(tab);
  const int* pre = reinterpret_cast<const int*>(tab + sizeof(BatchHdr)) + h->count + 1;
  const CompJob* jobs = reinterpret_cast<const CompJob*>(tab + tab_jobs_off(h->count));
  for_items(h->n_chunk, [&](int it) {
    const int f = find_job(pre, h->count, it);
    const CompJob& J = jobs[f];
    // (plain-SZp jobs take block mode's exact path: instantiating the plain
    // mode here too measured slower for the whole batch)
    if (J.ndim == 3) encode_body<3, WAVES>(J.enc, it - pre[f], sh);
    else encode_body<2, WAVES>(J.enc, it - pre[f], sh);
  });
}

__global__ __launch_bounds__(1024) void scan_batch_kernel(const uint8_t* __restrict__ tab) {
  const BatchHdr* h = reinterpret_cast<const BatchHdr*>(tab);
  const CompJob* jobs = reinterpret_cast<const CompJob*>(tab + tab_jobs_off(h->count));
  for_items(h->count, [&](int f) {
    if (!jobs[f].fin.fused) scan_body(jobs[f].scan);
  });
}

__global__ __launch_bounds__(256) void finalize_batch_kernel(const uint8_t* __restrict__ tab) {
  const BatchHdr* h = reinterpret_cast<const BatchHdr*>(tab);
  const int* pre = reinterpret_cast<const int*>(tab + sizeof(BatchHdr)) + h->count + 1;
  const CompJob* jobs = reinterpret_cast<const CompJob*>(tab + tab_jobs_off(h->count));
  for_items(h->n_chunk, [&](int it) {
    const int f = find_job(pre, h->count, it);
    finalize_body(jobs[f].fin, it - pre[f]);
  });
}

template <int WAVES>
__global__ __launch_bounds__(WAVES * 64) __attribute__((amdgpu_waves_per_eu(8))) void decode_batch_kernel(const uint8_t* __restrict__ tab) {
  const BatchHdr* h = reinterpret_cast<const BatchHdr*>(tab);
  const int* pre = reinterpret_cast<const int*>(tab + sizeof(BatchHdr));
  const DecJob* jobs = reinterpret_cast<const DecJob*>(tab + tab_jobs_off(h->count));
  for_items(h->n_slot, [&](int it) {
    const int f = find_job(pre, h->count, it);
    decode_body<WAVES>(jobs[f].dec, it - pre[f]);
  });
}

__global__ __launch_bounds__(kRefThreads) __attribute__((amdgpu_waves_per_eu(4))) void refine_batch_kernel(
    const uint8_t* __restrict__ tab) {
  __shared__ RefShared sh;
  const BatchHdr* h = reinterpret_cast<const BatchHdr*>(tab);
  const int* pre = reinterpret_cast<const int*>(tab + sizeof(BatchHdr));
  const DecJob* jobs = reinterpret_cast<const DecJob*>(tab + tab_jobs_off(h->count));
  for_items(h->n_slot, [&](int it) {
    const int f = find_job(pre, h->count, it);
    refine_body<false>(jobs[f].ref, it - pre[f], sh);
  });
}

__global__ __launch_bounds__(256) void tail_batch_kernel(const uint8_t* __restrict__ tab) {
  const BatchHdr* h = reinterpret_cast<const BatchHdr*>(tab);
  const DecJob* jobs = reinterpret_cast<const DecJob*>(tab + tab_jobs_off(h->count));
  for_items(h->count, [&](int f) { tail_body(jobs[f].ref); });
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

// timing (a diagnostic for one host thread: the events are shared)
std::atomic<bool> g_timing{false};
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

// Field-scope compression: sort keys and indices (in and out), ranks per
// point, and the per-chunk counts and their scan, after the compression
// region.
struct FieldLayout {
  uint64_t keys_in, vals_in, keys_out, vals_out, delta, ccnt, coff, end;
};
FieldLayout field_layout(const HostGeom& hg) {
  FieldLayout F;
  const uint64_t n = (uint64_t)hg.g.n;
  F.keys_in = al256(comp_layout(hg.nch, 1).end);
  F.vals_in = al256(F.keys_in + 8 * n);
  F.keys_out = al256(F.vals_in + 4 * n);
  F.vals_out = al256(F.keys_out + 8 * n);
  F.delta = al256(F.vals_out + 4 * n);
  F.ccnt = al256(F.delta + 4 * n);
  F.coff = al256(F.ccnt + 4 * hg.nch);
  F.end = al256(F.coff + 4 * (hg.nch + 1));
  return F;
}
size_t ws_need_field(const HostGeom& hg) {
  const uint64_t c = field_layout(hg).end, d = dec_layout(hg.nb, hg.nch).end;
  return (size_t)(c > d ? c : d);
}

size_t ws_need_n(uint64_t n) {
  const uint64_t nb = (n + kB - 1) / kB, nch = (nb + kB - 1) / kB;
  const uint64_t c = comp_layout(nch).end, d = dec_layout(nb, nch).end;
  return (size_t)al256(c > d ? c : d);
}

// Launch shapes (they change no byte of any result), one byte each in one
// word, so that a call on any host thread reads a consistent set.
std::atomic<uint32_t> g_tune{8u | 4u << 8 | 8u << 16 | 8u << 24};  // {8, 4, 8, 8}: measured fastest for one field
toposzp_tuning tune_now() {
  const uint32_t w = g_tune.load(std::memory_order_relaxed);
  return {(int32_t)(w & 255u), (int32_t)(w >> 8 & 255u), (int32_t)(w >> 16 & 255u), (int32_t)(w >> 24)};
}
void tune_set(const toposzp_tuning& t) {
  g_tune.store((uint32_t)t.encode_waves | (uint32_t)t.decode_waves << 8 | (uint32_t)t.compress_wgs_per_cu << 16 |
                   (uint32_t)t.decompress_wgs_per_cu << 24,
               std::memory_order_relaxed);
}

bool tuning_ok(const toposzp_tuning& t) {
  auto wgs = [](int v) { return v >= 1 && v <= 32; };
  return (t.encode_waves == 4 || t.encode_waves == 8) && (t.decode_waves == 4 || t.decode_waves == 8) &&
         wgs(t.compress_wgs_per_cu) && wgs(t.decompress_wgs_per_cu);
}

std::atomic<int> g_cus[64];  // compute units per device, 0 until first asked
int cu_count() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int c = g_cus[dev].load(std::memory_order_relaxed);
  if (!c) {
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 1) c = 256;
    g_cus[dev].store(c, std::memory_order_relaxed);
  }
  return c;
}

// Persistent grid: wgs_per_cu workgroups per CU, a multiple of 8, at most
// what the items need (rounded up to 8).
unsigned batch_grid(int items, int wgs_per_cu) {
  long long g = (long long)cu_count() * wgs_per_cu;
  const long long need = ((long long)items + 7) / 8 * 8;
  if (g > need) g = need;
  if (g < 8) g = 8;
  return (unsigned)((g + 7) / 8 * 8);
}

// Checks one compression request and fills its kernel arguments.
int build_comp(const float* d_field, uint32_t ndim, const uint64_t* dims, int eb_mode, double eb,
               const toposzp_params* params, uint8_t* d_ws, size_t ws_bytes, uint8_t* d_out, size_t out_cap,
               uint64_t* d_out_size, int32_t* d_status, CompJob* J, bool allow_field = true,
               bool comp_only = false) {
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
  const int field = p.rank_scope == 1 && p.topo ? 1 : 0;
  if (field && !allow_field) return TOPOSZP_E_UNSUPPORTED;
  if (out_cap < toposzp_compress_bound_ex(ndim, dims, field)) return TOPOSZP_E_CAPACITY;
  const size_t need = comp_only ? (size_t)al256(comp_layout(hg.nch).end) : field ? ws_need_field(hg) : ws_need(hg);
  if (ws_bytes < need) return TOPOSZP_E_CAPACITY;

  int nrange = (int)((hg.g.n / 4 + 256 * kRangeVec - 1) / (256 * kRangeVec));
  if (nrange > kRangeWG) nrange = kRangeWG;
  if (nrange < 1) nrange = 1;
  const float e_abs = host_round_down(eb);

  EncArgs& ea = J->enc;
  ea.f = d_field;
  ea.out = d_out;
  ea.ws = d_ws;
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
  ea.field = field;
  ea.keys = nullptr;
  ea.vals = nullptr;
  ea.skeys = nullptr;
  ea.svals = nullptr;
  ea.ccnt = nullptr;
  ea.delta = nullptr;
  if (field) {
    // the mark pass stages in the sort's output arrays, compacts into its input
    const FieldLayout F = field_layout(hg);
    ea.keys = reinterpret_cast<unsigned long long*>(d_ws + F.keys_in);
    ea.vals = reinterpret_cast<unsigned*>(d_ws + F.vals_in);
    ea.skeys = reinterpret_cast<unsigned long long*>(d_ws + F.keys_out);
    ea.svals = reinterpret_cast<unsigned*>(d_ws + F.vals_out);
    ea.ccnt = reinterpret_cast<unsigned*>(d_ws + F.ccnt);
    ea.delta = reinterpret_cast<const int*>(d_ws + F.delta);
  }

  ScanArgs& sa = J->scan;
  sa.ws = d_ws;
  sa.nch = ea.nch;
  sa.eb_mode = eb_mode;
  sa.nrange = nrange;
  sa.eb = eb;
  sa.e_abs = e_abs;
  sa.field = field;

  FinArgs& fa = J->fin;
  fa.out = d_out;
  fa.ws = d_ws;
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
  fa.e_abs = e_abs;
  fa.nrange = nrange;
  fa.fused = ea.nch <= kFuseMax ? 1 : 0;
  fa.field = field;
  memcpy(fa.off, ea.off, sizeof(ea.off));
  memcpy(fa.len, ea.len, sizeof(ea.len));
  const double sig[3] = {0.5, 0.75, 1.0};
  for (int t = 0; t < 3; ++t)
    for (int d2 = 0; d2 < 10; ++d2) fa.wtab[t][d2] = (float)exp(-(double)d2 / (2.0 * sig[t] * sig[t]));
  J->ndim = (int)ndim;
  J->nrange = eb_mode == TOPOSZP_EB_REL ? nrange : 0;
  return TOPOSZP_OK;
}

// Checks one decompression request and fills its kernel arguments; *slots
// receives the workgroup slots its capacity needs.
int build_dec(const uint8_t* d_in, size_t in_size, float* d_out, size_t out_cap_elems, uint8_t* d_ws,
              size_t ws_bytes, int32_t* d_status, DecJob* J, int* slots) {
  if (!d_in || !d_out || !d_ws || !d_status || out_cap_elems < 1) return TOPOSZP_E_INVALID_ARG;
  if (((uintptr_t)d_in & 7) || ((uintptr_t)d_out & 3) || ((uintptr_t)d_ws & 255) || ((uintptr_t)d_status & 3))
    return TOPOSZP_E_INVALID_ARG;
  if (ws_bytes < kRegionOff + 4096) return TOPOSZP_E_CAPACITY;
  uint64_t cap = out_cap_elems;
  if (cap > (1ull << 31)) cap = (1ull << 31);
  const uint64_t nch = ((cap + kB - 1) / kB + kB - 1) / kB;
  DecArgs& da = J->dec;
  da.in = d_in;
  da.in_size = in_size;
  da.out = d_out;
  da.out_cap = out_cap_elems;
  da.ws = d_ws;
  da.ws_bytes = ws_bytes;
  RefArgs& ra = J->ref;
  ra.in = d_in;
  ra.out = d_out;
  ra.ws = d_ws;
  ra.status = d_status;
  *slots = xcd_grid((int)nch);
  ra.slots = *slots;
  ra.split = 1;
  return TOPOSZP_OK;
}

void launch_encode(int ndim, int waves, unsigned grid, hipStream_t s, const EncArgs& ea) {
  if (!ea.topo) {
    if (ndim == 3 && waves == 8) hipLaunchKernelGGL((encode_kernel<3, 8, kModePlain>), dim3(grid), dim3(512), 0, s, ea);
    else if (ndim == 3) hipLaunchKernelGGL((encode_kernel<3, 4, kModePlain>), dim3(grid), dim3(256), 0, s, ea);
    else if (waves == 8) hipLaunchKernelGGL((encode_kernel<2, 8, kModePlain>), dim3(grid), dim3(512), 0, s, ea);
    else hipLaunchKernelGGL((encode_kernel<2, 4, kModePlain>), dim3(grid), dim3(256), 0, s, ea);
    return;
  }
  if (ndim == 3 && waves == 8) hipLaunchKernelGGL((encode_kernel<3, 8>), dim3(grid), dim3(512), 0, s, ea);
  else if (ndim == 3) hipLaunchKernelGGL((encode_kernel<3, 4>), dim3(grid), dim3(256), 0, s, ea);
  else if (waves == 8) hipLaunchKernelGGL((encode_kernel<2, 8>), dim3(grid), dim3(512), 0, s, ea);
  else hipLaunchKernelGGL((encode_kernel<2, 4>), dim3(grid), dim3(256), 0, s, ea);
}

// Batch workspace: the table, then one single-field workspace per job.
size_t comp_batch_layout(uint32_t count, const toposzp_compress_job* jobs, size_t* offs) {
  size_t off = (size_t)al256(tab_jobs_off((int)count) + count * sizeof(CompJob));
  for (uint32_t i = 0; i < count; ++i) {
    HostGeom hg;
    if (host_geom(jobs[i].ndim, jobs[i].dims, &hg) != TOPOSZP_OK) return 0;
    if (offs) offs[i] = off;
    off += ws_need(hg);
  }
  return off;
}
size_t dec_batch_layout(uint32_t count, const toposzp_decompress_job* jobs, size_t* offs) {
  size_t off = (size_t)al256(tab_jobs_off((int)count) + count * sizeof(DecJob));
  for (uint32_t i = 0; i < count; ++i) {
    uint64_t cap = jobs[i].out_cap_elems;
    if (cap < 1) return 0;
    if (cap > (1ull << 31)) cap = 1ull << 31;
    if (offs) offs[i] = off;
    off += ws_need_n(cap);
  }
  return off;
}

// Times `run` (one enqueue of the batch) under each candidate tuning and
// keeps the fastest: 2 untimed runs, then the median of 5 timed ones.
template <typename Run>
int autotune(const std::vector<toposzp_tuning>& cands, hipStream_t s, Run&& run, toposzp_tuning* out) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return TOPOSZP_E_DEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return TOPOSZP_E_DEVICE;
  }
  const toposzp_tuning saved = tune_now();
  toposzp_tuning best = saved;
  float best_ms = 1e30f;
  int rc = TOPOSZP_OK;
  for (const toposzp_tuning& t : cands) {
    tune_set(t);
    float ms[5];
    for (int r = 0; r < 7 && rc == TOPOSZP_OK; ++r) {
      if (r >= 2 && hipEventRecord(e0, s) != hipSuccess) rc = TOPOSZP_E_DEVICE;
      if (rc == TOPOSZP_OK) rc = run();
      if (rc == TOPOSZP_OK && r >= 2) {
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms[r - 2], e0, e1) != hipSuccess)
          rc = TOPOSZP_E_DEVICE;
      }
    }
    if (rc != TOPOSZP_OK) break;
    std::sort(ms, ms + 5);
    if (ms[2] < best_ms) {
      best_ms = ms[2];
      best = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  tune_set(rc == TOPOSZP_OK ? best : saved);
  if (out) *out = tune_now();
  return rc;
}

// Scratch of the allocation-free compression call: the compression region
// of a workspace for the largest field that call accepts.  Every device the
// library runs on holds one copy until the process ends.
constexpr uint64_t kNoAllocMaxPoints = 1ull << 24;
constexpr size_t kScratchBytes = (size_t)al256(comp_layout(kNoAllocMaxPoints / kChunk).end);
static_assert(kNoAllocMaxPoints / kChunk <= (uint64_t)kFuseMax, "the scratch path uses the fused scan");
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

// Device address of `scratch` on the current device, looked up once per
// device (host code must never pass the symbol itself to a kernel).
std::mutex g_scratch_mu;
std::atomic<uint8_t*> g_scratch[64];
int scratch_of_device(uint8_t** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return TOPOSZP_E_DEVICE;
  uint8_t* p = g_scratch[dev].load(std::memory_order_acquire);
  if (!p) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    p = g_scratch[dev].load(std::memory_order_relaxed);
    if (!p) {
      void* q = nullptr;
      if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || !q) return TOPOSZP_E_DEVICE;
      p = static_cast<uint8_t*>(q);
      g_scratch[dev].store(p, std::memory_order_release);
    }
  }
  *out = p;
  return TOPOSZP_OK;
}

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

size_t toposzp_compress_bound_ex(uint32_t ndim, const uint64_t* dims, int32_t rank_scope) {
  HostGeom hg;
  if (host_geom(ndim, dims, &hg) != TOPOSZP_OK || (rank_scope != 0 && rank_scope != 1)) return 0;
  uint64_t off[kNSeg], len[kNSeg];
  return (size_t)seg_layout(hg.nb, 1, hg.nb * kMaxWData, hg.nb * (uint64_t)rank_w(rank_scope), off, len);
}

size_t toposzp_workspace_size_ex(uint32_t ndim, const uint64_t* dims, int32_t rank_scope) {
  HostGeom hg;
  if (host_geom(ndim, dims, &hg) != TOPOSZP_OK || (rank_scope != 0 && rank_scope != 1)) return 0;
  return rank_scope ? ws_need_field(hg) : ws_need(hg);
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
  CompJob J;
  const int rc = build_comp(d_field, ndim, dims, eb_mode, eb, params, (uint8_t*)d_ws, ws_bytes, d_out, out_cap,
                            d_out_size, d_status, &J);
  if (rc != TOPOSZP_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  const EncArgs& ea = J.enc;
  if (g_timing)
    for (int k = 0; k < 3; ++k) g_ev_used[k] = false;
  if (eb_mode == TOPOSZP_EB_REL) {
    ev_begin(0, s);
    hipLaunchKernelGGL(range_kernel, dim3(ea.nrange), dim3(256), 0, s, d_field, ea.gd.n, (uint8_t*)d_ws);
    ev_end(0, s);
  }
  ev_begin(1, s);
  if (ea.field) {
    // field-scope ranks: the mark pass compacts the flattened extrema's sort
    // keys per chunk; their counts are scanned, the keys sorted by (class,
    // bin, order) and ranked, and the encode pass reads the ranks.  Every
    // count stays on the device.
    HostGeom hg;
    (void)host_geom(ndim, dims, &hg);
    const FieldLayout F = field_layout(hg);
    uint8_t* ws = (uint8_t*)d_ws;
    const unsigned grid = xcd_grid(ea.nch);
    if (ndim == 3) hipLaunchKernelGGL((encode_kernel<3, 8, kModeMark>), dim3(grid), dim3(512), 0, s, ea);
    else hipLaunchKernelGGL((encode_kernel<2, 8, kModeMark>), dim3(grid), dim3(512), 0, s, ea);
    auto K = [&](uint64_t o) { return reinterpret_cast<unsigned long long*>(ws + o); };
    auto V = [&](uint64_t o) { return reinterpret_cast<unsigned*>(ws + o); };
    const unsigned* ccnt = V(F.ccnt);
    const unsigned* coff = V(F.coff);
    // runs of one chunk into the "out" arrays, then four-way merges back and
    // forth; the sorted keys end where the last pass wrote them
    hipLaunchKernelGGL(fs_sort_kernel, dim3(ea.nch), dim3(kFsThreads), 0, s, K(F.keys_in), V(F.vals_in), ccnt,
                       V(F.coff), ea.nch, ws, K(F.keys_out), V(F.vals_out));
    const unsigned mg = (unsigned)std::min<uint64_t>(((uint64_t)hg.g.n + 1023) / 1024, 2048);
    bool in_out = true;  // the current run arrays are the "out" ones
    for (int L = 0; (1ll << (2 * L)) < ea.nch; ++L) {
      // one LDS workgroup per group while the groups are many, then the
      // grid-wide pass with its searches in L2
      const long long groups = ((long long)ea.nch + (1ll << (2 * L + 2)) - 1) >> (2 * L + 2);
      const unsigned long long* ik = K(in_out ? F.keys_out : F.keys_in);
      const unsigned* iv = V(in_out ? F.vals_out : F.vals_in);
      unsigned long long* ok = K(in_out ? F.keys_in : F.keys_out);
      unsigned* ov = V(in_out ? F.vals_in : F.vals_out);
      if (groups >= 64)
        hipLaunchKernelGGL(fs_merge_lds_kernel, dim3((unsigned)groups), dim3(1024), 0, s, ik, iv, coff, ea.nch, L, ok,
                           ov);
      else
        hipLaunchKernelGGL(fs_merge_kernel, dim3(mg), dim3(256), 0, s, ik, iv, coff, ea.nch, L, ok, ov);
      in_out = !in_out;
    }
    hipLaunchKernelGGL(fs_rank_kernel, dim3(mg), dim3(256), 0, s, K(in_out ? F.keys_out : F.keys_in),
                       V(in_out ? F.vals_out : F.vals_in), coff, ea.nch, reinterpret_cast<int*>(ws + F.delta));
    if (ndim == 3) hipLaunchKernelGGL((encode_kernel<3, 8, kModeField>), dim3(grid), dim3(512), 0, s, ea);
    else hipLaunchKernelGGL((encode_kernel<2, 8, kModeField>), dim3(grid), dim3(512), 0, s, ea);
  } else {
    launch_encode((int)ndim, tune_now().encode_waves, xcd_grid(ea.nch), s, ea);
  }
  ev_end(1, s);
  ev_begin(2, s);
  if (!J.fin.fused) hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, J.scan);
  hipLaunchKernelGGL(finalize_kernel, dim3(xcd_grid(ea.nch)), dim3(256), 0, s, J.fin);
  ev_end(2, s);
  return hipGetLastError() == hipSuccess ? TOPOSZP_OK : TOPOSZP_E_DEVICE;
}

int toposzp_compress_noalloc(const float* d_field, uint32_t ndim, const uint64_t* dims, int eb_mode, double eb,
                             const toposzp_params* params, uint8_t* d_out, size_t out_cap, uint64_t* d_out_size,
                             int32_t* d_status, void* stream) {
  // host checks first: nothing touches the device for a rejected request
  HostGeom hg;
  int rc = host_geom(ndim, dims, &hg);
  if (rc != TOPOSZP_OK) return rc;
  if ((uint64_t)hg.g.n > kNoAllocMaxPoints) return TOPOSZP_E_CAPACITY;
  if (params && params->rank_scope == 1 && params->topo) return TOPOSZP_E_UNSUPPORTED;
  uint8_t* ws = nullptr;
  rc = scratch_of_device(&ws);
  if (rc != TOPOSZP_OK) return rc;
  CompJob J;
  rc = build_comp(d_field, ndim, dims, eb_mode, eb, params, ws, kScratchBytes, d_out, out_cap, d_out_size,
                  d_status, &J, false, true);
  if (rc != TOPOSZP_OK) return rc;
  // the kernels of toposzp_compress on the scratch; each writes every byte
  // of the scratch that a later one reads, so nothing there needs clearing
  hipStream_t s = (hipStream_t)stream;
  const EncArgs& ea = J.enc;
  if (eb_mode == TOPOSZP_EB_REL)
    hipLaunchKernelGGL(range_kernel, dim3(ea.nrange), dim3(256), 0, s, d_field, ea.gd.n, ws);
  launch_encode((int)ndim, tune_now().encode_waves, xcd_grid(ea.nch), s, ea);
  hipLaunchKernelGGL(finalize_kernel, dim3(xcd_grid(ea.nch)), dim3(256), 0, s, J.fin);
  return hipGetLastError() == hipSuccess ? TOPOSZP_OK : TOPOSZP_E_DEVICE;
}

int toposzp_decompress(const uint8_t* d_in, size_t in_size, float* d_out, size_t out_cap_elems,
                       void* d_ws, size_t ws_bytes, int32_t* d_status, void* stream) {
  DecJob J;
  int slots = 0;
  const int rc = build_dec(d_in, in_size, d_out, out_cap_elems, (uint8_t*)d_ws, ws_bytes, d_status, &J, &slots);
  if (rc != TOPOSZP_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (g_timing)
    for (int k = 3; k < 5; ++k) g_ev_used[k] = false;
  ev_begin(3, s);
  if (tune_now().decode_waves == 8)
    hipLaunchKernelGGL(decode_kernel<8>, dim3(slots), dim3(512), 0, s, J.dec);
  else
    hipLaunchKernelGGL(decode_kernel<4>, dim3(slots), dim3(256), 0, s, J.dec);
  ev_end(3, s);
  ev_begin(4, s);
  // a small field divides each chunk's queue over up to 8 workgroups, so that
  // the few chunks with many clusters do not each hold one workgroup alone
  // (the division changes no result)
  while (J.ref.split < 8 && slots * J.ref.split < 1024) J.ref.split *= 2;
  if (J.ref.split > 1)
    hipLaunchKernelGGL(refine_split_kernel, dim3(slots * J.ref.split), dim3(kRefThreads), 0, s, J.ref);
  else
    hipLaunchKernelGGL(refine_kernel, dim3(slots), dim3(kRefThreads), 0, s, J.ref);
  hipLaunchKernelGGL(tail_kernel, dim3(1), dim3(256), 0, s, J.ref);
  ev_end(4, s);
  return hipGetLastError() == hipSuccess ? TOPOSZP_OK : TOPOSZP_E_DEVICE;
}

int toposzp_eval(const float* d_orig, const float* d_recon, uint32_t ndim, const uint64_t* dims,
                 int64_t* d_counts, double* d_max_err, void* stream) {
  HostGeom hg;
  const int rc = host_geom(ndim, dims, &hg);
  if (rc != TOPOSZP_OK) return rc;
  if (!d_orig || !d_recon || !d_counts || !d_max_err || ((uintptr_t)d_orig & 3) || ((uintptr_t)d_recon & 3) ||
      ((uintptr_t)d_counts & 7) || ((uintptr_t)d_max_err & 7))
    return TOPOSZP_E_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  GeomD g;
  g.n = hg.g.n;
  g.nx = hg.g.nx;
  g.ny = hg.g.ny;
  g.nz = hg.g.nz;
  g.nxy = hg.g.nx * hg.g.ny;
  g.dx = make_div((unsigned)g.nx);
  g.dy = make_div((unsigned)g.ny);
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(d_counts);
  hipLaunchKernelGGL(eval_clear_kernel, dim3(1), dim3(64), 0, s, cnt, d_max_err);
  const unsigned grid = (unsigned)std::min<long long>(((long long)g.n + 255) / 256, 4096);
  if (ndim == 3)
    hipLaunchKernelGGL(eval_kernel<3>, dim3(grid), dim3(256), 0, s, d_orig, d_recon, g, cnt, d_max_err);
  else
    hipLaunchKernelGGL(eval_kernel<2>, dim3(grid), dim3(256), 0, s, d_orig, d_recon, g, cnt, d_max_err);
  return hipGetLastError() == hipSuccess ? TOPOSZP_OK : TOPOSZP_E_DEVICE;
}

size_t toposzp_compress_batch_workspace_size(uint32_t count, const toposzp_compress_job* h_jobs) {
  if (count < 1 || count > (uint32_t)kBatchMax || !h_jobs) return 0;
  return comp_batch_layout(count, h_jobs, nullptr);
}

size_t toposzp_decompress_batch_workspace_size(uint32_t count, const toposzp_decompress_job* h_jobs) {
  if (count < 1 || count > (uint32_t)kBatchMax || !h_jobs) return 0;
  return dec_batch_layout(count, h_jobs, nullptr);
}

int toposzp_compress_batch(uint32_t count, const toposzp_compress_job* h_jobs, const toposzp_params* params,
                           void* d_ws, size_t ws_bytes, void* stream) {
  if (count < 1 || count > (uint32_t)kBatchMax || !h_jobs || !d_ws || ((uintptr_t)d_ws & 255))
    return TOPOSZP_E_INVALID_ARG;
  std::vector<size_t> offs(count);
  const size_t need = comp_batch_layout(count, h_jobs, offs.data());
  if (need == 0) return TOPOSZP_E_INVALID_ARG;
  if (ws_bytes < need) return TOPOSZP_E_CAPACITY;
  const size_t jo = tab_jobs_off((int)count);
  std::vector<uint8_t> tab(jo + count * sizeof(CompJob));
  BatchHdr* h = reinterpret_cast<BatchHdr*>(tab.data());
  int* pre_r = reinterpret_cast<int*>(tab.data() + sizeof(BatchHdr));
  int* pre_c = pre_r + count + 1;
  CompJob* jobs = reinterpret_cast<CompJob*>(tab.data() + jo);
  uint8_t* ws = (uint8_t*)d_ws;
  long long nr = 0, nc = 0;
  bool any_scan = false;
  for (uint32_t i = 0; i < count; ++i) {
    const toposzp_compress_job& q = h_jobs[i];
    const size_t wsz = (i + 1 < count ? offs[i + 1] : need) - offs[i];
    const int rc = build_comp(q.d_field, q.ndim, q.dims, q.eb_mode, q.eb, params, ws + offs[i], wsz, q.d_out,
                              q.out_cap, q.d_out_size, q.d_status, &jobs[i], false);
    if (rc != TOPOSZP_OK) return rc;
    pre_r[i] = (int)nr;
    pre_c[i] = (int)nc;
    nr += jobs[i].nrange;
    nc += jobs[i].enc.nch;
    any_scan |= !jobs[i].fin.fused;
    if (nr > INT32_MAX / 2 || nc > INT32_MAX / 2) return TOPOSZP_E_UNSUPPORTED;
  }
  pre_r[count] = (int)nr;
  pre_c[count] = (int)nc;
  h->count = (int)count;
  h->n_range = (int)nr;
  h->n_chunk = (int)nc;
  h->n_slot = 0;
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(ws, tab.data(), tab.size(), hipMemcpyHostToDevice, s) != hipSuccess) return TOPOSZP_E_DEVICE;
  const toposzp_tuning tn = tune_now();
  const int wpc = tn.compress_wgs_per_cu;
  if (nr > 0) hipLaunchKernelGGL(range_batch_kernel, dim3(batch_grid((int)nr, wpc)), dim3(256), 0, s, ws);
  if (tn.encode_waves == 8)
    hipLaunchKernelGGL(encode_batch_kernel<8>, dim3(batch_grid((int)nc, wpc)), dim3(512), 0, s, ws);
  else
    hipLaunchKernelGGL(encode_batch_kernel<4>, dim3(batch_grid((int)nc, wpc)), dim3(256), 0, s, ws);
  if (any_scan) hipLaunchKernelGGL(scan_batch_kernel, dim3(batch_grid((int)count, 1)), dim3(1024), 0, s, ws);
  hipLaunchKernelGGL(finalize_batch_kernel, dim3(batch_grid((int)nc, wpc)), dim3(256), 0, s, ws);
  return hipGetLastError() == hipSuccess ? TOPOSZP_OK : TOPOSZP_E_DEVICE;
}

int toposzp_decompress_batch(uint32_t count, const toposzp_decompress_job* h_jobs, void* d_ws, size_t ws_bytes,
                             void* stream) {
  if (count < 1 || count > (uint32_t)kBatchMax || !h_jobs || !d_ws || ((uintptr_t)d_ws & 255))
    return TOPOSZP_E_INVALID_ARG;
  std::vector<size_t> offs(count);
  const size_t need = dec_batch_layout(count, h_jobs, offs.data());
  if (need == 0) return TOPOSZP_E_INVALID_ARG;
  if (ws_bytes < need) return TOPOSZP_E_CAPACITY;
  const size_t jo = tab_jobs_off((int)count);
  std::vector<uint8_t> tab(jo + count * sizeof(DecJob));
  BatchHdr* h = reinterpret_cast<BatchHdr*>(tab.data());
  int* pre = reinterpret_cast<int*>(tab.data() + sizeof(BatchHdr));
  DecJob* jobs = reinterpret_cast<DecJob*>(tab.data() + jo);
  uint8_t* ws = (uint8_t*)d_ws;
  long long ns = 0;
  for (uint32_t i = 0; i < count; ++i) {
    const toposzp_decompress_job& q = h_jobs[i];
    const size_t wsz = (i + 1 < count ? offs[i + 1] : need) - offs[i];
    int slots = 0;
    const int rc = build_dec(q.d_in, q.in_size, q.d_out, q.out_cap_elems, ws + offs[i], wsz, q.d_status, &jobs[i],
                             &slots);
    if (rc != TOPOSZP_OK) return rc;
    pre[i] = (int)ns;
    ns += slots;
    if (ns > INT32_MAX / 2) return TOPOSZP_E_UNSUPPORTED;
  }
  pre[count] = (int)ns;
  h->count = (int)count;
  h->n_range = (int)ns;
  h->n_chunk = 0;
  h->n_slot = (int)ns;
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(ws, tab.data(), tab.size(), hipMemcpyHostToDevice, s) != hipSuccess) return TOPOSZP_E_DEVICE;
  const toposzp_tuning tn = tune_now();
  const int wpc = tn.decompress_wgs_per_cu;
  if (tn.decode_waves == 8)
    hipLaunchKernelGGL(decode_batch_kernel<8>, dim3(batch_grid((int)ns, wpc)), dim3(512), 0, s, ws);
  else
    hipLaunchKernelGGL(decode_batch_kernel<4>, dim3(batch_grid((int)ns, wpc)), dim3(256), 0, s, ws);
  hipLaunchKernelGGL(refine_batch_kernel, dim3(batch_grid((int)ns, 2 * wpc)), dim3(kRefThreads), 0, s, ws);
  hipLaunchKernelGGL(tail_batch_kernel, dim3(batch_grid((int)count, 1)), dim3(256), 0, s, ws);
  return hipGetLastError() == hipSuccess ? TOPOSZP_OK : TOPOSZP_E_DEVICE;
}

int toposzp_decompress_batch_stats(uint32_t count, const toposzp_decompress_job* h_jobs, void* d_ws,
                                   uint32_t index, int64_t out[5], void* stream) {
  if (count < 1 || count > (uint32_t)kBatchMax || !h_jobs || !d_ws || index >= count || !out)
    return TOPOSZP_E_INVALID_ARG;
  std::vector<size_t> offs(count);
  if (dec_batch_layout(count, h_jobs, offs.data()) == 0) return TOPOSZP_E_INVALID_ARG;
  return toposzp_decompress_stats((uint8_t*)d_ws + offs[index], out, stream);
}

int toposzp_set_tuning(const toposzp_tuning* t) {
  if (!t || !tuning_ok(*t)) return TOPOSZP_E_INVALID_ARG;
  tune_set(*t);
  return TOPOSZP_OK;
}

int toposzp_get_tuning(toposzp_tuning* t) {
  if (!t) return TOPOSZP_E_INVALID_ARG;
  *t = tune_now();
  return TOPOSZP_OK;
}

int toposzp_autotune_compress_batch(uint32_t count, const toposzp_compress_job* h_jobs,
                                    const toposzp_params* params, void* d_ws, size_t ws_bytes, void* stream,
                                    toposzp_tuning* out) {
  std::vector<toposzp_tuning> c;
  const toposzp_tuning cur = tune_now();
  for (int w : {4, 8})
    for (int g : {2, 4, 8, 16}) c.push_back({w, cur.decode_waves, g, cur.decompress_wgs_per_cu});
  return autotune(c, (hipStream_t)stream,
                  [&]() { return toposzp_compress_batch(count, h_jobs, params, d_ws, ws_bytes, stream); }, out);
}

int toposzp_autotune_decompress_batch(uint32_t count, const toposzp_decompress_job* h_jobs, void* d_ws,
                                      size_t ws_bytes, void* stream, toposzp_tuning* out) {
  std::vector<toposzp_tuning> c;
  const toposzp_tuning cur = tune_now();
  for (int w : {4, 8})
    for (int g : {2, 4, 8, 16}) c.push_back({cur.encode_waves, w, cur.compress_wgs_per_cu, g});
  return autotune(c, (hipStream_t)stream,
                  [&]() { return toposzp_decompress_batch(count, h_jobs, d_ws, ws_bytes, stream); }, out);
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

int toposzp_decompress_stats(void* d_ws, int64_t out[5], void* stream) {
  if (!d_ws || !out || ((uintptr_t)d_ws & 255)) return TOPOSZP_E_INVALID_ARG;
  const Ctrl* ct = (const Ctrl*)d_ws;
  unsigned long long st[5];
  hipLaunchKernelGGL(stats_kernel, dim3(1), dim3(1024), 0, (hipStream_t)stream, (uint8_t*)d_ws);
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(st, (const void*)ct->stats, sizeof(st), hipMemcpyDeviceToHost, (hipStream_t)stream) !=
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
