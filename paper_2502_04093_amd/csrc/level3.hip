// Fused per-level kernels for 3-D fields with the default chunk shape
// (2, 16, 64) level coordinates.
//
// One launch runs a whole level l (Sec. 4.1: the level's three 1-D
// interpolation passes along z, y, x) on the level grid G_{l-1}, reading the
// coarse grid G_l from a compact array and writing G_{l-1} compactly (or, for
// retrieval at level 1, the final field).  A workgroup owns a 16 x 64 column of
// chunks and marches along z, two level planes (one chunk row) per step:
//
//   pass A (along z) at the odd plane, from a ring of 4 coarse planes,
//   pass B (along y) at both planes, from the even rows,
//   pass C (along x) at both planes, from the even columns.
//
// Passes A and B are also evaluated on a halo (even rows y0-2, y0+16, y0+18
// and even columns x0-2, x0+64, x0+66) that neighbouring columns own; those
// values are recomputed from the same inputs, so workgroups never wait on each
// other.  Codes of the workgroup's own targets are buffered in LDS; one wave
// turns rows of 32 codes into plane words with an in-register bit transpose
// (Sec. 4.3), and in retrieval two waves turn the step's own and halo plane
// words back into codes.  Compression also accumulates the delta-y maxima of
// Thm. 1 from the buffered codes.
//
// Retrieval keeps its register count within five waves per SIMD: everything
// that follows from the thread index is worked out per step rather than held,
// a plane word's chunk advances by a fixed stride per step, passes B and C take
// two targets per thread from five neighbours, and pass C writes four finished
// points of the level grid per thread straight from its registers.  Code and
// outlier buffers alternate by step parity, so a step ends without a barrier.
//
// Tile-local arithmetic is 32-bit (the host limits extents to 2^24);
// only offsets into global arrays are 64-bit.  Per target the arithmetic is
// exactly that of the per-pass kernels (same stencils, same rounding), so
// streams and reconstructions are bit-identical.
#include <type_traits>

#include "kernels.h"

#include "ipc_internal.h"

namespace ipc {
namespace {

constexpr uint32_t NB_A = 0xAAAAAAAAu;
constexpr int WG3 = 256;
constexpr int TY = 16, TX = 64;   // chunk extents (level coordinates) in y, x
constexpr int NYE = 11;           // even rows y0-2 .. y0+18
constexpr int NXE = 35;           // even columns x0-2 .. x0+66
constexpr int NXP = 36;           // padded row length
constexpr int CA = 256, CB = 512, CC = 1024;  // codes per full chunk of pass A, B, C
constexpr int PADA = CA + CA / 32, PADB = CB + CB / 32, PADC = CC + CC / 32;
constexpr int NHA = 129, NHB = 48;  // halo targets of pass A and B per step

__device__ __forceinline__ int pidx(int j) { return j + (j >> 5); }
// a * b + c for small non-negative operands (tile-local indices, below 2^24)
__device__ __forceinline__ int mad24(int a, int b, int c) { return int(__umul24(uint32_t(a), uint32_t(b))) + c; }

template <typename T>
struct F3;
template <>
struct F3<float> {
  static __device__ __forceinline__ float add(float a, float b) { return __fadd_rn(a, b); }
  static __device__ __forceinline__ float sub(float a, float b) { return __fsub_rn(a, b); }
  static __device__ __forceinline__ float mul(float a, float b) { return __fmul_rn(a, b); }
  static __device__ __forceinline__ float rnd(float a) { return __builtin_rintf(a); }
  static __device__ __forceinline__ uint64_t bits(float a) { return __float_as_uint(a); }
  static __device__ __forceinline__ float from_bits(uint64_t b) { return __uint_as_float(uint32_t(b)); }
};
template <>
struct F3<double> {
  static __device__ __forceinline__ double add(double a, double b) { return __dadd_rn(a, b); }
  static __device__ __forceinline__ double sub(double a, double b) { return __dsub_rn(a, b); }
  static __device__ __forceinline__ double mul(double a, double b) { return __dmul_rn(a, b); }
  static __device__ __forceinline__ double rnd(double a) { return __builtin_rint(a); }
  static __device__ __forceinline__ uint64_t bits(double a) { return uint64_t(__double_as_longlong(a)); }
  static __device__ __forceinline__ double from_bits(uint64_t b) { return __longlong_as_double((long long)b); }
};

// Transpose a 32x32 bit matrix held as 32 words: afterwards bit j of a[k]
// is what bit k of a[j] was.
__device__ __forceinline__ void transpose32(uint32_t a[32]) {
  uint32_t m = 0x0000FFFFu;
#pragma unroll
  for (int j = 16; j != 0; j >>= 1, m ^= (m << j)) {
#pragma unroll
    for (int k = 0; k < 32; k = ((k | j) + 1) & ~j) {
      uint32_t t = ((a[k] >> j) ^ a[k | j]) & m;
      a[k] ^= t << j;
      a[k | j] ^= t;
    }
  }
}

// (m & a) | (~m & b) as one v_bfi_b32; written as an instruction so the
// transposes below keep one temporary per word pair instead of the
// and/shift/or sequences the scheduler would interleave
__device__ __forceinline__ uint32_t bfi(uint32_t m, uint32_t a, uint32_t b) {
  uint32_t r;
  asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "s"(m), "v"(a), "v"(b));
  return r;
}

// Same transpose: the 16- and 8-bit stages as byte permutes (v_perm_b32),
// the 4-, 2- and 1-bit stages as shifted bit-field inserts.
__device__ __forceinline__ void transpose32p(uint32_t a[32]) {
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const uint32_t lo = a[k], hi = a[k + 16];
    a[k] = __builtin_amdgcn_perm(hi, lo, 0x05040100u);
    a[k + 16] = __builtin_amdgcn_perm(hi, lo, 0x07060302u);
  }
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    if (k & 8) continue;
    const uint32_t lo = a[k], hi = a[k + 8];
    a[k] = __builtin_amdgcn_perm(hi, lo, 0x06020400u);
    a[k + 8] = __builtin_amdgcn_perm(hi, lo, 0x07030501u);
  }
  uint32_t m = 0x0F0F0F0Fu;
#pragma unroll
  for (int j = 4; j != 0; j >>= 1, m ^= (m << j)) {
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      if (k & j) continue;
      const uint32_t lo = a[k], hi = a[k | j];
      a[k] = bfi(m, lo, hi << j);
      a[k | j] = bfi(m, lo >> j, hi);
    }
  }
}

// The 16x16 bit transposes of the low and of the high halves of 16 words at
// once (the 8-, 4-, 2- and 1-bit stages above).  With 32 codes below 2^16,
// word k = code k | code k+16 << 16 turns into word k = plane k of the 32
// codes, and back: a 32x32 transpose whose zero half is never touched.
__device__ __forceinline__ void transpose16x2(uint32_t a[16]) {
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    if (k & 8) continue;
    const uint32_t lo = a[k], hi = a[k + 8];
    a[k] = __builtin_amdgcn_perm(hi, lo, 0x06020400u);
    a[k + 8] = __builtin_amdgcn_perm(hi, lo, 0x07030501u);
  }
  uint32_t m = 0x0F0F0F0Fu;
#pragma unroll
  for (int j = 4; j != 0; j >>= 1, m ^= (m << j)) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      if (k & j) continue;
      const uint32_t lo = a[k], hi = a[k | j];
      a[k] = bfi(m, lo, hi << j);
      a[k | j] = bfi(m, lo >> j, hi);
    }
  }
}

__device__ __forceinline__ uint32_t xenc(uint32_t v) { return v ^ (v >> 1) ^ (v >> 2); }
// (1 + x + x^2)^-1 = (1 + x)(1 + x^3)(1 + x^6)(1 + x^12)(1 + x^24) over GF(2)
__device__ __forceinline__ uint32_t xdec(uint32_t e) {
  uint32_t t = e ^ (e >> 1);
  t ^= t >> 3;
  t ^= t >> 6;
  t ^= t >> 12;
  t ^= t >> 24;
  return t;
}

// One-dimensional stencil on gathered neighbours (b, c at -+1; a, e at -+3);
// hc, ha, he say which of c, a, e exist.  Every lane evaluates the full cubic
// form; the boundary forms are evaluated only when some lane of the wave needs
// one, and then chosen by select (the neighbours of a missing point may hold
// anything: they are never selected).
template <typename T, int INTERP>
__device__ __forceinline__ T stencil(T a, T b, T c, T e, bool hc, bool ha, bool he) {
  using F = F3<T>;
  if (INTERP == IPC_LINEAR) return hc ? F::mul(F::add(b, c), T(0.5)) : b;
  const bool full = hc && ha && he;
  T r = F::mul(F::sub(F::mul(F::add(b, c), T(9.0)), F::add(a, e)), T(0.0625));
  if (__builtin_amdgcn_ballot_w64(!full)) {
    const T lin = F::mul(F::add(b, c), T(0.5));
    const T qr = F::mul(F::sub(F::add(F::mul(b, T(3.0)), F::mul(c, T(6.0))), e), T(0.125));
    const T ql = F::mul(F::sub(F::add(F::mul(c, T(3.0)), F::mul(b, T(6.0))), a), T(0.125));
    const T g = !hc ? b : (he ? qr : (ha ? ql : lin));
    r = full ? r : g;
  }
  return r;
}

// Quantization of Sec. 4.2.2 with the explicit check; returns the code (0 for
// an outlier) and the reconstruction.
template <typename T>
__device__ __forceinline__ int32_t quantize(T xv, T pred, double eb, T two_eb, T inv, T qmax,
                                            T &xhat, bool &out) {
  using F = F3<T>;
  T qf = F::rnd(F::mul(F::sub(xv, pred), inv));
  out = !(fabs(qf) <= qmax);
  int32_t q = out ? 0 : int32_t(qf);
  T xr = F::add(pred, F::mul(T(q), two_eb));
  if (!out) out = !(fabs(__dsub_rn(double(xr), double(xv))) <= eb);
  xhat = out ? xv : xr;
  return out ? 0 : q;
}

// Per-pass launch arguments picked by a pass number held in a register: a
// select chain, so no dynamically indexed read of the argument block
template <typename V>
__device__ __forceinline__ V sel3(int p, V a0, V a1, V a2) {
  return p == 0 ? a0 : (p == 1 ? a1 : a2);
}
#define LSEL(field, p) sel3((p), L.field[0], L.field[1], L.field[2])
#define LSEL2(field, p, j) sel3((p), L.field[0][j], L.field[1][j], L.field[2][j])

struct Ext {
  int ez, ey, ex, count;
};

__device__ __forceinline__ int clampi(int v, int hi) { return v < 0 ? 0 : (v > hi ? hi : v); }

// extents of chunk (tz, ty, tx) of pass p (0 = A, 1 = B, 2 = C)
__device__ __forceinline__ Ext chunk_ext(const Level3Args &L, int p, int tz, int ty, int tx) {
  Ext c;
  c.ez = clampi(LSEL2(tdims, p, 0) - tz * LSEL2(ct, p, 0), LSEL2(ct, p, 0));
  c.ey = clampi(LSEL2(tdims, p, 1) - ty * LSEL2(ct, p, 1), LSEL2(ct, p, 1));
  c.ex = clampi(LSEL2(tdims, p, 2) - tx * LSEL2(ct, p, 2), LSEL2(ct, p, 2));
  c.count = c.ez * c.ey * c.ex;
  return c;
}

__device__ __forceinline__ int64_t chunk_id(const Level3Args &L, int tz, int ty, int tx) {
  return (int64_t(tz) * L.tiles_y + ty) * L.tiles_x + tx;
}

// first payload word of a chunk's stored planes, and a plane's rank among them
__device__ __forceinline__ uint64_t chunk_words(const Level3Args &L, const RetrieveIn &in, int p,
                                                int64_t cid) {
  if (in.chunk_off) return in.chunk_off[LSEL(chunk_base, p) + cid];
  return LSEL(slot_base, p) + uint64_t(cid) * 32u * LSEL(wmax, p);
}
__device__ __forceinline__ uint32_t plane_rank(bool packed, uint32_t mask, int k) {
  return packed ? uint32_t(__popc((mask >> k) >> 1)) : uint32_t(31 - k);
}

// outlier lookup inside the sorted range [a0, a1) of one chunk
__device__ __forceinline__ bool find_outlier(const RetrieveIn &in, uint32_t a0, uint32_t a1,
                                             uint32_t local, uint64_t &bits) {
  const uint32_t end = a1;
  while (a0 < a1) {
    uint32_t m = (a0 + a1) >> 1;
    if (in.out_local[m] < local) a0 = m + 1; else a1 = m;
  }
  if (a0 < end && in.out_local[a0] == local) {
    bits = in.out_bits[a0];
    return true;
  }
  return false;
}

// Halo positions of one step (owned by neighbouring workgroups):
//   pass A: even rows {y0-2, y0+16, y0+18} x 35 even columns (105), then own
//           even rows x columns {x0-2, x0+64, x0+66} (24)                 = 129
//   pass B: 2 planes x 8 odd rows x columns {x0-2, x0+64, x0+66}         =  48
__device__ __forceinline__ void halo_a(int h, int &yj, int &xi) {
  if (h < 105) {
    int r = h / NXE;
    yj = r == 0 ? 0 : 8 + r;
    xi = h - r * NXE;
  } else {
    int hh = h - 105;
    int r = hh / 3;
    yj = 1 + r;
    int c = hh - r * 3;
    xi = c == 0 ? 0 : 32 + c;
  }
}
__device__ __forceinline__ void halo_b(int h, int &zz, int &k, int &xi) {
  zz = h >= 24 ? 1 : 0;
  int r = h - zz * 24;
  k = r / 3;
  int c = r - k * 3;
  xi = c == 0 ? 0 : 32 + c;
}
// Chunk column and in-chunk offset of halo index i (0 .. per + 2) around tile
// `tile` whose chunks hold `per` target coordinates: target coordinate
// tile * per - 1 + i lies in the tile before (i = 0), the tile, or the next.
__device__ __forceinline__ void halo_tile(int tile, int i, int per, int &tn, int &off) {
  int e = tile * per - 1 + i;
  tn = i == 0 ? tile - 1 : (i <= per ? tile : tile + 1);
  off = e - tn * per;
}

// Code of the target at offset (oz, oy, ox) of chunk (tz, tyn, txn) of pass p:
// every plane word is loaded independently (unrolled), then bits are gathered.
// Planes that are not loaded read word 0 of the payload, which always exists.
__device__ __forceinline__ uint32_t fetch_code(const Level3Args &L, const RetrieveIn &in, int p,
                                               int tz, int tyn, int txn, int oz, int oy, int ox,
                                               uint32_t keep) {
  const Ext e = chunk_ext(L, p, tz, tyn, txn);
  const uint32_t local = uint32_t((oz * e.ey + oy) * e.ex + ox);
  const int64_t cid = chunk_id(L, tz, tyn, txn);
  const uint32_t mask = in.masks[LSEL(chunk_base, p) + cid];
  const uint32_t load = mask & keep;
  const uint32_t W = uint32_t((e.count + 31) >> 5);
  const bool packed = in.chunk_off != nullptr;
  const uint32_t *base = in.payload + chunk_words(L, in, p, cid) + (local >> 5);
  const uint32_t bsel = local & 31;
  uint32_t code = 0;
#pragma unroll
  for (int k = 31; k >= 0; --k) {
    bool on = (load >> k) & 1u;
    uint32_t w = *(on ? base + plane_rank(packed, mask, k) * W : in.payload);
    code |= (on ? (w >> bsel) & 1u : 0u) << k;
  }
  return xdec(code) & keep;
}

// outliers of one chunk kept in LDS for a step (more are looked up in HBM)
constexpr int OCAP = 8;

// LDS of a retrieval workgroup.  Codes and outlier slots alternate between
// two buffers by step parity, so the next step's fetch never waits for this
// step's last pass.
template <typename T>
struct Shared3 {
  T ring[4][NYE][NXP];      // coarse planes m-1 .. m+2 (even rows x even columns, halo'd)
  T wa[NYE][NXP];           // pass A values of the step's odd plane (halo'd)
  T wb[2][8][NXP];          // pass B values of both planes (odd rows, halo'd columns)
  uint32_t hva[NYE][NXP];   // codes of pass-A halo targets
  uint32_t hvb[2][8][4];    // codes of pass-B halo targets
  uint32_t codes[2][PADA + PADB + PADC];
  uint32_t orng[2][13][2];     // outlier ranges of the step's chunks
  uint32_t oloc[2][13][OCAP];  // their entries, when a chunk holds at most OCAP
  uint64_t obits[2][13][OCAP];
};

// inputs of a compression step: the tile (both planes), then the halo targets
constexpr int XIN_HA = 2 * 16 * TX;           // pass-A halo inputs [NYE][NXP]
constexpr int XIN_HB = XIN_HA + NYE * NXP;    // pass-B halo inputs [2][8][4]
constexpr int XIN_N = XIN_HB + 2 * 8 * 4;

// residue bits of the delta-y set (see k_level3_compress)
constexpr int RB = 13;
constexpr int RW = (1 << RB) / 32;            // words of one pass's residue set

// LDS of a compression workgroup
constexpr int REC_CAP = 128;  // outlier records a compression step stages in LDS

template <typename T>
struct SharedC {
  T ring[4][NYE][NXP];
  T wa[NYE][NXP];
  T wb[2][8][NXP];
  T wc[2][16][32];
  T xin[XIN_N];
  uint32_t codes[PADA + PADB + PADC];
  uint32_t bm[3][RW];       // residues w mod 2^13 present among each pass's codes
  uint32_t eq[3][33];       // per workgroup delta-y of each pass
  uint32_t qa[3];           // largest |q| among 14-digit codes, per pass
  unsigned long long mxab;  // bits of the workgroup's largest finite |x^| (as a double)
  // the step's outlier records (pass << 16 | local, value bits), written out
  // with one slot reservation per step
  uint32_t rec_n;
  uint32_t rec_key[REC_CAP];
  unsigned long long rec_bits[REC_CAP];
};

// code buffers of one step (retrieval): pass A, B, C
__device__ __forceinline__ int code_off1(int p) { return p == 0 ? 0 : (p == 1 ? PADA : PADA + PADB); }


// The thread's role index.  Waves of a workgroup do different amounts of
// work (wave 0 carries the plane coding, the halo targets fall on the first
// waves), and every workgroup's wave i tends to land on the same SIMD of its
// compute unit; rotating the roles by the workgroup index spreads the heavy
// waves over the SIMDs.  The rotation is by whole waves, so lane numbers and
// wave-wide operations are unchanged.
__device__ __forceinline__ int role_thread() {
  return int((threadIdx.x + 64u * (blockIdx.x & 3u)) & 255u);
}

// Tile (tx, ty) and column segment zs of this workgroup.  Consecutive
// workgroup ids are dealt round-robin to the 8 XCDs; renumbering them so that
// each XCD works through a contiguous run of tiles keeps neighbouring columns,
// whose halos overlap, in the same L2.
__device__ __forceinline__ void block_tile(const Level3Args &L, int &tx, int &ty, int &zs) {
  const int nb = int(gridDim.x), b = int(blockIdx.x);
  const int lin = (nb & 7) == 0 ? (b & 7) * (nb >> 3) + (b >> 3) : b;
  tx = lin % L.tiles_x;
  const int r = lin / L.tiles_x;
  ty = r % L.tiles_y;
  zs = r / L.tiles_y;
}

// ring slots of the coarse planes m0 - 1 .. m0 + 1 (11 even rows x 35 even
// columns each; entry li[i] of a slot from offset ro[i] of its plane), every
// load issued before the first store.  Entries outside the coarse grid read
// the plane's first element and are never selected by a stencil.
template <typename T, typename SH>
__device__ __forceinline__ void load_ring(const Level3Args &L, const T *gin, SH &S, int m0,
                                          const int li[2], const uint32_t ro[2]) {
  const int64_t ps = int64_t(L.G[1]) * L.G[2];
  T v[3][2];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int cz = m0 - 1 + j;
    const T *gp = gin + (cz >= 0 && cz < L.G[0] ? int64_t(cz) * ps : 0);
#pragma unroll
    for (int i = 0; i < 2; ++i) v[j][i] = gp[ro[i]];
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int cz = m0 - 1 + j;
    if (cz < 0 || cz >= L.G[0]) continue;
    T *dst = &S.ring[cz & 3][0][0];
#pragma unroll
    for (int i = 0; i < 2; ++i)
      if (li[i] >= 0) dst[li[i]] = v[j][i];
  }
}

// even-column values of plane zz at tile row yy (0 .. 15), index i + 1 for the
// even column x0 + 2 i: the coarse plane (zz = 0, yy even), pass A (zz = 1,
// yy even) or pass B (yy odd)
template <typename T, typename SH>
__device__ __forceinline__ const T *even_row(SH &S, int m, int zz, int yy) {
  if (yy & 1) return S.wb[zz][yy >> 1];
  return zz == 0 ? S.ring[m & 3][(yy >> 1) + 1] : S.wa[(yy >> 1) + 1];
}

// write the 2 x 16 x 64 level points of a step from LDS to a compact grid,
// four consecutive points per thread and plane (thread t: row (t >> 4) & 15,
// columns 4 (t & 15) ..+3).  Level-grid indices fit 32 bits (the host limits
// fields to 2^31 points); interior tiles skip the bounds tests.
template <typename T, typename SH>
__device__ __forceinline__ void write_rows(const Level3Args &L, SH &S, T *gout, int m, int y0,
                                           int x0) {
  const int Lz = L.L[0], Ly = L.L[1], Lx = L.L[2];
  const int t = threadIdx.x;
  const int yy = (t >> 4) & 15, xq = (t & 15) * 4;
  const int y = y0 + yy, x = x0 + xq;
  const bool vec = (Lx & 3) == 0 && (reinterpret_cast<uintptr_t>(gout) & 15) == 0;
  const bool interior = vec && 2 * m + 1 < Lz && y0 + TY <= Ly && x0 + TX <= Lx;
  const uint32_t plane = uint32_t(Ly) * uint32_t(Lx);
  const uint32_t row = uint32_t(mad24(y, Lx, x));
#pragma unroll
  for (int zz = 0; zz < 2; ++zz) {
    const int z = 2 * m + zz;
    if (!interior && (z >= Lz || y >= Ly || x >= Lx)) continue;
    const T *ev = even_row<T>(S, m, zz, yy);
    const T v0 = ev[(xq >> 1) + 1];
    const T v1 = S.wc[zz][yy][xq >> 1];
    const T v2 = ev[(xq >> 1) + 2];
    const T v3 = S.wc[zz][yy][(xq >> 1) + 1];
    T *dst = gout + (uint32_t(z) * plane + row);
    if (vec) {
      if constexpr (sizeof(T) == 4) {
        *reinterpret_cast<float4 *>(dst) = make_float4(v0, v1, v2, v3);
      } else {
        reinterpret_cast<double2 *>(dst)[0] = make_double2(v0, v1);
        reinterpret_cast<double2 *>(dst)[1] = make_double2(v2, v3);
      }
    } else {
      dst[0] = v0;
      if (x + 1 < Lx) dst[1] = v1;
      if (x + 2 < Lx) dst[2] = v2;
      if (x + 3 < Lx) dst[3] = v3;
    }
  }
}

__device__ __forceinline__ uint32_t absdiff(uint32_t a, uint32_t b) { return a > b ? a - b : b - a; }

// Full-wave reductions (every lane active): within each row of 16 lanes by
// DPP lane swaps (quad permutes, then half-row and row mirrors; order does not
// matter for min / max), then the four row results through lane reads.  The
// result is uniform.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t v) {
  return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), CTRL, 0xF, 0xF, false));
}
template <typename Op>
__device__ __forceinline__ uint32_t wave_reduce(uint32_t v, Op op) {
  v = op(v, dpp<0xB1>(v));   // quad_perm [1, 0, 3, 2]
  v = op(v, dpp<0x4E>(v));   // quad_perm [2, 3, 0, 1]
  v = op(v, dpp<0x141>(v));  // row_half_mirror
  v = op(v, dpp<0x140>(v));  // row_mirror
  const uint32_t r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
  const uint32_t r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
  return op(op(r0, r1), op(r2, r3));
}
__device__ __forceinline__ int wave_min(int v) {
  return int(wave_reduce(uint32_t(v), [](uint32_t a, uint32_t b) { return int(a) < int(b) ? a : b; }));
}
__device__ __forceinline__ int wave_max(int v) {
  return int(wave_reduce(uint32_t(v), [](uint32_t a, uint32_t b) { return int(a) > int(b) ? a : b; }));
}
__device__ __forceinline__ uint64_t wave_max_bits(uint64_t v) {
  auto mx = [](uint64_t a, uint64_t b) { return a > b ? a : b; };
  auto sw = [](uint64_t x, auto ctrl) {
    constexpr int C = decltype(ctrl)::value;
    return uint64_t(dpp<C>(uint32_t(x))) | (uint64_t(dpp<C>(uint32_t(x >> 32))) << 32);
  };
  v = mx(v, sw(v, std::integral_constant<int, 0xB1>{}));
  v = mx(v, sw(v, std::integral_constant<int, 0x4E>{}));
  v = mx(v, sw(v, std::integral_constant<int, 0x141>{}));
  v = mx(v, sw(v, std::integral_constant<int, 0x140>{}));
  uint64_t r = 0;
#pragma unroll
  for (int l = 0; l < 64; l += 16) {
    const uint64_t x = uint64_t(uint32_t(__builtin_amdgcn_readlane(int(uint32_t(v)), l))) |
                       (uint64_t(uint32_t(__builtin_amdgcn_readlane(int(uint32_t(v >> 32)), l))) << 32);
    r = mx(r, x);
  }
  return r;
}
__device__ __forceinline__ uint32_t wave_max_bits(uint32_t v) { return uint32_t(wave_max(int(v))); }

// OR of v over a full wave (every lane active), uniform
__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
  return wave_reduce(v, [](uint32_t a, uint32_t b) { return a | b; });
}


// Delta-y for b >= 14 over the buffered codes lo .. hi - 1 of one chunk (see
// k_level3_compress), by one wave: nothing to do when none has more than 14
// digits; else, with nb the longest code's digit count, exact |q - q'_b| per
// code while b < nb and the range's largest |q| from there on, into the
// maxima eq[14..32].  One b at a time keeps the register footprint small.
__device__ __forceinline__ void errq_hi(uint32_t *eq, const uint32_t *v, int lo, int hi, int lane) {
  uint32_t qa = 0, orv = 0;
  for (int j = lo + lane; j < hi; j += 64) {
    const uint32_t c = v[pidx(j)];
    orv |= c;
    const int32_t q = int32_t((c ^ NB_A) - NB_A);
    const uint32_t aq = uint32_t(q < 0 ? -q : q);
    qa = aq > qa ? aq : qa;
  }
  // every code within 14 digits: the |q| tracked per code covers b >= 14
  const uint32_t o = wave_or(orv);
  const int nb = o ? 32 - __clz(o) : 0;
  if (nb <= 14) return;
  qa = uint32_t(wave_max(int(qa)));
#pragma unroll 1
  for (int b = 14; b < 33; ++b) {
    uint32_t d = qa;
    if (b < nb) {
      const uint32_t mb = (1u << b) - 1u, ab = NB_A & mb;
      d = 0;
      for (int j = lo + lane; j < hi; j += 64) {
        const uint32_t t = absdiff((v[pidx(j)] ^ NB_A) & mb, ab);
        d = t > d ? t : d;
      }
      d = uint32_t(wave_max(int(d)));
    }
    if (lane == 0 && d) atomicMax(&eq[b], d);
  }
}

// Delta-y for b <= 13 from the residue set of one pass (one wave): folding the
// 2^13-bit set onto 2^b bits gives the smallest and largest residue w mod 2^b,
// and |q - q'_b| is largest at one of them.  Results into eq[1..13].
__device__ __forceinline__ void errq_fold(const uint32_t *bm, uint32_t *eq, int lane) {
  auto emit = [&](int b, int mn, int mx) {
    mn = wave_min(mn);
    mx = wave_max(mx);
    if (lane == 0 && mx >= 0) {
      const uint32_t ab = NB_A & ((1u << b) - 1u);
      const uint32_t d1 = uint32_t(mx) >= ab ? uint32_t(mx) - ab : 0u;
      const uint32_t d2 = ab >= uint32_t(mn) ? ab - uint32_t(mn) : 0u;
      eq[b] = d1 > d2 ? d1 : d2;
    }
  };
  auto lo = [](uint32_t w, int base) { return w ? base + __builtin_ctz(w) : 0x7FFFFFFF; };
  auto hi = [](uint32_t w, int base) { return w ? base + 31 - __builtin_clz(w) : -1; };
  const uint32_t w0 = bm[lane], w1 = bm[lane + 64], w2 = bm[lane + 128], w3 = bm[lane + 192];
  // b = 13: word j of the set holds residues 32 j .. 32 j + 31
  {
    int mn = min(min(lo(w0, 32 * lane), lo(w1, 32 * (lane + 64))),
                 min(lo(w2, 32 * (lane + 128)), lo(w3, 32 * (lane + 192))));
    int mx = max(max(hi(w0, 32 * lane), hi(w1, 32 * (lane + 64))),
                 max(hi(w2, 32 * (lane + 128)), hi(w3, 32 * (lane + 192))));
    emit(13, mn, mx);
  }
  // b = 12: words j and j + 128 fold onto word j
  const uint32_t f0 = w0 | w2, f1 = w1 | w3;
  emit(12, min(lo(f0, 32 * lane), lo(f1, 32 * (lane + 64))),
       max(hi(f0, 32 * lane), hi(f1, 32 * (lane + 64))));
  // b = 11 .. 5: word j of 2^(b-5) words held by lane j
  uint32_t f = f0 | f1;
  emit(11, lo(f, 32 * lane), hi(f, 32 * lane));
#pragma unroll
  for (int b = 10; b >= 5; --b) {
    const int n = 1 << (b - 5);
    const uint32_t g = __shfl_down(f, n, 64);
    f = lane < n ? (f | g) : 0u;
    emit(b, lo(f, 32 * lane), hi(f, 32 * lane));
  }
  // b = 4 .. 1 inside the word of lane 0 (every lane computes the same, lane 0 writes)
  uint32_t g = __shfl(f, 0, 64);
#pragma unroll
  for (int b = 4; b >= 1; --b) {
    const int n = 1 << b;
    g = (g | (g >> n)) & ((1u << n) - 1u);
    if (lane == 0 && g) {
      const uint32_t ab = NB_A & ((1u << b) - 1u);
      const uint32_t mn = __builtin_ctz(g), mx = 31 - __builtin_clz(g);
      const uint32_t d1 = mx >= ab ? mx - ab : 0u;
      const uint32_t d2 = ab >= mn ? ab - mn : 0u;
      eq[b] = d1 > d2 ? d1 : d2;
    }
  }
}

template <typename T>
struct BitsOf;
template <>
struct BitsOf<float> {
  using U = uint32_t;
  static __device__ __forceinline__ U abs_bits(float a) { return __float_as_uint(a) & 0x7FFFFFFFu; }
  static __device__ __forceinline__ bool finite(float a) { return (__float_as_uint(a) & 0x7F800000u) != 0x7F800000u; }
  static __device__ __forceinline__ double to_double(U b) { return double(__uint_as_float(b)); }
};
template <>
struct BitsOf<double> {
  using U = uint64_t;
  static __device__ __forceinline__ U abs_bits(double a) {
    return uint64_t(__double_as_longlong(a)) & 0x7FFFFFFFFFFFFFFFull;
  }
  static __device__ __forceinline__ bool finite(double a) {
    return (uint64_t(__double_as_longlong(a)) & 0x7FF0000000000000ull) != 0x7FF0000000000000ull;
  }
  static __device__ __forceinline__ double to_double(U b) { return __longlong_as_double((long long)b); }
};

// ------------------------------------------------------------------ compress
//
// Delta-y of Thm. 1 in code units, errq[b] = max over a pass's codes of
// |q - q'_b|, q'_b being q with its b lowest negabinary digits cleared.  With
// w = q + A (mod 2^32, A = 0xAAAAAAAA; the code stored is v = w xor A) the
// low b digits are worth (w mod 2^b) - (A mod 2^b), which is q itself once b
// reaches the code's digit count.  The work is split by b:
//   b <= 13: the set of residues w mod 2^13 of the workgroup's codes (one LDS
//            OR per code); at the end, folding the set onto 2^b bits gives the
//            extreme residues mod 2^b and so the exact maximum;
//   b >= 14: a code within the 14-digit range [-0x2AAA, 0x1555] contributes
//            |q| (one max per code); chunks holding longer codes are scanned
//            exactly for b >= 14 once their codes are buffered (errq_hi).

// One column segment (tile tx, ty, chunk rows zs * zseg ..) of a level:
// the body of the level launch and of the batched launch.  `row` is the
// workgroup-row index of the segment.
template <typename T, int INTERP>
__device__ __forceinline__ void level3_compress_body(const Level3Args &L, const T *__restrict__ x,
                                                     const T *__restrict__ gin, T *gout,
                                                     double eb_arg, T two_eb_arg, T inv_arg,
                                                     T qmax_arg, const CompressOut &o, int tx, int ty,
                                                     int zs, uint32_t row_index, SharedC<T> &S) {
  using F = F3<T>;
  using BT = BitsOf<T>;
  using U = typename BT::U;
  // the quantizer's constants, held in vector registers: as scalars they are
  // spilled and re-read with a lane read at every use
  double eb = eb_arg;
  T two_eb = two_eb_arg, inv = inv_arg, qmax = qmax_arg;
  asm volatile("" : "+v"(eb), "+v"(two_eb), "+v"(inv), "+v"(qmax));
  const int tid0 = role_thread();
  const int x0 = tx * TX, y0 = ty * TY;
  const int m0 = zs * L.zseg;
  const int m1 = m0 + L.zseg < L.tiles_z ? m0 + L.zseg : L.tiles_z;
  const int Lz = L.L[0], Ly = L.L[1], Lx = L.L[2];

  for (int i = tid0; i < 3 * RW; i += WG3) (&S.bm[0][0])[i] = 0u;
  if (tid0 < 3 * 33) (&S.eq[0][0])[tid0] = 0u;
  if (tid0 < 3) S.qa[tid0] = 0u;
  if (tid0 == 0) S.mxab = 0ull;
  if (tid0 == 0) S.rec_n = 0u;

  uint32_t qaA = 0, qaB = 0, qaC = 0;
  U mxb = 0;
  // payload words stored per plane, accumulated by the encoding wave: lane j
  // holds plane j & 31 of pass C (j < 32) or B (j >= 32) in szCB, of pass A
  // (j < 32) in szA
  uint32_t szCB = 0, szA = 0;

  auto record = [&](int p, int m, int local, T xv) {
    const uint32_t k = atomicAdd(&S.rec_n, 1u);
    if (k < uint32_t(REC_CAP)) {
      S.rec_key[k] = uint32_t(p) << 16 | uint32_t(local);
      S.rec_bits[k] = (unsigned long long)F::bits(xv);
    } else if (unsigned long long slot = atomicAdd(o.n_out, 1ull); slot < o.out_cap) {
      // past the step's staging: a slot of its own
      OutlierRec *rr = reinterpret_cast<OutlierRec *>(o.out_recs) + slot;
      rr->pass = LSEL(pass_index, p);
      rr->chunk = uint32_t(chunk_id(L, m, ty, tx));
      rr->local = uint32_t(local);
      rr->pad = 0;
      rr->bits = F::bits(xv);
    }
    if (BT::finite(xv)) {
      const U b = BT::abs_bits(xv);
      mxb = b > mxb ? b : mxb;
    }
  };
  // one own target: code, residue, |q|, and the outlier record or max |x^|
  auto own_target = [&](int p, uint32_t *cb, int local, int32_t q, bool out, T xval, T xhat,
                        uint32_t &qa, int m) {
    const uint32_t w = uint32_t(q) + NB_A;
    cb[pidx(local)] = w ^ NB_A;
    atomicOr(&S.bm[p][(w >> 5) & (RW - 1)], 1u << (w & 31));
    const uint32_t aq = uint32_t(q < 0 ? -q : q);
    if (uint32_t(q) + 0x2AAAu <= 0x3FFFu) qa = aq > qa ? aq : qa;
    if (out) {
      record(p, m, local, xval);
    } else {
      const U b = BT::abs_bits(xhat);
      mxb = b > mxb ? b : mxb;
    }
  };

  // Inputs of a step, prefetched one step ahead (element offsets within the
  // two fine planes of the step fit 32 bits; the host checks 2 sZ < 2^31):
  //   xv[i]: tile row ly + 4 (i & 3) of plane ze + (i >> 2) at column lx (xin tid + 256 i)
  //   hv:    the halo input of this thread (pass A: tid < 129, pass B: 129 .. 176)
  //   rv[i]: coarse-plane entry tid + 256 i (< 385) of plane m + 2
  // Values at positions outside the level are loaded from the slab's first
  // element and never read by a stencil, so they are not cleared.
  T xv[8], hv, rv[2];
  const int lx = tid0 & 63, ly = tid0 >> 6;
  const bool colok = x0 + lx < Lx;
  const uint32_t xo0 = uint32_t(int64_t(y0 + ly) * L.sY + int64_t(x0 + lx) * L.sX);
  const uint32_t sZ32 = uint32_t(L.sZ), sY4 = uint32_t(4 * L.sY);
  int hidx = -1, hzz = 0;
  bool hxy = false;
  uint32_t ho = 0;
  if (tid0 < NHA) {
    int yj, xi;
    halo_a(tid0, yj, xi);
    const int y = y0 - 2 + 2 * yj, xg = x0 - 2 + 2 * xi;
    hzz = 1;
    hidx = XIN_HA + yj * NXP + xi;
    hxy = unsigned(y) < unsigned(Ly) && unsigned(xg) < unsigned(Lx);
    if (hxy) ho = uint32_t(L.sZ + int64_t(y) * L.sY + int64_t(xg) * L.sX);
  } else if (tid0 < NHA + NHB) {
    int zz, k, xi;
    halo_b(tid0 - NHA, zz, k, xi);
    const int y = y0 + 1 + 2 * k, xg = x0 - 2 + 2 * xi;
    hzz = zz;
    hidx = XIN_HB + (zz * 8 + k) * 4 + (xi & 3);
    hxy = y < Ly && unsigned(xg) < unsigned(Lx);
    if (hxy) ho = uint32_t(int64_t(zz) * L.sZ + int64_t(y) * L.sY + int64_t(xg) * L.sX);
  }
  int li[2];
  uint32_t ro[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int e = tid0 + i * WG3;
    const int yj = e / NXE, xi = e - (e / NXE) * NXE;
    const int cy = (y0 >> 1) - 1 + yj, cx = (x0 >> 1) - 1 + xi;
    const bool ok = e < NYE * NXE && unsigned(cy) < unsigned(L.G[1]) && unsigned(cx) < unsigned(L.G[2]);
    li[i] = e < NYE * NXE ? yj * NXP + xi : -1;
    ro[i] = ok ? uint32_t(cy * L.G[2] + cx) : 0u;
  }
  auto issue = [&](int m) {
    const int ze = 2 * m;
    const T *xs = x + int64_t(ze) * L.sZ;
    // offsets recomputed at each call rather than held across the loop
    uint32_t xo = xo0;
    asm volatile("" : "+v"(xo));
    if (y0 + TY <= Ly && x0 + TX <= Lx && ze + 1 < Lz) {
#pragma unroll
      for (int i = 0; i < 8; ++i) xv[i] = xs[xo + (i >> 2) * sZ32 + (i & 3) * sY4];
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const bool ok = ze + (i >> 2) < Lz && y0 + ly + 4 * (i & 3) < Ly && colok;
        xv[i] = xs[ok ? xo + (i >> 2) * sZ32 + (i & 3) * sY4 : 0u];
      }
    }
    hv = xs[hxy && ze + hzz < Lz ? ho : 0u];
    const int cz = m + 2;
    if (cz < L.G[0]) {
      const T *gp = gin + int64_t(cz) * L.G[1] * L.G[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) rv[i] = gp[ro[i]];
    }
  };

  // the first step's inputs requested before the ring's loads are waited for
  issue(m0);
  load_ring(L, gin, S, m0, li, ro);

  for (int m = m0; m < m1; ++m) {
    // a fresh copy of the thread index each step: values derived from it are
    // recomputed here instead of being held in registers across the loop
    int tid = tid0;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63;
    const int ze = 2 * m, zo = 2 * m + 1;
    // ---- stash the prefetched inputs, then prefetch the next step's
#pragma unroll
    for (int i = 0; i < 8; ++i) S.xin[tid + i * WG3] = xv[i];
    if (hidx >= 0) S.xin[hidx] = hv;
    if (m + 2 < L.G[0]) {
      T *rs = &S.ring[(m + 2) & 3][0][0];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        if (li[i] >= 0) rs[li[i]] = rv[i];
    }
    __syncthreads();
    if (m + 1 < m1) issue(m + 1);
    // ---- pass A (along z) at plane zo: the 8 x 32 own targets (one per
    // thread), then the 129 halo targets of the 11 x 35 even grid
    if (zo < Lz) {
      const bool hc = zo + 1 < Lz, ha = zo >= 3, he = zo + 3 < Lz;
      const T *rb = &S.ring[m & 3][0][0];
      const T *rc = &S.ring[(m + 1) & 3][0][0];
      const T *ra = &S.ring[(m - 1) & 3][0][0];
      const T *re = &S.ring[(m + 2) & 3][0][0];
      {
        const int r = tid >> 5, c = tid & 31;
        if (y0 + 2 * r < Ly && x0 + 2 * c < Lx) {
          const int ri = (r + 1) * NXP + c + 1;
          const T xval = S.xin[1024 + r * 2 * TX + 2 * c];
          const T pred = stencil<T, INTERP>(ra[ri], rb[ri], rc[ri], re[ri], hc, ha, he);
          T xhat;
          bool out;
          const int32_t q = quantize<T>(xval, pred, eb, two_eb, inv, qmax, xhat, out);
          (&S.wa[0][0])[ri] = xhat;
          const int ex = clampi(L.tdims[0][2] - tx * L.ct[0][2], L.ct[0][2]);
          own_target(0, S.codes + code_off1(0), mad24(r, ex, c), q, out, xval, xhat, qaA, m);
        }
      }
      if (tid < NHA) {
        int yj, xi;
        halo_a(tid, yj, xi);
        const int y = y0 - 2 + 2 * yj, xg = x0 - 2 + 2 * xi;
        if (unsigned(y) < unsigned(Ly) && unsigned(xg) < unsigned(Lx)) {
          const int ri = yj * NXP + xi;
          const T pred = stencil<T, INTERP>(ra[ri], rb[ri], rc[ri], re[ri], hc, ha, he);
          T xhat;
          bool out;
          quantize<T>(S.xin[XIN_HA + ri], pred, eb, two_eb, inv, qmax, xhat, out);
          (&S.wa[0][0])[ri] = xhat;
        }
      }
    }
    __syncthreads();
    // ---- pass B (along y) at planes ze, zo: 2 x 8 x 32 own targets (two per
    // thread), then the 48 halo targets at columns x0-2, x0+64, x0+66
    {
      const int ey = clampi(L.tdims[1][1] - ty * L.ct[1][1], L.ct[1][1]);
      const int ex = clampi(L.tdims[1][2] - tx * L.ct[1][2], L.ct[1][2]);
      const int k = tid >> 5, c = tid & 31;
      const int y = y0 + 1 + 2 * k;
      const bool hc = y + 1 < Ly, ha = y >= 3, he = y + 3 < Ly;
#pragma unroll
      for (int zz = 0; zz < 2; ++zz) {
        if (ze + zz >= Lz || y >= Ly || x0 + 2 * c >= Lx) continue;
        const T *src = zz == 0 ? S.ring[m & 3][0] : S.wa[0];
        const int ri = k * NXP + c + 1;
        const T pred = stencil<T, INTERP>(src[ri], src[ri + NXP], src[ri + 2 * NXP], src[ri + 3 * NXP], hc, ha, he);
        const T xval = S.xin[zz * 1024 + (2 * k + 1) * TX + 2 * c];
        T xhat;
        bool out;
        const int32_t q = quantize<T>(xval, pred, eb, two_eb, inv, qmax, xhat, out);
        S.wb[zz][k][c + 1] = xhat;
        own_target(1, S.codes + code_off1(1), mad24(mad24(zz, ey, k), ex, c), q, out, xval, xhat, qaB, m);
      }
      if (tid < NHB) {
        int zz, kh, xi;
        halo_b(tid, zz, kh, xi);
        const int yh = y0 + 1 + 2 * kh, xg = x0 - 2 + 2 * xi;
        if (ze + zz < Lz && yh < Ly && unsigned(xg) < unsigned(Lx)) {
          const T *src = zz == 0 ? S.ring[m & 3][0] : S.wa[0];
          const int ri = kh * NXP + xi;
          const bool hch = yh + 1 < Ly, hah = yh >= 3, heh = yh + 3 < Ly;
          const T pred = stencil<T, INTERP>(src[ri], src[ri + NXP], src[ri + 2 * NXP], src[ri + 3 * NXP], hch, hah, heh);
          T xhat;
          bool out;
          quantize<T>(S.xin[XIN_HB + (zz * 8 + kh) * 4 + (xi & 3)], pred, eb, two_eb, inv, qmax, xhat, out);
          S.wb[zz][kh][xi] = xhat;
        }
      }
    }
    __syncthreads();
    // ---- pass C (along x) at planes ze, zo: 16 rows x 32 odd columns
    {
      uint32_t *cb = S.codes + code_off1(2);
      const int ci = tid & 31, cr = (tid >> 5) & 7;
      const int cxg = x0 + 1 + 2 * ci;
      const bool chc = cxg + 1 < Lx, cha = cxg >= 3, che = cxg + 3 < Lx;
      const int cey = clampi(L.tdims[2][1] - ty * L.ct[2][1], L.ct[2][1]);
      const int cex = clampi(L.tdims[2][2] - tx * L.ct[2][2], L.ct[2][2]);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int zz = j >> 1, yy = cr + 8 * (j & 1);
        if (cxg >= Lx || y0 + yy >= Ly || ze + zz >= Lz) continue;
        const T *row = even_row<T>(S, m, zz, yy);
        const T pred = stencil<T, INTERP>(row[ci], row[ci + 1], row[ci + 2], row[ci + 3], chc, cha, che);
        const T xval = S.xin[zz * 1024 + yy * TX + 2 * ci + 1];
        T xhat;
        bool out;
        const int32_t q = quantize<T>(xval, pred, eb, two_eb, inv, qmax, xhat, out);
        S.wc[zz][yy][ci] = xhat;
        own_target(2, cb, mad24(mad24(zz, cey, yy), cex, ci), q, out, xval, xhat, qaC, m);
      }
    }
    __syncthreads();
    // ---- the level's output grid (compact), read by the next finer level
    if (gout) write_rows(L, S, gout, m, y0, x0);
    // ---- wave 0 encodes the step's chunks: 32 codes -> 32 plane words per
    // lane (pass C: lanes 0-31, B: 32-47, A: 48-55), chunk masks by OR
    // across each chunk's lanes.  The next step's first barrier orders these
    // reads of the code buffers before they are rewritten.
    if (tid < 64) {
      const int rp = lane < 32 ? 2 : (lane < 48 ? 1 : 0);
      const int rw = lane < 32 ? lane : (lane < 48 ? lane - 32 : lane - 48);
      // code counts of the step's chunk of each pass (uniform), this lane's
      const int cA = chunk_ext(L, 0, m, ty, tx).count, cB = chunk_ext(L, 1, m, ty, tx).count,
                cC = chunk_ext(L, 2, m, ty, tx).count;
      const int cnt = rp == 2 ? cC : (rp == 1 ? cB : cA);
      const int rW = (cnt + 31) >> 5;
      const bool work = lane < 56 && rw < rW;
      // codes 32 rw .. 32 rw + 31 sit at padded indices 33 rw + j
      const uint32_t *cb = S.codes + code_off1(rp) + 33 * rw;
      const int nv = work ? cnt - 32 * rw : 0;
      uint32_t r[32];
      if (cA == CA && cB == CB && cC == CC) {
        // every chunk full: lanes 0-55 all hold 32 codes (lanes 56-63 read
        // codes of the step that no mask, store or test below looks at)
#pragma unroll
        for (int j = 0; j < 32; ++j) r[j] = cb[j];
      } else {
#pragma unroll
        for (int j = 0; j < 32; ++j) r[j] = j < nv ? cb[j] : 0u;
      }
      uint32_t orv = 0;
#pragma unroll
      for (int j = 0; j < 32; ++j) orv |= r[j];
      orv = lane < 56 ? orv : 0u;
      const int64_t cid = chunk_id(L, m, ty, tx);
      // planes 0 .. NP-1 of v in r -> planes of e = v ^ (v >> 1) ^ (v >> 2)
      // (each materialized before it is tested: the scheduler would otherwise
      // keep pairwise partial XORs alive), the chunk masks from one ballot per
      // plane (pass C is lanes 0-31, B 32-47, A 48-55), the stores
      uint32_t mA = 0, mB = 0, mC = 0;
      auto finish = [&](auto npc) {
        constexpr int NP = decltype(npc)::value;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
          r[k] = k + 2 < NP ? (r[k] ^ r[k + 1] ^ r[k + 2]) : (k + 1 < NP ? (r[k] ^ r[k + 1]) : r[k]);
          asm volatile("" : "+v"(r[k]));
        }
#pragma unroll
        for (int k = 0; k < NP; ++k) {
          const uint64_t b = __builtin_amdgcn_ballot_w64(r[k] != 0u);
          mC |= uint32_t(uint32_t(b) != 0u) << k;
          mB |= uint32_t((uint32_t(b >> 32) & 0xFFFFu) != 0u) << k;
          mA |= uint32_t((uint32_t(b >> 48) & 0xFFu) != 0u) << k;
        }
        // planes up to the highest one any of the three chunks keeps; a
        // plane some chunk does not keep is written as zeros into its slot,
        // which no reader looks at
        const uint32_t top = 32u - uint32_t(__clz(mA | mB | mC));
        if (work) {
          uint32_t *q = o.payload + LSEL(slot_base, rp) + uint64_t(cid) * 32u * LSEL(wmax, rp) + rw +
                        31u * uint32_t(rW);
#pragma unroll
          for (int k = 0; k < NP; ++k) {
            if (uint32_t(k) < top) *q = r[k];
            q -= rW;
          }
        }
      };
      // every code of the wave below 2^16: planes 16 .. 31 are zero, and a
      // pair of 16x16 transposes gives planes 0 .. 15
      if (__builtin_amdgcn_ballot_w64(orv > 0xFFFFu) == 0) {
#pragma unroll
        for (int k = 0; k < 16; ++k) r[k] = __builtin_amdgcn_perm(r[k + 16], r[k], 0x05040100u);
        transpose16x2(r);
        finish(std::integral_constant<int, 16>{});
      } else {
        transpose32p(r);
        finish(std::integral_constant<int, 32>{});
      }
      const uint32_t rowor = rp == 2 ? mC : (rp == 1 ? mB : mA);
      // delta-y for b >= 14 of chunks holding codes longer than 14 digits
      {
        const uint32_t mk[3] = {mA, mB, mC};
        const int ck[3] = {cA, cB, cC};
#pragma unroll
        for (int p = 0; p < 3; ++p) {
          const int nb = mk[p] ? 32 - __clz(mk[p]) : 0;
          if (nb > 14) errq_hi(S.eq[p], S.codes + code_off1(p), 0, ck[p], lane);
        }
      }
      // (a 2-D field has no pass A: wmax 0 in its slot)
      if (lane < 56 && rw == 0 && (rp != 0 || L.wmax[0] != 0u)) o.masks[LSEL(chunk_base, rp) + cid] = rowor;
      {
        const int k = lane & 31;
        const uint32_t wA = uint32_t(cA + 31) >> 5, wB = uint32_t(cB + 31) >> 5, wC = uint32_t(cC + 31) >> 5;
        const uint32_t mcb = lane < 32 ? mC : mB;
        szCB += ((mcb >> k) & 1u) ? (lane < 32 ? wC : wB) : 0u;
        szA += ((mA >> k) & 1u) ? wA : 0u;
      }
    } else if ((tid >> 6) == 3) {
      {
        // meanwhile another wave writes the step's staged outlier records out
        // with one reservation of output slots; the count starts again from
        // zero for the next step (whose records come after its first barrier)
        const uint32_t nr = S.rec_n < uint32_t(REC_CAP) ? S.rec_n : uint32_t(REC_CAP);
        if (nr) {
          unsigned long long base = 0;
          if (lane == 0) base = atomicAdd(o.n_out, (unsigned long long)nr);
          base = (unsigned long long)uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(base)))) |
                 (unsigned long long)uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(base >> 32)))) << 32;
          const uint32_t cid = uint32_t(chunk_id(L, m, ty, tx));
          for (uint32_t i = uint32_t(lane); i < nr; i += 64u) {
            if (base + i < o.out_cap) {
              OutlierRec *rr = reinterpret_cast<OutlierRec *>(o.out_recs) + (base + i);
              const uint32_t key = S.rec_key[i];
              rr->pass = LSEL(pass_index, int(key >> 16));
              rr->chunk = cid;
              rr->local = key & 0xFFFFu;
              rr->pad = 0;
              rr->bits = S.rec_bits[i];
            }
          }
        }
        if (lane == 0) S.rec_n = 0u;
      }
    }
  }
  // ---- workgroup totals: per-pass |q| of 14-digit codes, max |x^|, then
  // the workgroup's row (reduced over the launch's workgroups afterwards)
  {
    const int lane = tid0 & 63, wave = tid0 >> 6;
    uint32_t qs[3] = {qaA, qaB, qaC};
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const int v = wave_max(int(qs[p]));
      if (lane == 0 && v > 0) atomicMax(&S.qa[p], uint32_t(v));
    }
    const U v = U(wave_max_bits(mxb));
    if (lane == 0 && v)
      atomicMax(&S.mxab, (unsigned long long)__double_as_longlong(BT::to_double(v)));
    __syncthreads();
    if (wave < 3) errq_fold(S.bm[wave], S.eq[wave], lane);
    __syncthreads();
  }
  uint32_t *row = o.wg_rows + size_t(row_index) * WG_ROW;
  if (tid0 < 3 * 33) {
    const int p = tid0 / 33, b = tid0 - p * 33;
    uint32_t val = b > 0 ? S.eq[p][b] : 0u;
    if (b >= 14) val = S.qa[p] > val ? S.qa[p] : val;
    row[tid0] = val;
  } else if (tid0 < 3 * 33 + 2) {
    const unsigned long long mx = S.mxab;
    row[tid0] = tid0 == 3 * 33 ? uint32_t(mx) : uint32_t(mx >> 32);
  }
  if (tid0 < 64) {
    row[ROW_SIZES + (tid0 < 32 ? 64 + tid0 : tid0)] = szCB;
    if (tid0 < 32) row[ROW_SIZES + tid0] = szA;
  }
}

template <typename T, int INTERP>
__global__ __launch_bounds__(WG3) void k_level3_compress(Level3Args L, const T *__restrict__ x,
                                                          const T *__restrict__ gin, T *gout,
                                                          double eb, T two_eb, T inv, T qmax,
                                                          CompressOut o) {
  __shared__ SharedC<T> S;
  int tx, ty, zs;
  block_tile(L, tx, ty, zs);
  level3_compress_body<T, INTERP>(L, x, gin, gout, eb, two_eb, inv, qmax, o, tx, ty, zs,
                                  L.row_base + blockIdx.x, S);
}

// Column segment `it` of a level launch, in plain order (tx fastest)
__device__ __forceinline__ void item_tile(const Level3Args &L, uint32_t it, int &tx, int &ty, int &zs) {
  tx = int(it % uint32_t(L.tiles_x));
  const uint32_t r = it / uint32_t(L.tiles_x);
  ty = int(r % uint32_t(L.tiles_y));
  zs = int(r / uint32_t(L.tiles_y));
}

// Work item of this workgroup in a work-list launch: consecutive workgroup
// ids are dealt round-robin to the 8 XCDs, so (as in block_tile) each XCD
// takes a contiguous run of items, whose halos overlap, in its own L2
__device__ __forceinline__ uint32_t work_item() {
  const uint32_t nb = gridDim.x, b = blockIdx.x;
  return (nb & 7) == 0 ? (b & 7) * (nb >> 3) + (b >> 3) : b;
}

// the field of work item `it` (fields in item order, a short uniform scan)
template <typename B>
__device__ __forceinline__ int item_field(const B *__restrict__ bf, int nf, uint32_t it) {
  int f = 0;
  while (f + 1 < nf && bf[f + 1].item0 <= it) ++f;
  return f;
}

// Batched compression of one level of several fields: one workgroup per
// column segment of the work list (the fields' segments in order).  The
// fields' launch arguments are read from memory.
template <typename T, int INTERP>
__global__ __launch_bounds__(WG3, sizeof(T) == 4 ? 4 : 2) void k_level3_compress_batch(const BatchC<T> *__restrict__ bf,
                                                                   int nf) {
  __shared__ SharedC<T> S;
  const uint32_t it = work_item();
  const BatchC<T> &b = bf[item_field(bf, nf, it)];
  const uint32_t li = it - b.item0;
  int tx, ty, zs;
  item_tile(b.L, li, tx, ty, zs);
  level3_compress_body<T, INTERP>(b.L, b.x, b.gin, b.gout, b.eb, b.two_eb, b.inv, b.qmax, b.o, tx,
                                  ty, zs, b.L.row_base + li, S);
}

// 32 plane words (p[k] = plane k of 32 codes, absent planes 0) -> the 32
// codes v with the digits outside `keep` cleared.  The XOR coding e = v ^
// (v >> 1) ^ (v >> 2) is undone plane by plane from the top (v_31 = e_31,
// v_30 = e_30 ^ v_31, v_k = e_k ^ v_k+1 ^ v_k+2), then the planes are
// transposed back into codes.
__device__ __forceinline__ void planes_to_codes(uint32_t p[32], uint32_t keep) {
  p[30] ^= p[31];
#pragma unroll
  for (int k = 29; k >= 0; --k) p[k] ^= p[k + 1] ^ p[k + 2];
  transpose32p(p);
#pragma unroll
  for (int j = 0; j < 32; ++j) p[j] &= keep;
}

// Planes 0 .. 15 only (every loaded plane below 16): the XOR coding undone
// on 16 planes, a pair of 16x16 transposes, then the halves split into codes
// j and j + 16.
__device__ __forceinline__ void planes_to_codes16(uint32_t p[32], uint32_t keep) {
  p[14] ^= p[15];
#pragma unroll
  for (int k = 13; k >= 0; --k) p[k] ^= p[k + 1] ^ p[k + 2];
  transpose16x2(p);
  const uint32_t kw = (keep & 0xFFFFu) | (keep << 16);
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const uint32_t w = p[j] & kw;
    p[j] = w & 0xFFFFu;
    p[j + 16] = w >> 16;
  }
}

// The plane word a retrieval thread fetches each step.  Roles are fixed for
// the workgroup (thread index):
//   t < 56:        word of the workgroup's own chunks (A: 8, B: 16, C: 32)
//   64 <= t < 121: a halo word (when every chunk column involved is 32
//                  targets wide, so that a chunk row is one word)
//     u 0 .. 8:   pass A rows y0-2, y0+16, y0+18 in chunk columns tx-1, tx, tx+1
//     u 9 .. 24:  pass A own rows, chunk columns tx-1 (code 31) and tx+1 (codes 0, 1)
//     u 25 .. 56: pass B rows (zz, k), chunk columns tx-1 and tx+1
// Everything that does not change along the column is worked out once: the
// chunk's global index and slot at chunk row 0 advance by a fixed stride per
// row.
struct WordRole {
  uint32_t bits;  // pass + 1 (0: no word) | sel << 2 | zlim << 4 | wd << 5 | dst << 10 | eyx << 20
  uint32_t g0;    // global chunk index at chunk row 0
  __device__ __forceinline__ int p() const { return int(bits & 3u) - 1; }
  __device__ __forceinline__ int sel() const { return int((bits >> 2) & 3u); }
  __device__ __forceinline__ int zlim() const { return int((bits >> 4) & 1u); }
  __device__ __forceinline__ uint32_t wd() const { return (bits >> 5) & 31u; }
  __device__ __forceinline__ int dst() const { return int((bits >> 10) & 1023u); }
  __device__ __forceinline__ uint32_t eyx() const { return bits >> 20; }
};

__device__ __forceinline__ WordRole word_role(const Level3Args &L, int t, int tx, int ty, int y0,
                                              bool wordhalo) {
  WordRole r{0u, 0u};
  int p = -1, sel = 3, dst = 0, dy = 0, dx = 0, row = 0, y = y0, zz = 0;
  if (t < 56) {
    p = t < 8 ? 0 : (t < 24 ? 1 : 2);
    row = t < 8 ? t : (t < 24 ? t - 8 : t - 24);
  } else if (wordhalo && t >= 64 && t < 121) {
    const int u = t - 64;
    if (u < 9) {
      const int q = u / 3, c = u - (u / 3) * 3;
      p = 0;
      dy = q == 0 ? -1 : 1;
      dx = c - 1;
      row = q == 0 ? 7 : q - 1;
      y = q == 0 ? y0 - 2 : y0 + 14 + 2 * q;
      sel = c;
      dst = (q == 0 ? 0 : 8 + q) * NXP;
    } else if (u < 25) {
      const int v = u - 9, yj = 1 + (v >> 1), side = v & 1;
      p = 0;
      dx = side ? 1 : -1;
      row = yj - 1;
      y = y0 - 2 + 2 * yj;
      sel = side ? 2 : 0;
      dst = yj * NXP;
    } else {
      const int v = u - 25, k = (v >> 1) & 7, side = v & 1;
      zz = v >> 4;
      p = 1;
      dx = side ? 1 : -1;
      row = k;
      y = y0 + 1 + 2 * k;
      sel = side ? 2 : 0;
      dst = (zz * 8 + k) * 4;
    }
  }
  const int tyn = ty + dy, txn = tx + dx;
  if (p < 0 || unsigned(tyn) >= unsigned(L.tiles_y) || unsigned(txn) >= unsigned(L.tiles_x) ||
      (sel != 3 && unsigned(y) >= unsigned(L.L[1])))
    return r;
  const int ey = clampi(LSEL2(tdims, p, 1) - tyn * LSEL2(ct, p, 1), LSEL2(ct, p, 1));
  const int ex = clampi(LSEL2(tdims, p, 2) - txn * LSEL2(ct, p, 2), LSEL2(ct, p, 2));
  const uint32_t wd = uint32_t(sel == 3 || p == 0 ? row : zz * ey + row);
  const uint32_t zlim = p == 0 ? 1u : uint32_t(zz);
  r.bits = uint32_t(p + 1) | uint32_t(sel) << 2 | zlim << 4 | wd << 5 | uint32_t(dst) << 10 |
           uint32_t(ey * ex) << 20;
  r.g0 = uint32_t(LSEL(chunk_base, p)) + uint32_t(tyn) * uint32_t(L.tiles_x) + uint32_t(txn);
  return r;
}

// the NP lowest plane words of word `w` of a chunk whose stored planes start
// at payload word `first` (its stored planes that `keep` selects; planes not
// loaded are 0, and planes from `top` up, which no lane of the wave loads,
// are not looked at).  Slot placement keeps plane k at (31 - k) W words;
// packed placement at the rank of k among the stored planes.
template <int NP>
__device__ __forceinline__ void load_planes_top(const RetrieveIn &in, bool packed, uint64_t first,
                                                uint32_t mask, uint32_t keep, uint32_t W, uint32_t w,
                                                int top, uint32_t p[32]) {
  uint32_t load = mask & keep;
  asm volatile("" : "+v"(load));
  const uint32_t *base = in.payload + first + w;
  if (!packed) {
    const uint32_t *q = base + 31u * W;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      uint32_t v = 0u;
      if (k < top && ((load >> k) & 1u)) v = *q;
      p[k] = v;
      q -= W;
    }
  } else {
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      uint32_t v = 0u;
      if (k < top && ((load >> k) & 1u)) v = base[__umul24(uint32_t(__popc((mask >> k) >> 1)), W)];
      p[k] = v;
    }
  }
}


template <typename T, int INTERP>
__device__ __forceinline__ void level3_retrieve_body(const Level3Args &L, const T *__restrict__ gin,
                                                     T *gout, int discA, int discB, int discC,
                                                     const RetrieveIn &in, T two_eb_arg, int tx,
                                                     int ty, int zs, Shared3<T> &S) {
  using F = F3<T>;
  T two_eb = two_eb_arg;  // in a vector register (see level3_compress_body)
  asm volatile("" : "+v"(two_eb));
  const int tid0 = role_thread();
  const int x0 = tx * TX, y0 = ty * TY;
  const int m0 = zs * L.zseg;
  const int m1 = m0 + L.zseg < L.tiles_z ? m0 + L.zseg : L.tiles_z;
  const int Lz = L.L[0], Ly = L.L[1], Lx = L.L[2];
  const uint32_t keepA = discA >= 32 ? 0u : (0xFFFFFFFFu << discA);
  const uint32_t keepB = discB >= 32 ? 0u : (0xFFFFFFFFu << discB);
  const uint32_t keepC = discC >= 32 ? 0u : (0xFFFFFFFFu << discC);
  const bool has_out = in.n_out > 0;
  const bool packed = in.chunk_off != nullptr;
  const uint32_t tyx = uint32_t(L.tiles_y) * uint32_t(L.tiles_x);
  // halo codes by plane words when every chunk column involved is 32 targets
  // wide (one chunk row = one word)
  const int txr = tx + 1 < L.tiles_x ? tx + 1 : L.tiles_x - 1;
  const bool wordhalo = L.tdims[0][2] - 32 * txr >= 32;

  // reconstruction pred + q * 2eb from the negabinary code v
  auto value = [&](T pred, uint32_t v) -> T {
    T tq;
    if constexpr (sizeof(T) == 4)
      tq = T(int32_t((v ^ NB_A) - NB_A));
    else
      tq = T(int64_t(v ^ NB_A) - int64_t(NB_A));
    return F::add(pred, F::mul(tq, two_eb));
  };

  // exact value of an outlier among the step's chunk oi, if `local` is one
  auto lookup = [&](int mb, int oi, uint32_t local, T &val) {
    const uint32_t a0 = S.orng[mb][oi][0], a1 = S.orng[mb][oi][1];
    if (a1 > a0) {
      if (a1 - a0 <= uint32_t(OCAP)) {
        for (uint32_t j = 0; j < a1 - a0; ++j)
          if (S.oloc[mb][oi][j] == local) val = F::from_bits(S.obits[mb][oi][j]);
      } else {
        uint64_t ob;
        if (find_outlier(in, a0, a1, local, ob)) val = F::from_bits(ob);
      }
    }
  };

  const WordRole R = word_role(L, tid0, tx, ty, y0, wordhalo);
  const uint32_t rkeep = R.p() < 0 ? 0u : sel3(R.p(), keepA, keepB, keepC);
  // mask and (packed placement) first payload word of the role's chunk,
  // fetched one step ahead
  uint32_t pmask = 0;
  uint64_t pword = 0;
  auto prefetch_word = [&](int m) {
    if (R.p() >= 0) {
      const uint32_t g = R.g0 + uint32_t(m) * tyx;
      pmask = in.masks[g];
      if (packed) pword = in.chunk_off[g];
    }
  };

  // coarse-plane entries t, t + 256 (< 385) of the ring, prefetched a step
  // ahead: entry i of thread t sits at li in its ring slot and at ro in its
  // coarse plane (worked out when needed rather than held in registers)
  T rv[2];
  auto ring_entry = [&](int t, int i, int &li, uint32_t &ro) {
    const int e = t + i * WG3;
    const int yj = e / NXE, xi = e - (e / NXE) * NXE;
    const int cy = (y0 >> 1) - 1 + yj, cx = (x0 >> 1) - 1 + xi;
    const bool ok = e < NYE * NXE && unsigned(cy) < unsigned(L.G[1]) && unsigned(cx) < unsigned(L.G[2]);
    li = e < NYE * NXE ? yj * NXP + xi : -1;
    ro = ok ? uint32_t(cy * L.G[2] + cx) : 0u;
  };
  auto issue_ring = [&](int t, int cz) {
    if (cz < L.G[0]) {
      const T *gp = gin + int64_t(cz) * L.G[1] * L.G[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        int li;
        uint32_t ro;
        ring_entry(t, i, li, ro);
        rv[i] = gp[ro];
      }
    }
  };

  const bool vec = (Lx & 3) == 0 && (reinterpret_cast<uintptr_t>(gout) & 15) == 0;
  const uint32_t plane = uint32_t(Ly) * uint32_t(Lx);

  // the first step's chunk words and coarse plane requested before the
  // ring's loads are waited for
  prefetch_word(m0);
  issue_ring(tid0, m0 + 2);
  {
    int li[2];
    uint32_t ro[2];
    ring_entry(tid0, 0, li[0], ro[0]);
    ring_entry(tid0, 1, li[1], ro[1]);
    load_ring(L, gin, S, m0, li, ro);
  }

  for (int m = m0; m < m1; ++m) {
    // a fresh copy of the thread index each step: values derived from it are
    // recomputed here instead of being held in registers across the loop
    int tid = tid0;
    asm volatile("" : "+v"(tid));
    const int ze = 2 * m, zo = 2 * m + 1;
    const int mb = m & 1;
    uint32_t *codes = S.codes[mb];
    // ---- stash the coarse plane m + 2
    if (m + 2 < L.G[0]) {
      T *rs = &S.ring[(m + 2) & 3][0][0];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        int li;
        uint32_t ro;
        ring_entry(tid, i, li, ro);
        if (li >= 0) rs[li] = rv[i];
      }
    }
    // ---- this step's plane words: own chunks and halo (waves 0 and 1)
    if (tid < 128) {
      const uint32_t mask = pmask;
      const int rp = R.p();
      // slot placement: chunk c of pass p at slot_base + c * 32 wmax words
      const uint64_t first =
          packed ? pword
                 : LSEL(slot_base, rp) + uint64_t(R.g0 + uint32_t(m) * tyx - uint32_t(LSEL(chunk_base, rp))) *
                                             (32u * LSEL(wmax, rp));
      const int ez = rp == 0 ? int(zo < Lz) : (Lz - ze < 2 ? Lz - ze : 2);
      const uint32_t W = (uint32_t(ez) * R.eyx() + 31u) >> 5;
      const bool ok = rp >= 0 && (R.sel() == 3 ? R.wd() < W : ze + R.zlim() < Lz);
      if (m + 1 < m1) prefetch_word(m + 1);
      // highest plane any lane of the wave loads
      const uint32_t ld = ok ? (mask & rkeep) : 0u;
      const int top = 32 - __clz(wave_or(ld));
      if (ok) {
        uint32_t p[32];
        if (top <= 16) {
          load_planes_top<16>(in, packed, first, mask, rkeep, W, R.wd(), top, p);
          planes_to_codes16(p, rkeep);
        } else {
          load_planes_top<32>(in, packed, first, mask, rkeep, W, R.wd(), top, p);
          planes_to_codes(p, rkeep);
        }
        if (R.sel() == 3) {
          // all 32 slots of the word, also past the chunk's last code: the
          // pass's buffer holds 33 slots per word of a full chunk, and only
          // slots of real targets are read
          uint32_t *cb = codes + code_off1(rp) + 33 * int(R.wd());
#pragma unroll
          for (int j = 0; j < 32; ++j) cb[j] = p[j];
        } else if (rp == 0) {
          uint32_t *d = &S.hva[0][0] + R.dst();
          if (R.sel() == 1) {
#pragma unroll
            for (int j = 0; j < 32; ++j) d[1 + j] = p[j];
          } else if (R.sel() == 0) {
            d[0] = p[31];
          } else {
            d[33] = p[0];
            d[34] = p[1];
          }
        } else {
          uint32_t *d = &S.hvb[0][0][0] + R.dst();
          if (R.sel() == 0) {
            d[0] = p[31];
          } else {
            d[1] = p[0];
            d[2] = p[1];
          }
        }
      }
    }
    // ---- halo codes one at a time where chunk rows are not single words
    if (!wordhalo && tid >= 64 && tid < 64 + NHA) {
      int yj, xi;
      halo_a(tid - 64, yj, xi);
      int y = y0 - 2 + 2 * yj, xg = x0 - 2 + 2 * xi;
      if (zo < Lz && unsigned(y) < unsigned(Ly) && unsigned(xg) < unsigned(Lx)) {
        int tyn, oy, txn, ox;
        halo_tile(ty, yj, 8, tyn, oy);
        halo_tile(tx, xi, 32, txn, ox);
        S.hva[yj][xi] = fetch_code(L, in, 0, m, tyn, txn, 0, oy, ox, keepA);
      }
    } else if (!wordhalo && tid >= 64 + NHA && tid < 64 + NHA + NHB) {
      int zz, k, xi;
      halo_b(tid - 64 - NHA, zz, k, xi);
      int z = ze + zz, y = y0 + 1 + 2 * k, xg = x0 - 2 + 2 * xi;
      if (z < Lz && y < Ly && unsigned(xg) < unsigned(Lx)) {
        int txn, ox;
        halo_tile(tx, xi, 32, txn, ox);
        S.hvb[zz][k][xi & 3] = fetch_code(L, in, 1, m, ty, txn, zz, k, ox, keepB);
      }
    }
    // outlier ranges of the chunks the step reads: pass A (m, ty-1..ty+1,
    // tx-1..tx+1), pass B (m, ty, tx-1..tx+1), pass C (m, ty, tx)
    int any_out = 0;
    if (has_out && tid >= 241 && tid < 254) {
      const int u = tid - 241;
      const int p = u < 9 ? 0 : (u < 12 ? 1 : 2);
      const int tyn = u < 9 ? ty - 1 + u / 3 : ty;
      const int txn = u < 9 ? tx - 1 + u % 3 : (u < 12 ? tx - 10 + u : tx);
      uint32_t a = 0, b = 0;
      if (unsigned(tyn) < unsigned(L.tiles_y) && unsigned(txn) < unsigned(L.tiles_x)) {
        const uint64_t g = uint64_t(LSEL(chunk_base, p) + chunk_id(L, m, tyn, txn));
        a = in.out_start[g];
        b = in.out_start[g + 1];
      }
      S.orng[mb][u][0] = a;
      S.orng[mb][u][1] = b;
      if (b - a <= uint32_t(OCAP))
        for (uint32_t j = 0; j < b - a; ++j) {
          S.oloc[mb][u][j] = in.out_local[a + j];
          S.obits[mb][u][j] = in.out_bits[a + j];
        }
      any_out = b > a;
    }
    any_out = __builtin_amdgcn_readfirstlane(__syncthreads_or(any_out));
    if (m + 1 < m1) issue_ring(tid, m + 3);
    // ---- pass A at plane zo: the 8 x 32 own targets (one per thread), then
    // the 129 halo targets of the 11 x 35 even grid
    if (zo < Lz) {
      const bool hc = zo + 1 < Lz, ha = zo >= 3, he = zo + 3 < Lz;
      const T *rb = &S.ring[m & 3][0][0];
      const T *rc = &S.ring[(m + 1) & 3][0][0];
      const T *ra = &S.ring[(m - 1) & 3][0][0];
      const T *re = &S.ring[(m + 2) & 3][0][0];
      {
        const int r = tid >> 5, c = tid & 31;
        if (y0 + 2 * r < Ly && x0 + 2 * c < Lx) {
          const int ri = (r + 1) * NXP + c + 1;
          const int ex = clampi(L.tdims[0][2] - tx * L.ct[0][2], L.ct[0][2]);
          const uint32_t local = uint32_t(mad24(r, ex, c));
          const T pred = stencil<T, INTERP>(ra[ri], rb[ri], rc[ri], re[ri], hc, ha, he);
          T val = value(pred, codes[code_off1(0) + pidx(int(local))]);
          if (any_out) lookup(mb, 4, local, val);
          (&S.wa[0][0])[ri] = val;
        }
      }
      if (tid < NHA) {
        int yj, xi;
        halo_a(tid, yj, xi);
        const int y = y0 - 2 + 2 * yj, xg = x0 - 2 + 2 * xi;
        if (unsigned(y) < unsigned(Ly) && unsigned(xg) < unsigned(Lx)) {
          const int ri = yj * NXP + xi;
          const T pred = stencil<T, INTERP>(ra[ri], rb[ri], rc[ri], re[ri], hc, ha, he);
          T val = value(pred, (&S.hva[0][0])[ri]);
          if (any_out) {
            const int oi = (yj == 0 ? 0 : (yj <= 8 ? 3 : 6)) + (xi == 0 ? 0 : (xi <= 32 ? 1 : 2));
            if (S.orng[mb][oi][1] > S.orng[mb][oi][0]) {
              int tyn, oy, txn, ox;
              halo_tile(ty, yj, 8, tyn, oy);
              halo_tile(tx, xi, 32, txn, ox);
              const Ext e = chunk_ext(L, 0, m, tyn, txn);
              lookup(mb, oi, uint32_t(oy * e.ex + ox), val);
            }
          }
          (&S.wa[0][0])[ri] = val;
        }
      }
    }
    __syncthreads();
    // ---- pass B at planes ze, zo: thread t takes plane t / 128, column
    // x0 + 2 (t % 32) and the odd rows y0 + 1 + 2 k of k = 2 s, 2 s + 1
    // (s = t / 32 % 4), from the five even rows around them; then the 48
    // halo targets at columns x0-2, x0+64, x0+66
    {
      const int zz = tid >> 7, s = (tid >> 5) & 3, c = tid & 31;
      const int ey = clampi(L.tdims[1][1] - ty * L.ct[1][1], L.ct[1][1]);
      const int ex = clampi(L.tdims[1][2] - tx * L.ct[1][2], L.ct[1][2]);
      if (ze + zz < Lz && x0 + 2 * c < Lx) {
        const T *src = (zz == 0 ? S.ring[m & 3][0] : S.wa[0]) + 2 * s * NXP + c + 1;
        const T v0 = src[0], v1 = src[NXP], v2 = src[2 * NXP], v3 = src[3 * NXP], v4 = src[4 * NXP];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int k = 2 * s + h;
          const int y = y0 + 1 + 2 * k;
          if (y >= Ly) continue;
          const bool hc = y + 1 < Ly, ha = y >= 3, he = y + 3 < Ly;
          const T pred = h == 0 ? stencil<T, INTERP>(v0, v1, v2, v3, hc, ha, he)
                                : stencil<T, INTERP>(v1, v2, v3, v4, hc, ha, he);
          const uint32_t local = uint32_t(mad24(mad24(zz, ey, k), ex, c));
          T val = value(pred, codes[code_off1(1) + pidx(int(local))]);
          if (any_out) lookup(mb, 10, local, val);
          S.wb[zz][k][c + 1] = val;
        }
      }
      if (tid < NHB) {
        int zh, kh, xi;
        halo_b(tid, zh, kh, xi);
        const int yh = y0 + 1 + 2 * kh, xg = x0 - 2 + 2 * xi;
        if (ze + zh < Lz && yh < Ly && unsigned(xg) < unsigned(Lx)) {
          const T *src = zh == 0 ? S.ring[m & 3][0] : S.wa[0];
          const int ri = kh * NXP + xi;
          const bool hch = yh + 1 < Ly, hah = yh >= 3, heh = yh + 3 < Ly;
          const T pred = stencil<T, INTERP>(src[ri], src[ri + NXP], src[ri + 2 * NXP], src[ri + 3 * NXP], hch, hah, heh);
          T val = value(pred, S.hvb[zh][kh][xi & 3]);
          if (any_out) {
            const int oi = 9 + (xi == 0 ? 0 : 2);
            if (S.orng[mb][oi][1] > S.orng[mb][oi][0]) {
              int txn, ox;
              halo_tile(tx, xi, 32, txn, ox);
              const Ext e = chunk_ext(L, 1, m, ty, txn);
              lookup(mb, oi, uint32_t((zh * e.ey + kh) * e.ex + ox), val);
            }
          }
          S.wb[zh][kh][xi] = val;
        }
      }
    }
    __syncthreads();
    // ---- pass C and the level grid's points (see above).  The next step
    // writes the other code buffer and outlier slots, and rewrites wa, wb
    // only after its first barrier, so no barrier closes the step.
    // pass C: thread t reconstructs row yy = t / 16 of both planes at the odd
    // columns x0 + 4 k + 1 and x0 + 4 k + 3 (k = t % 16), and writes the four
    // points x0 + 4 k .. + 3 of the row (two of them even columns it read)
    const int cyy = tid >> 4, ck = tid & 15;
    const int cx1 = x0 + 4 * ck + 1;
    if (y0 + cyy < Ly) {
      const int cexC = clampi(L.tdims[2][2] - tx * L.ct[2][2], L.ct[2][2]);
      const int ceyC = clampi(L.tdims[2][1] - ty * L.ct[2][1], L.ct[2][1]);
      const bool chc0 = cx1 + 1 < Lx, cha0 = cx1 >= 3, che0 = cx1 + 3 < Lx;
      const bool chc1 = cx1 + 3 < Lx, cha1 = cx1 + 2 >= 3, che1 = cx1 + 5 < Lx;
      const bool interior = vec && zo < Lz && x0 + TX <= Lx;
      const int y = y0 + cyy;
#pragma unroll
      for (int zz = 0; zz < 2; ++zz) {
        if (ze + zz >= Lz) continue;
        const T *row = even_row<T>(S, m, zz, cyy) + 2 * ck;
        const T e0 = row[0], e1 = row[1], e2 = row[2], e3 = row[3], e4 = row[4];
        const uint32_t lrow = uint32_t(mad24(mad24(zz, ceyC, cyy), cexC, 2 * ck));
        T v0 = e0, v1 = e0;
        if (cx1 < Lx) {
          v0 = value(stencil<T, INTERP>(e0, e1, e2, e3, chc0, cha0, che0), codes[code_off1(2) + pidx(int(lrow))]);
          if (any_out) lookup(mb, 12, lrow, v0);
        }
        if (cx1 + 2 < Lx) {
          v1 = value(stencil<T, INTERP>(e1, e2, e3, e4, chc1, cha1, che1), codes[code_off1(2) + pidx(int(lrow) + 1)]);
          if (any_out) lookup(mb, 12, lrow + 1u, v1);
        }
        T *dst = gout + (uint32_t(ze + zz) * plane + uint32_t(mad24(y, Lx, cx1 - 1)));
        if (interior) {
          if constexpr (sizeof(T) == 4) {
            *reinterpret_cast<float4 *>(dst) = make_float4(e1, v0, e2, v1);
          } else {
            reinterpret_cast<double2 *>(dst)[0] = make_double2(e1, v0);
            reinterpret_cast<double2 *>(dst)[1] = make_double2(e2, v1);
          }
        } else if (cx1 - 1 < Lx) {
          dst[0] = e1;
          if (cx1 < Lx) dst[1] = v0;
          if (cx1 + 1 < Lx) dst[2] = e2;
          if (cx1 + 2 < Lx) dst[3] = v1;
        }
      }
    }
  }
}

template <typename T, int INTERP>
__global__ __launch_bounds__(WG3) void k_level3_retrieve(Level3Args L, const T *__restrict__ gin,
                                                          T *gout, int discA, int discB, int discC,
                                                          RetrieveIn in, T two_eb) {
  __shared__ Shared3<T> S;
  int tx, ty, zs;
  block_tile(L, tx, ty, zs);
  level3_retrieve_body<T, INTERP>(L, gin, gout, discA, discB, discC, in, two_eb, tx, ty, zs, S);
}

// Batched retrieval of one level of several fields (work list, as
// k_level3_compress_batch)
template <typename T, int INTERP>
__global__ __launch_bounds__(WG3, sizeof(T) == 4 ? 5 : 4) void k_level3_retrieve_batch(const BatchR<T> *__restrict__ bf,
                                                                   int nf) {
  __shared__ Shared3<T> S;
  const uint32_t it = work_item();
  const BatchR<T> &b = bf[item_field(bf, nf, it)];
  int tx, ty, zs;
  item_tile(b.L, it - b.item0, tx, ty, zs);
  level3_retrieve_body<T, INTERP>(b.L, b.gin, b.gout, b.disc[0], b.disc[1], b.disc[2], b.in,
                                  b.two_eb, tx, ty, zs, S);
}

// anchors of a fused compression: quantize against 0 into the compact coarse grid
// (every thread of the workgroup calls it: it synchronizes the workgroup)
template <typename T>
__device__ __forceinline__ void anchor3_compress_body(const Level3Args &L, const T *__restrict__ x, T *gout,
                                                      double eb, T two_eb, T inv, T qmax,
                                                      const CompressOut &o, uint32_t *sv, uint32_t &sor) {
  using F = F3<T>;
  const int tid = threadIdx.x;
  const int n = L.L[0] * L.L[1] * L.L[2];  // anchor grid (<= 2 per dimension)
  if (tid == 0) sor = 0;
  __syncthreads();
  unsigned long long mb = 0;
  if (tid < n) {
    int az = tid / (L.L[1] * L.L[2]), r = tid - az * (L.L[1] * L.L[2]);
    int ay = r / L.L[2], ax = r - ay * L.L[2];
    T xv = x[int64_t(az) * L.sZ + int64_t(ay) * L.sY + int64_t(ax) * L.sX];
    T xhat;
    bool out;
    int32_t q = quantize<T>(xv, T(0), eb, two_eb, inv, qmax, xhat, out);
    gout[tid] = xhat;
    uint32_t v = (uint32_t(q) + NB_A) ^ NB_A;
    sv[tid] = v;
    atomicOr(&sor, xenc(v));
    if (out) {
      unsigned long long slot = atomicAdd(o.n_out, 1ull);
      if (slot < o.out_cap) {
        OutlierRec *rr = reinterpret_cast<OutlierRec *>(o.out_recs) + slot;
        rr->pass = 0;
        rr->chunk = 0;
        rr->local = uint32_t(tid);
        rr->pad = 0;
        rr->bits = F::bits(xv);
      }
    }
    double ax2 = fabs(double(xhat));
    if (ax2 <= 1.7976931348623157e308) mb = (unsigned long long)__double_as_longlong(ax2);
  }
  __syncthreads();
  const uint32_t mask = sor;
  if (tid == 0) {
    uint32_t r[32];
    for (int j = 0; j < 32; ++j) r[j] = j < n ? xenc(sv[j]) : 0u;
    transpose32(r);
    for (int k = 0; k < 32; ++k)
      if ((mask >> k) & 1u) o.payload[L.slot_base[0] + uint64_t(31 - k)] = r[k];
    o.masks[L.chunk_base[0]] = mask;
  }
  // plane sizes of the anchor chunk (one word per plane) and its delta-y
  // (always loaded; kept for completeness), one b per thread
  if (tid < 32 && ((mask >> tid) & 1u)) o.sizes[tid] = 4ull;
  if (tid < 32) {
    const int b = tid + 1;
    const uint32_t mm = b == 32 ? 0xFFFFFFFFu : ((1u << b) - 1u);
    const uint32_t ab = NB_A & mm;
    uint32_t mxv = 0;
    for (int j = 0; j < n; ++j) {
      const uint32_t t = (sv[j] ^ NB_A) & mm;
      const uint32_t d = t >= ab ? t - ab : ab - t;
      mxv = d > mxv ? d : mxv;
    }
    atomicMax(o.errq + b, mxv);
  }
  if (mb) atomicMax(o.maxabs_bits, mb);
}

// One wave (64 threads).  The cleared words are updated again by this wave's
// anchors (after the fence, which waits until the clearing stores have
// reached memory) and by later launches.
template <typename T>
__global__ __launch_bounds__(64) void k_anchor3_compress(Level3Args L, const T *__restrict__ x, T *gout,
                                                         double eb, T two_eb, T inv, T qmax,
                                                         CompressOut o, uint32_t *clear,
                                                         uint32_t clear_words) {
  __shared__ uint32_t sv[64];
  __shared__ uint32_t sor;
  if (clear_words) {
    for (uint32_t i = threadIdx.x; i < clear_words; i += 64) clear[i] = 0u;
    __threadfence();
  }
  anchor3_compress_body<T>(L, x, gout, eb, two_eb, inv, qmax, o, sv, sor);
}

// anchors of a fused retrieval: anchor `tid` of the anchor grid (the caller
// keeps tid below its size)
template <typename T>
__device__ __forceinline__ void anchor3_retrieve_one(const Level3Args &L, T *gout, const RetrieveIn &in,
                                                     T two_eb, int tid) {
  using F = F3<T>;
  const uint32_t mask = in.masks[L.chunk_base[0]];
  const bool packed = in.chunk_off != nullptr;
  const uint64_t base = packed ? in.chunk_off[L.chunk_base[0]] : L.slot_base[0];
  uint32_t e = 0;
  for (int k = 31; k >= 0; --k) {
    if (!((mask >> k) & 1u)) continue;
    e |= ((in.payload[base + plane_rank(packed, mask, k)] >> tid) & 1u) << k;
  }
  uint32_t v = xdec(e);
  int64_t q = int64_t(v ^ NB_A) - int64_t(NB_A);
  T tq = sizeof(T) == 4 ? T(int32_t(q)) : T(q);
  T val = F::add(T(0), F::mul(tq, two_eb));
  uint64_t ob;
  if (in.n_out > 0 && find_outlier(in, in.out_start[L.chunk_base[0]], in.out_start[L.chunk_base[0] + 1],
                                   uint32_t(tid), ob))
    val = F::from_bits(ob);
  gout[tid] = val;
}

template <typename T>
__global__ void k_anchor3_retrieve(Level3Args L, T *gout, RetrieveIn in, T two_eb) {
  const int tid = threadIdx.x;
  if (tid < L.L[0] * L.L[1] * L.L[2]) anchor3_retrieve_one<T>(L, gout, in, two_eb, tid);
}

template <typename T>
__global__ void k_gather_coarse(const T *__restrict__ field, int64_t fd1, int64_t fd2, int64_t s,
                                T *g, int64_t g0, int64_t g1, int64_t g2) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int64_t n = g0 * g1 * g2;
  if (i >= n) return;
  int64_t c2 = i % g2, r = i / g2, c1 = r % g1, c0 = r / g1;
  g[i] = field[((s * c0) * fd1 + s * c1) * fd2 + s * c2];
}

// ------------------------------------------------------------ queue launches

__global__ void k_queue_reset(uint32_t *claims) {
  if (threadIdx.x < QUEUE_LEVELS) claims[threadIdx.x] = 0u;
}

// Every head job of the table: the anchors of a field by workgroup
// (field mod grid), a gather spread over the whole grid.
template <typename T>
__global__ __launch_bounds__(256) void k_heads_retrieve(const QueueTable *__restrict__ tab) {
  const uint32_t n = tab->n_heads;
  const HeadR<T> *h = reinterpret_cast<const HeadR<T> *>(reinterpret_cast<const char *>(tab) + tab->heads_off);
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (uint32_t f = 0; f < n; ++f) {
    const HeadR<T> &hd = h[f];
    if (hd.mode == 0) {
      const int na = hd.A.L[0] * hd.A.L[1] * hd.A.L[2];
      if (blockIdx.x == f % gridDim.x && int(threadIdx.x) < na)
        anchor3_retrieve_one<T>(hd.A, hd.g, hd.in, hd.two_eb, int(threadIdx.x));
    } else {
      const int64_t g1 = hd.gd[1], g2 = hd.gd[2], total = hd.gd[0] * g1 * g2;
      for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += stride) {
        const int64_t c2 = i % g2, r = i / g2, c1 = r % g1, c0 = r / g1;
        hd.g[i] = hd.field[((hd.step * c0) * hd.fd[1] + hd.step * c1) * hd.fd[2] + hd.step * c2];
      }
    }
  }
}

// One level slot of a queue launch: a persistent grid whose workgroups take
// work items (column segments of the slot's fields, in work-list order) from
// the slot's claim counter until the list is exhausted.  Every workgroup
// leaves once a claim passes the item count, so the grid always drains.
template <typename T, int INTERP>
__global__ __launch_bounds__(WG3, sizeof(T) == 4 ? 5 : 4) void k_level3_retrieve_queue(
    const QueueTable *__restrict__ tab, int slot, uint32_t *claims) {
  __shared__ Shared3<T> S;
  __shared__ uint32_t s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(claims + slot, 1u);
    __syncthreads();
    const uint32_t it = s_item;
    // every thread has read the claim before the next one overwrites it
    __syncthreads();
    // the slot's description is re-read per item rather than held across
    // the body (it would take registers the body needs)
    const QueueLevel &q = tab->lev[slot];
    if (it >= q.items) break;
    const BatchR<T> *bf =
        reinterpret_cast<const BatchR<T> *>(reinterpret_cast<const char *>(tab) + tab->ent_off) + q.off;
    const BatchR<T> &b = bf[item_field(bf, int(q.nf), it)];
    int tx, ty, zs;
    item_tile(b.L, it - b.item0, tx, ty, zs);
    level3_retrieve_body<T, INTERP>(b.L, b.gin, b.gout, b.disc[0], b.disc[1], b.disc[2], b.in,
                                    b.two_eb, tx, ty, zs, S);
  }
}

// The anchor jobs of a queued compression batch: field f by workgroup
// f mod grid (the first 64 threads; the anchor grid has at most 8 points)
template <typename T>
__global__ __launch_bounds__(256) void k_heads_compress(const QueueTable *__restrict__ tab) {
  __shared__ uint32_t sv[64];
  __shared__ uint32_t sor;
  const uint32_t n = tab->n_heads;
  const HeadC<T> *h = reinterpret_cast<const HeadC<T> *>(reinterpret_cast<const char *>(tab) + tab->heads_off);
  for (uint32_t f = blockIdx.x; f < n; f += gridDim.x) {
    const HeadC<T> &hd = h[f];
    anchor3_compress_body<T>(hd.A, hd.x, hd.g, hd.eb, hd.two_eb, hd.inv, hd.qmax, hd.o, sv, sor);
    __syncthreads();
  }
}

// One level slot of a queued compression batch: a persistent grid whose
// workgroups claim work items (column segments of the slot's fields, in
// work-list order) from the slot's counter until the list is exhausted, as
// k_level3_retrieve_queue does; every workgroup leaves once a claim passes
// the item count.
template <typename T, int INTERP>
__global__ __launch_bounds__(WG3, sizeof(T) == 4 ? 4 : 2) void k_level3_compress_queue(
    const QueueTable *__restrict__ tab, int slot, uint32_t *claims) {
  __shared__ SharedC<T> S;
  __shared__ uint32_t s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(claims + slot, 1u);
    __syncthreads();
    const uint32_t it = s_item;
    // every thread has read the claim before the next one overwrites it
    __syncthreads();
    const QueueLevel &q = tab->lev[slot];
    if (it >= q.items) break;
    const BatchC<T> *bf =
        reinterpret_cast<const BatchC<T> *>(reinterpret_cast<const char *>(tab) + tab->ent_off) + q.off;
    const BatchC<T> &b = bf[item_field(bf, int(q.nf), it)];
    const uint32_t li = it - b.item0;
    int tx, ty, zs;
    item_tile(b.L, li, tx, ty, zs);
    level3_compress_body<T, INTERP>(b.L, b.x, b.gin, b.gout, b.eb, b.two_eb, b.inv, b.qmax, b.o, tx,
                                    ty, zs, b.L.row_base + li, S);
    // the body's last LDS reads are done before the next item clears it
    __syncthreads();
  }
}

// workgroup rows reduced by one workgroup of a row reduction
constexpr int RR_ROWS = 64;
// rows r0 .. r0 + RR_ROWS - 1 of one launch (its rows from row_base), pass p
__device__ __forceinline__ void rows_reduce_part(uint32_t row_base, uint32_t n, const uint32_t pass_index[3],
                                                 const uint32_t *rows, uint32_t *errq,
                                                 unsigned long long *maxabs_bits,
                                                 unsigned long long *sizes, int p, uint32_t r0) {
  __shared__ uint32_t s_max[33];
  __shared__ uint32_t s_sz[32];
  __shared__ unsigned long long s_mx;
  const int tid = threadIdx.x;
  if (r0 >= n) return;  // uniform: before any barrier
  const uint32_t nr = n - r0 < uint32_t(RR_ROWS) ? n - r0 : uint32_t(RR_ROWS);
  if (tid < 33) s_max[tid] = 0u;
  if (tid < 32) s_sz[tid] = 0u;
  if (tid == 0) s_mx = 0ull;
  __syncthreads();
  const uint32_t *base = rows + (size_t(row_base) + r0) * WG_ROW;
  // delta-y: thread t takes b = t % 33 of rows t / 33, + 7, ...
  if (tid < 7 * 33) {
    const int b = tid % 33, r = tid / 33;
    uint32_t v[10];
#pragma unroll
    for (int j = 0; j < 10; ++j) {
      const uint32_t rr = uint32_t(r + 7 * j);
      v[j] = rr < nr ? base[size_t(rr) * WG_ROW + p * 33 + b] : 0u;
    }
    uint32_t m = 0;
#pragma unroll
    for (int j = 0; j < 10; ++j) m = v[j] > m ? v[j] : m;
    if (m) atomicMax(&s_max[b], m);
  }
  // plane words: thread t takes plane t & 31 of rows t >> 5, + 8, ...
  {
    const int k = tid & 31, r = tid >> 5;
    uint32_t v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t rr = uint32_t(r + 8 * j);
      v[j] = rr < nr ? base[size_t(rr) * WG_ROW + ROW_SIZES + p * 32 + k] : 0u;
    }
    uint32_t t = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) t += v[j];
    if (t) atomicAdd(&s_sz[k], t);
  }
  if (p == 0 && uint32_t(tid) < nr) {
    const uint32_t *w = base + size_t(tid) * WG_ROW + 99;
    const unsigned long long v = (unsigned long long)w[0] | ((unsigned long long)w[1] << 32);
    if (v) atomicMax(&s_mx, v);
  }
  __syncthreads();
  const size_t pi = pass_index[p];
  if (tid > 0 && tid < 33 && s_max[tid]) atomicMax(errq + pi * 33 + tid, s_max[tid]);
  if (tid < 32 && s_sz[tid]) atomicAdd(sizes + pi * 32 + tid, 4ull * s_sz[tid]);
  if (p == 0 && tid == 0 && s_mx) atomicMax(maxabs_bits, s_mx);
}

// errq, max |x^| and plane sizes of a compression from the fused-level rows:
// grid (launch, pass, split), each workgroup reduces RR_ROWS rows of one
// launch for one pass with every load of a thread issued together, then one
// atomic per value.
__global__ __launch_bounds__(256) void k_rows_reduce(LevelRows lr, const uint32_t *rows, uint32_t *errq,
                                                     unsigned long long *maxabs_bits,
                                                     unsigned long long *sizes) {
  const int li = blockIdx.x;
  rows_reduce_part(lr.row_base[li], lr.n_rows[li], lr.pass_index[li], rows, errq, maxabs_bits, sizes,
                   int(blockIdx.y), blockIdx.z * RR_ROWS);
}

// ... of every field of a batch in one launch: grid (job, pass, split), a
// job being one level launch of one field with that field's outputs
__global__ __launch_bounds__(256) void k_rows_reduce_batch(const RowsJob *__restrict__ jobs,
                                                           const uint32_t *rows) {
  const RowsJob &j = jobs[blockIdx.x];
  rows_reduce_part(j.row_base, j.n_rows, j.pass_index, rows, j.errq, j.maxabs_bits, j.sizes,
                   int(blockIdx.y), blockIdx.z * RR_ROWS);
}

}  // namespace

hipError_t launch_rows_reduce(const LevelRows &lr, const uint32_t *rows, uint32_t *errq,
                              unsigned long long *maxabs_bits, unsigned long long *sizes,
                              hipStream_t stream) {
  uint32_t most = 0;
  for (int i = 0; i < lr.n; ++i) most = lr.n_rows[i] > most ? lr.n_rows[i] : most;
  if (lr.n == 0 || most == 0) return hipSuccess;
  dim3 grid(uint32_t(lr.n), 3, (most + RR_ROWS - 1) / RR_ROWS);
  hipLaunchKernelGGL(k_rows_reduce, grid, dim3(256), 0, stream, lr, rows, errq, maxabs_bits, sizes);
  return hipGetLastError();
}

hipError_t launch_rows_reduce_batch(const RowsJob *jobs_dev, uint32_t n_jobs, uint32_t most_rows,
                                    const uint32_t *rows, hipStream_t stream) {
  if (n_jobs == 0 || most_rows == 0) return hipSuccess;
  dim3 grid(n_jobs, 3, (most_rows + RR_ROWS - 1) / RR_ROWS);
  hipLaunchKernelGGL(k_rows_reduce_batch, grid, dim3(256), 0, stream, jobs_dev, rows);
  return hipGetLastError();
}

hipError_t launch_level3_compress_batch(int dtype, int interp, const void *batch_dev, int nf,
                                        uint32_t n_items, hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  const dim3 grid(n_items);
  if (dtype == IPC_F32) {
    const BatchC<float> *b = static_cast<const BatchC<float> *>(batch_dev);
    if (interp == IPC_LINEAR)
      hipLaunchKernelGGL((k_level3_compress_batch<float, IPC_LINEAR>), grid, dim3(WG3), 0, s, b,
                         nf);
    else
      hipLaunchKernelGGL((k_level3_compress_batch<float, IPC_CUBIC>), grid, dim3(WG3), 0, s, b,
                         nf);
  } else {
    const BatchC<double> *b = static_cast<const BatchC<double> *>(batch_dev);
    if (interp == IPC_LINEAR)
      hipLaunchKernelGGL((k_level3_compress_batch<double, IPC_LINEAR>), grid, dim3(WG3), 0, s,
                         b, nf);
    else
      hipLaunchKernelGGL((k_level3_compress_batch<double, IPC_CUBIC>), grid, dim3(WG3), 0, s,
                         b, nf);
  }
  return hipGetLastError();
}

hipError_t launch_level3_retrieve_batch(int dtype, int interp, const void *batch_dev, int nf,
                                        uint32_t n_items, hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  const dim3 grid(n_items);
  if (dtype == IPC_F32) {
    const BatchR<float> *b = static_cast<const BatchR<float> *>(batch_dev);
    if (interp == IPC_LINEAR)
      hipLaunchKernelGGL((k_level3_retrieve_batch<float, IPC_LINEAR>), grid, dim3(WG3), 0, s, b,
                         nf);
    else
      hipLaunchKernelGGL((k_level3_retrieve_batch<float, IPC_CUBIC>), grid, dim3(WG3), 0, s, b,
                         nf);
  } else {
    const BatchR<double> *b = static_cast<const BatchR<double> *>(batch_dev);
    if (interp == IPC_LINEAR)
      hipLaunchKernelGGL((k_level3_retrieve_batch<double, IPC_LINEAR>), grid, dim3(WG3), 0, s,
                         b, nf);
    else
      hipLaunchKernelGGL((k_level3_retrieve_batch<double, IPC_CUBIC>), grid, dim3(WG3), 0, s,
                         b, nf);
  }
  return hipGetLastError();
}

hipError_t launch_level3_compress(int dtype, int interp, const Level3Args &L, const void *x,
                                  const void *gin, void *gout, double eb, const CompressOut &o,
                                  hipStream_t s) {
  dim3 grid(uint32_t(L.tiles_x) * uint32_t(L.tiles_y) * uint32_t((L.tiles_z + L.zseg - 1) / L.zseg));
  if (dtype == IPC_F32) {
    float two_eb = float(2.0 * eb), inv = float(1.0 / (2.0 * eb)), qm = float(QMAX_F32);
    if (interp == IPC_LINEAR)
      hipLaunchKernelGGL((k_level3_compress<float, IPC_LINEAR>), grid, dim3(WG3), 0, s, L,
                         (const float *)x, (const float *)gin, (float *)gout, eb, two_eb, inv, qm, o);
    else
      hipLaunchKernelGGL((k_level3_compress<float, IPC_CUBIC>), grid, dim3(WG3), 0, s, L,
                         (const float *)x, (const float *)gin, (float *)gout, eb, two_eb, inv, qm, o);
  } else {
    double two_eb = 2.0 * eb, inv = 1.0 / (2.0 * eb), qm = double(QMAX_F64);
    if (interp == IPC_LINEAR)
      hipLaunchKernelGGL((k_level3_compress<double, IPC_LINEAR>), grid, dim3(WG3), 0, s, L,
                         (const double *)x, (const double *)gin, (double *)gout, eb, two_eb, inv, qm, o);
    else
      hipLaunchKernelGGL((k_level3_compress<double, IPC_CUBIC>), grid, dim3(WG3), 0, s, L,
                         (const double *)x, (const double *)gin, (double *)gout, eb, two_eb, inv, qm, o);
  }
  return hipGetLastError();
}

hipError_t launch_level3_retrieve(int dtype, int interp, const Level3Args &L, const void *gin,
                                  void *gout, const int disc[3], const RetrieveIn &in, double eb,
                                  hipStream_t s) {
  dim3 grid(uint32_t(L.tiles_x) * uint32_t(L.tiles_y) * uint32_t((L.tiles_z + L.zseg - 1) / L.zseg));
  if (dtype == IPC_F32) {
    float two_eb = float(2.0 * eb);
    if (interp == IPC_LINEAR)
      hipLaunchKernelGGL((k_level3_retrieve<float, IPC_LINEAR>), grid, dim3(WG3), 0, s, L,
                         (const float *)gin, (float *)gout, disc[0], disc[1], disc[2], in, two_eb);
    else
      hipLaunchKernelGGL((k_level3_retrieve<float, IPC_CUBIC>), grid, dim3(WG3), 0, s, L,
                         (const float *)gin, (float *)gout, disc[0], disc[1], disc[2], in, two_eb);
  } else {
    double two_eb = 2.0 * eb;
    if (interp == IPC_LINEAR)
      hipLaunchKernelGGL((k_level3_retrieve<double, IPC_LINEAR>), grid, dim3(WG3), 0, s, L,
                         (const double *)gin, (double *)gout, disc[0], disc[1], disc[2], in, two_eb);
    else
      hipLaunchKernelGGL((k_level3_retrieve<double, IPC_CUBIC>), grid, dim3(WG3), 0, s, L,
                         (const double *)gin, (double *)gout, disc[0], disc[1], disc[2], in, two_eb);
  }
  return hipGetLastError();
}

hipError_t launch_anchor3_compress(int dtype, const Level3Args &A, const void *x, void *gout,
                                   double eb, const CompressOut &o, uint32_t *clear,
                                   uint32_t clear_words, hipStream_t s) {
  if (dtype == IPC_F32)
    hipLaunchKernelGGL(k_anchor3_compress<float>, dim3(1), dim3(64), 0, s, A, (const float *)x,
                       (float *)gout, eb, float(2.0 * eb), float(1.0 / (2.0 * eb)), float(QMAX_F32), o,
                       clear, clear_words);
  else
    hipLaunchKernelGGL(k_anchor3_compress<double>, dim3(1), dim3(64), 0, s, A, (const double *)x,
                       (double *)gout, eb, 2.0 * eb, 1.0 / (2.0 * eb), double(QMAX_F64), o, clear,
                       clear_words);
  return hipGetLastError();
}

hipError_t launch_anchor3_retrieve(int dtype, const Level3Args &A, void *gout, const RetrieveIn &in,
                                   double eb, hipStream_t s) {
  if (dtype == IPC_F32)
    hipLaunchKernelGGL(k_anchor3_retrieve<float>, dim3(1), dim3(64), 0, s, A, (float *)gout, in,
                       float(2.0 * eb));
  else
    hipLaunchKernelGGL(k_anchor3_retrieve<double>, dim3(1), dim3(64), 0, s, A, (double *)gout, in,
                       2.0 * eb);
  return hipGetLastError();
}

hipError_t launch_queue_reset(uint32_t *claims, hipStream_t s) {
  hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, s, claims);
  return hipGetLastError();
}

hipError_t launch_heads_retrieve(int dtype, const QueueTable *tab, hipStream_t s) {
  if (dtype == IPC_F32)
    hipLaunchKernelGGL(k_heads_retrieve<float>, dim3(QUEUE_HEAD_WGS), dim3(256), 0, s, tab);
  else
    hipLaunchKernelGGL(k_heads_retrieve<double>, dim3(QUEUE_HEAD_WGS), dim3(256), 0, s, tab);
  return hipGetLastError();
}

hipError_t launch_level3_retrieve_queue(int dtype, int interp, const QueueTable *tab, int slot,
                                        uint32_t *claims, uint32_t grid, hipStream_t s) {
  if (grid == 0 || slot < 0 || slot >= QUEUE_LEVELS) return hipErrorInvalidValue;
  const dim3 g(grid);
  if (dtype == IPC_F32) {
    if (interp == IPC_LINEAR)
      hipLaunchKernelGGL((k_level3_retrieve_queue<float, IPC_LINEAR>), g, dim3(WG3), 0, s, tab, slot, claims);
    else
      hipLaunchKernelGGL((k_level3_retrieve_queue<float, IPC_CUBIC>), g, dim3(WG3), 0, s, tab, slot, claims);
  } else {
    if (interp == IPC_LINEAR)
      hipLaunchKernelGGL((k_level3_retrieve_queue<double, IPC_LINEAR>), g, dim3(WG3), 0, s, tab, slot, claims);
    else
      hipLaunchKernelGGL((k_level3_retrieve_queue<double, IPC_CUBIC>), g, dim3(WG3), 0, s, tab, slot, claims);
  }
  return hipGetLastError();
}

hipError_t launch_heads_compress(int dtype, const QueueTable *tab, hipStream_t s) {
  if (dtype == IPC_F32)
    hipLaunchKernelGGL(k_heads_compress<float>, dim3(QUEUE_HEAD_WGS), dim3(256), 0, s, tab);
  else
    hipLaunchKernelGGL(k_heads_compress<double>, dim3(QUEUE_HEAD_WGS), dim3(256), 0, s, tab);
  return hipGetLastError();
}

hipError_t launch_level3_compress_queue(int dtype, int interp, const QueueTable *tab, int slot,
                                        uint32_t *claims, uint32_t grid, hipStream_t s) {
  if (grid == 0 || slot < 0 || slot >= QUEUE_LEVELS) return hipErrorInvalidValue;
  const dim3 g(grid);
  if (dtype == IPC_F32) {
    if (interp == IPC_LINEAR)
      hipLaunchKernelGGL((k_level3_compress_queue<float, IPC_LINEAR>), g, dim3(WG3), 0, s, tab, slot, claims);
    else
      hipLaunchKernelGGL((k_level3_compress_queue<float, IPC_CUBIC>), g, dim3(WG3), 0, s, tab, slot, claims);
  } else {
    if (interp == IPC_LINEAR)
      hipLaunchKernelGGL((k_level3_compress_queue<double, IPC_LINEAR>), g, dim3(WG3), 0, s, tab, slot, claims);
    else
      hipLaunchKernelGGL((k_level3_compress_queue<double, IPC_CUBIC>), g, dim3(WG3), 0, s, tab, slot, claims);
  }
  return hipGetLastError();
}

hipError_t launch_gather_coarse(int dtype, const void *field, const int64_t fd[3], int64_t step,
                                void *g, const int64_t gd[3], hipStream_t s) {
  int64_t n = gd[0] * gd[1] * gd[2];
  if (n == 0) return hipSuccess;
  dim3 grid(uint32_t((n + 255) / 256));
  if (dtype == IPC_F32)
    hipLaunchKernelGGL(k_gather_coarse<float>, grid, dim3(256), 0, s, (const float *)field, fd[1],
                       fd[2], step, (float *)g, gd[0], gd[1], gd[2]);
  else
    hipLaunchKernelGGL(k_gather_coarse<double>, grid, dim3(256), 0, s, (const double *)field, fd[1],
                       fd[2], step, (double *)g, gd[0], gd[1], gd[2]);
  return hipGetLastError();
}

}  // namespace ipc
