// HIP kernels of the IPComp hot path for gfx950 (CDNA4, wave64).
//
// One workgroup handles one chunk of one pass (Sec. 4.1: a pass is one 1-D
// interpolation sweep of a level; its targets are independent of each other,
// all their neighbours come from earlier passes).
//
//  k_compress: prediction (Eq. interp-linear / interp-cubic) from the working
//    reconstruction, quantization with the explicit error check and in-place
//    write-back (Sec. 4.2.2), negabinary + 2-prefix-bit XOR (Sec. 4.4), exact
//    delta-y per discarded-plane count (Thm. 1), chunk plane mask, and an
//    in-register 32x32 bit transpose that turns 32 codes into 32 plane words
//    (Sec. 4.3), stored at the chunk's fixed slot.
//  k_retrieve: the inverse (Alg. 1): gather the loaded plane words, transpose
//    back, undo the XOR code and negabinary, dequantize on top of the same
//    prediction, and put the exactly stored outliers back.
//
// Arithmetic: one IEEE rounding per operation in the field's dtype through the
// *_rn intrinsics (no contraction), round-half-even quantization, the error
// check in double.  This is what makes the result bit-identical to a plain CPU
// evaluation of the same formulas.
#include "kernels.h"

#include <algorithm>
#include <type_traits>

#include "ipc_internal.h"

namespace ipc {
namespace {

constexpr uint32_t NB_A = 0xAAAAAAAAu;
constexpr int WG = 256;
constexpr int MAXC = int(MAX_CHUNK_CODES);
constexpr int LDS_WORDS = MAXC + MAXC / 32;
constexpr int PU = 4;  // codes per thread whose loads are issued together

__device__ __forceinline__ int lds_idx(int j) { return j + (j >> 5); }

template <typename T>
struct FP;
template <>
struct FP<float> {
  static __device__ __forceinline__ float add(float a, float b) { return __fadd_rn(a, b); }
  static __device__ __forceinline__ float sub(float a, float b) { return __fsub_rn(a, b); }
  static __device__ __forceinline__ float mul(float a, float b) { return __fmul_rn(a, b); }
  static __device__ __forceinline__ float rnd(float a) { return __builtin_rintf(a); }
  static __device__ __forceinline__ uint64_t bits(float a) { return __float_as_uint(a); }
  static __device__ __forceinline__ float from_bits(uint64_t b) { return __uint_as_float(uint32_t(b)); }
};
template <>
struct FP<double> {
  static __device__ __forceinline__ double add(double a, double b) { return __dadd_rn(a, b); }
  static __device__ __forceinline__ double sub(double a, double b) { return __dsub_rn(a, b); }
  static __device__ __forceinline__ double mul(double a, double b) { return __dmul_rn(a, b); }
  static __device__ __forceinline__ double rnd(double a) { return __builtin_rint(a); }
  static __device__ __forceinline__ uint64_t bits(double a) { return uint64_t(__double_as_longlong(a)); }
  static __device__ __forceinline__ double from_bits(uint64_t b) { return __longlong_as_double((long long)b); }
};

// Transpose a 32x32 bit matrix held as 32 words: afterwards bit j of a[k]
// is what bit k of a[j] was.  Five block-swap stages (16, 8, 4, 2, 1).
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

__device__ __forceinline__ uint32_t xor_encode(uint32_t v) { return v ^ (v >> 1) ^ (v >> 2); }

// (1 + x + x^2)^-1 = (1 + x)(1 + x^3)(1 + x^6)(1 + x^12)(1 + x^24) over GF(2)
__device__ __forceinline__ uint32_t xor_decode(uint32_t e) {
  uint32_t t = e ^ (e >> 1);
  t ^= t >> 3;
  t ^= t >> 6;
  t ^= t >> 12;
  t ^= t >> 24;
  return t;
}

struct ChunkGeo {
  int32_t e[3];
  int64_t m0[3];
  int32_t count;
};

__device__ __forceinline__ ChunkGeo chunk_geo(const PassArgs &a, int64_t c) {
  ChunkGeo g;
  int64_t t2 = c % a.tiles[2];
  int64_t r = c / a.tiles[2];
  int64_t t1 = r % a.tiles[1];
  int64_t t0 = r / a.tiles[1];
  int64_t t[3] = {t0, t1, t2};
  int32_t cnt = 1;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    int64_t base = t[j] * a.ct[j];
    int64_t e = a.tdims[j] - base;
    if (e > a.ct[j]) e = a.ct[j];
    if (e < 0) e = 0;
    g.e[j] = int32_t(e);
    g.m0[j] = base;
    cnt *= int32_t(e);
  }
  g.count = cnt;
  return g;
}

__device__ __forceinline__ int64_t level_coord(int64_t m, int kind) {
  return kind == KIND_ANY ? m : (kind == KIND_ODD ? 2 * m + 1 : 2 * m);
}

// Codes j = j0, j0 + WG, ... of a chunk walked in order: the chunk-local
// coordinates (o0, o1, o2) advance by WG in mixed radix (e0, e1, e2) with one
// carry per digit, instead of a division per code.
struct CodeWalk {
  int o0, o1, o2;     // chunk-local coordinates of the current code
  int s0, s1, s2;     // WG in mixed radix
  int e1, e2;
  __device__ __forceinline__ CodeWalk(const ChunkGeo &g, int j0) {
    e1 = g.e[1];
    e2 = g.e[2];
    o2 = j0 % e2;
    const int r = j0 / e2;
    o1 = r % e1;
    o0 = r / e1;
    s2 = WG % e2;
    const int t = WG / e2;
    s1 = t % e1;
    s0 = t / e1;
  }
  __device__ __forceinline__ void next() {
    o2 += s2;
    int c = o2 >= e2;
    o2 -= c ? e2 : 0;
    o1 += s1 + c;
    c = o1 >= e1;
    o1 -= c ? e1 : 0;
    o0 += s0 + c;
  }
};

// level coordinates and fine linear index of the walk's current code
__device__ __forceinline__ int64_t walk_position(const PassArgs &a, const ChunkGeo &g,
                                                 const CodeWalk &w, int64_t lev[3]) {
  lev[0] = level_coord(g.m0[0] + w.o0, a.kinds[0]);
  lev[1] = level_coord(g.m0[1] + w.o1, a.kinds[1]);
  lev[2] = level_coord(g.m0[2] + w.o2, a.kinds[2]);
  return ((a.h * lev[0]) * a.dims3[1] + a.h * lev[1]) * a.dims3[2] + a.h * lev[2];
}

__device__ __forceinline__ int64_t pass_stride(const PassArgs &a) {
  if (a.dim3 == 0) return a.h * a.dims3[1] * a.dims3[2];
  if (a.dim3 == 1) return a.h * a.dims3[2];
  return a.h;
}

// Prediction along the pass dimension from level neighbours -+1, -+3.
template <typename T, int INTERP>
__device__ __forceinline__ T predict(const T *w, int64_t idx, int64_t st, int64_t t, int64_t L) {
  using F = FP<T>;
  T b = w[idx - st];
  if (t + 1 >= L) return b;
  T c = w[idx + st];
  if (INTERP == IPC_LINEAR) return F::mul(F::add(b, c), T(0.5));
  bool ha = t >= 3;
  bool he = t + 3 < L;
  if (ha && he) {
    T a = w[idx - 3 * st];
    T e = w[idx + 3 * st];
    return F::mul(F::sub(F::mul(F::add(b, c), T(9.0)), F::add(a, e)), T(0.0625));
  }
  if (he) {
    T e = w[idx + 3 * st];
    return F::mul(F::sub(F::add(F::mul(b, T(3.0)), F::mul(c, T(6.0))), e), T(0.125));
  }
  if (ha) {
    T a = w[idx - 3 * st];
    return F::mul(F::sub(F::add(F::mul(c, T(3.0)), F::mul(b, T(6.0))), a), T(0.125));
  }
  return F::mul(F::add(b, c), T(0.5));
}

// Reductions over a full wave (every lane active) in registers: lane swaps
// within each row of 16 by DPP (quad permutes, half-row and row mirrors; order
// is irrelevant for OR and max), then the four row results read out.  The
// result is uniform.
template <int CTRL>
__device__ __forceinline__ uint32_t lane_swap(uint32_t v) {
  return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), CTRL, 0xF, 0xF, false));
}
template <typename Op>
__device__ __forceinline__ uint32_t wave_fold(uint32_t v, Op op) {
  v = op(v, lane_swap<0xB1>(v));   // quad_perm [1, 0, 3, 2]
  v = op(v, lane_swap<0x4E>(v));   // quad_perm [2, 3, 0, 1]
  v = op(v, lane_swap<0x141>(v));  // row_half_mirror
  v = op(v, lane_swap<0x140>(v));  // row_mirror
  const uint32_t r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
  const uint32_t r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
  return op(op(r0, r1), op(r2, r3));
}
__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
  return wave_fold(v, [](uint32_t a, uint32_t b) { return a | b; });
}
__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
  return wave_fold(v, [](uint32_t a, uint32_t b) { return a > b ? a : b; });
}
__device__ __forceinline__ unsigned long long wave_max64(unsigned long long v) {
  auto mx = [](unsigned long long a, unsigned long long b) { return a > b ? a : b; };
  auto sw = [](unsigned long long x, auto ctrl) {
    constexpr int C = decltype(ctrl)::value;
    return (unsigned long long)lane_swap<C>(uint32_t(x)) |
           ((unsigned long long)lane_swap<C>(uint32_t(x >> 32)) << 32);
  };
  v = mx(v, sw(v, std::integral_constant<int, 0xB1>{}));
  v = mx(v, sw(v, std::integral_constant<int, 0x4E>{}));
  v = mx(v, sw(v, std::integral_constant<int, 0x141>{}));
  v = mx(v, sw(v, std::integral_constant<int, 0x140>{}));
  unsigned long long r = 0;
#pragma unroll
  for (int l = 0; l < 64; l += 16) {
    const unsigned long long x =
        (unsigned long long)uint32_t(__builtin_amdgcn_readlane(int(uint32_t(v)), l)) |
        ((unsigned long long)uint32_t(__builtin_amdgcn_readlane(int(uint32_t(v >> 32)), l)) << 32);
    r = mx(r, x);
  }
  return r;
}

// Chunk c of one pass (the workgroup's share of a k_compress launch).
template <typename T, int INTERP>
__device__ __forceinline__ void compress_chunk(const PassArgs &a, const int64_t c,
                                               const T *__restrict__ x, T *xh, int write_back,
                                               double eb, T two_eb, T inv, T qmax,
                                               const CompressOut &o) {
  using F = FP<T>;
  __shared__ uint32_t s_v[LDS_WORDS];
  __shared__ uint32_t s_or_e, s_or_v, s_qmax;
  __shared__ uint32_t s_errq[33];
  __shared__ unsigned long long s_maxabs;

  const int tid = threadIdx.x;
  const ChunkGeo g = chunk_geo(a, c);
  const int count = g.count;
  uint32_t *mask_out = o.masks + a.chunk_base + c;
  if (count == 0) {
    if (tid == 0) *mask_out = 0;
    return;
  }
  if (tid == 0) {
    s_or_e = 0;
    s_or_v = 0;
    s_qmax = 0;
    s_maxabs = 0;
  }
  if (tid < 33) s_errq[tid] = 0;
  __syncthreads();

  const int64_t st = pass_stride(a);
  const int pd = a.dim3;
  uint32_t or_e = 0, or_v = 0, qabs = 0;
  unsigned long long mx = 0;
  CodeWalk cw(g, tid);
  // PU codes per thread at a time: their loads first, then their stores (the
  // targets of a pass are never neighbours within it, so no load here reads
  // what a store of the group writes; the compiler cannot know that)
  for (int j0 = tid; j0 < count; j0 += PU * WG) {
    int64_t idxu[PU];
    T xvu[PU], predu[PU];
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      if (j0 + u * WG < count) {
        int64_t lev[3];
        idxu[u] = walk_position(a, g, cw, lev);
        xvu[u] = x[idxu[u]];
        predu[u] = pd < 0 ? T(0) : predict<T, INTERP>(xh, idxu[u], st, lev[pd], a.ldims[pd]);
      }
      cw.next();
    }
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int j = j0 + u * WG;
      if (j >= count) break;
      const int64_t idx = idxu[u];
      const T xv = xvu[u];
      const T pred = predu[u];
      T diff = F::sub(xv, pred);
      T qf = F::rnd(F::mul(diff, inv));
      bool out = !(fabs(qf) <= qmax);
      int32_t q = out ? 0 : int32_t(qf);
      T xr = F::add(pred, F::mul(T(q), two_eb));
      if (!out) out = !(fabs(__dsub_rn(double(xr), double(xv))) <= eb);
      T xhat = xr;
      if (out) {
        q = 0;
        xhat = xv;
        unsigned long long slot = atomicAdd(o.n_out, 1ull);
        if (slot < o.out_cap) {
          OutlierRec *r = reinterpret_cast<OutlierRec *>(o.out_recs) + slot;
          r->pass = a.pass_index;
          r->chunk = uint32_t(c);
          r->local = uint32_t(j);
          r->pad = 0;
          r->bits = F::bits(xv);
        }
      }
      if (write_back) xh[idx] = xhat;
      uint32_t v = (uint32_t(q) + NB_A) ^ NB_A;
      s_v[lds_idx(j)] = v;
      or_v |= v;
      or_e |= xor_encode(v);
      uint32_t aq = q < 0 ? uint32_t(-int64_t(q)) : uint32_t(q);
      qabs = aq > qabs ? aq : qabs;
      double ax = fabs(double(xhat));
      if (ax <= 1.7976931348623157e308) {
        unsigned long long bx = (unsigned long long)__double_as_longlong(ax);
        mx = bx > mx ? bx : mx;
      }
    }
  }
  or_e = wave_or(or_e);
  or_v = wave_or(or_v);
  qabs = wave_max(qabs);
  mx = wave_max64(mx);
  if ((tid & 63) == 0) {
    atomicOr(&s_or_e, or_e);
    atomicOr(&s_or_v, or_v);
    atomicMax(&s_qmax, qabs);
    atomicMax(&s_maxabs, mx);
  }
  __syncthreads();
  const uint32_t mask = s_or_e;
  const uint32_t orv = s_or_v;
  const int nb = orv ? 32 - __clz(orv) : 0;  // significant negabinary digits in the chunk

  // delta-y: |q - q'_b| = |(w & M_b) - (A & M_b)| with w = v xor A, M_b = 2^b - 1
  if (nb > 1) {
    uint32_t acc[32];
#pragma unroll
    for (int b = 0; b < 32; ++b) acc[b] = 0;
    for (int j = tid; j < count; j += WG) {
      uint32_t w = s_v[lds_idx(j)] ^ NB_A;
#pragma unroll
      for (int b = 1; b < 32; ++b) {
        if (b < nb) {
          uint32_t m = (1u << b) - 1u;
          uint32_t d = __usad(w & m, NB_A & m, 0u);
          acc[b] = d > acc[b] ? d : acc[b];
        }
      }
    }
#pragma unroll
    for (int b = 1; b < 32; ++b) {
      if (b < nb) {
        uint32_t r = wave_max(acc[b]);
        if ((tid & 63) == 0) atomicMax(&s_errq[b], r);
      }
    }
  }
  __syncthreads();
  if (tid < 33 && tid > 0) {
    uint32_t val = tid < nb ? s_errq[tid] : s_qmax;
    uint32_t *dst = o.errq + size_t(a.pass_index) * 33 + tid;
    if (val > *dst) atomicMax(dst, val);
  }
  if (tid == 0) {
    *mask_out = mask;
    if (s_maxabs > *o.maxabs_bits) atomicMax(o.maxabs_bits, s_maxabs);
  }

  // planes: thread per word, 32 codes -> 32 plane words
  const int W = (count + 31) >> 5;
  uint32_t *slot = o.payload + a.slot_base + uint64_t(c) * 32u * a.wmax;
  for (int w = tid; w < W; w += WG) {
    uint32_t r[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) {
      int jj = 32 * w + j;
      uint32_t v = jj < count ? s_v[lds_idx(jj)] : 0u;
      r[j] = xor_encode(v);
    }
    transpose32(r);
#pragma unroll
    for (int k = 0; k < 32; ++k)
      if ((mask >> k) & 1u) slot[size_t(31 - k) * W + w] = r[k];
  }
}

template <typename T, int INTERP>
__global__ __launch_bounds__(WG) void k_compress(PassArgs a, const T *__restrict__ x, T *xh,
                                                  int write_back, double eb, T two_eb, T inv,
                                                  T qmax, CompressOut o) {
  compress_chunk<T, INTERP>(a, int64_t(blockIdx.x), x, xh, write_back, eb, two_eb, inv, qmax, o);
}

// discard_old >= 0 selects the additive form of Alg. 2: f is the difference
// field, the code is the difference between the codes truncated at `discard`
// and at `discard_old` planes, and outliers contribute zero.
template <typename T, int INTERP>
__device__ __forceinline__ void retrieve_chunk(const PassArgs &a, const int64_t c, T *f,
                                               int discard, const RetrieveIn &in, T two_eb,
                                               int discard_old) {
  using F = FP<T>;
  __shared__ uint32_t s_v[LDS_WORDS];
  const int tid = threadIdx.x;
  const ChunkGeo g = chunk_geo(a, c);
  const int count = g.count;
  if (count == 0) return;
  const int64_t gc = a.chunk_base + c;
  const uint32_t mask = in.masks[gc];
  const uint32_t keep = discard >= 32 ? 0u : (0xFFFFFFFFu << discard);
  const uint32_t load = mask & keep;
  const int W = (count + 31) >> 5;
  const bool packed = in.chunk_off != nullptr;
  const uint64_t off = packed ? in.chunk_off[gc] : a.slot_base + uint64_t(c) * 32u * a.wmax;
  // the chunk's words from one uniform base with 32-bit offsets
  const uint32_t *cbase = in.payload + off;
  for (int w = tid; w < W; w += WG) {
    uint32_t r[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      uint32_t rank = packed ? uint32_t(__popc(k == 31 ? 0u : (mask >> (k + 1)))) : uint32_t(31 - k);
      r[k] = ((load >> k) & 1u) ? cbase[rank * uint32_t(W) + uint32_t(w)] : 0u;
    }
    transpose32(r);
#pragma unroll
    for (int j = 0; j < 32; ++j) {
      int jj = 32 * w + j;
      if (jj < count) s_v[lds_idx(jj)] = xor_decode(r[j]) & keep;
    }
  }
  __syncthreads();
  // the chunk's outliers: records out_start[gc] .. out_start[gc + 1] (a
  // stream without outliers has no table)
  const bool any_out = in.n_out > 0;
  const uint64_t olo = any_out ? in.out_start[gc] : 0, ohi = any_out ? in.out_start[gc + 1] : 0;
  const int64_t st = pass_stride(a);
  const int pd = a.dim3;
  const bool additive = discard_old >= 0;
  const uint32_t keep_old = discard_old >= 32 || discard_old < 0 ? 0u : (0xFFFFFFFFu << discard_old);
  CodeWalk cw(g, tid);
  // PU codes per thread at a time: their loads first, then their stores (see
  // compress_chunk)
  for (int j0 = tid; j0 < count; j0 += PU * WG) {
    int64_t idxu[PU];
    T predu[PU];
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      if (j0 + u * WG < count) {
        int64_t lev[3];
        idxu[u] = walk_position(a, g, cw, lev);
        predu[u] = pd < 0 ? T(0) : predict<T, INTERP>(f, idxu[u], st, lev[pd], a.ldims[pd]);
      }
      cw.next();
    }
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int j = j0 + u * WG;
      if (j >= count) break;
      const int64_t idx = idxu[u];
      uint32_t v = s_v[lds_idx(j)];
      int64_t q = int64_t(v ^ NB_A) - int64_t(NB_A);
      const T pred = predu[u];
      T tq;
      if (additive) {
        // the planes above discard_old, as the previous plan held them
        const uint32_t vo = xor_decode(xor_encode(v) & keep_old) & keep_old;
        tq = T(q - (int64_t(vo ^ NB_A) - int64_t(NB_A)));
      } else {
        // float32 codes have at most 26 negabinary digits, so q fits in int32
        tq = sizeof(T) == 4 ? T(int32_t(q)) : T(q);
      }
      T val = F::add(pred, F::mul(tq, two_eb));
      if (ohi > olo) {
        uint64_t b0 = olo, b1 = ohi;
        while (b0 < b1) {
          uint64_t m = (b0 + b1) >> 1;
          if (in.out_local[m] < uint32_t(j)) b0 = m + 1; else b1 = m;
        }
        if (b0 < ohi && in.out_local[b0] == uint32_t(j))
          val = additive ? T(0) : F::from_bits(in.out_bits[b0]);
      }
      f[idx] = val;
    }
  }
}

template <typename T, int INTERP>
__global__ __launch_bounds__(WG) void k_retrieve(PassArgs a, T *f, int discard, RetrieveIn in,
                                                  T two_eb, int discard_old) {
  retrieve_chunk<T, INTERP>(a, int64_t(blockIdx.x), f, discard, in, two_eb, discard_old);
}

// Batched passes: step i of several fields in one launch, one workgroup per
// chunk of the work list (the fields' chunks in order); each workgroup finds
// its field by a uniform scan and reads that field's arguments from memory.
template <typename B>
__device__ __forceinline__ int pass_item_field(const B *__restrict__ bf, int nf, uint32_t it) {
  int f = 0;
  while (f + 1 < nf && bf[f + 1].item0 <= it) ++f;
  return f;
}

template <typename T, int INTERP>
__global__ __launch_bounds__(WG) void k_compress_batch(const PassBatchC<T> *__restrict__ bf, int nf) {
  const uint32_t it = blockIdx.x;
  // uniform field index: the arguments are read with scalar loads
  const PassBatchC<T> &b = bf[__builtin_amdgcn_readfirstlane(pass_item_field(bf, nf, it))];
  compress_chunk<T, INTERP>(b.a, int64_t(it - b.item0), b.x, b.xh, b.write_back, b.eb, b.two_eb,
                            b.inv, b.qmax, b.o);
}

template <typename T, int INTERP>
__global__ __launch_bounds__(WG) void k_retrieve_batch(const PassBatchR<T> *__restrict__ bf, int nf) {
  const uint32_t it = blockIdx.x;
  const PassBatchR<T> &b = bf[__builtin_amdgcn_readfirstlane(pass_item_field(bf, nf, it))];
  retrieve_chunk<T, INTERP>(b.a, int64_t(it - b.item0), b.f, b.discard, b.in, b.two_eb, -1);
}

// x_new = x_old + delta wherever delta is not zero (additive form of Alg. 2)
template <typename T>
__global__ __launch_bounds__(WG) void k_add_delta(T *f, const T *__restrict__ d, uint64_t n) {
  using F = FP<T>;
  for (uint64_t i = uint64_t(blockIdx.x) * WG + threadIdx.x; i < n; i += uint64_t(gridDim.x) * WG) {
    const T dv = d[i];
    if (dv != T(0)) f[i] = F::add(f[i], dv);
  }
}

// Points where a reconstruction misses the error bound: |x - x~| > eb
// (computed in float64) unless both hold the same bits (values that are not
// finite are stored exactly).  One atomic per workgroup with misses.
template <typename T>
__global__ __launch_bounds__(WG) void k_verify_bound(const T *__restrict__ x, const T *__restrict__ xt,
                                                      uint64_t n, double eb, unsigned long long *bad) {
  __shared__ unsigned int s_bad;
  if (threadIdx.x == 0) s_bad = 0u;
  __syncthreads();
  unsigned int mine = 0;
  for (uint64_t i = uint64_t(blockIdx.x) * WG + threadIdx.x; i < n; i += uint64_t(gridDim.x) * WG) {
    const T a = x[i], b = xt[i];
    const bool same = FP<T>::bits(a) == FP<T>::bits(b);
    if (!same && !(fabs(__dsub_rn(double(b), double(a))) <= eb)) ++mine;
  }
  if (mine) atomicAdd(&s_bad, mine);
  __syncthreads();
  if (threadIdx.x == 0 && s_bad) atomicAdd(bad, (unsigned long long)s_bad);
}

// ---- device-side outlier index: records (pass, chunk, local, bits) in any
// order -> arrays sorted by (global chunk, local) and the first record of
// every chunk.  Counting sort by chunk, then an insertion sort of each
// chunk's few records by local index.

__device__ __forceinline__ uint64_t rec_chunk(const PassArgs *args, const OutlierRec &r) {
  return uint64_t(args[r.pass].chunk_base) + r.chunk;
}

__global__ void k_out_hist(const OutlierRec *recs, const unsigned long long *n_out, uint64_t cap,
                           const PassArgs *args, uint32_t *cnt) {
  const uint64_t n = *n_out < cap ? *n_out : cap;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += uint64_t(gridDim.x) * blockDim.x)
    atomicAdd(&cnt[rec_chunk(args, recs[i])], 1u);
}

// exclusive scan of v[0 .. n) in blocks of 1024 (the counts also copied to
// cnt); block totals to bsum
__global__ __launch_bounds__(1024) void k_scan_block(uint32_t *v, uint64_t n, uint32_t *cnt,
                                                     uint32_t *bsum) {
  __shared__ uint32_t s[1024];
  const uint64_t i = uint64_t(blockIdx.x) * 1024 + threadIdx.x;
  const uint32_t x = i < n ? v[i] : 0u;
  if (i < n) cnt[i] = x;
  s[threadIdx.x] = x;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const uint32_t t = threadIdx.x >= unsigned(o) ? s[threadIdx.x - o] : 0u;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  if (i < n) v[i] = s[threadIdx.x] - x;
  if (threadIdx.x == 1023) bsum[blockIdx.x] = s[1023];
}

// adds to block b the sum of the totals of blocks 0 .. b-1 (each workgroup
// sums them itself)
__global__ __launch_bounds__(1024) void k_scan_add(uint32_t *v, uint64_t n, const uint32_t *bsum) {
  __shared__ uint32_t s[1024];
  uint32_t t = 0;
  for (uint32_t j = threadIdx.x; j < blockIdx.x; j += 1024) t += bsum[j];
  s[threadIdx.x] = t;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (threadIdx.x < unsigned(o)) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  const uint64_t i = uint64_t(blockIdx.x) * 1024 + threadIdx.x;
  if (i < n) v[i] += s[0];
}

// cnt holds the per-chunk counts; counting down gives every record its slot
__global__ void k_out_scatter(const OutlierRec *recs, const unsigned long long *n_out, uint64_t cap,
                              const PassArgs *args, const uint32_t *start, uint32_t *cnt,
                              uint64_t *gchunk, uint32_t *local, uint64_t *bits) {
  const uint64_t n = *n_out < cap ? *n_out : cap;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += uint64_t(gridDim.x) * blockDim.x) {
    const OutlierRec r = recs[i];
    const uint64_t g = rec_chunk(args, r);
    const uint32_t pos = start[g] + atomicSub(&cnt[g], 1u) - 1u;
    gchunk[pos] = g;
    local[pos] = r.local;
    bits[pos] = r.bits;
  }
}

__global__ void k_out_sort_chunks(const uint32_t *start, uint64_t n_chunks, uint32_t *local,
                                  uint64_t *bits) {
  for (uint64_t g = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < n_chunks;
       g += uint64_t(gridDim.x) * blockDim.x) {
    const uint32_t a = start[g], b = start[g + 1];
    for (uint32_t i = a + 1; i < b; ++i) {
      const uint32_t l = local[i];
      const uint64_t v = bits[i];
      uint32_t j = i;
      while (j > a && local[j - 1] > l) {
        local[j] = local[j - 1];
        bits[j] = bits[j - 1];
        --j;
      }
      local[j] = l;
      bits[j] = v;
    }
  }
}

// up to OUT_SMALL records sorted by (global chunk, local) in one workgroup:
// keys g << 32 | local (global chunks below 2^32, checked by the host) with
// their record indices, a bitonic sort over the next power of two (padding
// keys sort last), then the sorted arrays
__global__ __launch_bounds__(1024) void k_out_sort_small(const OutlierRec *__restrict__ recs, uint32_t n,
                                                         const PassArgs *__restrict__ args,
                                                         uint64_t *gchunk, uint32_t *local,
                                                         uint64_t *bits) {
  __shared__ uint64_t key[OUT_SMALL];
  __shared__ uint32_t idx[OUT_SMALL];
  uint32_t p2 = 1;
  while (p2 < n) p2 <<= 1;
  for (uint32_t i = threadIdx.x; i < p2; i += blockDim.x) {
    if (i < n) {
      const OutlierRec r = recs[i];
      key[i] = rec_chunk(args, r) << 32 | uint64_t(r.local);
    } else {
      key[i] = ~0ull;
    }
    idx[i] = i;
  }
  __syncthreads();
  for (uint32_t k = 2; k <= p2; k <<= 1)
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      // each pair (i, i ^ j) is ordered by its lower index alone
      for (uint32_t i = threadIdx.x; i < p2; i += blockDim.x) {
        const uint32_t l = i ^ j;
        if (l > i) {
          const uint64_t a = key[i], b = key[l];
          if ((a > b) == ((i & k) == 0)) {
            key[i] = b;
            key[l] = a;
            const uint32_t t = idx[i];
            idx[i] = idx[l];
            idx[l] = t;
          }
        }
      }
      __syncthreads();
    }
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
    gchunk[i] = key[i] >> 32;
    local[i] = uint32_t(key[i]);
    bits[i] = recs[idx[i]].bits;
  }
}

__global__ void k_out_start(const uint64_t *keys, uint64_t n, uint64_t n_chunks, uint32_t *start) {
  uint64_t c = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c > n_chunks) return;
  uint64_t a0 = 0, a1 = n;
  while (a0 < a1) {
    uint64_t m = (a0 + a1) >> 1;
    if (keys[m] < c) a0 = m + 1; else a1 = m;
  }
  start[c] = uint32_t(a0);
}

__global__ __launch_bounds__(WG) void k_pass_sizes(PassArgs a, const uint32_t *masks,
                                                    unsigned long long *sizes) {
  __shared__ unsigned long long s_acc;
  const int k = blockIdx.x;
  if (threadIdx.x == 0) s_acc = 0;
  __syncthreads();
  unsigned long long acc = 0;
  for (int64_t c = threadIdx.x; c < a.n_chunks; c += WG) {
    uint32_t mk = masks[a.chunk_base + c];
    if ((mk >> k) & 1u) {
      ChunkGeo g = chunk_geo(a, c);
      acc += 4ull * uint64_t((g.count + 31) >> 5);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(&s_acc, acc);
  __syncthreads();
  if (threadIdx.x == 0) sizes[k] = s_acc;
}

__global__ __launch_bounds__(WG) void k_pack(PassArgs a, const uint32_t *masks,
                                              const uint64_t *packed_off,
                                              const uint32_t *slot_payload, uint32_t *packed) {
  const int64_t c = blockIdx.x;
  const int64_t gc = a.chunk_base + c;
  const uint32_t mask = masks[gc];
  if (!mask) return;
  const ChunkGeo g = chunk_geo(a, c);
  const int W = (g.count + 31) >> 5;
  const uint32_t *src = slot_payload + a.slot_base + uint64_t(c) * 32u * a.wmax;
  uint32_t *dst = packed + packed_off[gc];
  int rank = 0;
  for (int k = 31; k >= 0; --k) {
    if (!((mask >> k) & 1u)) continue;
    for (int w = threadIdx.x; w < W; w += WG) dst[size_t(rank) * W + w] = src[size_t(31 - k) * W + w];
    ++rank;
  }
}

// sizes[p][k] += 4 * sum over chunks c of pass p with bit k of mask_c of W_c;
// grid (passes, splits), one chunk per thread (the mask loads all in flight).
constexpr int SIZES_CPT = 1;
__global__ __launch_bounds__(WG) void k_all_sizes(const PassArgs *args, const uint32_t *masks,
                                                   unsigned long long *sizes) {
  __shared__ unsigned long long s_acc[32];
  const PassArgs a = args[blockIdx.x];
  const int tid = threadIdx.x;
  const int64_t c0 = int64_t(blockIdx.y) * (SIZES_CPT * WG);
  if (c0 >= a.n_chunks) return;  // uniform: before any barrier
  if (tid < 32) s_acc[tid] = 0;
  __syncthreads();
  int64_t c1 = c0 + SIZES_CPT * WG;
  if (c1 > a.n_chunks) c1 = a.n_chunks;
  uint32_t acc[32];
#pragma unroll
  for (int k = 0; k < 32; ++k) acc[k] = 0;
  for (int64_t c = c0 + tid; c < c1; c += WG) {
    uint32_t mk = masks[a.chunk_base + c];
    if (!mk) continue;
    ChunkGeo g = chunk_geo(a, c);
    uint32_t W = uint32_t((g.count + 31) >> 5);
#pragma unroll
    for (int k = 0; k < 32; ++k) acc[k] += ((mk >> k) & 1u) * W;
  }
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    uint32_t v = acc[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((tid & 63) == 0 && v) atomicAdd(&s_acc[k], 4ull * v);
  }
  __syncthreads();
  if (tid < 32 && s_acc[tid]) atomicAdd(&sizes[size_t(blockIdx.x) * 32 + tid], s_acc[tid]);
}

template <typename T, int INTERP>
hipError_t launch_c(const PassArgs &pa, const void *x, void *xh, int wb, double eb,
                    const CompressOut &o, hipStream_t s) {
  T two_eb = T(2.0 * eb);
  T inv = T(1.0 / (2.0 * eb));
  T qmax = T(sizeof(T) == 4 ? QMAX_F32 : QMAX_F64);
  if (pa.n_chunks == 0) return hipSuccess;
  hipLaunchKernelGGL((k_compress<T, INTERP>), dim3(uint32_t(pa.n_chunks)), dim3(WG), 0, s, pa,
                     static_cast<const T *>(x), static_cast<T *>(xh), wb, eb, two_eb, inv, qmax, o);
  return hipGetLastError();
}

template <typename T, int INTERP>
hipError_t launch_r(const PassArgs &pa, void *f, int discard, const RetrieveIn &in, double eb,
                    hipStream_t s, int discard_old) {
  T two_eb = T(2.0 * eb);
  if (pa.n_chunks == 0) return hipSuccess;
  hipLaunchKernelGGL((k_retrieve<T, INTERP>), dim3(uint32_t(pa.n_chunks)), dim3(WG), 0, s, pa,
                     static_cast<T *>(f), discard, in, two_eb, discard_old);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_compress_pass(int dtype, int interp, const PassArgs &pa, const void *x, void *xh,
                                int write_back, double eb, const CompressOut &o,
                                hipStream_t stream) {
  if (dtype == IPC_F32)
    return interp == IPC_LINEAR ? launch_c<float, IPC_LINEAR>(pa, x, xh, write_back, eb, o, stream)
                                : launch_c<float, IPC_CUBIC>(pa, x, xh, write_back, eb, o, stream);
  return interp == IPC_LINEAR ? launch_c<double, IPC_LINEAR>(pa, x, xh, write_back, eb, o, stream)
                              : launch_c<double, IPC_CUBIC>(pa, x, xh, write_back, eb, o, stream);
}

hipError_t launch_retrieve_pass(int dtype, int interp, const PassArgs &pa, void *field,
                                int discard, const RetrieveIn &in, double eb, hipStream_t stream,
                                int discard_old) {
  const int d = discard, o = discard_old;
  if (dtype == IPC_F32)
    return interp == IPC_LINEAR ? launch_r<float, IPC_LINEAR>(pa, field, d, in, eb, stream, o)
                                : launch_r<float, IPC_CUBIC>(pa, field, d, in, eb, stream, o);
  return interp == IPC_LINEAR ? launch_r<double, IPC_LINEAR>(pa, field, d, in, eb, stream, o)
                              : launch_r<double, IPC_CUBIC>(pa, field, d, in, eb, stream, o);
}

hipError_t launch_compress_pass_batch(int dtype, int interp, const void *batch_dev, int nf,
                                      uint32_t n_items, hipStream_t stream) {
  if (n_items == 0) return hipSuccess;
  if (dtype == IPC_F32) {
    auto *b = static_cast<const PassBatchC<float> *>(batch_dev);
    if (interp == IPC_LINEAR)
      hipLaunchKernelGGL((k_compress_batch<float, IPC_LINEAR>), dim3(n_items), dim3(WG), 0, stream, b, nf);
    else
      hipLaunchKernelGGL((k_compress_batch<float, IPC_CUBIC>), dim3(n_items), dim3(WG), 0, stream, b, nf);
  } else {
    auto *b = static_cast<const PassBatchC<double> *>(batch_dev);
    if (interp == IPC_LINEAR)
      hipLaunchKernelGGL((k_compress_batch<double, IPC_LINEAR>), dim3(n_items), dim3(WG), 0, stream, b, nf);
    else
      hipLaunchKernelGGL((k_compress_batch<double, IPC_CUBIC>), dim3(n_items), dim3(WG), 0, stream, b, nf);
  }
  return hipGetLastError();
}

hipError_t launch_retrieve_pass_batch(int dtype, int interp, const void *batch_dev, int nf,
                                      uint32_t n_items, hipStream_t stream) {
  if (n_items == 0) return hipSuccess;
  if (dtype == IPC_F32) {
    auto *b = static_cast<const PassBatchR<float> *>(batch_dev);
    if (interp == IPC_LINEAR)
      hipLaunchKernelGGL((k_retrieve_batch<float, IPC_LINEAR>), dim3(n_items), dim3(WG), 0, stream, b, nf);
    else
      hipLaunchKernelGGL((k_retrieve_batch<float, IPC_CUBIC>), dim3(n_items), dim3(WG), 0, stream, b, nf);
  } else {
    auto *b = static_cast<const PassBatchR<double> *>(batch_dev);
    if (interp == IPC_LINEAR)
      hipLaunchKernelGGL((k_retrieve_batch<double, IPC_LINEAR>), dim3(n_items), dim3(WG), 0, stream, b, nf);
    else
      hipLaunchKernelGGL((k_retrieve_batch<double, IPC_CUBIC>), dim3(n_items), dim3(WG), 0, stream, b, nf);
  }
  return hipGetLastError();
}

hipError_t launch_add_delta(int dtype, void *field, const void *delta, uint64_t n,
                            hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const uint64_t want = (n + WG - 1) / WG;
  const uint32_t grid = uint32_t(want < 65536 ? want : 65536);
  if (dtype == IPC_F32)
    hipLaunchKernelGGL(k_add_delta<float>, dim3(grid), dim3(WG), 0, stream,
                       static_cast<float *>(field), static_cast<const float *>(delta), n);
  else
    hipLaunchKernelGGL(k_add_delta<double>, dim3(grid), dim3(WG), 0, stream,
                       static_cast<double *>(field), static_cast<const double *>(delta), n);
  return hipGetLastError();
}

hipError_t launch_verify_bound(int dtype, const void *x, const void *xt, uint64_t n, double eb,
                               unsigned long long *bad, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const uint32_t grid = uint32_t(std::min<uint64_t>((n + WG - 1) / WG, 4096));
  if (dtype == IPC_F32)
    hipLaunchKernelGGL(k_verify_bound<float>, dim3(grid), dim3(WG), 0, stream,
                       static_cast<const float *>(x), static_cast<const float *>(xt), n, eb, bad);
  else
    hipLaunchKernelGGL(k_verify_bound<double>, dim3(grid), dim3(WG), 0, stream,
                       static_cast<const double *>(x), static_cast<const double *>(xt), n, eb, bad);
  return hipGetLastError();
}

hipError_t launch_all_sizes(const PassArgs *args_dev, int n_passes, int64_t max_chunks,
                            const uint32_t *masks, unsigned long long *sizes, hipStream_t stream) {
  uint32_t splits = uint32_t((max_chunks + SIZES_CPT * WG - 1) / (SIZES_CPT * WG));
  if (splits == 0) splits = 1;
  hipLaunchKernelGGL(k_all_sizes, dim3(uint32_t(n_passes), splits), dim3(WG), 0, stream, args_dev,
                     masks, sizes);
  return hipGetLastError();
}

hipError_t launch_pass_sizes(const PassArgs &pa, const uint32_t *masks, unsigned long long *sizes,
                             hipStream_t stream) {
  hipLaunchKernelGGL(k_pass_sizes, dim3(32), dim3(WG), 0, stream, pa, masks, sizes);
  return hipGetLastError();
}

hipError_t launch_pack_payload(const PassArgs &pa, const uint32_t *masks,
                               const uint64_t *packed_off, const uint32_t *slot_payload,
                               uint32_t *packed, hipStream_t stream) {
  if (pa.n_chunks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack, dim3(uint32_t(pa.n_chunks)), dim3(WG), 0, stream, pa, masks,
                     packed_off, slot_payload, packed);
  return hipGetLastError();
}

hipError_t launch_out_start(const uint64_t *out_gchunk, uint64_t n_out, uint64_t n_chunks,
                            uint32_t *out_start, hipStream_t stream) {
  dim3 grid(uint32_t((n_chunks + 1 + 255) / 256));
  hipLaunchKernelGGL(k_out_start, grid, dim3(256), 0, stream, out_gchunk, n_out, n_chunks, out_start);
  return hipGetLastError();
}

hipError_t launch_outlier_index_n(const OutlierRec *recs, uint64_t n, const unsigned long long *n_out,
                                  const PassArgs *args, uint64_t n_chunks, uint32_t *start,
                                  uint32_t *cnt, uint32_t *bsum, uint64_t *gchunk, uint32_t *local,
                                  uint64_t *bits, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  if (n > OUT_SMALL || n_chunks >= (uint64_t(1) << 32))
    return launch_outlier_index(recs, n_out, n, args, n_chunks, start, cnt, bsum, gchunk, local, bits,
                                stream);
  hipLaunchKernelGGL(k_out_sort_small, dim3(1), dim3(1024), 0, stream, recs, uint32_t(n), args, gchunk,
                     local, bits);
  return launch_out_start(gchunk, n, n_chunks, start, stream);
}

hipError_t launch_outlier_index(const OutlierRec *recs, const unsigned long long *n_out,
                                uint64_t cap, const PassArgs *args, uint64_t n_chunks,
                                uint32_t *start, uint32_t *cnt, uint32_t *bsum, uint64_t *gchunk,
                                uint32_t *local, uint64_t *bits, hipStream_t stream) {
  // start[] doubles as the histogram (n_chunks + 1 entries, the last one 0)
  hipError_t e = hipMemsetAsync(start, 0, (n_chunks + 1) * 4, stream);
  if (e != hipSuccess) return e;
  const uint32_t rg = uint32_t(std::min<uint64_t>((cap + 255) / 256, 4096));
  hipLaunchKernelGGL(k_out_hist, dim3(rg), dim3(256), 0, stream, recs, n_out, cap, args, start);
  const uint64_t n = n_chunks + 1, nb = (n + 1023) / 1024;
  hipLaunchKernelGGL(k_scan_block, dim3(uint32_t(nb)), dim3(1024), 0, stream, start, n, cnt, bsum);
  hipLaunchKernelGGL(k_scan_add, dim3(uint32_t(nb)), dim3(1024), 0, stream, start, n,
                     (const uint32_t *)bsum);
  hipLaunchKernelGGL(k_out_scatter, dim3(rg), dim3(256), 0, stream, recs, n_out, cap, args,
                     (const uint32_t *)start, cnt, gchunk, local, bits);
  const uint32_t cg = uint32_t(std::min<uint64_t>((n_chunks + 255) / 256, 8192));
  hipLaunchKernelGGL(k_out_sort_chunks, dim3(cg), dim3(256), 0, stream, (const uint32_t *)start,
                     n_chunks, local, bits);
  return hipGetLastError();
}

}  // namespace ipc
