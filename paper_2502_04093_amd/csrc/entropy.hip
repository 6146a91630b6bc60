// Entropy stage for stored bitplane blocks (the stand-in for the paper's
// general-purpose lossless compressor, Sec. 6 setup): every block -- one stored
// plane of one chunk -- is coded on its own by an adaptive binary range coder,
// one block per thread, so retrieval still reads only the blocks of its plan.
//
// Coder: range coding (Martin, 1979) of the block's bits in code order with a
// 12-bit probability of a zero that moves 1/16 of the way toward every coded
// bit.  bound = (range >> 12) * p0; a zero keeps [low, low + bound), a one
// [low + bound, low + range); range is renormalized by bytes below 2^24.
// Output bytes are final when written: the encoder holds the last byte that a
// carry could still reach plus the run of 0xFF bytes behind it and releases
// them once the carry is decided.  The end is the shortest byte run inside the
// final interval, and trailing zero bytes are dropped (the decoder reads zeros
// past the end).  A block is stored coded only when that takes fewer words
// than the raw plane, else raw.
#include "kernels.h"

namespace ipc {
namespace {

constexpr int EC_WG = 128;
constexpr uint32_t PROB_ONE = 4096;
constexpr uint32_t TOP = 1u << 24;

// bytes of one block's code, packed little-endian into words of dst (at most
// cap words kept; only a code shorter than cap is ever used)
struct ByteSink {
  uint32_t *dst;
  uint32_t cap;
  uint32_t n = 0;       // bytes emitted
  uint32_t last_nz = 0; // bytes up to the last nonzero one
  uint32_t acc = 0;
  bool skip = true;     // the encoder's leading virtual zero byte

  __device__ ByteSink(uint32_t *d, uint32_t c) : dst(d), cap(c) {}
  __device__ __forceinline__ void put(uint32_t b) {
    if (skip) {
      skip = false;
      return;
    }
    acc |= b << (8 * (n & 3));
    if (b) last_nz = n + 1;
    ++n;
    if ((n & 3) == 0) {
      if ((n >> 2) <= cap) dst[(n >> 2) - 1] = acc;
      acc = 0;
    }
  }
  __device__ __forceinline__ void flush_word() {
    if ((n & 3) && (n >> 2) < cap) dst[n >> 2] = acc;
  }
};

struct Encoder {
  uint64_t low = 0;       // 32 bits plus the carry bit (low + range < 2^33)
  uint32_t range = 0xFFFFFFFFu;
  uint32_t cache = 0;     // last byte a carry can still change; at first a
                          // virtual zero byte ahead of the code (never carried
                          // into: the coded value stays below 1)
  uint32_t pending = 0;   // 0xFF bytes behind it

  // moves the top byte of low out (a renormalization step); a carry left in
  // bit 32 by the bits since the last step reaches the held bytes first
  __device__ __forceinline__ void shift(ByteSink &out) {
    const uint32_t top = uint32_t(low >> 24) & 0xFFu;
    const uint32_t carry = uint32_t(low >> 32);
    if (top != 0xFFu || carry) {
      // the held bytes are decided
      out.put((cache + carry) & 0xFFu);
      for (; pending; --pending) out.put((0xFFu + carry) & 0xFFu);
      cache = top;
    } else {
      ++pending;  // a 0xFF that a later carry would turn into 0x00
    }
    low = (low & 0x00FFFFFFull) << 8;
  }

  __device__ __forceinline__ void bit(uint32_t b, uint32_t &p0, ByteSink &out) {
    const uint32_t bound = (range >> 12) * p0;
    if (b) {
      low += bound;
      range -= bound;
      p0 -= p0 >> 4;
    } else {
      range = bound;
      p0 += (PROB_ONE - p0) >> 4;
    }
    while (range < TOP) {
      shift(out);
      range <<= 8;
    }
  }

  // the shortest byte run (then zeros) inside [low, low + range): zero bytes
  // when the value 0 (or the carry alone) lies inside, else one byte
  __device__ __forceinline__ void finish(ByteSink &out) {
    uint64_t v;
    const uint64_t hi = low + uint64_t(range);
    const uint64_t v0 = (low & 0xFFFFFFFFull) == 0 ? low : ((low >> 32) + 1) << 32;
    if (v0 < hi)
      v = v0;
    else
      v = ((low + 0xFFFFFFull) >> 24) << 24;
    low = v;
    for (int i = 0; i < 5; ++i) shift(out);
  }
};

// one thread per block
__global__ __launch_bounds__(EC_WG) void k_ec_encode(const EcBlock *__restrict__ blk, uint64_t n,
                                                     const uint32_t *__restrict__ raw,
                                                     uint32_t *__restrict__ scratch,
                                                     uint8_t *__restrict__ words) {
  const uint64_t i = uint64_t(blockIdx.x) * EC_WG + threadIdx.x;
  if (i >= n) return;
  const EcBlock b = blk[i];
  const uint32_t count = b.count;
  const uint32_t W = (count + 31) >> 5;
  const uint32_t *src = raw + b.raw_off;
  uint32_t *dst = scratch + b.raw_off;
  ByteSink out(dst, W);
  Encoder enc;
  uint32_t p0 = PROB_ONE / 2;
  // each word loaded one word ahead, while the one before it is coded
  uint32_t next = W ? src[0] : 0u;
  for (uint32_t w = 0; w < W; ++w) {
    const uint32_t word = next;
    if (w + 1 < W) next = src[w + 1];
    const uint32_t nb = count - 32 * w < 32 ? count - 32 * w : 32;
    for (uint32_t j = 0; j < nb; ++j) enc.bit((word >> j) & 1u, p0, out);
  }
  enc.finish(out);
  out.flush_word();
  const uint32_t used = (out.last_nz + 3) >> 2;
  if (used < W) {
    words[i] = uint8_t(used);
  } else {
    for (uint32_t w = 0; w < W; ++w) dst[w] = src[w];
    words[i] = uint8_t(W);
  }
}

// 16 lanes per block (a stored block holds at most 64 words, most far
// fewer): stored words from the scratch slot to their place in the coded
// payload
constexpr int EC_GATHER_LANES = 16;
__global__ __launch_bounds__(256) void k_ec_gather(const EcBlock *__restrict__ blk, uint64_t n,
                                                   const uint8_t *__restrict__ words,
                                                   const uint32_t *__restrict__ scratch,
                                                   uint32_t *__restrict__ coded) {
  const uint64_t i = uint64_t(blockIdx.x) * (256 / EC_GATHER_LANES) + threadIdx.x / EC_GATHER_LANES;
  if (i >= n) return;
  const uint32_t lane = threadIdx.x % EC_GATHER_LANES;
  const EcBlock b = blk[i];
  const uint32_t nw = words[i];
  for (uint32_t w = lane; w < nw; w += EC_GATHER_LANES) coded[b.coded_off + w] = scratch[b.raw_off + w];
}

// one thread per block: the raw plane (W words) back at raw_off
__global__ __launch_bounds__(EC_WG) void k_ec_decode(const EcBlock *__restrict__ blk, uint64_t n,
                                                     const uint8_t *__restrict__ words,
                                                     const uint32_t *__restrict__ coded,
                                                     uint32_t *__restrict__ raw) {
  const uint64_t i = uint64_t(blockIdx.x) * EC_WG + threadIdx.x;
  if (i >= n) return;
  const EcBlock b = blk[i];
  const uint32_t count = b.count;
  const uint32_t W = (count + 31) >> 5;
  const uint32_t nw = words[i];
  const uint32_t *src = coded + b.coded_off;
  uint32_t *dst = raw + b.raw_off;
  if (nw >= W) {
    for (uint32_t w = 0; w < W; ++w) dst[w] = src[w];
    return;
  }
  const uint32_t nbytes = 4 * nw;
  uint32_t pos = 0;                         // next byte to read
  uint32_t cur = nw ? src[0] : 0u;          // the word holding byte pos
  uint32_t nxt = nw > 1 ? src[1] : 0u;      // the word after it, loaded ahead
  auto next_byte = [&]() -> uint32_t {
    if (pos >= nbytes) {
      ++pos;
      return 0u;
    }
    if ((pos & 3) == 0 && pos) {
      cur = nxt;
      const uint32_t k = (pos >> 2) + 1;
      nxt = k < nw ? src[k] : 0u;
    }
    const uint32_t v = (cur >> (8 * (pos & 3))) & 0xFFu;
    ++pos;
    return v;
  };
  uint32_t code = 0;
  for (int k = 0; k < 4; ++k) code = (code << 8) | next_byte();
  uint32_t range = 0xFFFFFFFFu;
  uint32_t p0 = PROB_ONE / 2;
  for (uint32_t w = 0; w < W; ++w) {
    const uint32_t nb = count - 32 * w < 32 ? count - 32 * w : 32;
    uint32_t word = 0;
    for (uint32_t j = 0; j < nb; ++j) {
      const uint32_t bound = (range >> 12) * p0;
      if (code < bound) {
        range = bound;
        p0 += (PROB_ONE - p0) >> 4;
      } else {
        code -= bound;
        range -= bound;
        p0 -= p0 >> 4;
        word |= 1u << j;
      }
      while (range < TOP) {
        code = (code << 8) | next_byte();
        range <<= 8;
      }
    }
    dst[w] = word;
  }
}

// one thread per chunk: the descriptors of its stored blocks (planes from
// 31 down, each W = ceil(count / 32) words in the packed placement)
__global__ __launch_bounds__(256) void k_ec_blocks(const uint32_t *__restrict__ cblk,
                                                   const uint64_t *__restrict__ craw,
                                                   const uint32_t *__restrict__ ccount,
                                                   uint64_t n_chunks, EcBlock *__restrict__ blk) {
  const uint64_t c = uint64_t(blockIdx.x) * 256 + threadIdx.x;
  if (c >= n_chunks) return;
  const uint32_t b0 = cblk[c], b1 = cblk[c + 1];
  const uint32_t count = ccount[c];
  const uint64_t W = (count + 31) >> 5;
  for (uint32_t r = 0; r < b1 - b0; ++r) {
    EcBlock e;
    e.raw_off = craw[c] + uint64_t(r) * W;
    e.coded_off = 0;
    e.count = count;
    e.pad = 0;
    blk[b0 + r] = e;
  }
}

// exclusive scan of the stored word counts into the blocks' coded offsets:
// tiles of 1024 blocks scanned in LDS, tile totals to `tot`
__global__ __launch_bounds__(1024) void k_ec_scan_tiles(const uint8_t *__restrict__ words, uint64_t n,
                                                        EcBlock *__restrict__ blk,
                                                        uint64_t *__restrict__ tot) {
  __shared__ uint32_t s[1024];
  const uint64_t i = uint64_t(blockIdx.x) * 1024 + threadIdx.x;
  const uint32_t x = i < n ? words[i] : 0u;
  s[threadIdx.x] = x;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const uint32_t t = threadIdx.x >= unsigned(o) ? s[threadIdx.x - o] : 0u;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  if (i < n) blk[i].coded_off = s[threadIdx.x] - x;
  if (threadIdx.x == 1023) tot[blockIdx.x] = s[1023];
}

// adds to every tile the totals of the tiles before it (each workgroup sums
// them itself)
__global__ __launch_bounds__(1024) void k_ec_scan_add(uint64_t n, EcBlock *__restrict__ blk,
                                                      const uint64_t *__restrict__ tot) {
  __shared__ uint64_t s[1024];
  uint64_t t = 0;
  for (uint32_t j = threadIdx.x; j < blockIdx.x; j += 1024) t += tot[j];
  s[threadIdx.x] = t;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (threadIdx.x < unsigned(o)) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  const uint64_t i = uint64_t(blockIdx.x) * 1024 + threadIdx.x;
  if (i < n) blk[i].coded_off += s[0];
}

}  // namespace

hipError_t launch_ec_blocks(const uint32_t *cblk, const uint64_t *craw, const uint32_t *ccount,
                            uint64_t n_chunks, EcBlock *blk, hipStream_t s) {
  if (n_chunks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ec_blocks, dim3(uint32_t((n_chunks + 255) / 256)), dim3(256), 0, s, cblk, craw,
                     ccount, n_chunks, blk);
  return hipGetLastError();
}

hipError_t launch_ec_offsets(const uint8_t *words, uint64_t n, EcBlock *blk, uint64_t *tot,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint32_t tiles = uint32_t((n + 1023) / 1024);
  hipLaunchKernelGGL(k_ec_scan_tiles, dim3(tiles), dim3(1024), 0, s, words, n, blk, tot);
  hipLaunchKernelGGL(k_ec_scan_add, dim3(tiles), dim3(1024), 0, s, n, blk,
                     static_cast<const uint64_t *>(tot));
  return hipGetLastError();
}

hipError_t launch_ec_encode(const EcBlock *blk, uint64_t n, const uint32_t *raw, uint32_t *scratch,
                            uint8_t *words, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ec_encode, dim3(uint32_t((n + EC_WG - 1) / EC_WG)), dim3(EC_WG), 0, s, blk,
                     n, raw, scratch, words);
  return hipGetLastError();
}

hipError_t launch_ec_gather(const EcBlock *blk, uint64_t n, const uint8_t *words,
                            const uint32_t *scratch, uint32_t *coded, hipStream_t s) {
  if (n == 0) return hipSuccess;
  constexpr uint64_t per_wg = 256 / EC_GATHER_LANES;
  hipLaunchKernelGGL(k_ec_gather, dim3(uint32_t((n + per_wg - 1) / per_wg)), dim3(256), 0, s, blk, n,
                     words, scratch, coded);
  return hipGetLastError();
}

hipError_t launch_ec_decode(const EcBlock *blk, uint64_t n, const uint8_t *words,
                            const uint32_t *coded, uint32_t *raw, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ec_decode, dim3(uint32_t((n + EC_WG - 1) / EC_WG)), dim3(EC_WG), 0, s, blk,
                     n, words, coded, raw);
  return hipGetLastError();
}

}  // namespace ipc
