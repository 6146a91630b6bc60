// Level schedule and chunk geometry.
//
// Sec. 4.1 / Fig. interp-design: strides shrink by 2 per level and each level
// interpolates once along every dimension.  Reading used: K = max(1,
// ceil(log2(M - 1))) levels for the largest extent M (K = 0 when M = 1); the
// anchors are the points whose coordinates are all multiples of 2^K and are
// predicted from zero (Alg. 1).  In level coordinates (fine coordinate / h,
// h = 2^(l-1)) the pass along dimension k targets odd coordinates along k,
// even coordinates after k and any coordinate before k.  Codes of a pass are
// grouped in chunks: boxes of 2^chunk_log2 level coordinates, numbered in
// lexicographic tile order; codes inside a chunk are lexicographic.
#include "ipc_internal.h"

#include <algorithm>

namespace ipc {

static const int kDefaultChunk[4][3] = {{0, 0, 0}, {12, 0, 0}, {4, 6, 0}, {1, 4, 6}};

int ceil_log2_u64(uint64_t v) {
  int e = 0;
  while ((uint64_t(1) << e) < v) ++e;
  return e;
}

static int64_t parity_count(int64_t extent, int kind) {
  if (kind == KIND_ANY) return extent;
  if (kind == KIND_ODD) return extent / 2;
  return (extent + 1) / 2;
}

int64_t chunk_count(const PassGeom &p, int64_t c) {
  int64_t t2 = c % p.tiles[2];
  int64_t t1 = (c / p.tiles[2]) % p.tiles[1];
  int64_t t0 = c / (p.tiles[2] * p.tiles[1]);
  int64_t t[3] = {t0, t1, t2};
  int64_t n = 1;
  for (int j = 0; j < 3; ++j) {
    int64_t e = std::min(p.ct[j], p.tdims[j] - t[j] * p.ct[j]);
    if (e <= 0) return 0;
    n *= e;
  }
  return n;
}

void chunk_counts(const PassGeom &p, std::vector<uint32_t> &out) {
  out.assign(size_t(p.n_chunks), 0u);
  // extent of tile t along dimension j (0 past the lattice)
  auto ext = [&](int j, int64_t t) {
    const int64_t e = std::min(p.ct[j], p.tdims[j] - t * p.ct[j]);
    return e > 0 ? e : int64_t(0);
  };
  size_t c = 0;
  for (int64_t t0 = 0; t0 < p.tiles[0]; ++t0) {
    const int64_t e0 = ext(0, t0);
    for (int64_t t1 = 0; t1 < p.tiles[1]; ++t1) {
      const int64_t e01 = e0 * ext(1, t1);
      for (int64_t t2 = 0; t2 < p.tiles[2] && c < out.size(); ++t2, ++c)
        out[c] = uint32_t(e01 * ext(2, t2));
    }
  }
}

bool make_schedule(const int64_t *dims, int D, const int *chunk_log2, Schedule &s,
                   std::string &err) {
  if (D < 1 || D > 3) {
    err = "ndim must be 1, 2 or 3";
    return false;
  }
  s = Schedule();
  s.D = D;
  int64_t M = 0;
  s.n_points = 1;
  for (int j = 0; j < D; ++j) {
    if (dims[j] < 1 || dims[j] > (int64_t(1) << 40)) {
      err = "every dimension must be in [1, 2^40]";
      return false;
    }
    s.dims[j] = dims[j];
    s.dims3[3 - D + j] = dims[j];
    M = std::max(M, dims[j]);
    if (s.n_points > (int64_t(1) << 45) / dims[j]) {
      err = "field too large";
      return false;
    }
    s.n_points *= dims[j];
  }
  bool all_zero = true;
  if (chunk_log2)
    for (int j = 0; j < D; ++j) all_zero = all_zero && chunk_log2[j] == 0;
  for (int j = 0; j < D; ++j) {
    int c = (chunk_log2 && !all_zero) ? chunk_log2[j] : kDefaultChunk[D][j];
    if (c < 1 || c > 16) {
      err = "chunk_log2 entries must be in [1, 16]";
      return false;
    }
    s.chunk_log2[j] = c;
  }
  s.K = (M == 1) ? 0 : std::max(1, ceil_log2_u64(uint64_t(M - 1)));

  // chunk extents padded to 3-D (extent 1 in padded dims)
  int64_t C3[3] = {1, 1, 1};
  for (int j = 0; j < D; ++j) C3[3 - D + j] = int64_t(1) << s.chunk_log2[j];

  int64_t chunk_base = 0;
  uint64_t slot = 0;
  auto finish = [&](PassGeom &p) {
    p.n_chunks = p.tiles[0] * p.tiles[1] * p.tiles[2];
    p.n_targets = p.tdims[0] * p.tdims[1] * p.tdims[2];
    p.max_count = p.ct[0] * p.ct[1] * p.ct[2];
    p.wmax = (p.max_count + 31) / 32;
    p.chunk_base = chunk_base;
    p.slot_base = slot;
    chunk_base += p.n_chunks;
    slot += uint64_t(p.n_chunks) * uint64_t(32 * p.wmax);
    s.passes.push_back(p);
  };

  // pass 0: the anchors, one chunk
  {
    PassGeom p;
    p.index = 0;
    p.level = 0;
    p.dim = -1;
    p.dim3 = -1;
    p.h = int64_t(1) << s.K;
    for (int j = 0; j < 3; ++j) {
      p.ldims[j] = (s.dims3[j] - 1) / p.h + 1;
      p.kinds[j] = KIND_ANY;
      p.tdims[j] = p.ldims[j];
      p.ct[j] = p.ldims[j];
      p.tiles[j] = 1;
    }
    finish(p);
  }
  for (int lev = s.K; lev >= 1; --lev) {
    int64_t h = int64_t(1) << (lev - 1);
    for (int k = 0; k < D; ++k) {
      PassGeom p;
      p.index = int(s.passes.size());
      p.level = lev;
      p.dim = k;
      p.dim3 = k + 3 - D;
      p.h = h;
      for (int j = 0; j < 3; ++j) {
        p.ldims[j] = (s.dims3[j] - 1) / h + 1;
        p.kinds[j] = j < p.dim3 ? KIND_ANY : (j == p.dim3 ? KIND_ODD : KIND_EVEN);
        p.tdims[j] = parity_count(p.ldims[j], p.kinds[j]);
        p.ct[j] = p.kinds[j] == KIND_ANY ? C3[j] : C3[j] / 2;
        if (p.ct[j] < 1) p.ct[j] = 1;
        p.tiles[j] = (p.ldims[j] + C3[j] - 1) / C3[j];
      }
      finish(p);
    }
  }
  s.n_chunks = chunk_base;
  s.slot_words = slot;
  return true;
}

}  // namespace ipc
