// Serialized stream: header, delta-y table, chunk masks, outliers, payload.
//
// Fig. overall-design: the compressed data is a set of independently
// decompressible blocks, and the data loader reads only the ones a request
// needs.  A block here is one stored bitplane of one chunk.  Layout (little
// endian, every section zero-padded to 8 bytes):
//   header (128 B) | errq [P][33] u32 | masks [n_chunks] u32 |
//   outlier keys [n][3] u32 (pass, chunk, local) | outlier values [n] T |
//   [entropy-coded streams: stored words of every block, u8] |
//   payload u32 (per pass, per chunk, stored planes from 31 down to 0; each
//   block raw, or entropy coded when that is shorter).
// Header byte 11 holds the coding (0 raw, 1 entropy coded).
#include "ipc_internal.h"

#include <cmath>
#include <cstring>

namespace ipc {

static void put32(uint8_t *p, uint32_t v) { std::memcpy(p, &v, 4); }
static void put64(uint8_t *p, uint64_t v) { std::memcpy(p, &v, 8); }
static void putd(uint8_t *p, double v) { std::memcpy(p, &v, 8); }
static uint32_t get32(const uint8_t *p) {
  uint32_t v;
  std::memcpy(&v, p, 4);
  return v;
}
static uint64_t get64(const uint8_t *p) {
  uint64_t v;
  std::memcpy(&v, p, 8);
  return v;
}
static double getd(const uint8_t *p) {
  double v;
  std::memcpy(&v, p, 8);
  return v;
}

static int itemsize(int dtype) { return dtype == IPC_F32 ? 4 : 8; }

// header, errq, masks, outlier keys, outlier values, block words, payload
static void section_sizes(const StreamMeta &m, uint64_t sz[7]) {
  uint64_t P = m.sched.passes.size();
  uint64_t nout = m.n_outliers;
  sz[0] = HEADER_SIZE;
  sz[1] = pad8(4 * 33 * P);
  sz[2] = pad8(4 * uint64_t(m.sched.n_chunks));
  sz[3] = pad8(12 * nout);
  sz[4] = pad8(uint64_t(itemsize(m.dtype)) * nout);
  sz[5] = m.coding ? pad8(m.block_words.size()) : 0;
  sz[6] = pad8(4 * (m.coding ? m.coded_words : m.payload_words));
}

uint64_t serialized_size(const StreamMeta &m) {
  uint64_t sz[7];
  section_sizes(m, sz);
  return sz[0] + sz[1] + sz[2] + sz[3] + sz[4] + sz[5] + sz[6];
}

uint64_t payload_offset(const StreamMeta &m) {
  uint64_t sz[7];
  section_sizes(m, sz);
  return sz[0] + sz[1] + sz[2] + sz[3] + sz[4] + sz[5];
}

uint64_t n_blocks(const StreamMeta &m) {
  uint64_t n = 0;
  for (uint32_t mk : m.masks) n += uint64_t(__builtin_popcount(mk));
  return n;
}

void packed_chunk_offsets(const StreamMeta &m, std::vector<uint64_t> &off) {
  off.assign(size_t(m.sched.n_chunks) + 1, 0);
  uint64_t w = 0;
  std::vector<uint32_t> cnt;
  for (const PassGeom &p : m.sched.passes) {
    chunk_counts(p, cnt);
    for (int64_t c = 0; c < p.n_chunks; ++c) {
      size_t g = size_t(p.chunk_base + c);
      off[g] = w;
      uint32_t mk = m.masks[g];
      if (mk) w += uint64_t(__builtin_popcount(mk)) * uint64_t((cnt[size_t(c)] + 31) / 32);
    }
  }
  off[size_t(m.sched.n_chunks)] = w;
}

void write_serialized_head(const StreamMeta &m, uint8_t *dst) {
  uint64_t sz[7];
  section_sizes(m, sz);
  std::memset(dst, 0, size_t(sz[0] + sz[1] + sz[2] + sz[3] + sz[4] + sz[5]));
  const Schedule &s = m.sched;
  uint8_t *h = dst;
  put32(h + 0, MAGIC);
  put32(h + 4, VERSION);
  h[8] = uint8_t(m.dtype);
  h[9] = uint8_t(s.D);
  h[10] = uint8_t(m.interp);
  h[11] = uint8_t(m.coding);
  put32(h + 12, uint32_t(m.nonprog_levels));
  for (int j = 0; j < 3; ++j) put64(h + 16 + 8 * j, j < s.D ? uint64_t(s.dims[j]) : 1);
  putd(h + 40, m.eb);
  put32(h + 48, uint32_t(s.K));
  put32(h + 52, m.qmax);
  for (int j = 0; j < 3; ++j) h[56 + j] = j < s.D ? uint8_t(s.chunk_log2[j]) : 0;
  h[59] = 0;
  put32(h + 60, uint32_t(s.passes.size()));
  put64(h + 64, uint64_t(s.n_chunks));
  put64(h + 72, m.n_outliers);
  put64(h + 80, m.coding ? m.coded_words : m.payload_words);
  putd(h + 88, m.maxabs);
  uint8_t *p = dst + sz[0];
  std::memcpy(p, m.errq.data(), 4 * m.errq.size());
  p += sz[1];
  std::memcpy(p, m.masks.data(), 4 * m.masks.size());
  p += sz[2];
  for (size_t i = 0; i < m.outliers.size(); ++i) {
    put32(p + 12 * i + 0, m.outliers[i].pass);
    put32(p + 12 * i + 4, m.outliers[i].chunk);
    put32(p + 12 * i + 8, m.outliers[i].local);
  }
  p += sz[3];
  int is = itemsize(m.dtype);
  for (size_t i = 0; i < m.outliers.size(); ++i) {
    if (is == 4)
      put32(p + 4 * i, uint32_t(m.outliers[i].bits));
    else
      put64(p + 8 * i, m.outliers[i].bits);
  }
  p += sz[4];
  if (m.coding) std::memcpy(p, m.block_words.data(), m.block_words.size());
}

bool parse_serialized(const uint8_t *buf, uint64_t n, StreamMeta &m, const uint32_t **payload,
                      std::string &err) {
  if (!buf || n < HEADER_SIZE) {
    err = "stream shorter than its header";
    return false;
  }
  if (get32(buf) != MAGIC || get32(buf + 4) != VERSION) {
    err = "bad magic or version";
    return false;
  }
  m = StreamMeta();
  m.dtype = buf[8];
  int D = buf[9];
  m.interp = buf[10];
  m.coding = buf[11];
  if ((m.dtype != IPC_F32 && m.dtype != IPC_F64) || D < 1 || D > 3 ||
      (m.interp != IPC_LINEAR && m.interp != IPC_CUBIC) || m.coding > 1) {
    err = "bad dtype, ndim, interpolation or coding field";
    return false;
  }
  m.nonprog_levels = int(get32(buf + 12));
  int64_t dims[3];
  for (int j = 0; j < 3; ++j) dims[j] = int64_t(get64(buf + 16 + 8 * j));
  for (int j = D; j < 3; ++j)
    if (dims[j] != 1) {
      err = "unused dims must be 1";
      return false;
    }
  m.eb = getd(buf + 40);
  if (!(std::isfinite(m.eb) && m.eb > 0)) {
    err = "bad error bound";
    return false;
  }
  int cl[3] = {buf[56], buf[57], buf[58]};
  for (int j = 0; j < D; ++j)
    if (cl[j] < 1) {
      err = "bad chunk shape";
      return false;
    }
  if (!make_schedule(dims, D, cl, m.sched, err)) return false;
  if (get32(buf + 48) != uint32_t(m.sched.K)) {
    err = "level count does not match the dims";
    return false;
  }
  m.qmax = get32(buf + 52);
  if (m.qmax != (m.dtype == IPC_F32 ? QMAX_F32 : QMAX_F64)) {
    err = "bad QMAX";
    return false;
  }
  if (m.nonprog_levels < 0 || m.nonprog_levels > m.sched.K) {
    err = "bad nonprog_levels";
    return false;
  }
  uint64_t P = get32(buf + 60);
  uint64_t nch = get64(buf + 64);
  uint64_t nout = get64(buf + 72);
  uint64_t pw = get64(buf + 80);
  m.maxabs = getd(buf + 88);
  if (P != m.sched.passes.size() || nch != uint64_t(m.sched.n_chunks) || !(m.maxabs >= 0) ||
      !std::isfinite(m.maxabs) || nout > n || pw > n) {
    err = "header counts do not match the schedule";
    return false;
  }
  for (int i = 96; i < 128; ++i)
    if (buf[i]) {
      err = "reserved header bytes not zero";
      return false;
    }
  m.payload_words = pw;
  m.coded_words = m.coding ? pw : 0;
  m.n_outliers = nout;
  uint64_t sz[7];
  section_sizes(m, sz);
  if (sz[0] + sz[1] + sz[2] > n) {
    err = "stream shorter than its tables";
    return false;
  }
  if (m.coding) {
    // the block-length section's size follows from the masks
    m.masks.resize(nch);
    std::memcpy(m.masks.data(), buf + sz[0] + sz[1], 4 * nch);
    m.block_words.assign(size_t(n_blocks(m)), 0);
    section_sizes(m, sz);
  }
  if (sz[0] + sz[1] + sz[2] + sz[3] + sz[4] + sz[5] + sz[6] != n) {
    err = "stream size does not match its header";
    return false;
  }
  m.outliers.resize(nout);
  const uint8_t *p = buf + sz[0];
  m.errq.resize(33 * P);
  std::memcpy(m.errq.data(), p, 4 * m.errq.size());
  for (uint64_t s = 0; s < P; ++s)
    if (m.errq[33 * s] != 0) {
      err = "delta-y with no discarded plane must be zero";
      return false;
    }
  p += sz[1];
  m.masks.resize(nch);
  std::memcpy(m.masks.data(), p, 4 * nch);
  p += sz[2];
  for (uint64_t i = 0; i < nout; ++i) {
    m.outliers[i].pass = get32(p + 12 * i);
    m.outliers[i].chunk = get32(p + 12 * i + 4);
    m.outliers[i].local = get32(p + 12 * i + 8);
    m.outliers[i].pad = 0;
  }
  p += sz[3];
  int is = itemsize(m.dtype);
  for (uint64_t i = 0; i < nout; ++i) m.outliers[i].bits = is == 4 ? get32(p + 4 * i) : get64(p + 8 * i);
  p += sz[4];
  if (m.coding) {
    std::memcpy(m.block_words.data(), p, m.block_words.size());
    for (uint64_t i = m.block_words.size(); i < sz[5]; ++i)
      if (p[i]) {
        err = "nonzero padding";
        return false;
      }
    p += sz[5];
  }
  // masks and payload size; a coded block stores at most its raw words
  uint64_t words = 0, stored = 0;
  size_t blk = 0;
  std::vector<uint32_t> counts;
  for (const PassGeom &g : m.sched.passes) {
    chunk_counts(g, counts);
    for (int64_t c = 0; c < g.n_chunks; ++c) {
      uint32_t mk = m.masks[size_t(g.chunk_base + c)];
      int64_t cnt = int64_t(counts[size_t(c)]);
      if (cnt == 0 && mk) {
        err = "empty chunk with stored planes";
        return false;
      }
      const uint64_t W = uint64_t((cnt + 31) / 32);
      words += uint64_t(__builtin_popcount(mk)) * W;
      if (m.coding)
        for (int k = 0; k < __builtin_popcount(mk); ++k, ++blk) {
          if (m.block_words[blk] > W) {
            err = "block longer than its raw plane";
            return false;
          }
          stored += m.block_words[blk];
        }
    }
  }
  if (m.coding ? stored != pw : words != pw) {
    err = "payload size does not match the chunk masks";
    return false;
  }
  m.payload_words = words;
  // outlier keys: in range and strictly increasing
  for (uint64_t i = 0; i < nout; ++i) {
    const OutlierRec &o = m.outliers[i];
    if (o.pass >= P) {
      err = "outlier pass out of range";
      return false;
    }
    const PassGeom &g = m.sched.passes[o.pass];
    if (int64_t(o.chunk) >= g.n_chunks || int64_t(o.local) >= chunk_count(g, o.chunk)) {
      err = "outlier position out of range";
      return false;
    }
    if (i > 0) {
      const OutlierRec &a = m.outliers[i - 1];
      bool inc = a.pass < o.pass || (a.pass == o.pass && (a.chunk < o.chunk ||
                                                          (a.chunk == o.chunk && a.local < o.local)));
      if (!inc) {
        err = "outliers not sorted";
        return false;
      }
    }
  }
  // padding bytes must be zero
  for (uint64_t i = 4 * pw; i < sz[6]; ++i)
    if (p[i]) {
      err = "nonzero padding";
      return false;
    }
  *payload = reinterpret_cast<const uint32_t *>(p);
  m.serialized_bytes = n;
  return true;
}

}  // namespace ipc
