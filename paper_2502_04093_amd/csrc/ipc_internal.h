// Internal declarations of the IPComp library (host runtime + kernel launchers).
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ipcomp.h"

namespace ipc {

constexpr int KIND_ANY = 0;   // every level coordinate
constexpr int KIND_ODD = 1;   // odd level coordinates (the pass dimension)
constexpr int KIND_EVEN = 2;  // even level coordinates (dimensions after it)

constexpr int64_t MAX_CHUNK_CODES = 4096;  // codes per chunk supported by the kernels
constexpr uint32_t QMAX_F32 = 1u << 24;
constexpr uint32_t QMAX_F64 = 1u << 30;

// Geometry of one pass (Sec. 4.1: one 1-D interpolation sweep of one level).
// Arrays are padded to 3 dimensions: a D-dimensional field is treated as
// (1, .., d_0, .., d_{D-1}); padded dimensions have extent 1 everywhere.
struct PassGeom {
  int index = 0;     // position in stream order (0 = anchors)
  int level = 0;     // l (0 = anchors)
  int dim = -1;      // pass dimension in the field's own numbering (-1 anchors)
  int dim3 = -1;     // same, in padded 3-D numbering
  int64_t h = 1;     // stride in fine coordinates
  int64_t ldims[3];  // level-grid extents
  int kinds[3];
  int64_t tdims[3];  // target-lattice extents
  int64_t ct[3];     // chunk extent in target-lattice coordinates
  int64_t tiles[3];  // chunk grid
  int64_t n_chunks = 0;
  int64_t n_targets = 0;
  int64_t chunk_base = 0;   // first chunk of this pass in the stream's chunk table
  int64_t max_count = 0;    // codes in a full chunk
  int64_t wmax = 0;         // ceil(max_count / 32)
  uint64_t slot_base = 0;   // first word of this pass in slot placement
};

struct Schedule {
  int D = 0;
  int64_t dims[3] = {1, 1, 1};   // the field's own dims (first D used)
  int64_t dims3[3] = {1, 1, 1};  // padded to 3-D
  int K = 0;
  int chunk_log2[3] = {0, 0, 0};  // first D used
  std::vector<PassGeom> passes;
  int64_t n_chunks = 0;
  uint64_t slot_words = 0;
  int64_t n_points = 0;
};

bool make_schedule(const int64_t *dims, int D, const int *chunk_log2, Schedule &out,
                   std::string &err);
// codes in chunk c of pass p
int64_t chunk_count(const PassGeom &p, int64_t c);
// the same for every chunk of pass p, in chunk order (out[c], no division per
// chunk: host loops over every chunk of a stream use it)
void chunk_counts(const PassGeom &p, std::vector<uint32_t> &out);
int ceil_log2_u64(uint64_t v);

// ---------------------------------------------------------------- planner
struct PlanTables {
  int P = 0;
  std::vector<uint32_t> errq;      // [P][33]
  std::vector<int64_t> sizes;      // [P][32] bytes of plane k of pass s
  std::vector<uint8_t> progressive;
  std::vector<double> amp, tail;
  double two_eb = 0, eb = 0, unit_roundoff = 0, maxabs = 0;
  int64_t n_points = 0;
  int64_t total_bytes = 0, fixed_bytes = 0;
  std::vector<int> level;          // [P] level of every pass (0: the anchors)
};

struct PlanResult {
  std::vector<int> plan;
  uint32_t flags = 0;
  double bound = 0;
  int64_t loaded = 0;
};

// mode 0 = error bound, 1 = bitrate, optionally or-ed with
// IPC_TARGET_LEVEL_GROUPS (one discarded-plane count per level); limit may be
// null
PlanResult plan_request(const PlanTables &t, int mode, double value, const int *limit);
double plan_bound(const PlanTables &t, const std::vector<int> &plan, double M);
int64_t plan_loaded(const PlanTables &t, const std::vector<int> &plan);
// bound of the additive form of Alg. 2 after refining old_plan to plan
// (`reported` = plan_request's bound for plan)
double plan_additive_bound(const PlanTables &t, const std::vector<int> &plan,
                           const std::vector<int> &old_plan, int mode, double value, double reported);

// ---------------------------------------------------------------- format
constexpr uint32_t MAGIC = 0x4D435049u;  // "IPCM"
constexpr uint32_t VERSION = 1;
constexpr size_t HEADER_SIZE = 128;

struct OutlierRec {   // one exactly stored value
  uint32_t pass;
  uint32_t chunk;     // chunk index within the pass
  uint32_t local;     // position inside the chunk
  uint32_t pad;
  uint64_t bits;      // raw bits of the value (low 32 for float32)
};

// Host-side description of a stream (everything but the payload words).
struct StreamMeta {
  int dtype = 0;          // 0 f32, 1 f64
  int interp = 1;
  int nonprog_levels = 0;
  double eb = 0;
  double maxabs = 0;
  uint32_t qmax = 0;
  Schedule sched;
  std::vector<uint32_t> errq;       // [P][33]
  std::vector<uint32_t> masks;      // [n_chunks]
  std::vector<OutlierRec> outliers; // sorted by (pass, chunk, local); may be left on the device
  uint64_t n_outliers = 0;
  uint64_t payload_words = 0;       // packed raw payload size
  uint64_t serialized_bytes = 0;
  // entropy stage: 0 raw blocks, 1 every stored block entropy coded (then the
  // serialized form holds the stored words of every block and coded_words
  // payload words)
  int coding = 0;
  std::vector<uint8_t> block_words;  // [n_blocks], payload order
  uint64_t coded_words = 0;
};

inline uint64_t pad8(uint64_t n) { return (n + 7) & ~uint64_t(7); }
uint64_t serialized_size(const StreamMeta &m);
void packed_chunk_offsets(const StreamMeta &m, std::vector<uint64_t> &off);  // words
PlanTables plan_tables(const StreamMeta &m);
PlanTables plan_tables_from_sizes(const StreamMeta &m, const std::vector<uint64_t> &sizes);
// parse + validate serialized bytes into meta and the packed payload pointer
bool parse_serialized(const uint8_t *buf, uint64_t n, StreamMeta &m, const uint32_t **payload,
                      std::string &err);
void write_serialized_head(const StreamMeta &m, uint8_t *dst);  // everything before payload
uint64_t payload_offset(const StreamMeta &m);
// stored blocks (chunk planes) of a stream: sum of the mask popcounts
uint64_t n_blocks(const StreamMeta &m);

}  // namespace ipc
