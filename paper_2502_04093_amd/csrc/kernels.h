// Kernel launchers of the IPComp library (implemented in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ipc {

struct OutlierRec;

// Geometry of one pass, as the kernels see it (3-D padded).
struct PassArgs {
  int64_t dims3[3];   // fine extents
  int64_t ldims[3];   // level-grid extents
  int64_t tdims[3];   // target-lattice extents
  int64_t ct[3];      // chunk extent (target coordinates)
  int64_t tiles[3];   // chunk grid
  int32_t kinds[3];
  int32_t dim3;       // pass dimension, -1 for the anchors
  int64_t h;          // stride in fine coordinates
  int64_t n_chunks;
  int64_t chunk_base; // first chunk of the pass in the stream's tables
  uint64_t slot_base; // first payload word of the pass (slot placement)
  uint32_t wmax;      // words per plane of a full chunk
  uint32_t pass_index;
};

// Everything a compression pass reads or writes besides the field.
struct CompressOut {
  uint32_t *payload;     // slot placement: chunk c at slot_base + c*32*wmax
  uint32_t *masks;       // [n_chunks total]
  uint32_t *errq;        // [P][33], max-reduced
  unsigned long long *maxabs_bits;  // max |x^| over finite values, as double bits
  unsigned long long *n_out;        // outlier counter
  void *out_recs;        // OutlierRec array
  unsigned long long out_cap;
  uint32_t *wg_rows;     // fused levels: one row of WG_ROW words per workgroup (see below)
  unsigned long long *sizes;  // [P][32] stored bytes per plane (fused path: anchors and rows)
};

// Row of a fused-level compression workgroup, reduced after the level
// launches so that no two workgroups update one word:
//   words 0 .. 98:   delta-y maxima errq[p][b] (3 passes x 33, b = 0 unused)
//   words 99, 100:   its largest finite |x^| as double bits (low, high)
//   words 104 .. :   payload words stored per plane, [p][k] (3 x 32)
constexpr int ROW_SIZES = 104;
constexpr int WG_ROW = ROW_SIZES + 96;

// the fused level launches of one compression, for the row reduction
constexpr int MAX_LEVEL_LAUNCHES = 32;
struct LevelRows {
  int32_t n;                                  // launches
  uint32_t row_base[MAX_LEVEL_LAUNCHES];      // first row of each launch
  uint32_t n_rows[MAX_LEVEL_LAUNCHES];        // its workgroups
  uint32_t pass_index[MAX_LEVEL_LAUNCHES][3]; // its passes A, B, C
};
// One level launch of one field of a compression batch, for the batched row
// reduction: its rows and passes, and the field's outputs
struct RowsJob {
  uint32_t row_base;
  uint32_t n_rows;
  uint32_t pass_index[3];
  uint32_t pad;
  uint32_t *errq;
  unsigned long long *maxabs_bits;
  unsigned long long *sizes;
};
// the same reduction for every job of `jobs_dev` (n_jobs entries; most_rows
// is the largest n_rows among them) in one launch
hipError_t launch_rows_reduce_batch(const RowsJob *jobs_dev, uint32_t n_jobs, uint32_t most_rows,
                                    const uint32_t *rows, hipStream_t stream);
// errq[pass][b] and maxabs_bits <- max over the rows of every launch;
// sizes[pass][k] += 4 x the rows' plane words
hipError_t launch_rows_reduce(const LevelRows &lr, const uint32_t *rows, uint32_t *errq,
                              unsigned long long *maxabs_bits, unsigned long long *sizes,
                              hipStream_t stream);

struct RetrieveIn {
  const uint32_t *payload;
  const uint32_t *masks;
  const uint64_t *chunk_off;  // packed placement: word offset per chunk (null = slot)
  const uint64_t *out_gchunk; // outliers sorted by (global chunk, local)
  const uint32_t *out_local;
  const uint64_t *out_bits;
  const uint32_t *out_start;  // first outlier of each global chunk (n_chunks + 1 entries)
  uint64_t n_out;
  const uint32_t *zero;       // a device word holding 0 (read for planes not loaded)
};

// A whole level of a 3-D field in one launch (chunk shape (2, 16, 64)).
// Level-grid extents are below 2^30 (checked by the host).
struct Level3Args {
  int32_t L[3];          // level-grid extents (z, y, x)
  int32_t G[3];          // coarse-grid extents ((L - 1) >> 1) + 1
  int64_t sZ, sY;        // fine-field index strides of one level step in z and y
  int32_t sX;            // ... and in x (the level stride h)
  int32_t tiles_z, tiles_y, tiles_x;  // chunk grid (shared by the 3 passes)
  int32_t zseg;          // chunk rows per workgroup (even)
  int32_t tdims[3][3];   // target lattice of passes A, B, C
  int32_t ct[3][3];      // chunk extents in target coordinates
  int64_t chunk_base[3];
  uint64_t slot_base[3];
  uint32_t wmax[3];
  uint32_t pass_index[3];
  uint32_t row_base;     // compression: row of the launch's first workgroup in wg_rows
};

// One field of a batched level launch (compression): its level, buffers,
// outputs and quantizer constants; item0 = its first work item (column
// segment) in the launch, fields in increasing item0.
template <typename T>
struct BatchC {
  Level3Args L;
  const T *x;
  const T *gin;
  T *gout;
  CompressOut o;
  double eb;
  T two_eb, inv, qmax;
  uint32_t item0;
};
// ... and retrieval (disc: planes discarded per pass A, B, C)
template <typename T>
struct BatchR {
  Level3Args L;
  const T *gin;
  T *gout;
  RetrieveIn in;
  int32_t disc[3];
  T two_eb;
  uint32_t item0;
};
// Batched level launches over a work list: one workgroup per column segment
// of the nf fields in `batch_dev` (device array of BatchC<T> / BatchR<T>,
// n_items segments in all).
hipError_t launch_level3_compress_batch(int dtype, int interp, const void *batch_dev, int nf,
                                        uint32_t n_items, hipStream_t s);
hipError_t launch_level3_retrieve_batch(int dtype, int interp, const void *batch_dev, int nf,
                                        uint32_t n_items, hipStream_t s);

// Queue launches of a batched retrieval, replayable from one captured HIP
// graph whatever the batch holds: everything that varies from batch to batch
// sits in a device-resident table, and each level launch is a persistent grid
// whose workgroups claim work items from a device counter until its work list
// is exhausted.  The table (QueueTable, then the head jobs, then the level
// work lists, at the byte offsets the table gives) is uploaded before the
// graph runs.
constexpr int QUEUE_LEVELS = 32;
struct QueueLevel {
  uint32_t off;    // first BatchR entry of the level's work list
  uint32_t nf;     // its fields
  uint32_t items;  // its work items (0: the slot is empty)
  uint32_t pad;
};
struct QueueTable {
  uint32_t n_heads;
  uint32_t heads_off;  // byte offset of the HeadR array from the table
  uint32_t ent_off;    // byte offset of the BatchR array from the table
  uint32_t pad;
  QueueLevel lev[QUEUE_LEVELS];
};
// The job that fills a field's first coarse grid before its level launches:
// its anchors (mode 0) or, for a refinement, a strided gather of the
// resident reconstruction (mode 1).
template <typename T>
struct HeadR {
  Level3Args A;
  RetrieveIn in;
  T *g;
  const T *field;
  int64_t fd[3];
  int64_t step;
  int64_t gd[3];
  T two_eb;
  int32_t mode;
};
// Anchor job of a queued compression batch (one per field)
template <typename T>
struct HeadC {
  Level3Args A;
  const T *x;
  T *g;
  CompressOut o;
  double eb;
  T two_eb, inv, qmax;
};
// every anchor job of a compression table (grid of QUEUE_HEAD_WGS workgroups)
hipError_t launch_heads_compress(int dtype, const QueueTable *tab, hipStream_t s);
// one level slot of a compression table (its work list holds BatchC<T>)
hipError_t launch_level3_compress_queue(int dtype, int interp, const QueueTable *tab, int slot,
                                        uint32_t *claims, uint32_t grid, hipStream_t s);
// claim counters (QUEUE_LEVELS words) set to zero
hipError_t launch_queue_reset(uint32_t *claims, hipStream_t s);
// every head job of the table (grid of QUEUE_HEAD_WGS workgroups)
constexpr int QUEUE_HEAD_WGS = 256;
hipError_t launch_heads_retrieve(int dtype, const QueueTable *tab, hipStream_t s);
// level slot `slot` of the table: `grid` persistent workgroups
hipError_t launch_level3_retrieve_queue(int dtype, int interp, const QueueTable *tab, int slot,
                                        uint32_t *claims, uint32_t grid, hipStream_t s);

hipError_t launch_level3_compress(int dtype, int interp, const Level3Args &L, const void *x,
                                  const void *gin, void *gout, double eb, const CompressOut &o,
                                  hipStream_t s);
hipError_t launch_level3_retrieve(int dtype, int interp, const Level3Args &L, const void *gin,
                                  void *gout, const int disc[3], const RetrieveIn &in, double eb,
                                  hipStream_t s);
// `clear`: clear_words words zeroed before the anchors write anything (the
// call's summary block, which the anchors are the first to update)
hipError_t launch_anchor3_compress(int dtype, const Level3Args &A, const void *x, void *gout,
                                   double eb, const CompressOut &o, uint32_t *clear,
                                   uint32_t clear_words, hipStream_t s);
hipError_t launch_anchor3_retrieve(int dtype, const Level3Args &A, void *gout, const RetrieveIn &in,
                                   double eb, hipStream_t s);
// g[c] = field[step * c] over the coarse grid gd
hipError_t launch_gather_coarse(int dtype, const void *field, const int64_t fd[3], int64_t step,
                                void *g, const int64_t gd[3], hipStream_t s);

hipError_t launch_compress_pass(int dtype, int interp, const PassArgs &pa, const void *x, void *xh,
                                int write_back, double eb, const CompressOut &o,
                                hipStream_t stream);
// discard_old >= 0: the additive form of Alg. 2 (field is the difference
// field; codes are the differences of the truncations at discard and
// discard_old planes; outliers add zero)
hipError_t launch_retrieve_pass(int dtype, int interp, const PassArgs &pa, void *field,
                                int discard, const RetrieveIn &in, double eb, hipStream_t stream,
                                int discard_old = -1);
// Batched passes (one step of several fields in one launch): the arguments
// of one field's pass and the first work item of its chunks.
template <typename T>
struct PassBatchC {
  PassArgs a;
  const T *x;
  T *xh;
  CompressOut o;
  double eb;
  T two_eb, inv, qmax;
  int32_t write_back;
  uint32_t item0;
};
template <typename T>
struct PassBatchR {
  PassArgs a;
  T *f;
  RetrieveIn in;
  T two_eb;
  int32_t discard;
  uint32_t item0;
};
// one workgroup per chunk of the nf fields' passes in `batch_dev` (device
// array of PassBatchC<T> / PassBatchR<T>, n_items chunks in all)
hipError_t launch_compress_pass_batch(int dtype, int interp, const void *batch_dev, int nf,
                                      uint32_t n_items, hipStream_t stream);
hipError_t launch_retrieve_pass_batch(int dtype, int interp, const void *batch_dev, int nf,
                                      uint32_t n_items, hipStream_t stream);
// field[i] += delta[i] wherever delta[i] != 0
// *bad += points where |x - xt| > eb (float64) and the bits differ
hipError_t launch_verify_bound(int dtype, const void *x, const void *xt, uint64_t n, double eb,
                               unsigned long long *bad, hipStream_t stream);
hipError_t launch_add_delta(int dtype, void *field, const void *delta, uint64_t n,
                            hipStream_t stream);
// Outlier index built on the device from the compression kernels' records
// (any order, count *n_out, at most cap used): gchunk/local/bits sorted by
// (global chunk, local) and start[c] = first record of chunk c (n_chunks + 1
// entries).  cnt: n_chunks + 1 words of scratch; bsum: (n_chunks + 1024) / 1024.
hipError_t launch_outlier_index(const OutlierRec *recs, const unsigned long long *n_out,
                                uint64_t cap, const PassArgs *args, uint64_t n_chunks,
                                uint32_t *start, uint32_t *cnt, uint32_t *bsum, uint64_t *gchunk,
                                uint32_t *local, uint64_t *bits, hipStream_t stream);
// The same index for a record count n known on the host (at most cap
// records): up to OUT_SMALL records are sorted by one workgroup and start[]
// comes from a binary search per chunk (two launches), more take the path
// above.  cnt and bsum are used by the larger path only.
constexpr uint32_t OUT_SMALL = 2048;
hipError_t launch_outlier_index_n(const OutlierRec *recs, uint64_t n, const unsigned long long *n_out,
                                  const PassArgs *args, uint64_t n_chunks, uint32_t *start,
                                  uint32_t *cnt, uint32_t *bsum, uint64_t *gchunk, uint32_t *local,
                                  uint64_t *bits, hipStream_t stream);
// out_start[c] = index of the first outlier whose global chunk is >= c, for
// c = 0 .. n_chunks (outliers sorted by global chunk)
hipError_t launch_out_start(const uint64_t *out_gchunk, uint64_t n_out, uint64_t n_chunks,
                            uint32_t *out_start, hipStream_t stream);
// sizes[p][k] for every pass at once (args_dev: the passes' PassArgs on the device)
hipError_t launch_all_sizes(const PassArgs *args_dev, int n_passes, int64_t max_chunks,
                            const uint32_t *masks, unsigned long long *sizes, hipStream_t stream);
// sizes[k] (bytes of plane k summed over the pass's chunks), one pass
hipError_t launch_pass_sizes(const PassArgs &pa, const uint32_t *masks,
                             unsigned long long *sizes, hipStream_t stream);
// copy the stored planes of one pass from slot placement to packed placement
hipError_t launch_pack_payload(const PassArgs &pa, const uint32_t *masks,
                               const uint64_t *packed_off, const uint32_t *slot_payload,
                               uint32_t *packed, hipStream_t stream);

// ---- entropy stage (entropy.hip): one stored plane block of one chunk
struct EcBlock {
  uint64_t raw_off;    // first word of the raw plane (W = ceil(count / 32) words)
  uint64_t coded_off;  // first word of its stored form in the coded payload
  uint32_t count;      // codes of the chunk (bits of the block)
  uint32_t pad;
};
// codes every block of raw into its scratch slot (scratch + raw_off, W words:
// the code when shorter than W words, else the raw plane) and its stored word
// count into words[i]
hipError_t launch_ec_encode(const EcBlock *blk, uint64_t n, const uint32_t *raw, uint32_t *scratch,
                            uint8_t *words, hipStream_t s);
// the blocks of n_chunks chunks: chunk c holds blocks cblk[c] .. cblk[c+1]
// (its stored planes from 31 down), raw planes from word craw[c], ccount[c]
// codes each
hipError_t launch_ec_blocks(const uint32_t *cblk, const uint64_t *craw, const uint32_t *ccount,
                            uint64_t n_chunks, EcBlock *blk, hipStream_t s);
// coded_off of every block: exclusive prefix sum of words[] (tot: one u64 per
// 1024 blocks of scratch)
hipError_t launch_ec_offsets(const uint8_t *words, uint64_t n, EcBlock *blk, uint64_t *tot,
                             hipStream_t s);
// words[i] stored words of every block from its scratch slot to coded_off
hipError_t launch_ec_gather(const EcBlock *blk, uint64_t n, const uint8_t *words,
                            const uint32_t *scratch, uint32_t *coded, hipStream_t s);
// the raw plane of every block back from its stored form
hipError_t launch_ec_decode(const EcBlock *blk, uint64_t n, const uint8_t *words,
                            const uint32_t *coded, uint32_t *raw, hipStream_t s);

}  // namespace ipc
