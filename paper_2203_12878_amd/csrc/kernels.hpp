// Launch wrappers of the gfx950 kernels (defined in kernels.hip).
#pragma once
#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "drf_layout.hpp"

namespace drf {

constexpr int WG = 256;            // lanes per workgroup of the evaluator kernels
constexpr int MAXSPAN = 2048;      // phases one count / emit item may cover
constexpr int TILE = 8192;         // access events one LDS tile holds (64 KiB)
constexpr int FUSED_PACK = 8192;   // events of a fused group of several phases
constexpr int CHUNK = 8192;        // records per partition chunk (one workgroup)
constexpr int RADIX = 1024;        // largest partition digit: 10 bits (starts stride per segment)
constexpr uint32_t FILTER_BITS = 18; // singleton filter bitmap bits (direct below 2^18 cells of span, else hashed)

// Big-phase segment being partitioned by its next 8 (or fewer) index bits.
struct Seg {
    uint64_t start;       // first record in the input buffer
    uint64_t len;
    uint64_t obase;       // first record of the segment in the output buffer
    uint64_t hbase;       // histogram base: chunk-major (chunk c, digit d at hbase + c * 2^dbits + d)
    uint32_t nchunks;
    uint32_t proto;
    uint32_t phase;       // local phase
    uint32_t shift;       // digit = (index >> shift) & (2^dbits - 1)
    uint32_t dbits;
    uint32_t sbase;       // first of the segment's 2^dbits bucket starts
};

struct Chunk {
    uint32_t seg;
    uint32_t c;           // chunk number within the segment
};

// Records of one phase (or a sub-bucket of it) that fit one LDS tile, or
// a group of one index value that does not.
struct Tile {
    uint64_t start;
    uint32_t len;
    uint32_t proto;
    uint32_t phase;       // local phase
    uint32_t pad;
};

struct Group {
    uint64_t start;
    uint64_t len;
    uint32_t proto;
    uint32_t phase;
};

struct Best {             // per protocol
    unsigned long long key;   // local phase << 32 | index, ~0 when none
    unsigned long long pair;  // tid_i << 32 | tid_j
};

struct SingleAcc {        // per single-index group
    uint32_t t0, w0, tmax, t1;
};

hipError_t launch_count(const Item *items, uint32_t nitems, bool wide, const NestDesc *nests,
                        const ProtoDesc *protos, const FixedVal *fixed, const uint32_t *code,
                        unsigned long long *phase_counts, uint32_t *item_cnt, uint32_t *proto_ovf,
                        hipStream_t s);

hipError_t launch_emit(const Item *items, uint32_t nitems, bool wide, const NestDesc *nests,
                       const ProtoDesc *protos, const FixedVal *fixed, const uint32_t *code,
                       const uint32_t *item_cnt, const unsigned long long *big_base,
                       unsigned long long *cursor, uint64_t win_lo, uint64_t win_n, unsigned long long *recs,
                       unsigned long long cap, hipStream_t s, bool table = false);

// A big phase decided by its table (table path): offset of its three cell
// arrays in the table region (in 32-bit words), its cell count (a power of
// two), its protocol and local phase.
struct TablePhase {
    uint64_t off;
    uint32_t cells;
    uint32_t proto;
    uint32_t phase;
    uint32_t pad;
};
hipError_t launch_table_scan(const TablePhase *tp, uint32_t ntp, const uint32_t *tabs, uint32_t *tmin,
                             uint32_t blocks_per_table, hipStream_t s);
hipError_t launch_table_offer(const TablePhase *tp, uint32_t ntp, const uint32_t *tabs, const uint32_t *tmin,
                              Cand *cands, Best *best, hipStream_t s);

hipError_t launch_fused(const Unit *units, uint32_t nunits, uint32_t *qhead, bool wide, const NestDesc *nests,
                        const ProtoDesc *protos, const FixedVal *fixed, const uint32_t *code,
                        unsigned long long *phase_counts, unsigned long long *nrec, uint32_t *ovf_flags,
                        Cand *cands, Best *best, uint32_t grid, uint32_t tile, hipStream_t s,
                        const uint32_t *nunits_dev = nullptr);

hipError_t launch_hist(const Seg *segs, const Chunk *chunks, uint32_t nchunks, const unsigned long long *in,
                       unsigned long long *hist, hipStream_t s);

hipError_t launch_offsets(const Seg *segs, uint32_t nsegs, unsigned long long *hist, unsigned long long *starts,
                          hipStream_t s);

hipError_t launch_scatter(const Seg *segs, const Chunk *chunks, uint32_t nchunks, const unsigned long long *in,
                          const unsigned long long *offs, unsigned long long *out, unsigned long long cap,
                          hipStream_t s);

hipError_t launch_tiles(const Tile *tiles, uint32_t ntiles, const unsigned long long *recs, Cand *cands,
                        Best *best, hipStream_t s);

hipError_t launch_single(const Group *groups, uint32_t ngroups, const unsigned long long *recs,
                         SingleAcc *acc, Cand *cands, Best *best, hipStream_t s);

// (n_dev / count_dev / nunits_dev: counts read on the device, for graph
// replays; the host count then bounds the grid)
hipError_t launch_pick(const Cand *cands, uint64_t ncands, Best *best, hipStream_t s,
                       const uint32_t *n_dev = nullptr);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, uint64_t n, hipStream_t s);
// best[p] = the lesser of best[p] and best2[p] by key (with its pair)
hipError_t launch_best_min(Best *best, const Best *best2, uint32_t count, hipStream_t s);

// Up to FILL_MAX word fills in one launch (passed by value).
constexpr int FILL_MAX = 8;
struct FillList {
    uint32_t *p[FILL_MAX];
    uint64_t n[FILL_MAX];        // words
    uint32_t v[FILL_MAX];
    uint32_t b0[FILL_MAX];       // first block of each fill (set by the launcher)
    uint32_t count;
};
hipError_t launch_fill_multi(FillList L, hipStream_t s);
hipError_t launch_init_acc(SingleAcc *a, uint32_t n, hipStream_t s);

// Final per-protocol result (same layout as drf_result of the C ABI).
struct drf_result_dev {
    int32_t status;
    uint32_t racy;
    uint32_t phase, index, tid_i, tid_j;
    uint64_t num_records;
    uint32_t num_phases;
    uint32_t reserved;
};

constexpr uint32_t RESULT_FROM_DEVICE = 1;   // record total and overflow come from the fused path
// per-protocol flags set on the device
constexpr uint32_t OVF_RANGE = 1;   // an evaluated value reached 2^63 or an index 2^32
constexpr uint32_t OVF_LIMIT = 2;   // a fused group held more events than its bound

struct ResultIn {
    int32_t status;
    uint32_t num_phases;
    uint64_t num_records;
    uint32_t flags;
    uint32_t pad;
};

hipError_t launch_result(uint32_t count, const ResultIn *rin, const Best *best, const unsigned long long *nrec,
                         const uint32_t *ovf_flags, drf_result_dev *out, hipStream_t s,
                         const uint32_t *count_dev = nullptr);

// Bytes of the per-device scratch array of the allocation-free checking
// call (a file-scope device array in kernels.hip, held until the process
// ends).
constexpr uint64_t FIXED_SCRATCH_BYTES = 64ull << 20;   // DRF_FIXED_SCRATCH_BYTES of the C ABI
// Device address of that array on `device` (looked up once per device with
// the device current, then cached).
hipError_t fixed_scratch_address(int device, void **ptr);

}  // namespace drf
