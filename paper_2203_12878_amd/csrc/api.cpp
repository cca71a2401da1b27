// C ABI of libdrf: contexts, planning and the checking pipeline.
//
// Pipeline of one call (plain = one protocol, batch = many, same code):
//   plan (host)          decode, static checks, leaf nests, leaf code
//   count (GPU)          every access event counted per phase; dynamic
//                        range overflow flagged per protocol
//   -- one stream sync: per-phase counts come back to the host --
//   fused (GPU)          phases with at most TILE events: evaluated again
//                        straight into LDS, sorted, scanned (no HBM records)
//   big phases (GPU)     in waves that fit the scratch budget: emit records
//                        to HBM, MSD radix partition by 8 index bits per
//                        level until every bucket fits one LDS tile, then
//                        LDS sort + segmented scan per tile; buckets of a
//                        single index value reduce directly
//   results (GPU)        witness (least phase, index, pair), counts, status
// Protocols whose planner bound proves every phase fits one LDS tile skip
// the count pass and the host round trip: their fused units count, sort
// and scan in one kernel.
//
// A prepared batch runs this once while recording every device operation,
// then captures the recorded sequence into one hipGraph that replays the
// whole device work (fills are kernels, never memset nodes).
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <functional>
#include <thread>
#include <tuple>
#include <initializer_list>
#include <memory>
#include <new>
#include <vector>

#include "../../include/drf.h"
#include "host.hpp"
#include "kernels.hpp"

using namespace drf;

static_assert(FIXED_SCRATCH_BYTES == DRF_FIXED_SCRATCH_BYTES, "fixed scratch size of the C ABI");

enum KClass { K_COUNT, K_FUSED, K_EMIT, K_HIST, K_SCAN, K_SCATTER, K_TILE, K_SINGLE, K_TABLE, K_OTHER, K_NCLASS };
static const char *KNAMES[K_NCLASS] = {"count", "fused", "emit", "hist", "scan", "scatter", "tile", "single", "table",
                                       "other"};

struct drf_ctx {
    int device = 0;
    uint64_t limit = 0;
    void *poolA = nullptr;
    size_t sizeA = 0;
    void *poolB = nullptr;
    size_t sizeB = 0;
    hipEvent_t done = nullptr;
    hipEvent_t counted = nullptr;
    hipEvent_t parted = nullptr;        // a partition level's bucket starts are on the host
    // the counted protocols' fused units beside the HBM path: their
    // stream, its start and its end
    hipStream_t side = nullptr;
    hipEvent_t side_go = nullptr, side_done = nullptr;
    void *h_starts = nullptr;           // pinned host copy of those starts
    size_t h_starts_cap = 0;
    // pinned host staging of uploads and read-backs: blocks kept for the
    // context's life, handed out in order during a call and reused once the
    // call's stream has drained
    std::vector<std::pair<char *, size_t>> pin_blocks;
    size_t pin_bi = 0, pin_off = 0;
    void *h_counts = nullptr;           // pinned read-back of per-phase counts and overflow flags
    size_t h_counts_cap = 0;
    void *fixed = nullptr;              // the device's fixed scratch array (allocation-free calls)
    bool done_valid = false;
    uint32_t cus = 256;
    drf_tuning tune = {(uint32_t)drf::TILE, 10, 1u << 15, 1u << 16, 0};
    // per-kernel-class timing
    bool prof = false;
    std::vector<hipEvent_t> ev_free;
    struct Pending { int cls; hipEvent_t a, b; uint64_t records, bytes; };
    std::vector<Pending> pending;
    drf_kernel_stat stats[K_NCLASS] = {};
};

namespace {

// Host stage timings on stderr when the environment sets DRF_TRACE (a
// development aid; off by default).
struct Trace {
    using clock = std::chrono::steady_clock;
    bool on;
    clock::time_point t0, last;
    Trace() : on(getenv("DRF_TRACE") != nullptr) { t0 = last = clock::now(); }
    void mark(const char *what, unsigned long long a = 0) {
        if (!on) return;
        const clock::time_point n = clock::now();
        fprintf(stderr, "[drf] %-22s +%9.3f ms  (%9.3f)  %llu\n", what,
                std::chrono::duration<double, std::milli>(n - last).count(),
                std::chrono::duration<double, std::milli>(n - t0).count(), a);
        last = n;
    }
};


constexpr uint64_t CAND_CAP = 1ull << 20;      // candidates per launch
constexpr bool FUSED_BESIDE = true;            // counted fused units beside the HBM path
constexpr uint64_t BESIDE_MIN = 1ull << 24;    // ... when both sides hold at least this many events
constexpr uint64_t ALIGN = 256;

struct Bump {
    char *base = nullptr;
    size_t cap = 0, used = 0;
    size_t reserve(size_t bytes) {
        size_t off = (used + ALIGN - 1) & ~(ALIGN - 1);
        used = off + bytes;
        return off;
    }
};

template <class T>
T *at(void *base, size_t off) { return (T *)((char *)base + off); }

struct Fail {
    int code;
};

void hipck(hipError_t e) {
    if (e != hipSuccess) throw Fail{DRF_E_HIP};
}

hipEvent_t take_event(drf_ctx *c) {
    if (c->ev_free.empty()) {
        hipEvent_t e;
        hipck(hipEventCreate(&e));
        return e;
    }
    hipEvent_t e = c->ev_free.back();
    c->ev_free.pop_back();
    return e;
}

// Brackets one launch with events when profiling is on.
struct Prof {
    drf_ctx *c;
    hipStream_t st;
    int cls;
    hipEvent_t a = nullptr;
    uint64_t records, bytes;
    Prof(drf_ctx *ctx, hipStream_t s, int k, uint64_t rec, uint64_t b) : c(ctx), st(s), cls(k), records(rec), bytes(b) {
        if (c->prof) {
            a = take_event(c);
            hipck(hipEventRecord(a, st));
        }
    }
    ~Prof() noexcept(false) {
        if (!c->prof || !a) return;
        hipEvent_t b = take_event(c);
        hipck(hipEventRecord(b, st));
        c->pending.push_back({cls, a, b, records, bytes});
    }
};

// After the stream is idle: fold pending event pairs into the totals.
void prof_collect(drf_ctx *c) {
    for (auto &p : c->pending) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            drf_kernel_stat &s = c->stats[p.cls];
            s.launches++;
            s.ms += ms;
            s.records += p.records;
            s.bytes += p.bytes;
        }
        c->ev_free.push_back(p.a);
        c->ev_free.push_back(p.b);
    }
    c->pending.clear();
}

// Grows one of the context's two pools to at least `need` bytes, keeping
// both pools together within the context's limit (DRF_E_NOMEM beyond it).
// The old block is released and the new one taken in stream order on the
// call's stream (which already waits for the context's previous call), so
// no other stream or context is stalled.  Contents are not preserved.
void grow(drf_ctx *c, void *&p, size_t &size, size_t need, hipStream_t st) {
    if (need <= size) return;
    const uint64_t other = c->sizeA + c->sizeB - size;
    size_t want = (need + (64ull << 20) - 1) & ~((64ull << 20) - 1);
    if (other + want > c->limit) want = (need + ALIGN - 1) & ~(ALIGN - 1);
    if (other + want > c->limit) throw Fail{DRF_E_NOMEM};
    if (p) {
        hipck(hipFreeAsync(p, st));
        p = nullptr;
        size = 0;
    }
    if (hipMallocAsync(&p, want, st) != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        throw Fail{DRF_E_NOMEM};
    }
    size = want;
}

// Host copies of uploaded arrays (and read-back buffers) in pinned memory,
// so that copies never wait for the stream; they stay untouched until the
// call's next stream sync.
struct Keep {
    drf_ctx *ctx = nullptr;
    // allocation-free calls stage on the host heap instead: blocks owned by
    // the call, never reused within it, freed after its final stream sync
    bool heap = false;
    std::vector<std::unique_ptr<char[]>> heap_blocks;
    void *take(size_t bytes) {
        bytes = (bytes + 255) & ~(size_t)255;
        if (heap) {
            heap_blocks.emplace_back(new char[bytes]);
            return heap_blocks.back().get();
        }
        auto &B = ctx->pin_blocks;
        while (ctx->pin_bi < B.size() && ctx->pin_off + bytes > B[ctx->pin_bi].second) {
            ctx->pin_bi++;
            ctx->pin_off = 0;
        }
        if (ctx->pin_bi == B.size()) {
            const size_t want = std::max<size_t>(bytes, B.empty() ? (8u << 20) : 2 * B.back().second);
            void *p = nullptr;
            if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                throw Fail{DRF_E_NOMEM};
            }
            B.push_back({(char *)p, want});
            ctx->pin_off = 0;
        }
        void *r = B[ctx->pin_bi].first + ctx->pin_off;
        ctx->pin_off += bytes;
        return r;
    }
    template <class T>
    const void *hold(const std::vector<T> &v) {
        void *p = take(v.size() * sizeof(T));
        memcpy(p, v.data(), v.size() * sizeof(T));
        return p;
    }
    void clear() {
        if (heap) return;
        ctx->pin_bi = 0;
        ctx->pin_off = 0;
    }
};

template <class T>
void upload(Keep &keep, void *dst, const std::vector<T> &v, hipStream_t s) {
    if (v.empty()) return;
    hipck(hipMemcpyAsync(dst, keep.hold(v), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

uint64_t nest_phase(const NestDesc &nd, uint64_t f) {
    uint64_t ph = nd.phase_base, rem = f;
    for (int l = (int)nd.nloops - 1; l >= 0; l--) {
        ph += (rem % nd.trip[l]) * nd.stride[l];
        rem /= nd.trip[l];
    }
    return ph;
}

struct BigPhase {
    uint64_t k;        // global phase id
    uint64_t count;
    uint32_t proto;
    uint32_t local;
};

// Device operations of a recorded call, and the device memory they use.
struct Recorder {
    std::vector<std::function<hipError_t(hipStream_t)>> ops;
    std::vector<void *> owned;     // device allocations kept for the replays
    char *arena = nullptr;
    size_t arena_cap = 0, arena_used = 0;
    uint64_t limit = ~0ull, total = 0;   // bytes the recording may own, and owns

    void *alloc(size_t bytes) {
        size_t off = (arena_used + ALIGN - 1) & ~(ALIGN - 1);
        if (!arena || off + bytes > arena_cap) {
            size_t cap = std::max<size_t>(bytes + ALIGN, 64ull << 20);
            if (total + cap > limit) cap = bytes + ALIGN;
            if (total + cap > limit) throw Fail{DRF_E_NOMEM};
            void *p = nullptr;
            if (hipMalloc(&p, cap) != hipSuccess) {
                (void)hipGetLastError();
                throw Fail{DRF_E_NOMEM};
            }
            owned.push_back(p);
            total += cap;
            arena = (char *)p;
            arena_cap = cap;
            off = 0;
        }
        arena_used = off + bytes;
        return arena + off;
    }
};

// Phases of at most this many events are decided in the fused kernel (in
// LDS, no HBM records); larger ones go through HBM and the tile kernel.
uint32_t small_events(const drf_ctx *ctx) { return ctx->tune.tile_events; }

struct Call {
    drf_ctx *ctx;
    hipStream_t st;
    uint32_t count;
    Recorder *rec = nullptr;
    bool noalloc = false;              // pools come from the fixed scratch array
    void *A = nullptr, *B = nullptr;   // pool A / pool B of this call
    Trace tr;

    // run a device operation on the call's stream (and record it)
    template <class F>
    void dev(F f) {
        hipck(f(st));
        if (rec) rec->ops.emplace_back(f);
    }
    void fill32(void *p, uint32_t word, size_t bytes) {
        uint32_t *q = (uint32_t *)p;
        const uint64_t n = bytes / 4;
        dev([=](hipStream_t s) { return launch_fill_u32(q, word, n, s); });
    }
    // several fills (pointer, word, bytes) as one launch
    void fill_many(std::initializer_list<std::tuple<void *, uint32_t, size_t>> fs) {
        FillList L{};
        for (const auto &f : fs) {
            if (L.count == (uint32_t)FILL_MAX) {
                const FillList M = L;
                dev([=](hipStream_t s) { return launch_fill_multi(M, s); });
                L = FillList{};
            }
            L.p[L.count] = (uint32_t *)std::get<0>(f);
            L.v[L.count] = std::get<1>(f);
            L.n[L.count] = std::get<2>(f) / 4;
            L.count++;
        }
        if (L.count) dev([=](hipStream_t s) { return launch_fill_multi(L, s); });
    }
    // upload host data; a recorded call gives every upload its own memory
    template <class T>
    T *put(void *region, const std::vector<T> &v) {
        if (v.empty()) return (T *)region;
        void *dst = rec ? rec->alloc(v.size() * sizeof(T)) : region;
        upload(keep, dst, v, st);
        return (T *)dst;
    }
    // upload n elements that fill(dst) writes straight into the staging
    // memory (no intermediate vector)
    template <class T, class F>
    T *put_fill(void *region, size_t n, F fill) {
        if (n == 0) return (T *)region;
        void *dst = rec ? rec->alloc(n * sizeof(T)) : region;
        void *h = keep.take(n * sizeof(T));
        fill((T *)h);
        hipck(hipMemcpyAsync(dst, h, n * sizeof(T), hipMemcpyHostToDevice, st));
        return (T *)dst;
    }
    void sync() {
        hipck(hipStreamSynchronize(st));
        keep.clear();
    }

    std::vector<Plan> plans;
    std::vector<int32_t> status;
    std::vector<uint64_t> poff;
    std::vector<ProtoDesc> protos;
    std::vector<NestDesc> nests;
    std::vector<uint32_t> nest_tids;   // per nest: tids that may access memory
    const Item *ditems[2] = {nullptr, nullptr};   // the items as uploaded (pool A or a recording)
    std::vector<FixedVal> fixed;
    std::vector<uint32_t> code;
    std::vector<Item> items[2];        // narrow, wide
    std::vector<char> stat;            // phases proven to fit one LDS tile: no count pass
    std::vector<Unit> sunits[2];       // fused units of those protocols, narrow / wide
    uint64_t item_cnt_words = 0;
    uint64_t total_phases = 0;
    Keep keep;

    // pool A offsets
    bool beside = false;       // pool A holds the counted units' own witness candidates:
    size_t o_best2, o_cand2;   // ... when they run beside the HBM path
    size_t o_protos, o_nests, o_fixed, o_code, o_items[2], o_itemcnt, o_ovf, o_nrec, o_qhead, o_best, o_cand, o_units,
        o_sunits[2], o_rin, o_res;
    size_t needA = 0;

    void plan_all(const uint32_t *codep, const uint64_t *code_off, const uint32_t *nthreads) {
        plans.resize(count);
        auto work = [&](uint32_t lo, uint32_t hi) {
            for (uint32_t i = lo; i < hi; i++) {
                const uint64_t len = code_off[i + 1] - code_off[i];
                if (code_off[i + 1] < code_off[i] || len > 0xFFFFFFFFull) { plans[i].status = DRF_E_BYTECODE; continue; }
                plan_protocol(codep + code_off[i], (uint32_t)len, nthreads[i], plans[i]);
            }
        };
        uint32_t nt = std::min<uint32_t>(std::max(1u, std::thread::hardware_concurrency()), 16);
        if (count < 64) nt = 1;
        std::vector<std::thread> th;
        for (uint32_t t = 0; t < nt; t++) th.emplace_back(work, count * t / nt, count * (t + 1) / nt);
        for (auto &t : th) t.join();
    }

    // Events per fused unit: the tuned size, made smaller when the work is
    // too little to give every persistent workgroup a few units.
    uint64_t unit_size(uint64_t events) const {
        const uint64_t slots = 4ull * 2 * ctx->cus;
        uint64_t u = std::max<uint64_t>(events / slots, small_events(ctx));
        return std::min<uint64_t>(u, std::max<uint64_t>(ctx->tune.unit_events, small_events(ctx)));
    }

    void build_blob() {
        uint64_t static_events = 0;
        for (uint32_t i = 0; i < count; i++) {
            const Plan &p = plans[i];
            if (!p.status && p.max_phase_records <= (uint64_t)small_events(ctx))
                static_events += (uint64_t)std::min<uint64_t>(p.num_phases * std::max<uint64_t>(1, p.max_phase_records),
                                                              1ull << 50);
        }
        const uint64_t static_unit = unit_size(static_events);
        status.assign(count, 0);
        stat.assign(count, 0);
        poff.assign(count, 0);
        protos.assign(count, ProtoDesc{});
        for (uint32_t i = 0; i < count; i++) {
            const Plan &p = plans[i];
            status[i] = p.status;
            poff[i] = total_phases;
            ProtoDesc &pd = protos[i];
            pd.n = p.n;
            pd.wide = p.wide ? 1 : 0;
            pd.nest0 = (uint32_t)nests.size();
            pd.nnests = 0;
            pd.phase_off = total_phases;
            pd.nphases = 0;
            {
                uint32_t tb = 0;
                while (tb < 31 && p.n > 1 && ((uint64_t)(p.n - 1) >> tb) != 0) tb++;
                pd.tb = tb;
                pd.ib = p.index_bits;
                pd.pack = (!p.wide && p.index_bits + tb + 1 <= 48) ? 1 : 0;
                pd.phase_bound = (uint32_t)std::min<uint64_t>(p.max_phase_records, 0xFFFFFFFFu);
            }
            if (p.status) continue;
            pd.nphases = p.num_phases;
            total_phases += p.num_phases;
            std::vector<uint32_t> leaf_off(p.leaf_code.size());
            for (size_t j = 0; j < p.leaf_code.size(); j++) {
                leaf_off[j] = (uint32_t)code.size();
                code.insert(code.end(), p.leaf_code[j].begin(), p.leaf_code[j].end());
            }
            for (size_t j = 0; j < p.nests.size(); j++) {
                const Nest &ne = p.nests[j];
                NestDesc nd{};
                nd.proto = i;
                nd.code_off = leaf_off[p.nest_leaf_code[j]];
                nd.nloops = (uint32_t)ne.loops.size();
                nd.nfixed = (uint32_t)ne.fixed.size();
                nd.fixed_off = (uint32_t)fixed.size();
                nd.rec_bound = ne.rec_bound;
                {
                    const int g = p.leaf_guard[p.nest_leaf_code[j]];
                    nd.guard_off = g < 0 ? NONE32 : leaf_off[p.nest_leaf_code[j]] + (uint32_t)g;
                    const int cl = p.leaf_cal[p.nest_leaf_code[j]];
                    nd.cal_off = cl < 0 ? NONE32 : leaf_off[p.nest_leaf_code[j]] + (uint32_t)cl;
                }
                nd.iters = ne.iters;
                nd.phase_base = pd.phase_off + ne.phase_base;
                nd.phase_last = pd.phase_off + ne.phase_last;
                for (size_t l = 0; l < ne.loops.size(); l++) {
                    nd.slot[l] = ne.loops[l].slot;
                    nd.lo[l] = ne.loops[l].lo;
                    nd.trip[l] = ne.loops[l].trip;
                    nd.stride[l] = ne.loops[l].stride;
                }
                for (auto &f : ne.fixed) fixed.push_back(FixedVal{f.first, 0, f.second});
                nests.push_back(nd);
                nest_tids.push_back(ne.tid_bound);
                pd.nnests++;
            }
            stat[i] = p.max_phase_records <= (uint64_t)small_events(ctx);
            if (stat[i]) {
                if (pd.nnests == 0) continue;
                // units of about unit_events (by the static bound), one phase at least
                const uint64_t per = std::max<uint64_t>(1, p.max_phase_records);
                const uint64_t step = std::max<uint64_t>(1, static_unit / per);
                for (uint64_t k = 0; k < pd.nphases; k += step)
                    sunits[pd.wide].push_back(Unit{i, UNIT_STATIC, pd.phase_off + k,
                                                   pd.phase_off + std::min<uint64_t>(pd.nphases, k + step)});
            } else {
                for (uint32_t j = pd.nest0; j < pd.nest0 + pd.nnests; j++) make_items(j, p.n, p.wide);
            }
        }
    }

    void make_items(uint32_t ni, uint32_t n, bool wide) {
        const NestDesc &nd = nests[ni];
        n = std::min(n, nest_tids[ni]);   // blocks past the guard's bound never access memory
        if (n == 0) return;
        const uint64_t lanes = std::min<uint64_t>(n, WG);
        const uint64_t per_iter = lanes * std::max<uint64_t>(1, nd.rec_bound);
        const uint64_t F = std::max<uint64_t>(1, ctx->tune.item_events / per_iter);
        const uint32_t nb = (n + WG - 1) / WG;
        for (uint64_t f0 = 0; f0 < nd.iters;) {
            uint64_t f1 = std::min(nd.iters, f0 + F);
            const uint64_t k0 = nest_phase(nd, f0);
            while (f1 - f0 > 1 && nest_phase(nd, f1 - 1) - k0 + 1 > (uint64_t)MAXSPAN) f1 = f0 + (f1 - f0) / 2;
            const uint32_t span = (uint32_t)(nest_phase(nd, f1 - 1) - k0 + 1);
            // several tid blocks per item when one block's share of the
            // iterations holds few events (fewer items to build and launch;
            // such an item may hold twice the events of a one-block item)
            const uint64_t blk_events = per_iter * (f1 - f0);
            const uint32_t per_item = (uint32_t)std::max<uint64_t>(
                1, std::min<uint64_t>(2 * (uint64_t)ctx->tune.item_events / std::max<uint64_t>(1, blk_events), 64));
            for (uint32_t b = 0; b < nb; b += per_item) {
                Item it{};
                it.nest = ni;
                it.tid0 = b * WG;
                it.nblk = std::min<uint32_t>(per_item, nb - b);
                it.f0 = f0;
                it.f1 = f1;
                it.k_lo = k0;
                it.span = span;
                it.cnt_off = item_cnt_words;
                item_cnt_words += span;
                items[wide ? 1 : 0].push_back(it);
            }
            f0 = f1;
        }
    }

    // (beside: room for the counted units' own witness candidates, which
    // ordinary calls run on the context's second stream)
    void layout_a(uint64_t nunits_max, bool beside) {
        Bump b;
        o_protos = b.reserve(protos.size() * sizeof(ProtoDesc));
        o_nests = b.reserve(nests.size() * sizeof(NestDesc));
        o_fixed = b.reserve(fixed.size() * sizeof(FixedVal));
        o_code = b.reserve(code.size() * sizeof(uint32_t));
        o_items[0] = b.reserve(items[0].size() * sizeof(Item));
        o_items[1] = b.reserve(items[1].size() * sizeof(Item));
        o_itemcnt = b.reserve(item_cnt_words * sizeof(uint32_t));
        o_ovf = b.reserve(count * sizeof(uint32_t));
        o_nrec = b.reserve(count * sizeof(uint64_t));
        o_qhead = b.reserve(64 * sizeof(uint32_t));
        o_best = b.reserve(count * sizeof(Best));
        o_cand = b.reserve(CAND_CAP * sizeof(Cand));
        o_units = b.reserve(std::min<uint64_t>(nunits_max, CAND_CAP) * sizeof(Unit));
        o_best2 = o_cand2 = 0;
        this->beside = beside;
        if (beside) {
            o_best2 = b.reserve(count * sizeof(Best));
            o_cand2 = b.reserve(std::min<uint64_t>(nunits_max, CAND_CAP) * sizeof(Cand));
        }
        o_sunits[0] = b.reserve(sunits[0].size() * sizeof(Unit));
        o_sunits[1] = b.reserve(sunits[1].size() * sizeof(Unit));
        o_rin = b.reserve(count * sizeof(ResultIn));
        o_res = b.used;
        needA = b.used + ALIGN;
    }
};

// Layout of pool B for one wave of `recs` big-phase records over a window
// of win_n phases.
struct WaveLayout {
    size_t o_bb, o_cur, o_ra, o_rb, o_hist, o_starts, o_segs, o_chunks, o_tiles, o_groups, o_acc, o_wi0, o_wi1;
    size_t bytes;
    uint64_t hist_max, nsegs_max, chunks_max, tiles_cap, groups_cap;
    uint32_t sstride;
};

// A segment of any level holds more than `small` records (level 0: a big
// phase; deeper: a bucket above the tile size, which is at least `small`).
WaveLayout wave_layout(uint64_t recs, uint64_t win_n, uint64_t nbig, uint64_t nitems0, uint64_t nitems1,
                       uint32_t tile, uint32_t small, uint32_t dbits) {
    WaveLayout L{};
    (void)tile;
    L.nsegs_max = recs / ((uint64_t)small + 1) + 1;
    L.chunks_max = recs / CHUNK + L.nsegs_max + 1;
    L.hist_max = L.chunks_max << dbits;
    const uint64_t tiles_max = std::min<uint64_t>(L.nsegs_max << dbits, recs) + 1;
    L.sstride = 1u << dbits;
    Bump b;
    L.o_bb = b.reserve(win_n * 8);
    L.o_cur = b.reserve(win_n * 8);
    L.o_ra = b.reserve(recs * 8);
    L.o_rb = b.reserve(recs * 8);
    L.o_hist = b.reserve(L.hist_max * 8);
    L.o_starts = b.reserve(L.nsegs_max * L.sstride * 8);
    L.o_segs = b.reserve(L.nsegs_max * sizeof(Seg));
    L.o_chunks = b.reserve(L.chunks_max * sizeof(Chunk));
    L.tiles_cap = std::min<uint64_t>(tiles_max, CAND_CAP);
    L.groups_cap = std::min<uint64_t>(L.nsegs_max + nbig, CAND_CAP);
    L.o_tiles = b.reserve(L.tiles_cap * sizeof(Tile));
    L.o_groups = b.reserve(L.groups_cap * sizeof(Group));
    L.o_acc = b.reserve(std::min<uint64_t>(L.nsegs_max + nbig, CAND_CAP) * sizeof(SingleAcc));
    L.o_wi0 = b.reserve(nitems0 * sizeof(Item));
    L.o_wi1 = b.reserve(nitems1 * sizeof(Item));
    L.bytes = b.used + ALIGN;
    return L;
}

// Index bits of one partition level for a segment of len records: buckets
// of about 512 records on average (skewed index distributions then still
// fit tiles in one level), at least 4 bits, at most the tuned maximum.
uint32_t digit_bits_for(uint64_t len, uint32_t max_bits) {
    uint32_t b = 4;
    while (b < max_bits && (len >> b) > 1024) b++;
    return b;
}

struct Wave {
    size_t bi, be;
    uint64_t recs;
    bool all = false;              // the wave needs every item: use the copy in pool A
    std::vector<Item> witems[2];
};

// One wave of big phases [bi, be) of the global big-phase list: emit, then
// partition levels until every bucket fits an LDS tile (or holds a single
// index value).  Pool B has been sized for the largest wave.
void run_wave(Call &C, const std::vector<BigPhase> &big, const Wave &W, Best *best, Cand *cand) {
    drf_ctx *ctx = C.ctx;
    hipStream_t st = C.st;
    void *A = C.A;
    void *B = C.B;
    const size_t bi = W.bi, be = W.be;
    const uint64_t recs = W.recs;
    const uint64_t win_lo = big[bi].k;
    const uint64_t win_n = big[be - 1].k - win_lo + 1;
    const uint32_t tile = ctx->tune.tile_events;
    const uint32_t dbits = ctx->tune.digit_bits;
    const WaveLayout L =
        wave_layout(recs, win_n, be - bi, W.witems[0].size(), W.witems[1].size(), tile, small_events(ctx), dbits);
    const uint32_t sstride = L.sstride;

    // ---- emit the wave's records, phase-major
    std::vector<unsigned long long> bb(win_n, ~0ull);
    std::vector<uint64_t> pos(be - bi);
    uint64_t p = 0;
    for (size_t j = bi; j < be; j++) {
        bb[big[j].k - win_lo] = p;
        pos[j - bi] = p;
        p += big[j].count;
    }
    const unsigned long long *dbb = C.put(at<void>(B, L.o_bb), bb);
    unsigned long long *dcur = at<unsigned long long>(B, L.o_cur);
    C.fill32(dcur, 0, win_n * 8);
    const Item *dwi[2];
    size_t nwi[2];
    for (int w = 0; w < 2; w++) {
        if (W.all) {
            dwi[w] = C.ditems[w];
            nwi[w] = C.items[w].size();
        } else {
            dwi[w] = C.put(at<void>(B, w ? L.o_wi1 : L.o_wi0), W.witems[w]);
            nwi[w] = W.witems[w].size();
        }
    }
    unsigned long long *in = at<unsigned long long>(B, L.o_ra), *out = at<unsigned long long>(B, L.o_rb);
    const NestDesc *dnests = at<NestDesc>(A, C.o_nests);
    const ProtoDesc *dprotos = at<ProtoDesc>(A, C.o_protos);
    const FixedVal *dfixed = at<FixedVal>(A, C.o_fixed);
    const uint32_t *dcode = at<uint32_t>(A, C.o_code);
    const uint32_t *ditemcnt = at<uint32_t>(A, C.o_itemcnt);
    for (int w = 0; w < 2; w++) {
        const Item *it = dwi[w];
        for (uint64_t s0 = 0; s0 < nwi[w]; s0 += 1u << 30) {
            const uint32_t n = (uint32_t)std::min<uint64_t>(nwi[w] - s0, 1u << 30);
            const bool wide = w == 1;
            unsigned long long *recbuf = in;
            Prof pr(ctx, st, K_EMIT, w == 0 ? recs : 0, w == 0 ? recs * 8 : 0);
            C.dev([=](hipStream_t s) {
                return launch_emit(it + s0, n, wide, dnests, dprotos, dfixed, dcode, ditemcnt, dbb, dcur, win_lo,
                                   win_n, recbuf, recs, s);
            });
        }
    }

    C.tr.mark("wave emit launched", recs);
    // (more groups than candidate slots: launches of at most CAND_CAP
    // groups, each followed by its pick, in stream order without host waits)
    auto run_groups = [&](const std::vector<Group> &groups, const unsigned long long *recbuf) {
        for (uint64_t g0 = 0; g0 < groups.size(); g0 += CAND_CAP) {
            const uint64_t n = std::min<uint64_t>(groups.size() - g0, CAND_CAP);
            std::vector<Group> part(groups.begin() + g0, groups.begin() + g0 + n);
            if (n > L.groups_cap) throw Fail{DRF_E_NOMEM};   // beyond the reserved region
            const Group *dg = C.put(at<void>(B, L.o_groups), part);
            SingleAcc *dacc = C.rec ? (SingleAcc *)C.rec->alloc(n * sizeof(SingleAcc)) : at<SingleAcc>(B, L.o_acc);
            C.dev([=](hipStream_t s) { return launch_init_acc(dacc, (uint32_t)n, s); });
            uint64_t gl = 0;
            for (auto &g : part) gl += g.len;
            {
                Prof pr(ctx, st, K_SINGLE, gl, gl * 16);
                C.dev([=](hipStream_t s) { return launch_single(dg, (uint32_t)n, recbuf, dacc, cand, best, s); });
            }
            {
                Prof pr(ctx, st, K_OTHER, 0, 0);
                C.dev([=](hipStream_t s) { return launch_pick(cand, n, best, s); });
            }
        }
    };
    // (as for the groups above: launches of at most CAND_CAP tiles, each
    // followed by its pick; stream order keeps a launch from writing
    // candidates or tile lists that the previous one still reads, so the
    // host does not wait between them)
    auto run_tiles = [&](const std::vector<Tile> &tiles, const unsigned long long *recbuf) {
        for (uint64_t t0 = 0; t0 < tiles.size(); t0 += CAND_CAP) {
            const uint64_t n = std::min<uint64_t>(tiles.size() - t0, CAND_CAP);
            std::vector<Tile> part(tiles.begin() + t0, tiles.begin() + t0 + n);
            if (n > L.tiles_cap) throw Fail{DRF_E_NOMEM};   // beyond the reserved region
            const Tile *dt = C.put(at<void>(B, L.o_tiles), part);
            uint64_t tl = 0;
            for (auto &t : part) tl += t.len;
            {
                Prof pr(ctx, st, K_TILE, tl, tl * 8);
                C.dev([=](hipStream_t s) { return launch_tiles(dt, (uint32_t)n, recbuf, cand, best, s); });
            }
            {
                Prof pr(ctx, st, K_OTHER, 0, 0);
                C.dev([=](hipStream_t s) { return launch_pick(cand, n, best, s); });
            }
        }
    };

    // ---- level 0 segments: one per big phase
    std::vector<Seg> segs;
    std::vector<Group> groups;
    for (size_t j = bi; j < be; j++) {
        const uint32_t r = C.plans[big[j].proto].index_bits;
        if (r == 0) {
            groups.push_back(Group{pos[j - bi], big[j].count, big[j].proto, big[j].local});
            continue;
        }
        Seg sg{};
        sg.start = pos[j - bi];
        sg.len = big[j].count;
        sg.proto = big[j].proto;
        sg.phase = big[j].local;
        sg.dbits = std::min<uint32_t>(digit_bits_for(sg.len, dbits), r);
        sg.shift = r - sg.dbits;
        segs.push_back(sg);
    }
    if (!groups.empty()) run_groups(groups, in);

    unsigned long long *hist = at<unsigned long long>(B, L.o_hist);
    unsigned long long *dstarts = at<unsigned long long>(B, L.o_starts);
    while (!segs.empty()) {
        std::vector<Chunk> chunks;
        std::vector<uint64_t> out_start(segs.size());
        uint64_t hb = 0, op = 0, nstarts = 0;
        for (size_t s2 = 0; s2 < segs.size(); s2++) {
            Seg &sg = segs[s2];
            sg.nchunks = (uint32_t)((sg.len + CHUNK - 1) / CHUNK);
            sg.hbase = hb;
            hb += (uint64_t)sg.nchunks << sg.dbits;
            sg.sbase = (uint32_t)nstarts;
            nstarts += 1ull << sg.dbits;
            out_start[s2] = op;
            sg.obase = op;
            op += sg.len;
            for (uint32_t c = 0; c < sg.nchunks; c++) chunks.push_back(Chunk{(uint32_t)s2, c});
        }
        // the level must fit the regions the wave layout reserved
        if (segs.size() > L.nsegs_max || chunks.size() > L.chunks_max || hb > L.hist_max ||
            nstarts > L.nsegs_max * sstride || nstarts > 0xFFFFFFFFull)
            throw Fail{DRF_E_NOMEM};
        const Seg *dsegs = C.put(at<void>(B, L.o_segs), segs);
        const Chunk *dch = C.put(at<void>(B, L.o_chunks), chunks);
        const uint32_t nch = (uint32_t)chunks.size(), nsg = (uint32_t)segs.size();
        const unsigned long long *cin = in;
        unsigned long long *cout = out;
        {
            Prof pr(ctx, st, K_HIST, op, op * 8);
            C.dev([=](hipStream_t s) { return launch_hist(dsegs, dch, nch, cin, hist, s); });
        }
        // The bucket starts are only read by the host: the offsets kernel
        // writes them straight into pinned host memory, and the host builds
        // the next tiles while the scatter runs.  A recorded call writes them
        // to device memory and copies them back (its replays must not write
        // host memory that may since have been released); so does an
        // allocation-free call, into host heap memory, reading them once the
        // stream has drained (it takes no pinned memory).
        std::vector<uint64_t> heap_starts;
        const uint64_t *starts = nullptr;
        unsigned long long *wstarts = dstarts;
        if (C.noalloc) {
            heap_starts.resize(nstarts);
            starts = heap_starts.data();
        } else {
            if (nstarts * 8 > ctx->h_starts_cap) {
                if (ctx->h_starts) hipck(hipHostFree(ctx->h_starts));
                ctx->h_starts = nullptr;
                ctx->h_starts_cap = 0;
                const size_t want = std::max<size_t>(nstarts * 8, 8u << 20);
                if (hipHostMalloc(&ctx->h_starts, want, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
                    ctx->h_starts = nullptr;
                    (void)hipGetLastError();
                    throw Fail{DRF_E_NOMEM};
                }
                ctx->h_starts_cap = want;
            }
            starts = (const uint64_t *)ctx->h_starts;
            if (!C.rec) hipck(hipHostGetDevicePointer((void **)&wstarts, ctx->h_starts, 0));
        }
        {
            // counts in, output positions out (read twice, written once)
            Prof pr(ctx, st, K_SCAN, 0, hb * 24);
            C.dev([=](hipStream_t s) { return launch_offsets(dsegs, nsg, hist, wstarts, s); });
        }
        if (C.rec) hipck(hipMemcpyAsync(ctx->h_starts, dstarts, nstarts * 8, hipMemcpyDeviceToHost, st));
        if (C.noalloc) hipck(hipMemcpyAsync(heap_starts.data(), dstarts, nstarts * 8, hipMemcpyDeviceToHost, st));
        hipck(hipEventRecord(ctx->parted, st));
        {
            Prof pr(ctx, st, K_SCATTER, op, op * 16);
            C.dev([=](hipStream_t s) { return launch_scatter(dsegs, dch, nch, cin, hist, cout, recs, s); });
        }
        if (C.noalloc) hipck(hipStreamSynchronize(st));
        else hipck(hipEventSynchronize(ctx->parted));
        C.tr.mark("level partitioned", segs.size());

        std::vector<Seg> next;
        std::vector<Tile> tiles;
        std::vector<Group> g2;
        for (size_t s2 = 0; s2 < segs.size(); s2++) {
            const Seg &sg = segs[s2];
            const uint32_t nd = 1u << sg.dbits;
            const uint64_t *S = starts + sg.sbase;
            const uint64_t send = out_start[s2] + sg.len;
            auto end = [&](uint32_t x) { return x + 1 < nd ? S[x + 1] : send; };
            // consecutive small buckets of one segment are contiguous and
            // hold disjoint index values: one tile takes the longest run of
            // them that fits (a tile wider than the direct filter bitmap
            // hashes its cells into it; fuller tiles are fewer)
            uint32_t d = 0;
            while (d < nd) {
                const uint64_t a0 = S[d], len = end(d) - a0;
                if (len == 0) {
                    d++;
                    continue;
                }
                if (len > (uint64_t)tile) {
                    if (sg.shift == 0) {
                        g2.push_back(Group{a0, len, sg.proto, sg.phase});
                    } else {
                        Seg ns{};
                        ns.start = a0;
                        ns.len = len;
                        ns.proto = sg.proto;
                        ns.phase = sg.phase;
                        ns.dbits = std::min<uint32_t>(digit_bits_for(len, dbits), sg.shift);
                        ns.shift = sg.shift - ns.dbits;
                        next.push_back(ns);
                    }
                    d++;
                    continue;
                }
                // largest x in [d, nd) with end(x) - a0 <= tile (ends are nondecreasing)
                uint32_t lo = d, hi = nd - 1;
                const uint64_t lim = a0 + tile;
                while (lo < hi) {
                    const uint32_t m = (lo + hi + 1) >> 1;
                    if (end(m) <= lim) lo = m;
                    else hi = m - 1;
                }
                tiles.push_back(Tile{a0, (uint32_t)(end(lo) - a0), sg.proto, sg.phase, 0});
                d = lo + 1;
            }
        }
        run_tiles(tiles, out);
        if (!g2.empty()) run_groups(g2, out);
        segs.swap(next);
        std::swap(in, out);
        C.tr.mark("level tiles launched", tiles.size());
    }
}

// Big phases decided by tables (table path): a protocol with at most
// 2^table_bits cells whose phase holds at least as many events as cells.
// In waves of up to TABLE_WAVE_WORDS table words: tables cleared, the
// phases' items evaluated again with every event updating its cell, then
// the least racy cell of each table offered as a witness candidate.  No
// record reaches HBM.
constexpr uint64_t TABLE_WAVE_WORDS = 1ull << 28;   // 1 GiB of tables per wave

bool table_phase(const Call &C, const BigPhase &b, uint64_t cap_words) {
    const uint32_t tb = C.ctx->tune.table_bits, ib = C.plans[b.proto].index_bits;
    return tb && ib > 0 && ib <= tb && b.count >= (1ull << ib) && (3ull << ib) <= cap_words;
}

void run_table_waves(Call &C, const std::vector<BigPhase> &tbig, uint64_t cap_words, Best *best, Cand *cand) {
    drf_ctx *ctx = C.ctx;
    hipStream_t st = C.st;
    void *A = C.A;
    size_t bi = 0;
    while (bi < tbig.size()) {
        // the wave: consecutive table phases within the table budget and
        // one window of phases
        uint64_t words = 0;
        size_t be = bi;
        while (be < tbig.size()) {
            const uint64_t w = 3ull << C.plans[tbig[be].proto].index_bits;
            if (be > bi && (words + w > cap_words || tbig[be].k - tbig[bi].k >= (1ull << 26))) break;
            words += w;
            be++;
        }
        const uint64_t win_lo = tbig[bi].k, win_n = tbig[be - 1].k - win_lo + 1;
        std::vector<unsigned long long> tb(win_n, ~0ull);
        std::vector<TablePhase> tp(be - bi);
        uint64_t off = 0;
        for (size_t j = bi; j < be; j++) {
            const uint32_t cells = 1u << C.plans[tbig[j].proto].index_bits;
            tb[tbig[j].k - win_lo] = off;
            tp[j - bi] = TablePhase{off, cells, tbig[j].proto, tbig[j].local, 0};
            off += 3ull * cells;
        }
        std::vector<Item> witems[2];
        const bool all = bi == 0 && be == tbig.size();
        if (!all)
            for (int w = 0; w < 2; w++)
                for (const Item &it : C.items[w])
                    if (it.k_lo < win_lo + win_n && it.k_lo + it.span > win_lo) witems[w].push_back(it);
        Bump b;
        const size_t o_tab = b.reserve(words * 4);
        const size_t o_tb = b.reserve(win_n * 8);
        const size_t o_tp = b.reserve(tp.size() * sizeof(TablePhase));
        const size_t o_tmin = b.reserve(tp.size() * 4);
        const size_t o_wi0 = b.reserve(witems[0].size() * sizeof(Item));
        const size_t o_wi1 = b.reserve(witems[1].size() * sizeof(Item));
        grow(ctx, ctx->poolB, ctx->sizeB, b.used + ALIGN, st);
        void *B = ctx->poolB;
        uint32_t *tabs = at<uint32_t>(B, o_tab);
        uint32_t *tmin = at<uint32_t>(B, o_tmin);
        const unsigned long long *dtb = C.put(at<void>(B, o_tb), tb);
        const TablePhase *dtp = C.put(at<void>(B, o_tp), tp);
        C.fill_many({{tabs, 0xFFFFFFFFu, words * 4}, {tmin, 0xFFFFFFFFu, tp.size() * 4}});
        const NestDesc *dnests = at<NestDesc>(A, C.o_nests);
        const ProtoDesc *dprotos = at<ProtoDesc>(A, C.o_protos);
        const FixedVal *dfixed = at<FixedVal>(A, C.o_fixed);
        const uint32_t *dcode = at<uint32_t>(A, C.o_code);
        const uint32_t *ditemcnt = at<uint32_t>(A, C.o_itemcnt);
        uint64_t recs = 0;
        for (size_t j = bi; j < be; j++) recs += tbig[j].count;
        for (int w = 0; w < 2; w++) {
            const Item *it = all ? C.ditems[w] : C.put(at<void>(B, w ? o_wi1 : o_wi0), witems[w]);
            const size_t nit = all ? C.items[w].size() : witems[w].size();
            unsigned long long *tptr = reinterpret_cast<unsigned long long *>(tabs);
            for (uint64_t s0 = 0; s0 < nit; s0 += 1u << 30) {
                const uint32_t n = (uint32_t)std::min<uint64_t>(nit - s0, 1u << 30);
                const bool wide = w == 1;
                Prof pr(ctx, st, K_TABLE, w == 0 ? recs : 0, 0);
                C.dev([=](hipStream_t s) {
                    return launch_emit(it + s0, n, wide, dnests, dprotos, dfixed, dcode, ditemcnt, dtb, nullptr,
                                       win_lo, win_n, tptr, 0, s, true);
                });
            }
        }
        const uint32_t ntp = (uint32_t)tp.size();
        uint32_t bpt = 1;
        {
            const uint64_t per = words / 3 / ntp;   // mean cells per table
            while (bpt < 64 && (uint64_t)bpt * WG * 16 < per) bpt <<= 1;
        }
        {
            Prof pr(ctx, st, K_TABLE, 0, words * 4);
            C.dev([=](hipStream_t s) { return launch_table_scan(dtp, ntp, tabs, tmin, bpt, s); });
            C.dev([=](hipStream_t s) { return launch_table_offer(dtp, ntp, tabs, tmin, cand, best, s); });
        }
        {
            Prof pr(ctx, st, K_OTHER, 0, 0);
            C.dev([=](hipStream_t s) { return launch_pick(cand, ntp, best, s); });
        }
        C.tr.mark("table wave", be - bi);
        bi = be;
    }
}

// Fused units in launch order: largest first by the power of two of their
// work, input order within one power (a counting sort, linear in the units),
// written to out[0 .. units.size()).
void order_units_to(const std::vector<Unit> &units, const std::vector<uint64_t> &work, Unit *out) {
    auto bucket = [](uint64_t w) { return w ? 64 - __builtin_clzll(w) : 0; };
    size_t start[66] = {};
    for (uint64_t w : work) start[65 - bucket(w)]++;
    for (size_t b = 1; b < 66; b++) start[b] += start[b - 1];
    for (size_t i = 0; i < units.size(); i++) out[start[64 - bucket(work[i])]++] = units[i];
}
std::vector<Unit> order_units(const std::vector<Unit> &units, const std::vector<uint64_t> &work) {
    std::vector<Unit> out(units.size());
    order_units_to(units, work, out.data());
    return out;
}

// Profiling off for the duration of one call (an allocation-free call
// creates no timing events).
struct ProfOff {
    drf_ctx *c;
    bool was;
    explicit ProfOff(drf_ctx *ctx, bool on) : c(ctx), was(ctx->prof) { if (on) c->prof = false; }
    ~ProfOff() { c->prof = was; }
};

int check_impl(drf_ctx *ctx, const uint32_t *code, const uint64_t *code_off, const uint32_t *nthreads,
               uint32_t count, drf_result *d_results, uint64_t *d_phase_counts, uint64_t phase_cap,
               hipStream_t st, Recorder *rec = nullptr, bool noalloc = false) {
    if (!ctx || !code_off || !nthreads || (count && (!code || !d_results))) return DRF_E_ARG;
    if (count == 0) return DRF_OK;
    if (noalloc && (rec || !ctx->fixed)) return DRF_E_ARG;
    Call C;
    C.ctx = ctx;
    C.st = st;
    C.count = count;
    C.rec = rec;
    C.noalloc = noalloc;
    C.keep.ctx = ctx;
    C.keep.heap = noalloc;
    ProfOff prof_off(ctx, noalloc);
    try {
        hipck(hipSetDevice(ctx->device));
        if (ctx->done_valid) hipck(hipStreamWaitEvent(st, ctx->done, 0));
        C.plan_all(code, code_off, nthreads);
        C.tr.mark("plan", count);
        C.build_blob();
        C.tr.mark("blob", C.items[0].size() + C.items[1].size());
        if (C.total_phases > phase_cap || (C.total_phases && !d_phase_counts)) return DRF_E_ARG;
        // upper bound on fused units: one per small phase at most
        C.layout_a(C.total_phases + 1, !noalloc && !rec);
        // the previous call's device work may still read the pinned staging
        // and read-back buffers: wait for it on the host before reusing them
        // (planning above overlapped with it)
        if (ctx->done_valid) hipck(hipEventSynchronize(ctx->done));
        prof_collect(ctx);
        C.keep.clear();
        if (noalloc) {
            // pool A at the start of the fixed array, pool B after it
            if (C.needA > FIXED_SCRATCH_BYTES) throw Fail{DRF_E_NOMEM};
            C.A = ctx->fixed;
        } else {
            grow(ctx, ctx->poolA, ctx->sizeA, C.needA, st);
            C.A = ctx->poolA;
        }
        void *A = C.A;
        unsigned long long *phase_counts = (unsigned long long *)d_phase_counts;
        Best *best = at<Best>(A, C.o_best);
        Cand *cand = at<Cand>(A, C.o_cand);
        uint32_t *ovf = at<uint32_t>(A, C.o_ovf);
        const ProtoDesc *dprotos;
        const NestDesc *dnests;
        const FixedVal *dfixed;
        const uint32_t *dcode;
        if (!rec) {
            // the blob's parts are consecutive in pool A: one staged image,
            // one copy
            const size_t lo = C.o_protos, hi = C.o_items[1] + C.items[1].size() * sizeof(Item);
            char *img = (char *)C.keep.take(hi - lo);
            auto stage = [&](size_t off, const void *src, size_t bytes) {
                if (bytes) memcpy(img + (off - lo), src, bytes);
            };
            stage(C.o_protos, C.protos.data(), C.protos.size() * sizeof(ProtoDesc));
            stage(C.o_nests, C.nests.data(), C.nests.size() * sizeof(NestDesc));
            stage(C.o_fixed, C.fixed.data(), C.fixed.size() * sizeof(FixedVal));
            stage(C.o_code, C.code.data(), C.code.size() * sizeof(uint32_t));
            stage(C.o_items[0], C.items[0].data(), C.items[0].size() * sizeof(Item));
            stage(C.o_items[1], C.items[1].data(), C.items[1].size() * sizeof(Item));
            if (hi > lo) hipck(hipMemcpyAsync(at<char>(A, lo), img, hi - lo, hipMemcpyHostToDevice, st));
            dprotos = at<ProtoDesc>(A, C.o_protos);
            dnests = at<NestDesc>(A, C.o_nests);
            dfixed = at<FixedVal>(A, C.o_fixed);
            dcode = at<uint32_t>(A, C.o_code);
            C.ditems[0] = at<Item>(A, C.o_items[0]);
            C.ditems[1] = at<Item>(A, C.o_items[1]);
        } else {
            dprotos = C.put(at<void>(A, C.o_protos), C.protos);
            dnests = C.put(at<void>(A, C.o_nests), C.nests);
            dfixed = C.put(at<void>(A, C.o_fixed), C.fixed);
            dcode = C.put(at<void>(A, C.o_code), C.code);
            C.ditems[0] = C.put(at<void>(A, C.o_items[0]), C.items[0]);
            C.ditems[1] = C.put(at<void>(A, C.o_items[1]), C.items[1]);
        }
        const Item *const *ditems = C.ditems;
        // the emit pass reads the blob through pool A offsets
        if (rec) {
            // recorded calls keep the blob at its pool A offsets too (the
            // wave code addresses it there); pool A belongs to the recording
            upload(C.keep, at<void>(A, C.o_protos), C.protos, st);
            upload(C.keep, at<void>(A, C.o_nests), C.nests, st);
            upload(C.keep, at<void>(A, C.o_fixed), C.fixed, st);
            upload(C.keep, at<void>(A, C.o_code), C.code, st);
        }
        uint32_t *item_cnt = at<uint32_t>(A, C.o_itemcnt);
        unsigned long long *nrec_dev = at<unsigned long long>(A, C.o_nrec);
        uint32_t *qhead = at<uint32_t>(A, C.o_qhead);
        C.fill_many({{phase_counts, 0u, C.total_phases * sizeof(uint64_t)},
                     {ovf, 0u, count * sizeof(uint32_t)},
                     {best, 0xFFFFFFFFu, count * sizeof(Best)},
                     {nrec_dev, 0u, count * sizeof(uint64_t)},
                     {qhead, 0u, 64 * sizeof(uint32_t)}});
        const uint32_t fgrid = ctx->cus * 2;
        bool overlap = false;   // the counted units on the second stream
        const uint32_t small = small_events(ctx);
        int qslot = 0;

        // fused launches (persistent, units largest first), pair pick after each
        // (side: on the context's second stream, one workgroup per CU, with
        // their own witness candidates; the call's stream does the HBM path
        // meanwhile)
        auto fused = [&](std::vector<Unit> &units, bool wide, size_t dst_off, const std::vector<uint64_t> &work,
                         uint64_t events, bool side = false) {
            if (units.empty()) return;
            Cand *fc = side ? at<Cand>(A, C.o_cand2) : cand;
            Best *fb = side ? at<Best>(A, C.o_best2) : best;
            const uint32_t fg = side ? ctx->cus : fgrid;
            // one launch (the common case): the ordered units go straight
            // into the upload's staging memory
            std::vector<Unit> ord;
            if (units.size() > CAND_CAP) ord = order_units(units, work);
            for (uint64_t b0 = 0; b0 < units.size(); b0 += CAND_CAP) {
                const uint64_t n = std::min<uint64_t>(units.size() - b0, CAND_CAP);
                const Unit *du =
                    ord.empty() ? C.put_fill<Unit>(at<void>(A, dst_off), n,
                                                   [&](Unit *d) { order_units_to(units, work, d); })
                                : C.put(at<void>(A, dst_off),
                                        std::vector<Unit>(ord.begin() + b0, ord.begin() + b0 + n));
                if (qslot >= 64) {
                    C.fill32(qhead, 0, 64 * sizeof(uint32_t));
                    qslot = 0;
                }
                uint32_t *qh = qhead + qslot++;
                if (side) {
                    // after everything the call's stream has queued so far
                    hipck(hipEventRecord(ctx->side_go, st));
                    hipck(hipStreamWaitEvent(ctx->side, ctx->side_go, 0));
                    Prof pr(ctx, ctx->side, K_FUSED, events, 0);
                    events = 0;
                    hipck(launch_fused(du, (uint32_t)n, qh, wide, dnests, dprotos, dfixed, dcode, phase_counts, nrec_dev,
                                       ovf, fc, fb, fg, small, ctx->side));
                    hipck(launch_pick(fc, n, fb, ctx->side));
                    hipck(hipEventRecord(ctx->side_done, ctx->side));
                    continue;
                }
                {
                    Prof pr(ctx, st, K_FUSED, events, 0);
                    events = 0;
                    C.dev([=](hipStream_t s) {
                        return launch_fused(du, (uint32_t)n, qh, wide, dnests, dprotos, dfixed, dcode, phase_counts,
                                            nrec_dev, ovf, fc, fb, fg, small, s);
                    });
                }
                {
                    Prof pr(ctx, st, K_OTHER, 0, 0);
                    C.dev([=](hipStream_t s) { return launch_pick(fc, n, fb, s); });
                }
                if (b0 + CAND_CAP < units.size()) C.sync();
            }
        };

        // ---- count pass (protocols whose phases are not proven small)
        bool dynamic = false;
        for (uint32_t i = 0; i < count; i++) dynamic |= (C.status[i] == 0 && !C.stat[i]);
        for (int w = 0; w < 2; w++) {
            const Item *it = ditems[w];
            for (uint64_t b0 = 0; b0 < C.items[w].size(); b0 += 1u << 30) {
                const uint32_t n = (uint32_t)std::min<uint64_t>(C.items[w].size() - b0, 1u << 30);
                const bool wide = w == 1;
                Prof pr(ctx, st, K_COUNT, 0, 0);
                C.dev([=](hipStream_t s) {
                    return launch_count(it + b0, n, wide, dnests, dprotos, dfixed, dcode, phase_counts, item_cnt,
                                        ovf, s);
                });
            }
        }
        C.tr.mark("count launched");
        uint64_t *counts = nullptr;
        uint32_t *hovf = nullptr;
        std::vector<uint64_t> heap_counts;
        std::vector<uint32_t> heap_ovf;
        if (dynamic && noalloc) {
            // host heap read-back, read once the stream has drained
            heap_counts.resize(std::max<uint64_t>(1, C.total_phases));
            heap_ovf.resize(count);
            counts = heap_counts.data();
            hovf = heap_ovf.data();
            if (C.total_phases)
                hipck(hipMemcpyAsync(counts, phase_counts, C.total_phases * sizeof(uint64_t),
                                     hipMemcpyDeviceToHost, st));
            hipck(hipMemcpyAsync(hovf, ovf, count * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        } else if (dynamic) {
            // pinned read-back buffers of the context (not the upload staging,
            // which a sync in between may recycle)
            const size_t need = (std::max<uint64_t>(1, C.total_phases) * sizeof(uint64_t) + 255) & ~(size_t)255;
            const size_t want = need + count * sizeof(uint32_t);
            if (want > ctx->h_counts_cap) {
                if (ctx->h_counts) hipck(hipHostFree(ctx->h_counts));
                ctx->h_counts = nullptr;
                ctx->h_counts_cap = 0;
                if (hipHostMalloc(&ctx->h_counts, want, hipHostMallocDefault) != hipSuccess) {
                    ctx->h_counts = nullptr;
                    (void)hipGetLastError();
                    throw Fail{DRF_E_NOMEM};
                }
                ctx->h_counts_cap = want;
            }
            counts = (uint64_t *)ctx->h_counts;
            hovf = (uint32_t *)((char *)ctx->h_counts + need);
            if (C.total_phases)
                hipck(hipMemcpyAsync(counts, phase_counts, C.total_phases * sizeof(uint64_t),
                                     hipMemcpyDeviceToHost, st));
            hipck(hipMemcpyAsync(hovf, ovf, count * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
            hipck(hipEventRecord(ctx->counted, st));
        }

        // ---- fused path of protocols proven small: no host round trip;
        // runs on the device while the host classifies the counted ones
        for (int w = 0; w < 2; w++) {
            std::vector<uint64_t> work(C.sunits[w].size());
            for (size_t j = 0; j < work.size(); j++) {
                const Unit &u = C.sunits[w][j];
                work[j] = (u.k1 - u.k0) * C.plans[u.proto].max_phase_records;
            }
            fused(C.sunits[w], w == 1, C.o_sunits[w], work, 0);
        }

        C.tr.mark("static fused launched");
        // ---- classification of the counted protocols
        std::vector<uint64_t> nrec(count, 0);
        std::vector<Unit> units[2];
        std::vector<BigPhase> big;
        if (dynamic) {
            if (noalloc) hipck(hipStreamSynchronize(st));
            else hipck(hipEventSynchronize(ctx->counted));
            uint64_t dyn_events = 0;
            for (uint32_t i = 0; i < count; i++) {
                if (C.status[i] || C.stat[i] || hovf[i]) continue;
                const ProtoDesc &pd = C.protos[i];
                for (uint64_t k = pd.phase_off; k < pd.phase_off + pd.nphases; k++)
                    if (counts[k] <= (uint64_t)small) dyn_events += counts[k];
            }
            const uint64_t dyn_unit = C.unit_size(dyn_events);
            C.tr.mark("counts on host");
            for (uint32_t i = 0; i < count; i++) {
                if (C.status[i] || C.stat[i]) continue;
                if (hovf[i]) { C.status[i] = DRF_E_RANGE; continue; }
                const ProtoDesc &pd = C.protos[i];
                uint64_t acc = 0, ustart = ~0ull, last_small = 0;
                for (uint64_t k = pd.phase_off; k < pd.phase_off + pd.nphases; k++) {
                    const uint64_t c = counts[k];
                    nrec[i] += c;
                    if (c == 0) continue;
                    if (c > (uint64_t)small) {
                        big.push_back(BigPhase{k, c, i, (uint32_t)(k - pd.phase_off)});
                        continue;
                    }
                    if (ustart == ~0ull) ustart = k;
                    last_small = k;
                    acc += c;
                    if (acc >= dyn_unit) {
                        units[pd.wide].push_back(Unit{i, 0, ustart, k + 1});
                        ustart = ~0ull;
                        acc = 0;
                    }
                }
                if (ustart != ~0ull) units[pd.wide].push_back(Unit{i, 0, ustart, last_small + 1});
            }
            if (ctx->prof) {
                uint64_t tot = 0;
                for (uint32_t i = 0; i < count; i++) tot += nrec[i];
                for (auto &pp : ctx->pending) if (pp.cls == K_COUNT) { pp.records = tot; break; }
            }
            std::vector<uint64_t> work[2];
            uint64_t ev[2] = {0, 0};
            for (int w = 0; w < 2; w++) {
                work[w].assign(units[w].size(), 0);
                for (size_t j = 0; j < work[w].size(); j++) {
                    for (uint64_t k = units[w][j].k0; k < units[w][j].k1; k++)
                        if (counts[k] <= (uint64_t)small) work[w][j] += counts[k];
                    ev[w] += work[w][j];
                }
            }
            // the counted units run beside the HBM path when both are large
            // and the path is long enough to cover them (one launch of units
            // at most, narrow or wide: the second stream's candidates hold
            // one launch; not in recorded or allocation-free calls).  At one
            // workgroup per CU the fused kernel takes about 2.1 times as long
            // per event as at two, and the HBM-path kernels beside it about
            // 1.4 times their time alone: the overlap saves time while the
            // path's records are at least about 5/8 of the counted events.
            uint64_t big_recs = 0;
            for (const BigPhase &bp : big) big_recs += bp.count;
            overlap = FUSED_BESIDE && C.beside && ctx->side && ev[0] + ev[1] >= BESIDE_MIN && big_recs >= BESIDE_MIN &&
                      big_recs * 8 >= (ev[0] + ev[1]) * 5 &&
                      qslot + 2 <= 64 && units[0].size() <= CAND_CAP && units[1].size() <= CAND_CAP &&
                      (units[0].empty() || units[1].empty());
            if (overlap) C.fill32(at<Best>(A, C.o_best2), 0xFFFFFFFFu, count * sizeof(Best));
            C.tr.mark("counted events", ev[0] + ev[1]);
            C.tr.mark("big-phase records", big_recs);
            for (int w = 0; w < 2; w++) fused(units[w], w == 1, C.o_units, work[w], ev[w], overlap);
            C.tr.mark("fused launched", units[0].size() + units[1].size());
        }

        // ---- big phases decided by tables (when enabled), then the rest in
        // waves under the scratch budget
        // (not in allocation-free or recorded calls: their pool B is fixed
        // once for the call)
        if (ctx->tune.table_bits && !noalloc && !rec && !big.empty()) {
            const uint64_t cap_words =
                std::min<uint64_t>(TABLE_WAVE_WORDS, (ctx->limit > ctx->sizeA ? ctx->limit - ctx->sizeA : 0) / 8);
            std::vector<BigPhase> tbig, rest;
            for (const BigPhase &bp : big) (table_phase(C, bp, cap_words) ? tbig : rest).push_back(bp);
            big.swap(rest);
            if (!tbig.empty()) run_table_waves(C, tbig, cap_words, best, cand);
        }
        if (!big.empty()) {
            const uint64_t a_end = (C.needA + ALIGN - 1) & ~(ALIGN - 1);
            uint64_t budget = noalloc ? (FIXED_SCRATCH_BYTES > a_end ? FIXED_SCRATCH_BYTES - a_end : 0)
                                      : (ctx->limit > ctx->sizeA ? ctx->limit - ctx->sizeA : 0);
            std::vector<Wave> waves;
            size_t needB = 0;
            const std::vector<int32_t> status0 = C.status;
            for (int shrink = 0;; shrink++) {
            C.status = status0;
            // records per wave: about 21 bytes of pool B per record (two
            // record buffers and the partition metadata); the cap shrinks
            // until the largest wave's layout fits the budget
            uint64_t rec_cap = budget / 24;
            for (int attempt = 0;; attempt++) {
                waves.clear();
                std::vector<int32_t> st_try = C.status;
                size_t bi = 0;
                while (bi < big.size()) {
                    if (big[bi].count > rec_cap) {   // a phase that can never fit
                        st_try[big[bi].proto] = DRF_E_NOMEM;
                        bi++;
                        continue;
                    }
                    Wave W;
                    W.bi = bi;
                    W.recs = 0;
                    size_t be = bi;
                    while (be < big.size() && big[be].count <= rec_cap && W.recs + big[be].count <= rec_cap &&
                           big[be].k - big[bi].k < (1ull << 26)) {
                        W.recs += big[be].count;
                        be++;
                    }
                    W.be = be;
                    waves.push_back(std::move(W));
                    bi = be;
                }
                // one wave takes every item as uploaded; several take the
                // items overlapping their phase window
                if (waves.size() == 1) {
                    waves[0].all = true;
                } else {
                    for (Wave &W : waves) {
                        const uint64_t win_lo = big[W.bi].k, win_n = big[W.be - 1].k - win_lo + 1;
                        for (int w = 0; w < 2; w++)
                            for (const Item &it : C.items[w])
                                if (it.k_lo < win_lo + win_n && it.k_lo + it.span > win_lo) W.witems[w].push_back(it);
                    }
                }
                needB = 0;
                for (const Wave &W : waves) {
                    const uint64_t win_n = big[W.be - 1].k - big[W.bi].k + 1;
                    needB = std::max(needB, wave_layout(W.recs, win_n, W.be - W.bi, W.witems[0].size(),
                                                        W.witems[1].size(), ctx->tune.tile_events, small,
                                                        ctx->tune.digit_bits).bytes);
                }
                if (needB <= budget || rec_cap == 0 || attempt == 8) {
                    C.status.swap(st_try);
                    break;
                }
                rec_cap = (uint64_t)((double)rec_cap * ((double)budget / (double)needB) * 0.98);
            }
            if (noalloc) {
                if (needB > budget) throw Fail{DRF_E_NOMEM};
                C.B = (char *)ctx->fixed + a_end;
                break;
            }
            try {
                grow(ctx, ctx->poolB, ctx->sizeB, needB, st);
            } catch (Fail f) {
                // the device could not give a pool this large, although it
                // is within the limit: plan smaller waves
                if (f.code != DRF_E_NOMEM || shrink == 6 || needB <= (256ull << 20)) throw;
                C.tr.mark("pool B allocation failed", needB);
                budget = needB / 2;
                continue;
            }
            C.B = ctx->poolB;
            break;
            }
            C.tr.mark("waves planned", waves.size());
            for (const Wave &W : waves) run_wave(C, big, W, best, cand);
            C.tr.mark("waves done");
        }
        if (overlap) {
            // join the second stream; its witnesses into the call's
            hipck(hipStreamWaitEvent(st, ctx->side_done, 0));
            Best *b2 = at<Best>(A, C.o_best2);
            C.dev([=](hipStream_t s) { return launch_best_min(best, b2, count, s); });
        }

        // ---- results
        std::vector<ResultIn> rin(count);
        for (uint32_t i = 0; i < count; i++) {
            rin[i].status = C.status[i];
            rin[i].num_phases = C.status[i] ? 0 : (uint32_t)C.protos[i].nphases;
            rin[i].num_records = C.status[i] ? 0 : nrec[i];
            rin[i].flags = (C.status[i] == 0 && C.stat[i]) ? RESULT_FROM_DEVICE : 0;
        }
        const ResultIn *drin = C.put(at<void>(A, C.o_rin), rin);
        {
            Prof pr(ctx, st, K_OTHER, 0, 0);
            drf_result_dev *dres = (drf_result_dev *)d_results;
            C.dev([=](hipStream_t s) { return launch_result(count, drin, best, nrec_dev, ovf, dres, s); });
        }
        hipck(hipEventRecord(ctx->done, st));
        ctx->done_valid = true;
        // an allocation-free call's staging lives on the host heap until
        // this call returns: wait for the stream before releasing it
        if (noalloc) hipck(hipStreamSynchronize(st));
        // every upload came from pinned staging that the context keeps until
        // its next call has waited for this event: return without waiting
        C.tr.mark("enqueued");
        return DRF_OK;
    } catch (Fail f) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(st);
        if (ctx->side) (void)hipStreamSynchronize(ctx->side);
        return f.code;
    } catch (...) {
        (void)hipStreamSynchronize(st);
        if (ctx->side) (void)hipStreamSynchronize(ctx->side);
        return DRF_E_NOMEM;
    }
}

// Device scratch one call checking these plans may take: pool A (the
// uploaded metadata, per-phase bookkeeping and witness candidates) plus pool
// B for every record of the phases above one tile in a single wave.  The
// tuning of `tuned` is used (the library default when null).  An upper
// bound: the count pass may find fewer big-phase records than the plans
// allow, and a context whose limit is smaller splits the records into
// waves instead.
uint64_t scratch_estimate(const drf_ctx *tuned, std::vector<Plan> &&plans) {
    drf_ctx tmp;
    if (tuned) {
        tmp.tune = tuned->tune;
        tmp.cus = tuned->cus;
    }
    Call C;
    C.ctx = &tmp;
    C.count = (uint32_t)plans.size();
    C.plans = std::move(plans);
    C.build_blob();
    C.layout_a(C.total_phases + 1, true);
    const uint32_t small = small_events(&tmp);
    uint64_t bigrec = 0, nbig = 0;
    for (const Plan &p : C.plans) {
        if (p.status || p.max_phase_records <= (uint64_t)small) continue;
        bigrec += std::min<uint64_t>(p.max_records, 1ull << 40);
        nbig += p.num_phases;
    }
    uint64_t b = 0;
    if (bigrec)
        b = wave_layout(bigrec, nbig, nbig, C.items[0].size(), C.items[1].size(), tmp.tune.tile_events, small,
                        tmp.tune.digit_bits).bytes;
    return C.needA + b;
}

// The context's synchronization events and (for contexts whose calls are
// not recorded) its second stream, created up front so that no checking
// call creates any.
bool ctx_events(drf_ctx *c, bool side) {
    return hipEventCreateWithFlags(&c->done, hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&c->counted, hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&c->parted, hipEventDisableTiming) == hipSuccess &&
           (!side || (hipEventCreateWithFlags(&c->side_go, hipEventDisableTiming) == hipSuccess &&
                      hipEventCreateWithFlags(&c->side_done, hipEventDisableTiming) == hipSuccess &&
                      hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) == hipSuccess));
}

void fill_plan(const Plan &p, drf_plan *out) {
    memset(out, 0, sizeof *out);
    out->status = p.status;
    if (!p.status) {
        out->num_phases = (uint32_t)p.num_phases;
        out->index_bits = p.index_bits;
        out->wide = p.wide ? 1 : 0;
        out->max_records = p.max_records;
        out->nests = p.nests.size();
        out->max_phase_records = p.max_phase_records;
    }
}

}  // namespace

// ================================================================ C ABI
extern "C" {

const char *drf_version(void) { return "libdrf 0.1 (gfx950)"; }

int drf_compile_text(const char *text, size_t len, uint32_t *out, uint32_t cap, uint32_t *nwords) {
    if (!text || !nwords) return DRF_E_ARG;
    try {
        std::vector<uint32_t> w;
        int rc = compile_text(text, len, w);
        if (rc) return rc;
        *nwords = (uint32_t)w.size();
        if (w.size() > cap || !out) return DRF_E_NOMEM;
        memcpy(out, w.data(), w.size() * sizeof(uint32_t));
        return DRF_OK;
    } catch (...) {
        return DRF_E_NOMEM;
    }
}

int drf_plan_protocol(const uint32_t *code, uint32_t words, uint32_t num_threads, drf_plan *out) {
    if (!out) return DRF_E_ARG;
    try {
        std::vector<Plan> ps(1);
        plan_protocol(code, words, num_threads, ps[0]);
        fill_plan(ps[0], out);
        out->scratch_bytes = scratch_estimate(nullptr, std::move(ps));
        return DRF_OK;
    } catch (...) {
        memset(out, 0, sizeof *out);
        return DRF_E_NOMEM;
    }
}

int drf_plan_batch(const drf_ctx *ctx, const uint32_t *code, const uint64_t *code_off, const uint32_t *nthreads,
                   uint32_t count, drf_plan *plans, uint64_t *scratch_bytes_total) {
    if (!code_off || !nthreads || (count && (!code || !plans))) return DRF_E_ARG;
    try {
        drf_ctx tmp;
        if (ctx) {
            tmp.tune = ctx->tune;
            tmp.cus = ctx->cus;
        }
        Call C;
        C.ctx = &tmp;
        C.count = count;
        C.plan_all(code, code_off, nthreads);
        for (uint32_t i = 0; i < count; i++) {
            fill_plan(C.plans[i], &plans[i]);
            std::vector<Plan> one(1, C.plans[i]);
            plans[i].scratch_bytes = scratch_estimate(&tmp, std::move(one));
        }
        if (scratch_bytes_total) *scratch_bytes_total = count ? scratch_estimate(&tmp, std::move(C.plans)) : 0;
        return DRF_OK;
    } catch (...) {
        return DRF_E_NOMEM;
    }
}

int drf_ctx_create(int hip_device, uint64_t scratch_limit_bytes, drf_ctx **out) {
    if (!out) return DRF_E_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) {
        (void)hipGetLastError();
        return DRF_E_HIP;
    }
    if (hipSetDevice(hip_device) != hipSuccess) return DRF_E_HIP;
    drf_ctx *c = new (std::nothrow) drf_ctx();
    if (!c) return DRF_E_NOMEM;
    c->device = hip_device;
    if (scratch_limit_bytes == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) { delete c; return DRF_E_HIP; }
        scratch_limit_bytes = fr / 4 * 3;
    }
    c->limit = scratch_limit_bytes;
    // the fixed scratch array's address on this device (looked up once per
    // device, with the device current) for allocation-free calls
    if (!ctx_events(c, true) || fixed_scratch_address(hip_device, &c->fixed) != hipSuccess) {
        (void)hipGetLastError();
        drf_ctx_destroy(c);
        return DRF_E_HIP;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, hip_device) == hipSuccess && cus > 0)
        c->cus = (uint32_t)cus;
    *out = c;
    return DRF_OK;
}

int drf_ctx_release(drf_ctx *ctx, uint64_t keep_bytes) {
    if (!ctx) return DRF_E_ARG;
    if (ctx->sizeA + ctx->sizeB <= keep_bytes) return DRF_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return DRF_E_HIP;
    // freed in stream order after the context's last call, on a stream of
    // its own, so that neither the host nor other streams wait
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        return DRF_E_HIP;
    }
    int rc = DRF_OK;
    if (ctx->done_valid && hipStreamWaitEvent(st, ctx->done, 0) != hipSuccess) rc = DRF_E_HIP;
    if (rc == DRF_OK && ctx->poolB) {
        if (hipFreeAsync(ctx->poolB, st) == hipSuccess) {
            ctx->poolB = nullptr;
            ctx->sizeB = 0;
        } else {
            rc = DRF_E_HIP;
        }
    }
    if (rc == DRF_OK && ctx->poolA && ctx->sizeA > keep_bytes) {
        if (hipFreeAsync(ctx->poolA, st) == hipSuccess) {
            ctx->poolA = nullptr;
            ctx->sizeA = 0;
        } else {
            rc = DRF_E_HIP;
        }
    }
    (void)hipStreamDestroy(st);
    if (rc != DRF_OK) (void)hipGetLastError();
    return rc;
}

int drf_ctx_destroy(drf_ctx *ctx) {
    if (!ctx) return DRF_E_ARG;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    // the pools come from the stream-ordered allocator
    if (ctx->poolA) (void)hipFreeAsync(ctx->poolA, nullptr);
    if (ctx->poolB) (void)hipFreeAsync(ctx->poolB, nullptr);
    (void)hipDeviceSynchronize();
    if (ctx->done) (void)hipEventDestroy(ctx->done);
    if (ctx->counted) (void)hipEventDestroy(ctx->counted);
    if (ctx->parted) (void)hipEventDestroy(ctx->parted);
    if (ctx->side_go) (void)hipEventDestroy(ctx->side_go);
    if (ctx->side_done) (void)hipEventDestroy(ctx->side_done);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    if (ctx->h_starts) (void)hipHostFree(ctx->h_starts);
    for (auto &b : ctx->pin_blocks) (void)hipHostFree(b.first);
    if (ctx->h_counts) (void)hipHostFree(ctx->h_counts);
    for (auto e : ctx->ev_free) (void)hipEventDestroy(e);
    for (auto &p : ctx->pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    delete ctx;
    return DRF_OK;
}

int drf_ctx_set_profiling(drf_ctx *ctx, int on) {
    if (!ctx) return DRF_E_ARG;
    ctx->prof = on != 0;
    return DRF_OK;
}

int drf_ctx_set_tuning(drf_ctx *ctx, const drf_tuning *t) {
    if (!ctx || !t) return DRF_E_ARG;
    drf_tuning n = ctx->tune;
    if (t->tile_events) {
        if (t->tile_events < 256 || t->tile_events > (uint32_t)TILE || (t->tile_events & (t->tile_events - 1)))
            return DRF_E_ARG;
        n.tile_events = t->tile_events;
    }
    if (t->digit_bits) {
        if (t->digit_bits < 4 || t->digit_bits > 10) return DRF_E_ARG;
        n.digit_bits = t->digit_bits;
    }
    if (t->unit_events) n.unit_events = t->unit_events;
    if (t->item_events) {
        if (t->item_events < 256) return DRF_E_ARG;
        n.item_events = t->item_events;
    }
    if (t->table_bits) {
        if (t->table_bits == DRF_TABLE_OFF) n.table_bits = 0;
        else if (t->table_bits > 24) return DRF_E_ARG;
        else n.table_bits = t->table_bits;
    }
    ctx->tune = n;
    return DRF_OK;
}

int drf_ctx_get_tuning(drf_ctx *ctx, drf_tuning *t) {
    if (!ctx || !t) return DRF_E_ARG;
    *t = ctx->tune;
    return DRF_OK;
}

int drf_ctx_kernel_stats(drf_ctx *ctx, drf_kernel_stat *out, uint32_t cap, uint32_t *n, int reset) {
    if (!ctx || !n) return DRF_E_ARG;
    if (ctx->done_valid) {
        (void)hipSetDevice(ctx->device);
        if (hipEventSynchronize(ctx->done) != hipSuccess) {
            (void)hipGetLastError();
            return DRF_E_HIP;
        }
    }
    prof_collect(ctx);
    *n = K_NCLASS;
    for (uint32_t i = 0; i < K_NCLASS && i < cap && out; i++) {
        out[i] = ctx->stats[i];
        snprintf(out[i].name, sizeof out[i].name, "%s", KNAMES[i]);
    }
    if (reset) memset(ctx->stats, 0, sizeof ctx->stats);
    return DRF_OK;
}

struct drf_prepared {
    drf_ctx *priv = nullptr;       // private context: its pools belong to the recording
    Recorder rec;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

int drf_prepared_destroy(drf_prepared *p) {
    if (!p) return DRF_E_ARG;
    if (p->priv) (void)hipSetDevice(p->priv->device);
    (void)hipDeviceSynchronize();
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    for (void *q : p->rec.owned) (void)hipFree(q);
    if (p->priv) drf_ctx_destroy(p->priv);
    delete p;
    return DRF_OK;
}

int drf_prepare_batch(drf_ctx *ctx, const uint32_t *code, const uint64_t *code_off, const uint32_t *nthreads,
                      uint32_t count, drf_result *d_results, uint64_t *d_phase_counts, uint64_t phase_cap,
                      void *stream, drf_prepared **out) {
    if (!ctx || !out) return DRF_E_ARG;
    *out = nullptr;
    drf_prepared *p = new drf_prepared();
    p->priv = new drf_ctx();
    p->priv->device = ctx->device;
    p->priv->limit = ctx->limit;
    p->priv->tune = ctx->tune;
    p->priv->cus = ctx->cus;
    p->rec.limit = ctx->limit;
    if (!ctx_events(p->priv, false)) {
        (void)hipGetLastError();
        drf_prepared_destroy(p);
        return DRF_E_HIP;
    }
    int rc = check_impl(p->priv, code, code_off, nthreads, count, d_results, d_phase_counts, phase_cap,
                        (hipStream_t)stream, &p->rec);
    if (rc != DRF_OK) {
        drf_prepared_destroy(p);
        return rc;
    }
    hipStream_t cs = nullptr;
    bool ok = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        for (auto &op : p->rec.ops)
            if (op(cs) != hipSuccess) ok = false;
        hipGraph_t g = nullptr;
        if (hipStreamEndCapture(cs, &g) != hipSuccess) ok = false;
        p->graph = g;
    }
    ok = ok && p->graph && hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) == hipSuccess;
    if (cs) (void)hipStreamDestroy(cs);
    if (!ok) {
        (void)hipGetLastError();
        drf_prepared_destroy(p);
        return DRF_E_HIP;
    }
    *out = p;
    return DRF_OK;
}

int drf_run_prepared(drf_prepared *p, void *stream) {
    if (!p || !p->exec) return DRF_E_ARG;
    if (hipSetDevice(p->priv->device) != hipSuccess) return DRF_E_HIP;
    if (hipGraphLaunch(p->exec, (hipStream_t)stream) != hipSuccess) {
        (void)hipGetLastError();
        return DRF_E_HIP;
    }
    return DRF_OK;
}

uint64_t drf_prepared_launches(const drf_prepared *p) { return p ? p->rec.ops.size() : 0; }

// ------------------------------------------------------ shape-class graphs
// A hipGraph captured once over fixed device buffers sized by capacities,
// replayed for every batch of the class: batches whose protocols are all
// statically small (their planner bound puts every phase in one LDS tile),
// so the whole device work is fills, the fused launches, witness picks and
// results, with no host round trip.  Counts that change from batch to batch
// (protocols, fused units) are read by the kernels from a header uploaded
// with the batch.
struct GraphHdr {
    uint32_t count;
    uint32_t nunits[2];
    uint32_t pad;
};

struct drf_graph {
    drf_ctx *priv = nullptr;          // tuning, device, compute units
    drf_graph_caps caps{};
    char *dev = nullptr;              // device buffers of the class
    char *pin = nullptr;              // pinned staging of one batch's upload
    size_t o_hdr = 0, o_protos = 0, o_nests = 0, o_fixed = 0, o_code = 0, o_units[2] = {0, 0}, o_rin = 0;
    size_t o_counts = 0, o_results = 0, o_ovf = 0, o_nrec = 0, o_qhead = 0, o_best = 0, o_cand = 0, bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t staged = nullptr;      // the previous batch's upload has been read
    bool staged_valid = false;
};

int drf_graph_destroy(drf_graph *g) {
    if (!g) return DRF_E_ARG;
    if (g->priv) (void)hipSetDevice(g->priv->device);
    if (g->staged) {
        if (g->staged_valid) (void)hipEventSynchronize(g->staged);
        (void)hipEventDestroy(g->staged);
    }
    (void)hipDeviceSynchronize();
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->dev) (void)hipFree(g->dev);
    if (g->pin) (void)hipHostFree(g->pin);
    if (g->priv) drf_ctx_destroy(g->priv);
    delete g;
    return DRF_OK;
}

int drf_graph_create(drf_ctx *ctx, const drf_graph_caps *caps, void *stream, drf_graph **out) {
    if (!ctx || !caps || !out) return DRF_E_ARG;
    *out = nullptr;
    const drf_graph_caps c = *caps;
    if (c.max_protocols == 0 || c.max_units == 0 || c.max_units > CAND_CAP || c.max_phases > (1ull << 40))
        return DRF_E_ARG;
    drf_graph *g = new (std::nothrow) drf_graph();
    if (!g) return DRF_E_NOMEM;
    g->caps = c;
    int rc = DRF_OK;
    hipStream_t cs = nullptr;
    try {
        hipck(hipSetDevice(ctx->device));
        g->priv = new drf_ctx();
        g->priv->device = ctx->device;
        g->priv->limit = ctx->limit;
        g->priv->tune = ctx->tune;
        g->priv->cus = ctx->cus;
        if (!ctx_events(g->priv, false)) throw Fail{DRF_E_HIP};
        hipck(hipEventCreateWithFlags(&g->staged, hipEventDisableTiming));
        // uploaded part first (one staging image), then the device-only part
        Bump b;
        g->o_hdr = b.reserve(sizeof(GraphHdr));
        g->o_protos = b.reserve((size_t)c.max_protocols * sizeof(ProtoDesc));
        g->o_nests = b.reserve((size_t)c.max_nests * sizeof(NestDesc));
        g->o_fixed = b.reserve((size_t)c.max_fixed * sizeof(FixedVal));
        g->o_code = b.reserve((size_t)c.max_code_words * sizeof(uint32_t));
        g->o_units[0] = b.reserve((size_t)c.max_units * sizeof(Unit));
        g->o_units[1] = b.reserve((size_t)c.max_units * sizeof(Unit));
        g->o_rin = b.reserve((size_t)c.max_protocols * sizeof(ResultIn));
        const size_t staged_bytes = b.used;
        g->o_counts = b.reserve(std::max<uint64_t>(1, c.max_phases) * sizeof(uint64_t));
        g->o_results = b.reserve((size_t)c.max_protocols * sizeof(drf_result));
        g->o_ovf = b.reserve((size_t)c.max_protocols * sizeof(uint32_t));
        g->o_nrec = b.reserve((size_t)c.max_protocols * sizeof(uint64_t));
        g->o_qhead = b.reserve(64 * sizeof(uint32_t));
        g->o_best = b.reserve((size_t)c.max_protocols * sizeof(Best));
        g->o_cand = b.reserve((size_t)c.max_units * sizeof(Cand));
        g->bytes = b.used + ALIGN;
        if (hipMalloc((void **)&g->dev, g->bytes) != hipSuccess) {
            g->dev = nullptr;
            (void)hipGetLastError();
            throw Fail{DRF_E_NOMEM};
        }
        if (hipHostMalloc((void **)&g->pin, staged_bytes + ALIGN, hipHostMallocDefault) != hipSuccess) {
            g->pin = nullptr;
            (void)hipGetLastError();
            throw Fail{DRF_E_NOMEM};
        }
        char *D = g->dev;
        const GraphHdr *hdr = (const GraphHdr *)(D + g->o_hdr);
        const ProtoDesc *dprotos = (const ProtoDesc *)(D + g->o_protos);
        const NestDesc *dnests = (const NestDesc *)(D + g->o_nests);
        const FixedVal *dfixed = (const FixedVal *)(D + g->o_fixed);
        const uint32_t *dcode = (const uint32_t *)(D + g->o_code);
        unsigned long long *counts = (unsigned long long *)(D + g->o_counts);
        unsigned long long *nrec = (unsigned long long *)(D + g->o_nrec);
        uint32_t *ovf = (uint32_t *)(D + g->o_ovf);
        uint32_t *qhead = (uint32_t *)(D + g->o_qhead);
        Best *best = (Best *)(D + g->o_best);
        Cand *cand = (Cand *)(D + g->o_cand);
        const ResultIn *rin = (const ResultIn *)(D + g->o_rin);
        drf_result_dev *res = (drf_result_dev *)(D + g->o_results);
        hipck(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipck(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        FillList L{};
        auto add = [&](void *p, uint32_t v, size_t bytes) {
            L.p[L.count] = (uint32_t *)p;
            L.v[L.count] = v;
            L.n[L.count] = bytes / 4;
            L.count++;
        };
        add(counts, 0u, std::max<uint64_t>(1, c.max_phases) * sizeof(uint64_t));
        add(ovf, 0u, (size_t)c.max_protocols * sizeof(uint32_t));
        add(best, 0xFFFFFFFFu, (size_t)c.max_protocols * sizeof(Best));
        add(nrec, 0u, (size_t)c.max_protocols * sizeof(uint64_t));
        add(qhead, 0u, 64 * sizeof(uint32_t));
        hipError_t e = launch_fill_multi(L, cs);
        const uint32_t grid = g->priv->cus * 2, tile = small_events(g->priv);
        for (int w = 0; w < 2 && e == hipSuccess; w++) {
            const Unit *du = (const Unit *)(D + g->o_units[w]);
            e = launch_fused(du, c.max_units, qhead + w, w == 1, dnests, dprotos, dfixed, dcode, counts, nrec, ovf,
                             cand, best, grid, tile, cs, &hdr->nunits[w]);
            if (e == hipSuccess) e = launch_pick(cand, c.max_units, best, cs, &hdr->nunits[w]);
        }
        if (e == hipSuccess) e = launch_result(c.max_protocols, rin, best, nrec, ovf, res, cs, &hdr->count);
        hipGraph_t gr = nullptr;
        const hipError_t e2 = hipStreamEndCapture(cs, &gr);
        g->graph = gr;
        if (e != hipSuccess || e2 != hipSuccess || !gr) throw Fail{DRF_E_HIP};
        hipck(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
        // one replay on the caller's stream initializes nothing the runs rely
        // on; the class is ready
        (void)stream;
    } catch (Fail f) {
        rc = f.code;
    } catch (...) {
        rc = DRF_E_NOMEM;
    }
    if (cs) (void)hipStreamDestroy(cs);
    if (rc != DRF_OK) {
        (void)hipGetLastError();
        drf_graph_destroy(g);
        return rc;
    }
    *out = g;
    return DRF_OK;
}

int drf_graph_check(drf_graph *g, const uint32_t *code, const uint64_t *code_off, const uint32_t *nthreads,
                    uint32_t count, drf_result *d_results, uint64_t *d_phase_counts, uint64_t phase_cap,
                    void *stream) {
    if (!g || !code_off || !nthreads || (count && (!code || !d_results))) return DRF_E_ARG;
    if (count == 0) return DRF_OK;
    const hipStream_t st = (hipStream_t)stream;
    try {
        hipck(hipSetDevice(g->priv->device));
        Call C;
        C.ctx = g->priv;
        C.st = st;
        C.count = count;
        C.keep.ctx = g->priv;
        C.plan_all(code, code_off, nthreads);
        C.build_blob();
        // the class: statically small protocols within the capacities
        for (uint32_t i = 0; i < count; i++)
            if (C.status[i] == 0 && !C.stat[i]) return DRF_E_LIMIT;
        const drf_graph_caps &c = g->caps;
        if (count > c.max_protocols || C.nests.size() > c.max_nests || C.code.size() > c.max_code_words ||
            C.fixed.size() > c.max_fixed || C.total_phases > c.max_phases || C.sunits[0].size() > c.max_units ||
            C.sunits[1].size() > c.max_units)
            return DRF_E_LIMIT;
        if (C.total_phases > phase_cap || (C.total_phases && !d_phase_counts)) return DRF_E_ARG;
        // the upload, staged at the device offsets: header, blob, units
        // (largest first, as in a direct check), result inputs
        if (g->staged_valid) hipck(hipEventSynchronize(g->staged));
        char *P = g->pin;
        GraphHdr h{count, {0, 0}, 0};
        std::vector<std::pair<size_t, size_t>> parts;
        auto stage = [&](size_t off, const void *src, size_t bytes) {
            if (!bytes) return;
            memcpy(P + off, src, bytes);
            parts.push_back({off, bytes});
        };
        for (int w = 0; w < 2; w++) {
            std::vector<Unit> &us = C.sunits[w];
            std::vector<uint64_t> work(us.size());
            for (size_t j = 0; j < us.size(); j++) work[j] = (us[j].k1 - us[j].k0) * C.plans[us[j].proto].max_phase_records;
            std::vector<Unit> ord = order_units(us, work);
            h.nunits[w] = (uint32_t)ord.size();
            stage(g->o_units[w], ord.data(), ord.size() * sizeof(Unit));
        }
        std::vector<ResultIn> rin(count);
        for (uint32_t i = 0; i < count; i++) {
            rin[i].status = C.status[i];
            rin[i].num_phases = C.status[i] ? 0 : (uint32_t)C.protos[i].nphases;
            rin[i].num_records = 0;
            rin[i].flags = C.status[i] == 0 ? RESULT_FROM_DEVICE : 0;
        }
        stage(g->o_hdr, &h, sizeof h);
        stage(g->o_protos, C.protos.data(), C.protos.size() * sizeof(ProtoDesc));
        stage(g->o_nests, C.nests.data(), C.nests.size() * sizeof(NestDesc));
        stage(g->o_fixed, C.fixed.data(), C.fixed.size() * sizeof(FixedVal));
        stage(g->o_code, C.code.data(), C.code.size() * sizeof(uint32_t));
        stage(g->o_rin, rin.data(), rin.size() * sizeof(ResultIn));
        for (auto &pt : parts)
            hipck(hipMemcpyAsync(g->dev + pt.first, P + pt.first, pt.second, hipMemcpyHostToDevice, st));
        hipck(hipEventRecord(g->staged, st));
        g->staged_valid = true;
        hipck(hipGraphLaunch(g->exec, st));
        hipck(hipMemcpyAsync(d_results, g->dev + g->o_results, (size_t)count * sizeof(drf_result),
                             hipMemcpyDeviceToDevice, st));
        if (C.total_phases)
            hipck(hipMemcpyAsync(d_phase_counts, g->dev + g->o_counts, C.total_phases * sizeof(uint64_t),
                                 hipMemcpyDeviceToDevice, st));
        return DRF_OK;
    } catch (Fail f) {
        (void)hipGetLastError();
        return f.code;
    } catch (...) {
        return DRF_E_NOMEM;
    }
}

int drf_babycuda_infer(const char *text, size_t len, const char *params, char *out, size_t cap, size_t *needed,
                       int32_t *status) {
    if (!text || !needed || !status) return DRF_E_ARG;
    try {
        std::string map;
        const int st = babycuda_infer(text, len, params, map);
        if (st == DRF_E_ARG) return DRF_E_ARG;
        *status = st;
        *needed = st ? 0 : map.size() + 1;
        if (st) return DRF_OK;
        if (!out || cap < map.size() + 1) return DRF_E_NOMEM;
        memcpy(out, map.c_str(), map.size() + 1);
        return DRF_OK;
    } catch (...) {
        return DRF_E_NOMEM;
    }
}

int drf_text_slot(const char *text, size_t len, const char *name, uint32_t *slot) {
    if (!text || !name || !slot) return DRF_E_ARG;
    try {
        const int s2 = text_slot(text, len, name);
        if (s2 < 0) return DRF_E_ARG;
        *slot = (uint32_t)s2;
        return DRF_OK;
    } catch (...) {
        return DRF_E_NOMEM;
    }
}

int drf_protocol_arrays(const uint32_t *code, uint32_t words, uint32_t *num_arrays) {
    if (!num_arrays) return DRF_E_ARG;
    try {
        IR ir;
        const int st = decode(code, words, ir);
        if (st) return st;
        *num_arrays = ir_arrays(ir);
        return DRF_OK;
    } catch (...) {
        return DRF_E_NOMEM;
    }
}

int drf_bind_param(const uint32_t *code, uint32_t words, uint32_t slot, uint64_t value, uint32_t *out,
                   uint32_t cap, uint32_t *nwords) {
    if (!nwords) return DRF_E_ARG;
    try {
        IR ir;
        const int st = decode(code, words, ir);
        if (st) return st;
        if (slot >= ir.nslots || !ir_bind(ir, slot, value)) return DRF_E_ARG;
        std::vector<uint32_t> w;
        encode(ir, w);
        *nwords = (uint32_t)w.size();
        if (w.size() > cap || !out) return DRF_E_NOMEM;
        memcpy(out, w.data(), w.size() * sizeof(uint32_t));
        return DRF_OK;
    } catch (...) {
        return DRF_E_NOMEM;
    }
}

namespace {

// The instances of a parameter sweep, packed as a batch: instance i is the
// protocol with variable `slot` bound to first + i.
int sweep_codes(const uint32_t *code, uint32_t words, uint32_t slot, uint64_t first, uint32_t count,
                std::vector<uint32_t> &all, std::vector<uint64_t> &off) {
    IR ir;
    const int st = decode(code, words, ir);
    if (st) return st;
    if (slot >= ir.nslots) return DRF_E_ARG;
    for (const SNode &s2 : ir.s)
        if ((s2.kind == B_FORU || s2.kind == B_FORS) && s2.slot == slot) return DRF_E_ARG;
    if (count && first + (uint64_t)(count - 1) < first) return DRF_E_ARG;
    off.assign(1, 0);
    std::vector<uint32_t> w;
    for (uint32_t i = 0; i < count; i++) {
        IR c = ir;
        ir_bind(c, slot, first + i);
        encode(c, w);
        all.insert(all.end(), w.begin(), w.end());
        off.push_back(all.size());
    }
    return DRF_OK;
}

// The protocol of each array of a multi-array protocol, packed as a batch.
int array_codes(const uint32_t *code, uint32_t words, std::vector<uint32_t> &all, std::vector<uint64_t> &off) {
    IR ir;
    const int st = decode(code, words, ir);
    if (st) return st;
    const uint32_t na = ir_arrays(ir);
    off.assign(1, 0);
    std::vector<uint32_t> w;
    for (uint32_t a = 0; a < na; a++) {
        IR c = ir;
        ir_project(c, a);
        encode(c, w);
        all.insert(all.end(), w.begin(), w.end());
        off.push_back(all.size());
    }
    return DRF_OK;
}

}  // namespace

int drf_plan_sweep(const uint32_t *code, uint32_t words, uint32_t num_threads, uint32_t slot, uint64_t first,
                   uint32_t count, drf_plan *plans, uint64_t *scratch_bytes_total) {
    if (count && !plans) return DRF_E_ARG;
    try {
        std::vector<uint32_t> all;
        std::vector<uint64_t> off;
        const int rc = sweep_codes(code, words, slot, first, count, all, off);
        if (rc) return rc;
        std::vector<uint32_t> nth(count, num_threads);
        return drf_plan_batch(nullptr, all.data(), off.data(), nth.data(), count, plans, scratch_bytes_total);
    } catch (...) {
        return DRF_E_NOMEM;
    }
}

int drf_check_sweep(drf_ctx *ctx, const uint32_t *code, uint32_t words, uint32_t num_threads, uint32_t slot,
                    uint64_t first, uint32_t count, drf_result *d_results, uint64_t *d_phase_counts,
                    uint64_t phase_cap, void *stream) {
    if (!ctx) return DRF_E_ARG;
    try {
        std::vector<uint32_t> all;
        std::vector<uint64_t> off;
        const int rc = sweep_codes(code, words, slot, first, count, all, off);
        if (rc) return rc;
        std::vector<uint32_t> nth(count, num_threads);
        return check_impl(ctx, all.data(), off.data(), nth.data(), count, d_results, d_phase_counts, phase_cap,
                          (hipStream_t)stream);
    } catch (...) {
        return DRF_E_NOMEM;
    }
}

int drf_plan_arrays(const uint32_t *code, uint32_t words, uint32_t num_threads, drf_plan *plans, uint32_t cap,
                    uint64_t *scratch_bytes_total) {
    if (!plans) return DRF_E_ARG;
    try {
        std::vector<uint32_t> all;
        std::vector<uint64_t> off;
        const int rc = array_codes(code, words, all, off);
        if (rc) return rc;
        const uint32_t na = (uint32_t)(off.size() - 1);
        if (na > cap) return DRF_E_ARG;
        std::vector<uint32_t> nth(na, num_threads);
        return drf_plan_batch(nullptr, all.data(), off.data(), nth.data(), na, plans, scratch_bytes_total);
    } catch (...) {
        return DRF_E_NOMEM;
    }
}

int drf_check_arrays(drf_ctx *ctx, const uint32_t *code, uint32_t words, uint32_t num_threads,
                     drf_result *d_results, uint64_t *d_phase_counts, uint64_t phase_cap, void *stream) {
    if (!ctx) return DRF_E_ARG;
    try {
        std::vector<uint32_t> all;
        std::vector<uint64_t> off;
        const int rc = array_codes(code, words, all, off);
        if (rc) return rc;
        const uint32_t na = (uint32_t)(off.size() - 1);
        std::vector<uint32_t> nth(na, num_threads);
        return check_impl(ctx, all.data(), off.data(), nth.data(), na, d_results, d_phase_counts, phase_cap,
                          (hipStream_t)stream);
    } catch (...) {
        return DRF_E_NOMEM;
    }
}

int drf_check_protocol(drf_ctx *ctx, const uint32_t *code, uint32_t words, uint32_t num_threads,
                       drf_result *d_result, uint64_t *d_phase_counts, uint64_t phase_cap, void *stream) {
    const uint64_t off[2] = {0, words};
    return check_impl(ctx, code, off, &num_threads, 1, d_result, d_phase_counts, phase_cap, (hipStream_t)stream);
}

int drf_check_batch(drf_ctx *ctx, const uint32_t *code, const uint64_t *code_off, const uint32_t *nthreads,
                    uint32_t count, drf_result *d_results, uint64_t *d_phase_counts, uint64_t phase_cap,
                    void *stream) {
    return check_impl(ctx, code, code_off, nthreads, count, d_results, d_phase_counts, phase_cap,
                      (hipStream_t)stream);
}

int drf_check_batch_noalloc(drf_ctx *ctx, const uint32_t *code, const uint64_t *code_off, const uint32_t *nthreads,
                            uint32_t count, drf_result *d_results, uint64_t *d_phase_counts, uint64_t phase_cap,
                            void *stream) {
    return check_impl(ctx, code, code_off, nthreads, count, d_results, d_phase_counts, phase_cap,
                      (hipStream_t)stream, nullptr, true);
}

}  // extern "C"
