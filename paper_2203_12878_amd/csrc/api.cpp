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
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <thread>
#include <vector>

#include "../../include/drf.h"
#include "host.hpp"
#include "kernels.hpp"

using namespace drf;

enum KClass { K_COUNT, K_FUSED, K_EMIT, K_HIST, K_SCAN, K_SCATTER, K_TILE, K_SINGLE, K_OTHER, K_NCLASS };
static const char *KNAMES[K_NCLASS] = {"count", "fused", "emit", "hist", "scan", "scatter", "tile", "single", "other"};

struct drf_ctx {
    int device = 0;
    uint64_t limit = 0;
    void *poolA = nullptr;
    size_t sizeA = 0;
    void *poolB = nullptr;
    size_t sizeB = 0;
    hipEvent_t done = nullptr;
    bool done_valid = false;
    // per-kernel-class timing
    bool prof = false;
    std::vector<hipEvent_t> ev_free;
    struct Pending { int cls; hipEvent_t a, b; uint64_t records, bytes; };
    std::vector<Pending> pending;
    drf_kernel_stat stats[K_NCLASS] = {};
};

namespace {

constexpr uint64_t ITEM_EVENTS = 1ull << 16;   // target access events per count/emit item
constexpr uint64_t UNIT_EVENTS = 1ull << 12;   // target access events per fused unit
constexpr uint64_t CAND_CAP = 1ull << 20;      // candidates per launch
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

void grow(void *&p, size_t &size, size_t need) {
    if (need <= size) return;
    if (p) {
        hipck(hipDeviceSynchronize());
        hipck(hipFree(p));
        p = nullptr;
        size = 0;
    }
    size_t want = (need + (64ull << 20) - 1) & ~((64ull << 20) - 1);
    if (hipMalloc(&p, want) != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        throw Fail{DRF_E_NOMEM};
    }
    size = want;
}

// host copies of uploaded arrays stay alive until the call's next sync
struct Keep {
    std::vector<std::vector<char>> bufs;
    template <class T>
    const void *hold(const std::vector<T> &v) {
        bufs.emplace_back((const char *)v.data(), (const char *)v.data() + v.size() * sizeof(T));
        return bufs.back().data();
    }
    void clear() { bufs.clear(); }
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

struct Call {
    drf_ctx *ctx;
    hipStream_t st;
    uint32_t count;
    std::vector<Plan> plans;
    std::vector<int32_t> status;
    std::vector<uint64_t> poff;
    std::vector<ProtoDesc> protos;
    std::vector<NestDesc> nests;
    std::vector<FixedVal> fixed;
    std::vector<uint32_t> code;
    std::vector<Item> items[2];        // narrow, wide
    uint64_t item_cnt_words = 0;
    uint64_t total_phases = 0;
    Keep keep;

    // pool A offsets
    size_t o_protos, o_nests, o_fixed, o_code, o_items[2], o_itemcnt, o_ovf, o_best, o_cand, o_units, o_rin, o_res;
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

    void build_blob() {
        status.assign(count, 0);
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
                pd.nnests++;
                make_items((uint32_t)nests.size() - 1, p.n, p.wide);
            }
        }
    }

    void make_items(uint32_t ni, uint32_t n, bool wide) {
        const NestDesc &nd = nests[ni];
        if (n == 0) return;
        const uint64_t lanes = std::min<uint64_t>(n, WG);
        const uint64_t per_iter = lanes * std::max<uint64_t>(1, nd.rec_bound);
        const uint64_t F = std::max<uint64_t>(1, ITEM_EVENTS / per_iter);
        const uint32_t nb = (n + WG - 1) / WG;
        for (uint64_t f0 = 0; f0 < nd.iters;) {
            uint64_t f1 = std::min(nd.iters, f0 + F);
            const uint64_t k0 = nest_phase(nd, f0);
            while (f1 - f0 > 1 && nest_phase(nd, f1 - 1) - k0 + 1 > (uint64_t)MAXSPAN) f1 = f0 + (f1 - f0) / 2;
            const uint32_t span = (uint32_t)(nest_phase(nd, f1 - 1) - k0 + 1);
            for (uint32_t b = 0; b < nb; b++) {
                Item it{};
                it.nest = ni;
                it.tid0 = b * WG;
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

    void layout_a(uint64_t nunits_max) {
        Bump b;
        o_protos = b.reserve(protos.size() * sizeof(ProtoDesc));
        o_nests = b.reserve(nests.size() * sizeof(NestDesc));
        o_fixed = b.reserve(fixed.size() * sizeof(FixedVal));
        o_code = b.reserve(code.size() * sizeof(uint32_t));
        o_items[0] = b.reserve(items[0].size() * sizeof(Item));
        o_items[1] = b.reserve(items[1].size() * sizeof(Item));
        o_itemcnt = b.reserve(item_cnt_words * sizeof(uint32_t));
        o_ovf = b.reserve(count * sizeof(uint32_t));
        o_best = b.reserve(count * sizeof(Best));
        o_cand = b.reserve(CAND_CAP * sizeof(Cand));
        o_units = b.reserve(std::min<uint64_t>(nunits_max, CAND_CAP) * sizeof(Unit));
        o_rin = b.reserve(count * sizeof(ResultIn));
        o_res = b.used;
        needA = b.used + ALIGN;
    }
};

// One wave of big phases [bi, be) of the global big-phase list, holding
// `recs` records in total: emit, then partition levels until every bucket
// fits an LDS tile (or holds a single index value).
void run_wave(Call &C, const std::vector<BigPhase> &big, size_t bi, size_t be, uint64_t recs, Best *best,
              Cand *cand) {
    drf_ctx *ctx = C.ctx;
    hipStream_t st = C.st;
    void *A = ctx->poolA;
    const uint64_t win_lo = big[bi].k;
    const uint64_t win_n = big[be - 1].k - win_lo + 1;

    std::vector<Item> witems[2];
    for (int w = 0; w < 2; w++)
        for (const Item &it : C.items[w])
            if (it.k_lo < win_lo + win_n && it.k_lo + it.span > win_lo) witems[w].push_back(it);

    const uint64_t nsegs_max = recs / TILE + 1;
    const uint64_t chunks_max = recs / CHUNK + nsegs_max + 1;
    const uint64_t hist_max = chunks_max * RADIX;
    const uint64_t tiles_max = std::min<uint64_t>(nsegs_max * RADIX, recs) + 1;
    Bump b;
    const size_t o_bb = b.reserve(win_n * 8), o_cur = b.reserve(win_n * 8);
    const size_t o_ra = b.reserve(recs * 8), o_rb = b.reserve(recs * 8);
    const size_t o_hist = b.reserve((hist_max + scan_tmp_words(hist_max)) * 8);
    const size_t o_starts = b.reserve(nsegs_max * RADIX * 8);
    const size_t o_segs = b.reserve(nsegs_max * sizeof(Seg));
    const size_t o_chunks = b.reserve(chunks_max * sizeof(Chunk));
    const size_t o_tiles = b.reserve(std::min<uint64_t>(tiles_max, CAND_CAP) * sizeof(Tile));
    const size_t o_groups = b.reserve(std::min<uint64_t>(nsegs_max + (be - bi), CAND_CAP) * sizeof(Group));
    const size_t o_acc = b.reserve(std::min<uint64_t>(nsegs_max + (be - bi), CAND_CAP) * sizeof(SingleAcc));
    const size_t o_wi0 = b.reserve(witems[0].size() * sizeof(Item));
    const size_t o_wi1 = b.reserve(witems[1].size() * sizeof(Item));
    grow(ctx->poolB, ctx->sizeB, b.used + ALIGN);
    void *B = ctx->poolB;

    // ---- emit the wave's records, phase-major
    std::vector<unsigned long long> bb(win_n, ~0ull);
    std::vector<uint64_t> pos(be - bi);
    uint64_t p = 0;
    for (size_t j = bi; j < be; j++) {
        bb[big[j].k - win_lo] = p;
        pos[j - bi] = p;
        p += big[j].count;
    }
    upload(C.keep, at<void>(B, o_bb), bb, st);
    hipck(hipMemsetAsync(at<void>(B, o_cur), 0, win_n * 8, st));
    upload(C.keep, at<void>(B, o_wi0), witems[0], st);
    upload(C.keep, at<void>(B, o_wi1), witems[1], st);
    unsigned long long *in = at<unsigned long long>(B, o_ra), *out = at<unsigned long long>(B, o_rb);
    const size_t o_wi[2] = {o_wi0, o_wi1};
    for (int w = 0; w < 2; w++) {
        const Item *it = at<Item>(B, o_wi[w]);
        for (uint64_t s0 = 0; s0 < witems[w].size(); s0 += 1u << 30) {
            const uint32_t n = (uint32_t)std::min<uint64_t>(witems[w].size() - s0, 1u << 30);
            Prof pr(ctx, st, K_EMIT, w == 0 ? recs : 0, w == 0 ? recs * 8 : 0);
            hipck(launch_emit(it + s0, n, w == 1, at<NestDesc>(A, C.o_nests), at<ProtoDesc>(A, C.o_protos),
                              at<FixedVal>(A, C.o_fixed), at<uint32_t>(A, C.o_code), at<uint32_t>(A, C.o_itemcnt),
                              at<unsigned long long>(B, o_bb), at<unsigned long long>(B, o_cur), win_lo, win_n, in,
                              recs, st));
        }
    }

    auto run_groups = [&](const std::vector<Group> &groups, const unsigned long long *recbuf) {
        for (uint64_t g0 = 0; g0 < groups.size(); g0 += CAND_CAP) {
            const uint64_t n = std::min<uint64_t>(groups.size() - g0, CAND_CAP);
            std::vector<Group> part(groups.begin() + g0, groups.begin() + g0 + n);
            std::vector<SingleAcc> acc(n, SingleAcc{NONE32, NONE32, 0, NONE32});
            upload(C.keep, at<void>(B, o_groups), part, st);
            upload(C.keep, at<void>(B, o_acc), acc, st);
            uint64_t gl = 0;
            for (auto &g : part) gl += g.len;
            {
                Prof pr(ctx, st, K_SINGLE, gl, gl * 16);
                hipck(launch_single(at<Group>(B, o_groups), (uint32_t)n, recbuf, at<SingleAcc>(B, o_acc), cand, best,
                                    st));
            }
            {
                Prof pr(ctx, st, K_OTHER, 0, 0);
                hipck(launch_pick(cand, n, best, st));
            }
            hipck(hipStreamSynchronize(st));
            C.keep.clear();
        }
    };
    auto run_tiles = [&](const std::vector<Tile> &tiles, const unsigned long long *recbuf) {
        for (uint64_t t0 = 0; t0 < tiles.size(); t0 += CAND_CAP) {
            const uint64_t n = std::min<uint64_t>(tiles.size() - t0, CAND_CAP);
            std::vector<Tile> part(tiles.begin() + t0, tiles.begin() + t0 + n);
            upload(C.keep, at<void>(B, o_tiles), part, st);
            uint64_t tl = 0;
            for (auto &t : part) tl += t.len;
            {
                Prof pr(ctx, st, K_TILE, tl, tl * 8);
                hipck(launch_tiles(at<Tile>(B, o_tiles), (uint32_t)n, recbuf, cand, best, st));
            }
            {
                Prof pr(ctx, st, K_OTHER, 0, 0);
                hipck(launch_pick(cand, n, best, st));
            }
            if (t0 + CAND_CAP < tiles.size()) { hipck(hipStreamSynchronize(st)); C.keep.clear(); }
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
        sg.dbits = std::min<uint32_t>(8, r);
        sg.shift = r - sg.dbits;
        segs.push_back(sg);
    }
    if (!groups.empty()) run_groups(groups, in);

    unsigned long long *hist = at<unsigned long long>(B, o_hist);
    while (!segs.empty()) {
        std::vector<Chunk> chunks;
        std::vector<uint64_t> out_start(segs.size());
        uint64_t hb = 0, op = 0;
        for (size_t s2 = 0; s2 < segs.size(); s2++) {
            Seg &sg = segs[s2];
            sg.nchunks = (uint32_t)((sg.len + CHUNK - 1) / CHUNK);
            sg.hbase = hb;
            hb += (uint64_t)sg.nchunks << sg.dbits;
            out_start[s2] = op;
            op += sg.len;
            for (uint32_t c = 0; c < sg.nchunks; c++) chunks.push_back(Chunk{(uint32_t)s2, c});
        }
        upload(C.keep, at<void>(B, o_segs), segs, st);
        upload(C.keep, at<void>(B, o_chunks), chunks, st);
        const Seg *dsegs = at<Seg>(B, o_segs);
        const Chunk *dch = at<Chunk>(B, o_chunks);
        {
            Prof pr(ctx, st, K_HIST, op, op * 8);
            hipck(launch_hist(dsegs, dch, (uint32_t)chunks.size(), in, hist, st));
        }
        {
            Prof pr(ctx, st, K_SCAN, 0, hb * 16);
            hipck(launch_scan_u64(hist, hb, hist + hb, st));
        }
        {
            Prof pr(ctx, st, K_SCATTER, op, op * 16);
            hipck(launch_scatter(dsegs, dch, (uint32_t)chunks.size(), in, hist, out, recs, st));
        }
        {
            Prof pr(ctx, st, K_OTHER, 0, 0);
            hipck(launch_starts(dsegs, (uint32_t)segs.size(), hist, at<unsigned long long>(B, o_starts), st));
        }
        std::vector<uint64_t> starts(segs.size() * RADIX);
        hipck(hipMemcpyAsync(starts.data(), at<void>(B, o_starts), starts.size() * 8, hipMemcpyDeviceToHost, st));
        hipck(hipStreamSynchronize(st));
        C.keep.clear();

        std::vector<Seg> next;
        std::vector<Tile> tiles;
        std::vector<Group> g2;
        for (size_t s2 = 0; s2 < segs.size(); s2++) {
            const Seg &sg = segs[s2];
            const uint32_t nd = 1u << sg.dbits;
            // consecutive small buckets of one segment are contiguous and
            // hold disjoint index values: one tile takes several of them
            Tile cur{0, 0, sg.proto, sg.phase, 0};
            for (uint32_t d = 0; d < nd; d++) {
                const uint64_t a = starts[s2 * RADIX + d];
                const uint64_t e = (d + 1 < nd) ? starts[s2 * RADIX + d + 1] : out_start[s2] + sg.len;
                const uint64_t len = e - a;
                if (len == 0) continue;
                if (len <= (uint64_t)TILE) {
                    if (cur.len && cur.start + cur.len == a && cur.len + len <= (uint64_t)TILE) {
                        cur.len += (uint32_t)len;
                    } else {
                        if (cur.len) tiles.push_back(cur);
                        cur.start = a;
                        cur.len = (uint32_t)len;
                    }
                    continue;
                }
                if (cur.len) { tiles.push_back(cur); cur.len = 0; }
                if (sg.shift == 0) {
                    g2.push_back(Group{a, len, sg.proto, sg.phase});
                } else {
                    Seg ns{};
                    ns.start = a;
                    ns.len = len;
                    ns.proto = sg.proto;
                    ns.phase = sg.phase;
                    ns.dbits = std::min<uint32_t>(8, sg.shift);
                    ns.shift = sg.shift - ns.dbits;
                    next.push_back(ns);
                }
            }
            if (cur.len) tiles.push_back(cur);
        }
        run_tiles(tiles, out);
        if (!g2.empty()) run_groups(g2, out);
        segs.swap(next);
        std::swap(in, out);
        hipck(hipStreamSynchronize(st));
        C.keep.clear();
    }
}

int check_impl(drf_ctx *ctx, const uint32_t *code, const uint64_t *code_off, const uint32_t *nthreads,
               uint32_t count, drf_result *d_results, uint64_t *d_phase_counts, uint64_t phase_cap,
               hipStream_t st) {
    if (!ctx || !code_off || !nthreads || (count && (!code || !d_results))) return DRF_E_ARG;
    if (count == 0) return DRF_OK;
    Call C;
    C.ctx = ctx;
    C.st = st;
    C.count = count;
    try {
        hipck(hipSetDevice(ctx->device));
        if (ctx->done_valid) hipck(hipStreamWaitEvent(st, ctx->done, 0));
        C.plan_all(code, code_off, nthreads);
        C.build_blob();
        if (C.total_phases > phase_cap || (C.total_phases && !d_phase_counts)) return DRF_E_ARG;
        // upper bound on fused units: one per small phase at most
        C.layout_a(C.total_phases + 1);
        grow(ctx->poolA, ctx->sizeA, C.needA);
        void *A = ctx->poolA;
        unsigned long long *phase_counts = (unsigned long long *)d_phase_counts;
        Best *best = at<Best>(A, C.o_best);
        Cand *cand = at<Cand>(A, C.o_cand);
        uint32_t *ovf = at<uint32_t>(A, C.o_ovf);
        upload(C.keep, at<void>(A, C.o_protos), C.protos, st);
        upload(C.keep, at<void>(A, C.o_nests), C.nests, st);
        upload(C.keep, at<void>(A, C.o_fixed), C.fixed, st);
        upload(C.keep, at<void>(A, C.o_code), C.code, st);
        for (int w = 0; w < 2; w++) upload(C.keep, at<void>(A, C.o_items[w]), C.items[w], st);
        if (C.total_phases) hipck(hipMemsetAsync(phase_counts, 0, C.total_phases * sizeof(uint64_t), st));
        hipck(hipMemsetAsync(ovf, 0, count * sizeof(uint32_t), st));
        hipck(hipMemsetAsync(best, 0xFF, count * sizeof(Best), st));
        const ProtoDesc *dprotos = at<ProtoDesc>(A, C.o_protos);
        const NestDesc *dnests = at<NestDesc>(A, C.o_nests);
        const FixedVal *dfixed = at<FixedVal>(A, C.o_fixed);
        const uint32_t *dcode = at<uint32_t>(A, C.o_code);
        uint32_t *item_cnt = at<uint32_t>(A, C.o_itemcnt);

        // ---- count pass
        for (int w = 0; w < 2; w++) {
            const Item *it = at<Item>(A, C.o_items[w]);
            for (uint64_t b = 0; b < C.items[w].size(); b += 1u << 30) {
                uint32_t n = (uint32_t)std::min<uint64_t>(C.items[w].size() - b, 1u << 30);
                Prof pr(ctx, st, K_COUNT, 0, 0);
                hipck(launch_count(it + b, n, w == 1, dnests, dprotos, dfixed, dcode, phase_counts, item_cnt, ovf, st));
            }
        }
        std::vector<uint64_t> counts(C.total_phases);
        std::vector<uint32_t> hovf(count);
        if (C.total_phases)
            hipck(hipMemcpyAsync(counts.data(), phase_counts, C.total_phases * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
        hipck(hipMemcpyAsync(hovf.data(), ovf, count * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        hipck(hipStreamSynchronize(st));
        C.keep.clear();

        // ---- classification
        std::vector<uint64_t> nrec(count, 0);
        std::vector<Unit> units[2];
        std::vector<BigPhase> big;
        for (uint32_t i = 0; i < count; i++) {
            if (C.status[i]) continue;
            if (hovf[i]) { C.status[i] = DRF_E_RANGE; continue; }
            const ProtoDesc &pd = C.protos[i];
            uint64_t acc = 0, ustart = ~0ull, last_small = 0;
            for (uint64_t k = pd.phase_off; k < pd.phase_off + pd.nphases; k++) {
                const uint64_t c = counts[k];
                nrec[i] += c;
                if (c == 0) continue;
                if (c > (uint64_t)TILE) {
                    big.push_back(BigPhase{k, c, i, (uint32_t)(k - pd.phase_off)});
                    continue;
                }
                if (ustart == ~0ull) ustart = k;
                last_small = k;
                acc += c;
                if (acc >= UNIT_EVENTS) {
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
            for (auto &p : ctx->pending) if (p.cls == K_COUNT) { p.records = tot; break; }
        }

        // ---- fused path
        for (int w = 0; w < 2; w++) {
            for (uint64_t b = 0; b < units[w].size(); b += CAND_CAP) {
                const uint64_t n = std::min<uint64_t>(units[w].size() - b, CAND_CAP);
                std::vector<Unit> part(units[w].begin() + b, units[w].begin() + b + n);
                upload(C.keep, at<void>(A, C.o_units), part, st);
                uint64_t ev = 0;
                for (uint64_t u = b; u < b + n; u++)
                    for (uint64_t k = units[w][u].k0; k < units[w][u].k1; k++)
                        if (counts[k] <= (uint64_t)TILE) ev += counts[k];
                {
                    Prof pr(ctx, st, K_FUSED, ev, 0);
                    hipck(launch_fused(at<Unit>(A, C.o_units), (uint32_t)n, w == 1, dnests, dprotos, dfixed, dcode,
                                       phase_counts, cand, best, st));
                }
                {
                    Prof pr(ctx, st, K_OTHER, 0, 0);
                    hipck(launch_pick(cand, n, best, st));
                }
                if (b + CAND_CAP < units[w].size()) { hipck(hipStreamSynchronize(st)); C.keep.clear(); }
            }
        }

        // ---- big phases, in waves under the scratch budget
        if (!big.empty()) {
            const uint64_t budget = ctx->limit > C.needA ? ctx->limit - C.needA : 0;
            const uint64_t per_rec = 20;   // two record buffers + partition metadata
            const uint64_t rec_cap = budget / per_rec;
            size_t bi = 0;
            while (bi < big.size()) {
                // skip phases that can never fit
                if (big[bi].count > rec_cap) {
                    C.status[big[bi].proto] = DRF_E_NOMEM;
                    bi++;
                    continue;
                }
                size_t be = bi;
                uint64_t recs = 0;
                while (be < big.size() && big[be].count <= rec_cap && recs + big[be].count <= rec_cap &&
                       big[be].k - big[bi].k < (1ull << 26)) {
                    recs += big[be].count;
                    be++;
                }
                run_wave(C, big, bi, be, recs, best, cand);
                bi = be;
            }
        }

        // ---- results
        std::vector<ResultIn> rin(count);
        for (uint32_t i = 0; i < count; i++) {
            rin[i].status = C.status[i];
            rin[i].num_phases = C.status[i] ? 0 : (uint32_t)C.protos[i].nphases;
            rin[i].num_records = C.status[i] ? 0 : nrec[i];
        }
        upload(C.keep, at<void>(A, C.o_rin), rin, st);
        {
            Prof pr(ctx, st, K_OTHER, 0, 0);
            hipck(launch_result(count, at<ResultIn>(A, C.o_rin), best, (drf_result_dev *)d_results, st));
        }
        if (!ctx->done) hipck(hipEventCreateWithFlags(&ctx->done, hipEventDisableTiming));
        hipck(hipEventRecord(ctx->done, st));
        ctx->done_valid = true;
        // pageable uploads are staged synchronously; the last ones must
        // still be complete before the host copies go away
        hipck(hipStreamSynchronize(st));
        prof_collect(ctx);
        return DRF_OK;
    } catch (Fail f) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(st);
        return f.code;
    } catch (...) {
        (void)hipStreamSynchronize(st);
        return DRF_E_NOMEM;
    }
}

}  // namespace

// ================================================================ C ABI
extern "C" {

const char *drf_version(void) { return "libdrf 0.1 (gfx950)"; }

int drf_compile_text(const char *text, size_t len, uint32_t *out, uint32_t cap, uint32_t *nwords) {
    if (!text || !nwords) return DRF_E_ARG;
    std::vector<uint32_t> w;
    int rc = compile_text(text, len, w);
    if (rc) return rc;
    *nwords = (uint32_t)w.size();
    if (w.size() > cap || !out) return DRF_E_NOMEM;
    memcpy(out, w.data(), w.size() * sizeof(uint32_t));
    return DRF_OK;
}

int drf_plan_protocol(const uint32_t *code, uint32_t words, uint32_t num_threads, drf_plan *out) {
    if (!out) return DRF_E_ARG;
    Plan p;
    plan_protocol(code, words, num_threads, p);
    memset(out, 0, sizeof *out);
    out->status = p.status;
    if (!p.status) {
        out->num_phases = (uint32_t)p.num_phases;
        out->index_bits = p.index_bits;
        out->wide = p.wide ? 1 : 0;
        out->max_records = p.max_records;
        out->nests = p.nests.size();
    }
    return DRF_OK;
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
    drf_ctx *c = new drf_ctx();
    c->device = hip_device;
    if (scratch_limit_bytes == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) { delete c; return DRF_E_HIP; }
        scratch_limit_bytes = fr / 4 * 3;
    }
    c->limit = scratch_limit_bytes;
    *out = c;
    return DRF_OK;
}

int drf_ctx_destroy(drf_ctx *ctx) {
    if (!ctx) return DRF_E_ARG;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->poolA) (void)hipFree(ctx->poolA);
    if (ctx->poolB) (void)hipFree(ctx->poolB);
    if (ctx->done) (void)hipEventDestroy(ctx->done);
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

int drf_ctx_kernel_stats(drf_ctx *ctx, drf_kernel_stat *out, uint32_t cap, uint32_t *n, int reset) {
    if (!ctx || !n) return DRF_E_ARG;
    *n = K_NCLASS;
    for (uint32_t i = 0; i < K_NCLASS && i < cap && out; i++) {
        out[i] = ctx->stats[i];
        snprintf(out[i].name, sizeof out[i].name, "%s", KNAMES[i]);
    }
    if (reset) memset(ctx->stats, 0, sizeof ctx->stats);
    return DRF_OK;
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

}  // extern "C"
