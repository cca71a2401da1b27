// gfx950 kernels of libdrf.
//
// Evaluation.  One lane per thread id of the checked protocol; all lanes of
// a wave execute the same leaf-code instruction (the opcode is read with
// readfirstlane, so dispatch is a scalar branch) and carry per-lane
// activity for if / for^U (bit stacks of saved activity and conditions).
// This is rule par of the paper's semantics: every thread runs the leaf
// independently; lanes that took the other branch simply stay inactive.
// for^S loops are not interpreted at all: the planner turned them into an
// odometer over symbolic loop digits with an affine phase map.
//
// Conflict detection.  Records are u64: index << 32 | tid << 1 | is_write.
// Within one phase, sorting records groups equal indices and orders each
// group by tid.  A group (phase, index) is racy iff some record writes and
// two distinct tids occur (Definition 1); its least pair (tid_i < tid_j)
// with a writer is (t0, t1) when the least tid t0 writes, else (t0, w0)
// with w0 the least writing tid.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "kernels.hpp"

namespace drf {

#define DEV __device__ __forceinline__

DEV uint32_t rfl(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
DEV uint64_t rfl64(uint64_t x) {
    return ((uint64_t)rfl((uint32_t)(x >> 32)) << 32) | (uint64_t)rfl((uint32_t)x);
}
DEV uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }
DEV uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
DEV uint64_t ballot(bool p) { return __ballot(p); }
DEV uint32_t readlane(uint32_t v, uint32_t l) { return __builtin_amdgcn_readlane(v, l); }

// ------------------------------------------------------------ expressions
template <typename T, bool WIDE>
DEV T ovf_add(T a, T b, bool &o) {
    T r = a + b;
    if constexpr (WIDE) o |= (r >> 63) != 0;
    return r;
}
template <typename T, bool WIDE>
DEV T ovf_mul(T a, T b, bool &o) {
    T r = a * b;
    if constexpr (WIDE) o |= (__umul64hi(a, b) != 0) || ((r >> 63) != 0);
    return r;
}

template <typename T, bool WIDE>
DEV T eval_expr(const uint32_t *__restrict__ c, uint32_t len, const T *vars, T tid, bool &o) {
    T st[MAXSTACK];
    uint32_t sp = 0;
    uint32_t i = 0;
    while (i < len) {
        const uint32_t op = rfl(c[i]);
        if (op == X_CONST) {
            T v;
            if constexpr (WIDE) {
                v = ((uint64_t)rfl(c[i + 2]) << 32) | (uint64_t)rfl(c[i + 1]);
                o |= (v >> 63) != 0;
            } else {
                v = rfl(c[i + 1]);
            }
            st[sp++] = v;
            i += 3;
        } else if (op == X_TID) {
            st[sp++] = tid;
            i += 1;
        } else if (op == X_VAR) {
            st[sp++] = vars[rfl(c[i + 1])];
            i += 2;
        } else if (op >= X_ADDC && op <= X_SHRC) {
            const T k = (T)rfl(c[i + 1]);
            const T a = st[sp - 1];
            T r;
            switch (op) {
            case X_ADDC: r = ovf_add<T, WIDE>(a, k, o); break;
            case X_MULC: r = ovf_mul<T, WIDE>(a, k, o); break;
            case X_DIVC: r = a / k; break;
            case X_MODC: r = a % k; break;
            case X_ANDC: r = a & k; break;
            default: r = a >> k; break;   // X_SHRC
            }
            st[sp - 1] = r;
            i += 2;
        } else if (op == X_AFF) {
            // c0 + sum coef * var (var NONE32 = tid); multipliers below 2^32
            const uint32_t nt = rfl(c[i + 1]);
            T acc;
            if constexpr (WIDE) {
                acc = ((uint64_t)rfl(c[i + 3]) << 32) | (uint64_t)rfl(c[i + 2]);
            } else {
                acc = rfl(c[i + 2]);
            }
            for (uint32_t t = 0; t < nt; t++) {
                const uint32_t v = rfl(c[i + 4 + 2 * t]);
                const T k = (T)rfl(c[i + 5 + 2 * t]);
                const uint32_t vi = (v == NONE32) ? 0u : v;
                const T x = (v == NONE32) ? tid : vars[vi];
                if constexpr (WIDE) {
                    const T p = x * k;
                    o |= (__umul64hi(x, k) != 0) || ((p >> 63) != 0);
                    acc += p;
                    o |= (acc >> 63) != 0;
                } else {
                    acc += x * k;
                }
            }
            st[sp++] = acc;
            i += 4 + 2 * nt;
        } else if (op == X_TRUE || op == X_FALSE) {
            st[sp++] = (op == X_TRUE) ? 1 : 0;
            i += 1;
        } else if (op == X_NOT) {
            st[sp - 1] = st[sp - 1] ? 0 : 1;
            i += 1;
        } else {
            const T b = st[--sp];
            const T a = st[sp - 1];
            T r;
            switch (op) {
            case X_ADD: r = ovf_add<T, WIDE>(a, b, o); break;
            case X_MONUS: r = a > b ? a - b : 0; break;
            case X_MUL: r = ovf_mul<T, WIDE>(a, b, o); break;
            case X_DIV: r = b ? a / b : 0; break;
            case X_MOD: r = b ? a % b : a; break;
            case X_SHL:
                if constexpr (WIDE) {
                    if (a == 0) r = 0;
                    else if (b >= 63) { o = true; r = 0; }
                    else { r = a << b; o |= ((r >> b) != a) || ((r >> 63) != 0); }
                } else {
                    r = b >= 32 ? 0 : a << b;
                }
                break;
            case X_SHR: r = b >= (T)(8 * sizeof(T)) ? 0 : a >> b; break;
            case X_MIN: r = a < b ? a : b; break;
            case X_MAX: r = a > b ? a : b; break;
            case X_LT: r = a < b; break;
            case X_LE: r = a <= b; break;
            case X_EQ: r = a == b; break;
            case X_NE: r = a != b; break;
            case X_GT: r = a > b; break;
            case X_GE: r = a >= b; break;
            case X_AND: r = (a && b) ? 1 : 0; break;
            default: r = (a || b) ? 1 : 0; break;   // X_OR
            }
            st[sp - 1] = r;
            i += 1;
        }
    }
    return st[0];
}

// --------------------------------------------------------------- leaf code
// Runs one unsynchronized leaf for this lane's thread id.  sink.acc(active,
// index, mode) is called by all lanes of the wave at every access.
template <typename T, bool WIDE, typename Sink>
DEV void run_leaf(const uint32_t *__restrict__ code, T *vars, T tid, bool act0, bool &ovf, Sink &sink) {
    T his[MAXSLOTS];
    uint32_t msave = 0, mcond = 0;
    bool act = act0;
    uint32_t pc = 0;
    for (;;) {
        const uint32_t op = rfl(code[pc]);
        if (op == U_ACC) {
            const uint32_t mode = rfl(code[pc + 1]);
            const uint32_t len = rfl(code[pc + 2]);
            bool o = false;
            const T v = eval_expr<T, WIDE>(code + pc + 3, len, vars, tid, o);
            if constexpr (WIDE) {
                o |= (v >> 32) != 0;
                ovf |= act && o;
            }
            sink.acc(act, (uint32_t)v, mode);
            pc += 3 + len;
        } else if (op == U_IF) {
            const uint32_t len = rfl(code[pc + 1]);
            bool o = false;
            const T c = eval_expr<T, WIDE>(code + pc + 2, len, vars, tid, o);
            if constexpr (WIDE) ovf |= act && o;
            const bool cv = c != 0;
            msave = (msave << 1) | (act ? 1u : 0u);
            mcond = (mcond << 1) | (cv ? 1u : 0u);
            act = act && cv;
            pc = __any(act) ? pc + 3 + len : rfl(code[pc + 2 + len]);
        } else if (op == U_ELSE) {
            act = (msave & 1u) && !(mcond & 1u);
            pc = __any(act) ? pc + 2 : rfl(code[pc + 1]);
        } else if (op == U_ENDIF) {
            act = (msave & 1u) != 0;
            msave >>= 1;
            mcond >>= 1;
            pc += 1;
        } else if (op == U_FOR) {
            const uint32_t slot = rfl(code[pc + 1]);
            const uint32_t ll = rfl(code[pc + 2]);
            bool o = false;
            const T lo = eval_expr<T, WIDE>(code + pc + 3, ll, vars, tid, o);
            const uint32_t hl = rfl(code[pc + 3 + ll]);
            const T hi = eval_expr<T, WIDE>(code + pc + 4 + ll, hl, vars, tid, o);
            if constexpr (WIDE) ovf |= act && o;
            const uint32_t end_pc = rfl(code[pc + 4 + ll + hl]);
            vars[slot] = lo;
            his[slot] = hi;
            msave = (msave << 1) | (act ? 1u : 0u);
            act = act && (lo < hi);
            if (__any(act)) {
                pc = pc + 5 + ll + hl;
            } else {
                act = (msave & 1u) != 0;
                msave >>= 1;
                pc = end_pc;
            }
        } else if (op == U_ENDFOR) {
            const uint32_t slot = rfl(code[pc + 1]);
            const T x = vars[slot] + 1;
            vars[slot] = x;
            act = (msave & 1u) && (x < his[slot]);
            if (__any(act)) {
                pc = rfl(code[pc + 2]);
            } else {
                act = (msave & 1u) != 0;
                msave >>= 1;
                pc += 3;
            }
        } else {
            break;   // U_END
        }
    }
}

// --------------------------------------------------- nest iteration state
// Symbolic for^S loops of a nest as an odometer of digits (loop 0 outermost).
// The loops are unrolled to MAXLOOPS so the digits stay in registers.
template <typename T>
struct Odo {
    uint32_t nloops;
    uint64_t digit[MAXLOOPS];
    uint64_t phase;

    DEV void start(const NestDesc &nd, uint64_t f, T *vars) {
        nloops = nd.nloops;
        phase = nd.phase_base;
        const bool narrow = nd.iters <= 0xFFFFFFFFull;   // every trip and f fit 32 bits
        uint64_t rem = f;
#pragma unroll
        for (int l = MAXLOOPS - 1; l >= 0; l--) {
            digit[l] = 0;
            if (l < (int)nloops) {
                const uint64_t t = nd.trip[l];
                uint64_t d;
                if (narrow) {
                    const uint32_t r32 = (uint32_t)rem, t32 = (uint32_t)t;
                    d = r32 % t32;
                    rem = r32 / t32;
                } else {
                    d = rem % t;
                    rem /= t;
                }
                digit[l] = d;
                vars[nd.slot[l]] = (T)(nd.lo[l] + d);
                phase += d * nd.stride[l];
            }
        }
    }
    DEV void next(const NestDesc &nd, T *vars) {
        bool carry = true;
#pragma unroll
        for (int l = MAXLOOPS - 1; l >= 0; l--) {
            if (carry && l < (int)nloops) {
                const uint64_t d = digit[l] + 1;
                phase += nd.stride[l];
                if (d < nd.trip[l]) {
                    digit[l] = d;
                    vars[nd.slot[l]] = (T)(nd.lo[l] + d);
                    carry = false;
                } else {
                    phase -= nd.trip[l] * nd.stride[l];
                    digit[l] = 0;
                    vars[nd.slot[l]] = (T)nd.lo[l];
                }
            }
        }
    }
};

template <typename T>
DEV void load_fixed(const NestDesc &nd, const FixedVal *__restrict__ fixed, T *vars) {
    for (uint32_t i = 0; i < nd.nfixed; i++) {
        const FixedVal fv = fixed[nd.fixed_off + i];
        vars[rfl(fv.slot)] = (T)rfl64(fv.value);
    }
}

// Tids that can access memory in the current iteration: [0, limit).
template <typename T>
DEV uint32_t tid_limit(const NestDesc &nd, const uint32_t *__restrict__ code, const T *vars, uint32_t n) {
    if (nd.guard_off == NONE32) return n;
    bool o = false;
    const uint32_t *g = code + nd.guard_off;
    const T e = eval_expr<T, false>(g + 1, rfl(g[0]), vars, (T)0, o);
    return (uint64_t)e < (uint64_t)n ? (uint32_t)e : n;
}

// Phase of iteration f (digits decoded from scratch).
DEV uint64_t phase_of(const NestDesc &nd, uint64_t f) {
    uint64_t ph = nd.phase_base, rem = f;
    if (nd.iters <= 0xFFFFFFFFull) {
        uint32_t r32 = (uint32_t)rem;
        for (int l = (int)nd.nloops - 1; l >= 0; l--) {
            const uint32_t t32 = (uint32_t)nd.trip[l];
            ph += (uint64_t)(r32 % t32) * nd.stride[l];
            r32 /= t32;
        }
        return ph;
    }
    for (int l = (int)nd.nloops - 1; l >= 0; l--) {
        ph += (rem % nd.trip[l]) * nd.stride[l];
        rem /= nd.trip[l];
    }
    return ph;
}

// First iteration whose phase is >= k (phases are non-decreasing in f).
// First iteration of the nest whose phase is at least k (iters if none).
// One iteration of loop l runs every iteration of the loops inside it, so
// its stride is at least the phases those can add (rem below) and the
// phase map is monotone: digits are chosen outermost first, each the least
// that still lets the inner loops reach k.
DEV uint64_t first_iter_at(const NestDesc &nd, uint64_t k) {
    if (k <= nd.phase_base) return 0;
    if (k > nd.phase_last) return nd.iters;
    uint64_t rem = 0;
    for (uint32_t l = 0; l < nd.nloops; l++) rem += (nd.trip[l] - 1) * nd.stride[l];
    uint64_t p = nd.phase_base, f = 0;
    for (uint32_t l = 0; l < nd.nloops; l++) {
        rem -= (nd.trip[l] - 1) * nd.stride[l];   // what the loops inside l can add
        uint64_t d = 0;
        if (nd.stride[l] && p + rem < k) {
            d = (k - p - rem + nd.stride[l] - 1) / nd.stride[l];
            if (d > nd.trip[l] - 1) d = nd.trip[l] - 1;
        }
        p += d * nd.stride[l];
        f = f * nd.trip[l] + d;
    }
    return f;
}

// ============================================================= count pass
// Compiled leaf: every lane below the thread limit performs every access
// once per iteration, so one lane per iteration finds the counts.
template <typename T>
DEV void count_cal(const Item &it, const NestDesc &nd, const ProtoDesc &pd, const FixedVal *__restrict__ fixed,
                   const uint32_t *__restrict__ code, uint32_t *lds_cnt) {
    const uint32_t nacc = rfl(code[nd.cal_off]);
    const uint64_t nit = it.f1 - it.f0;
    for (uint64_t q = threadIdx.x; q < nit; q += WG) {
        T vars[MAXSLOTS];
        for (int z = 0; z < MAXSLOTS; z++) vars[z] = 0;
        load_fixed<T>(nd, fixed, vars);
        Odo<T> odo;
        odo.start(nd, it.f0 + q, vars);
        const uint32_t lim = tid_limit<T>(nd, code, vars, pd.n);
        const uint32_t tids = it.nblk * (uint32_t)WG;   // the item's tids, all blocks
        const uint32_t na = lim > it.tid0 ? (lim - it.tid0 < tids ? lim - it.tid0 : tids) : 0u;
        if (na) atomicAdd(&lds_cnt[odo.phase - it.k_lo], nacc * na);
    }
}

struct CountSink {
    uint32_t n;   // wave-uniform running count of the current phase
    DEV void acc(bool act, uint32_t, uint32_t) { n += __builtin_popcountll(ballot(act)); }
};

template <typename T, bool WIDE>
__global__ __launch_bounds__(WG) void k_count(const Item *__restrict__ items, const NestDesc *__restrict__ nests,
                                               const ProtoDesc *__restrict__ protos,
                                               const FixedVal *__restrict__ fixed, const uint32_t *__restrict__ code,
                                               unsigned long long *__restrict__ phase_counts,
                                               uint32_t *__restrict__ item_cnt, uint32_t *__restrict__ proto_ovf) {
    __shared__ uint32_t lds_cnt[MAXSPAN];
    const Item it = items[blockIdx.x];
    const NestDesc &nd = nests[it.nest];
    const ProtoDesc pd = protos[nd.proto];
    const uint32_t span = it.span;
    for (uint32_t i = threadIdx.x; i < span; i += WG) lds_cnt[i] = 0;
    __syncthreads();

    bool compiled = false;
    if constexpr (!WIDE) compiled = nd.cal_off != NONE32;
    if (compiled) {
        count_cal<T>(it, nd, pd, fixed, code, lds_cnt);
    } else {
        bool ovf = false;
        for (uint32_t blk = 0; blk < it.nblk; blk++) {
            const uint32_t tid0 = it.tid0 + blk * (uint32_t)WG;
            T vars[MAXSLOTS];
            for (int s = 0; s < MAXSLOTS; s++) vars[s] = 0;
            load_fixed<T>(nd, fixed, vars);
            Odo<T> odo;
            odo.start(nd, it.f0, vars);
            const uint32_t tid = tid0 + threadIdx.x;
            const bool act0 = tid < pd.n;
            const uint32_t *leaf = code + nd.code_off;
            CountSink sink{0};
            uint64_t cur = odo.phase;
            for (uint64_t f = it.f0; f < it.f1; f++) {
                if (odo.phase != cur) {
                    if (lane_id() == 0 && sink.n) atomicAdd(&lds_cnt[cur - it.k_lo], sink.n);
                    sink.n = 0;
                    cur = odo.phase;
                }
                // leaf loops never write for^S slots (binders are distinct)
                if (tid0 < tid_limit<T>(nd, code, vars, pd.n)) run_leaf<T, WIDE>(leaf, vars, (T)tid, act0, ovf, sink);
                odo.next(nd, vars);
            }
            if (lane_id() == 0 && sink.n) atomicAdd(&lds_cnt[cur - it.k_lo], sink.n);
        }
        if (ballot(ovf) != 0 && lane_id() == 0) atomicOr(&proto_ovf[nd.proto], 1u);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < span; i += WG) {
        const uint32_t c = lds_cnt[i];
        item_cnt[it.cnt_off + i] = c;
        if (c) atomicAdd(&phase_counts[it.k_lo + i], (unsigned long long)c);
    }
}

// ============================================================== emit pass
struct EmitSink {
    uint32_t *cur;              // LDS cursor of the current phase
    unsigned long long base;    // record position of this item's share of the phase
    unsigned long long *recs;
    unsigned long long cap;     // records the buffer holds
    uint32_t tid;
    DEV void acc(bool act, uint32_t idx, uint32_t mode) {
        const uint64_t m = ballot(act);
        if (m == 0) return;
        uint32_t off = 0;
        if (lane_id() == 0) off = atomicAdd(cur, (uint32_t)__builtin_popcountll(m));
        off = __shfl(off, 0);
        const unsigned long long pos = base + off + mbcnt(m);
        if (act && pos < cap) recs[pos] = ((unsigned long long)idx << 32) | ((unsigned long long)tid << 1) | mode;
    }
};

// Table path of a big phase: each access event updates its cell of the
// phase's table in device memory (least tid, second least tid, least
// writing tid; three arrays of 2^index_bits words at `tab`), with the same
// one-pass rule as the LDS aggregation: atomicMin on the least tid returns
// the minimum before it, and the larger of two different tids is offered to
// the second least.
DEV void table_update(uint32_t *tab, uint32_t cells, uint32_t idx, uint32_t tid, bool wr) {
    const uint32_t old = atomicMin(tab + idx, tid);
    if (old != NONE32 && old != tid) atomicMin(tab + cells + idx, old > tid ? old : tid);
    if (wr) atomicMin(tab + 2 * cells + idx, tid);
}

struct TableSink {
    uint32_t *tab;              // the current phase's table
    uint32_t cells;
    uint32_t tid;
    DEV void acc(bool act, uint32_t idx, uint32_t mode) {
        if (act) table_update(tab, cells, idx, tid, (mode & 1u) != 0);
    }
};

// Compiled leaf: per chunk of iterations the workgroup first evaluates the
// uniform slots (slot-major, iterations padded to whole waves so every wave
// runs one slot program), the phase and the thread limit of each iteration
// into LDS; then each lane runs its access chains.
constexpr uint32_t CAL_U = 2048;    // staged uniform values per chunk
constexpr uint32_t CAL_CH = 256;    // iterations per chunk

// Runs the chain of one compiled access on tid; uniform slot z reads
// U[z * ustride].
DEV uint32_t cal_chain(const uint32_t *__restrict__ ap, uint32_t nops, uint32_t tid, const uint32_t *U,
                       uint32_t ustride) {
    uint32_t v = tid;
    for (uint32_t o = 0; o < nops; o++) {
        const uint32_t opw = rfl(ap[2 * o]), arg = rfl(ap[2 * o + 1]);
        const uint32_t x = (opw & C_UNI) ? rfl(U[arg * ustride]) : arg;
        switch (opw & 0xFFu) {
        case C_ADD: v += x; break;
        case C_MUL: v *= x; break;
        case C_MONUS: v = v > x ? v - x : 0u; break;
        case C_RMONUS: v = x > v ? x - v : 0u; break;
        case C_DIV: v = x ? v / x : 0u; break;
        case C_MOD: v = x ? v % x : v; break;
        case C_SHL: v = x >= 32u ? 0u : v << x; break;
        case C_SHR: v = x >= 32u ? 0u : v >> x; break;
        case C_MIN: v = v < x ? v : x; break;
        case C_MAX: v = v > x ? v : x; break;
        default: v &= x; break;   // C_AND
        }
    }
    return v;
}

// One modulus step of a compiled access's fixed form: v & d, v mod d (the
// quotient by the stored division magic of d >= 1, then the remainder) or
// v unchanged.
DEV uint32_t fixed_op(uint32_t v, uint32_t kind, uint32_t d, uint32_t mag, uint32_t sh) {
    if (kind == CAL_K_AND) return v & d;
    if (kind == CAL_K_MOD) {
        const uint32_t t = __umulhi(mag, v);
        const uint32_t q = (t + ((v - t) >> (sh & 0xFFu))) >> (sh >> 8);
        return v - q * d;
    }
    return v;
}

// Index of one compiled access (block at ap) for tid: the fixed form with
// its parameters read once, else the chain.
DEV uint32_t cal_index(const uint32_t *__restrict__ ap, uint32_t tid, const uint32_t *U, uint32_t ustride) {
    if (rfl(ap[1]) == 1u) {
        const uint32_t c0 = rfl(ap[2]), m0k = rfl(ap[3]), m0 = rfl(ap[4]), a = rfl(ap[5]), us = rfl(ap[6]);
        const uint32_t pk = rfl(ap[7]), pa = rfl(ap[8]);
        uint32_t v = fixed_op(tid + c0, m0k, m0, rfl(ap[9]), rfl(ap[10])) * a;
        if (us != NONE32) v += rfl(U[us * ustride]);
        return fixed_op(v, pk, pa, rfl(ap[11]), rfl(ap[12]));
    }
    return cal_chain(ap + CAL_HDR, rfl(ap[CAL_HDR - 1]), tid, U, ustride);
}

// A compiled access's header read once (uniform), for several iterations.
struct CalHdr {
    uint32_t mode, form, c0, m0k, m0, a, us, pk, pa, m0mag, m0sh, pamag, pash, nops;
    const uint32_t *ops;
};
DEV CalHdr cal_hdr(const uint32_t *__restrict__ ap) {
    CalHdr h;
    h.mode = rfl(ap[0]);
    h.form = rfl(ap[1]);
    h.c0 = rfl(ap[2]);
    h.m0k = rfl(ap[3]);
    h.m0 = rfl(ap[4]);
    h.a = rfl(ap[5]);
    h.us = rfl(ap[6]);
    h.pk = rfl(ap[7]);
    h.pa = rfl(ap[8]);
    h.m0mag = rfl(ap[9]);
    h.m0sh = rfl(ap[10]);
    h.pamag = rfl(ap[11]);
    h.pash = rfl(ap[12]);
    h.nops = rfl(ap[CAL_HDR - 1]);
    h.ops = ap + CAL_HDR;
    return h;
}
DEV uint32_t cal_eval(const CalHdr &h, uint32_t tid, const uint32_t *U, uint32_t ustride) {
    if (h.form == 1u) {
        uint32_t v = fixed_op(tid + h.c0, h.m0k, h.m0, h.m0mag, h.m0sh) * h.a;
        if (h.us != NONE32) v += rfl(U[h.us * ustride]);
        return fixed_op(v, h.pk, h.pa, h.pamag, h.pash);
    }
    return cal_chain(h.ops, h.nops, tid, U, ustride);
}

struct CalLds {
    uint32_t u[CAL_U];
    uint32_t ph[CAL_CH];
    uint32_t lim[CAL_CH];
    uint32_t uoff[CAL_MAXU + 1];
};

// TABLE: lds_base holds each phase's table offset (in words from recs as
// uint32_t*) instead of its record position; events update the tables.
template <typename T, bool TABLE>
DEV void emit_cal(const Item &it, const NestDesc &nd, const ProtoDesc &pd, const FixedVal *__restrict__ fixed,
                  const uint32_t *__restrict__ code, const unsigned long long *lds_base, uint32_t *lds_cur,
                  unsigned long long *__restrict__ recs, unsigned long long cap, CalLds &L) {
    const uint32_t *cal = code + nd.cal_off;
    const uint32_t nacc = rfl(cal[0]), nuni = rfl(cal[1]);
    if (threadIdx.x == 0) {
        uint32_t o = 3;
        for (uint32_t z = 0; z < nuni; z++) {
            L.uoff[z] = o;
            o += 1 + cal[o];
        }
        L.uoff[CAL_MAXU] = cal[2];
    }
    __syncthreads();
    const uint32_t *acc0 = cal + rfl(L.uoff[CAL_MAXU]);
    const uint32_t nu = nuni ? nuni : 1u;
    static_assert(CAL_U / CAL_MAXU >= 64, "a chunk must hold one wave of iterations");
    const uint32_t chmax = (CAL_U / nu) / 64 * 64 < CAL_CH ? (CAL_U / nu) / 64 * 64 : CAL_CH;   // >= 64
    for (uint64_t fc = it.f0; fc < it.f1; fc += chmax) {
        const uint32_t ch = (uint32_t)(it.f1 - fc < chmax ? it.f1 - fc : chmax);
        const uint32_t chp = (ch + 63) & ~63u;
        for (uint32_t q = threadIdx.x; q < chp * nu; q += WG) {
            const uint32_t z = rfl(q / chp), fi = q - z * chp;   // slot is uniform per wave
            if (fi >= ch) continue;
            T vars[MAXSLOTS];
            for (int y = 0; y < MAXSLOTS; y++) vars[y] = 0;
            load_fixed<T>(nd, fixed, vars);
            Odo<T> odo;
            odo.start(nd, fc + fi, vars);
            if (z == 0) {
                L.ph[fi] = (uint32_t)(odo.phase - it.k_lo);
                L.lim[fi] = tid_limit<T>(nd, code, vars, pd.n);
            }
            if (z < nuni) {
                bool o = false;
                const uint32_t *up = cal + rfl(L.uoff[z]);
                L.u[q] = (uint32_t)eval_expr<T, false>(up + 1, rfl(up[0]), vars, (T)0, o);
            }
        }
        __syncthreads();
        // the item's tid blocks reuse the chunk's staging; EB iterations at
        // a time: their reservations are issued together and each access
        // header is read once for all of them (eight measured best)
        constexpr uint32_t EB = 8;
        for (uint32_t blk = 0; blk < it.nblk; blk++) {
            const uint32_t tid0 = it.tid0 + blk * (uint32_t)WG;
            const uint32_t tid = tid0 + threadIdx.x;
            const bool act0 = tid < pd.n;
            for (uint32_t i0 = 0; i0 < ch; i0 += EB) {
                unsigned long long p0[EB];
                uint32_t na[EB];
                bool go[EB], act[EB];
#pragma unroll
                for (uint32_t q = 0; q < EB; q++) {
                    const uint32_t i = i0 + q;
                    go[q] = false;
                    act[q] = false;
                    na[q] = 0;
                    p0[q] = 0;
                    if (i >= ch) continue;
                    const uint32_t pi = rfl(L.ph[i]);
                    const unsigned long long b = lds_base[pi];
                    const uint32_t lim = rfl(L.lim[i]);
                    if (b == ~0ull || tid0 >= lim) continue;
                    // a compiled leaf has no branches: the wave's active lanes are
                    // the same for every access of the iteration, so one
                    // reservation covers all of them (access j, lane l at
                    // r0 + j * na + rank of l)
                    act[q] = act0 && tid < lim;
                    const uint64_t m = ballot(act[q]);
                    if (m == 0) continue;
                    go[q] = true;
                    if constexpr (TABLE) {
                        p0[q] = b;
                        continue;
                    }
                    na[q] = (uint32_t)__builtin_popcountll(m);
                    uint32_t r0 = 0;
                    if (lane_id() == 0) r0 = atomicAdd(&lds_cur[pi], na[q] * nacc);
                    p0[q] = b + readlane(r0, 0) + mbcnt(m);
                }
                bool any = false;
#pragma unroll
                for (uint32_t q = 0; q < EB; q++) any |= go[q];
                if (!any) continue;
                const uint32_t *ap = acc0;
                for (uint32_t j = 0; j < nacc; j++) {
                    const CalHdr h = cal_hdr(ap);
#pragma unroll
                    for (uint32_t q = 0; q < EB; q++) {
                        if (!go[q]) continue;
                        const uint32_t v = cal_eval(h, tid, L.u + i0 + q, chp);
                        if constexpr (TABLE) {
                            if (act[q])   // a table phase: its protocol's index bits are at most 31
                                table_update(reinterpret_cast<uint32_t *>(recs) + p0[q], 1u << (pd.ib & 31u), v,
                                             tid, (h.mode & 1u) != 0);
                            continue;
                        }
                        const unsigned long long pos = p0[q] + (unsigned long long)j * na[q];
                        if (act[q] && pos < cap)
                            recs[pos] = ((unsigned long long)v << 32) | ((unsigned long long)tid << 1) | h.mode;
                    }
                    ap += CAL_HDR + 2 * h.nops;
                }
            }
        }
        __syncthreads();
    }
}

template <typename T, bool WIDE, bool TABLE>
__global__ __launch_bounds__(WG) void k_emit(const Item *__restrict__ items, const NestDesc *__restrict__ nests,
                                              const ProtoDesc *__restrict__ protos,
                                              const FixedVal *__restrict__ fixed, const uint32_t *__restrict__ code,
                                              const uint32_t *__restrict__ item_cnt,
                                              const unsigned long long *__restrict__ big_base,
                                              unsigned long long *__restrict__ cursor, uint64_t win_lo,
                                              uint64_t win_n, unsigned long long *__restrict__ recs,
                                              unsigned long long cap) {
    __shared__ unsigned long long lds_base[MAXSPAN];
    __shared__ uint32_t lds_cur[MAXSPAN];
    __shared__ CalLds lds_cal;
    const Item it = items[blockIdx.x];
    const NestDesc &nd = nests[it.nest];
    const ProtoDesc pd = protos[nd.proto];
    const uint32_t span = it.span;
    for (uint32_t i = threadIdx.x; i < span; i += WG) {
        const uint64_t k = it.k_lo + i;
        const uint32_t c = item_cnt[it.cnt_off + i];
        unsigned long long v = ~0ull;
        if (c && k >= win_lo && k - win_lo < win_n) {
            const unsigned long long b = big_base[k - win_lo];
            if constexpr (TABLE) v = b;   // the phase's table (or none)
            else if (b != ~0ull) v = b + atomicAdd(&cursor[k - win_lo], (unsigned long long)c);
        }
        lds_base[i] = v;
        lds_cur[i] = 0;
    }
    __syncthreads();
    if constexpr (!WIDE) {
        if (nd.cal_off != NONE32) {
            emit_cal<T, TABLE>(it, nd, pd, fixed, code, lds_base, lds_cur, recs, cap, lds_cal);
            return;
        }
    }

    for (uint32_t blk = 0; blk < it.nblk; blk++) {
        const uint32_t tid0 = it.tid0 + blk * (uint32_t)WG;
        T vars[MAXSLOTS];
        for (int s = 0; s < MAXSLOTS; s++) vars[s] = 0;
        load_fixed<T>(nd, fixed, vars);
        Odo<T> odo;
        odo.start(nd, it.f0, vars);
        const uint32_t tid = tid0 + threadIdx.x;
        const bool act0 = tid < pd.n;
        const uint32_t *leaf = code + nd.code_off;
        bool ovf = false;
        EmitSink sink{nullptr, 0, recs, cap, tid};
        TableSink tsink{nullptr, 0, tid};
        for (uint64_t f = it.f0; f < it.f1; f++) {
            const uint32_t i = (uint32_t)(odo.phase - it.k_lo);
            const unsigned long long b = lds_base[i];
            if (b != ~0ull && tid0 < tid_limit<T>(nd, code, vars, pd.n)) {
                if constexpr (TABLE) {
                    tsink.tab = reinterpret_cast<uint32_t *>(recs) + b;
                    tsink.cells = 1u << (pd.ib & 31u);
                    run_leaf<T, WIDE>(leaf, vars, (T)tid, act0, ovf, tsink);
                } else {
                    sink.cur = &lds_cur[i];
                    sink.base = b;
                    run_leaf<T, WIDE>(leaf, vars, (T)tid, act0, ovf, sink);
                }
            }
            odo.next(nd, vars);
        }
    }
}

// ======================================================= LDS sort + scan
// LDS record arrays are padded by one slot per 32 keys: thread blocks of
// E consecutive keys then start in different banks (no 64-way conflicts
// when a thread loads or stores its block).
constexpr uint32_t TILE_LDS = TILE + TILE / 32;
DEV uint32_t ph(uint32_t i) { return i + (i >> 5); }

// Bitonic sort of n = NT * E u64 keys in LDS by an NT-thread workgroup.
// Thread t keeps a[E*t .. E*t+E) in registers for every stride below E;
// larger strides exchange through LDS, with all loads of a stage issued
// before any store (pairs of one stage are disjoint).
template <int E, int NT = WG>
DEV void block_sort_e(unsigned long long *a, uint32_t n) {
    constexpr int PAIRS = (E / 2 > 0) ? E / 2 : 1;
    const uint32_t t = threadIdx.x;
    const uint32_t g0 = t * E;
    const uint32_t half = n >> 1;
    unsigned long long v[E];
#pragma unroll
    for (int j = 0; j < E; j++) v[j] = a[ph(g0 + j)];
    for (uint32_t size = 2; size <= n; size <<= 1) {
        if ((size >> 1) >= (uint32_t)E) {
            __syncthreads();
#pragma unroll
            for (int j = 0; j < E; j++) a[ph(g0 + j)] = v[j];
            __syncthreads();
            for (uint32_t stride = size >> 1; stride >= (uint32_t)E; stride >>= 1) {
                unsigned long long x[PAIRS], y[PAIRS];
                uint32_t lo[PAIRS];
#pragma unroll
                for (int j = 0; j < PAIRS; j++) {
                    const uint32_t i = t + (uint32_t)j * (uint32_t)NT;
                    lo[j] = 2 * i - (i & (stride - 1));
                    if (i < half) {
                        x[j] = a[ph(lo[j])];
                        y[j] = a[ph(lo[j] + stride)];
                    }
                }
#pragma unroll
                for (int j = 0; j < PAIRS; j++) {
                    const uint32_t i = t + (uint32_t)j * (uint32_t)NT;
                    if (i < half) {
                        const bool asc = (lo[j] & size) == 0;
                        const bool sw = (x[j] > y[j]) == asc;
                        a[ph(lo[j])] = sw ? y[j] : x[j];
                        a[ph(lo[j] + stride)] = sw ? x[j] : y[j];
                    }
                }
                __syncthreads();
            }
#pragma unroll
            for (int j = 0; j < E; j++) v[j] = a[ph(g0 + j)];
        }
#pragma unroll
        for (int st = E / 2; st >= 1; st >>= 1) {
            if ((uint32_t)st <= (size >> 1)) {
#pragma unroll
                for (int j = 0; j < E; j++) {
                    if ((j & st) == 0) {
                        const bool asc = ((g0 + (uint32_t)j) & size) == 0;
                        const unsigned long long x = v[j], y = v[j + st];
                        const bool sw = (x > y) == asc;
                        v[j] = sw ? y : x;
                        v[j + st] = sw ? x : y;
                    }
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < E; j++) a[ph(g0 + j)] = v[j];
    __syncthreads();
}

// Bitonic sort of a[0..n) (n a power of two, n >= 2) in LDS by an
// NT-thread workgroup with every stage through LDS: no record stays in
// registers between stages, and a thread holds four pairs at a time (for
// callers at their register budget).
template <int NT>
DEV void block_sort_lds(unsigned long long *a, uint32_t n) {
    const uint32_t half = n >> 1;
    __syncthreads();
    for (uint32_t size = 2; size <= n; size <<= 1) {
        for (uint32_t stride = size >> 1; stride >= 1; stride >>= 1) {
            for (uint32_t i0 = threadIdx.x; i0 < half; i0 += 4 * NT) {
                unsigned long long x[4], y[4];
                uint32_t lo[4];
#pragma unroll
                for (int d = 0; d < 4; d++) {
                    const uint32_t i = i0 + (uint32_t)d * NT;
                    lo[d] = 2 * i - (i & (stride - 1));
                    if (i < half) {
                        x[d] = a[ph(lo[d])];
                        y[d] = a[ph(lo[d] + stride)];
                    }
                }
#pragma unroll
                for (int d = 0; d < 4; d++) {
                    if (i0 + (uint32_t)d * NT < half) {
                        const bool asc = (lo[d] & size) == 0;
                        const bool sw = (x[d] > y[d]) == asc;
                        a[ph(lo[d])] = sw ? y[d] : x[d];
                        a[ph(lo[d] + stride)] = sw ? x[d] : y[d];
                    }
                }
            }
            __syncthreads();
        }
    }
}

DEV uint32_t rec_idx(unsigned long long r) { return (uint32_t)(r >> 32); }
DEV uint32_t rec_tid(unsigned long long r) { return (uint32_t)(r >> 1) & 0x7FFFFFFFu; }

// Run state of the segmented conflict scan (all wave-uniform).
struct RunState {
    bool open;
    unsigned long long key;
    uint32_t t0, t1, wf;
    bool t0w, in_t0;
};

DEV uint64_t bits_from(uint32_t s) { return s >= 64 ? 0ull : (~0ull << s); }
DEV uint64_t bits_range(uint32_t s, uint32_t e) { return bits_from(s) & ~bits_from(e); }

// Folds lanes [s, e) of the current chunk into the open run.
DEV void run_segment(RunState &st, uint32_t s, uint32_t e, uint64_t G, uint64_t Wm, uint32_t tidv) {
    uint64_t seg = bits_range(s, e);
    uint64_t rest = seg;
    if (st.in_t0) {
        const uint64_t g = G & seg;
        if (g) {
            const uint32_t gb = (uint32_t)__builtin_ctzll(g);
            st.t0w = st.t0w || ((Wm & bits_range(s, gb)) != 0);
            st.in_t0 = false;
            st.t1 = readlane(tidv, gb);
            rest = bits_range(gb, e);
        } else {
            st.t0w = st.t0w || ((Wm & seg) != 0);
            rest = 0;
        }
    }
    if (!st.in_t0 && st.wf == NONE32) {
        const uint64_t wm = Wm & rest;
        if (wm) st.wf = readlane(tidv, (uint32_t)__builtin_ctzll(wm));
    }
}

DEV bool run_close(const RunState &st, unsigned long long &rkey, uint32_t &ri1, uint32_t &ri2) {
    if (st.t1 != NONE32 && (st.t0w || st.wf != NONE32)) {
        rkey = st.key;
        ri1 = st.t0;
        ri2 = st.t0w ? st.t1 : st.wf;
        return true;
    }
    return false;
}

DEV uint32_t ctz64(uint64_t m) { return (uint32_t)__builtin_ctzll(m); }

// First racy run (in sorted order) whose head lies in [a, b) of the sorted
// array rec[0..cnt); runs starting before a belong to the previous wave and
// the last run may extend past b.  The array is read 64 records at a time:
// group heads (index changes), tid changes and writers are three ballots.
// Every head lane resolves its own group when the group ends inside the
// chunk (lane-parallel mask arithmetic plus one cross-lane read); only a
// group that crosses into the next chunk is carried in wave-uniform state.
DEV bool wave_first_racy(const unsigned long long *rec, uint32_t cnt, uint32_t a, uint32_t b, uint32_t tb,
                         unsigned long long &rkey, uint32_t &ri1, uint32_t &ri2) {
    RunState st{false, 0, 0, NONE32, NONE32, false, false};
    const uint32_t lane = lane_id();
    const uint32_t gsh = tb + 1;
    const uint32_t tmask = tb >= 32 ? 0xFFFFFFFFu : ((1u << tb) - 1u);
    for (uint32_t base = a; base < cnt; base += 64) {
        if (!st.open && base >= b) break;
        const uint32_t i = base + lane;
        const bool valid = i < cnt;
        const unsigned long long r = valid ? rec[ph(i)] : ~0ull;
        const unsigned long long rp = (valid && i > 0) ? rec[ph(i - 1)] : ~0ull;
        const unsigned long long grp = r >> gsh;
        const uint32_t tidv = (uint32_t)(r >> 1) & tmask;
        const bool head = valid && (i == 0 || (rp >> gsh) != grp);
        const bool gch = valid && !head && ((uint32_t)(rp >> 1) & tmask) != tidv;
        const uint32_t glo = (uint32_t)grp, ghi = (uint32_t)(grp >> 32);
        const uint64_t H = ballot(head), G = ballot(gch), Wm = ballot(valid && (r & 1ull));
        const uint32_t nvalid = (uint32_t)__builtin_popcountll(ballot(valid));   // valid lanes are a prefix
        const bool at_end = base + nvalid >= cnt;
        uint32_t pos = 0;
        if (st.open) {
            // the group carried in from the previous chunk
            const uint32_t end = H ? ctz64(H) : nvalid;
            run_segment(st, 0, end, G, Wm, tidv);
            if (end < nvalid || at_end) {
                st.open = false;
                if (run_close(st, rkey, ri1, ri2)) return true;
            } else {
                continue;   // the group spans the whole chunk
            }
            pos = end;
        }
        const uint32_t lim = (b > base) ? (b - base < 64 ? b - base : 64) : 0;
        const uint64_t mine_m = H & bits_range(pos, lim);
        // per head lane: its group [lane, e)
        const uint64_t after = H & bits_from(lane + 1);
        const uint32_t e = after ? ctz64(after) : nvalid;
        const bool closed = e < nvalid || at_end;
        const bool mine = ((mine_m >> lane) & 1ull) != 0;
        bool racy = false;
        uint32_t src = lane;
        if (mine && closed) {
            const uint64_t g = G & bits_range(lane, e);
            const uint32_t gb = g ? ctz64(g) : e;
            const bool t0w = (Wm & bits_range(lane, gb)) != 0;
            const uint64_t wl = Wm & bits_range(gb, e);
            racy = gb < e && (t0w || wl != 0);
            if (racy) src = t0w ? gb : ctz64(wl);
        }
        const uint32_t partner = __shfl(tidv, (int)src);
        const uint64_t R = ballot(racy);
        if (R) {
            const uint32_t f = ctz64(R);
            rkey = ((unsigned long long)readlane(ghi, f) << 32) | readlane(glo, f);
            ri1 = readlane(tidv, f);
            ri2 = readlane(partner, f);
            return true;
        }
        // a group of this wave that continues in the next chunk
        const uint64_t open_m = mine_m & ~ballot(closed);
        if (open_m) {
            const uint32_t h = ctz64(open_m);
            st.open = true;
            st.key = ((unsigned long long)readlane(ghi, h) << 32) | readlane(glo, h);
            st.t0 = readlane(tidv, h);
            st.t1 = NONE32;
            st.wf = NONE32;
            st.in_t0 = true;
            st.t0w = false;
            run_segment(st, h, nvalid, G, Wm, tidv);
        }
    }
    if (st.open && run_close(st, rkey, ri1, ri2)) return true;
    return false;
}

// Workgroup-wide: first racy group of the sorted LDS array (records with
// tid bits tb).  Returns found (uniform across the block) and the group
// key (record >> (tb + 1)) with its pair.
DEV bool block_first_racy(const unsigned long long *rec, uint32_t cnt, uint32_t tb,
                          uint32_t *lds_res /* 5 words per wave */, unsigned long long &key, uint32_t &i1, uint32_t &i2) {
    const uint32_t wave = threadIdx.x >> 6;
    const uint32_t nw = blockDim.x >> 6;
    const uint32_t per = (cnt + nw - 1) / nw;
    const uint32_t a = wave * per, b = (a + per < cnt) ? a + per : cnt;
    unsigned long long rk = 0;
    uint32_t r1 = 0, r2 = 0;
    bool f = (a < cnt) ? wave_first_racy(rec, cnt, a, b, tb, rk, r1, r2) : false;
    if (lane_id() == 0) {
        lds_res[wave * 5 + 0] = f ? 1u : 0u;
        lds_res[wave * 5 + 1] = (uint32_t)rk;
        lds_res[wave * 5 + 2] = (uint32_t)(rk >> 32);
        lds_res[wave * 5 + 3] = r1;
        lds_res[wave * 5 + 4] = r2;
    }
    __syncthreads();
    bool found = false;
    for (uint32_t w = 0; w < nw; w++) {
        if (lds_res[w * 5]) {
            found = true;
            key = ((unsigned long long)lds_res[w * 5 + 2] << 32) | lds_res[w * 5 + 1];
            i1 = lds_res[w * 5 + 3];
            i2 = lds_res[w * 5 + 4];
            break;
        }
    }
    __syncthreads();
    return found;
}

DEV void offer(Best *best, Cand *cand, uint32_t proto, uint32_t phase, uint32_t idx, uint32_t i1, uint32_t i2) {
    const unsigned long long key = ((unsigned long long)phase << 32) | idx;
    cand->key = key;
    cand->pair = ((unsigned long long)i1 << 32) | i2;
    cand->proto = proto;
    atomicMin(&best[proto].key, key);
}

// ======================================================= group decision
DEV uint32_t wave_min(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) { uint32_t w = __shfl_xor(v, o); v = w < v ? w : v; }
    return v;
}
DEV uint32_t wave_max(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) { uint32_t w = __shfl_xor(v, o); v = w > v ? w : v; }
    return v;
}

// Workgroup min of a u32 through red[0 .. waves) (barriers on entry and exit).
DEV uint32_t block_min(uint32_t v, uint32_t *red) {
    v = wave_min(v);
    __syncthreads();
    if (lane_id() == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    uint32_t r = red[0];
    for (uint32_t w = 1; w < (blockDim.x >> 6); w++) r = red[w] < r ? red[w] : r;
    __syncthreads();
    return r;
}

// Wave min / max of a u64 (a butterfly over the 64 lanes).
DEV unsigned long long wave_min64(unsigned long long v) {
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long w = __shfl_xor(v, o);
        v = w < v ? w : v;
    }
    return v;
}
DEV unsigned long long wave_max64(unsigned long long v) {
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long w = __shfl_xor(v, o);
        v = w > v ? w : v;
    }
    return v;
}
// Workgroup min and max of a u64 in one reduction (red[0 .. 4 * waves)).
DEV void block_minmax64(unsigned long long &lo, unsigned long long &hi, uint32_t *red) {
    lo = wave_min64(lo);
    hi = wave_max64(hi);
    __syncthreads();
    if (lane_id() == 0) {
        const uint32_t w = threadIdx.x >> 6;
        red[4 * w] = (uint32_t)lo;
        red[4 * w + 1] = (uint32_t)(lo >> 32);
        red[4 * w + 2] = (uint32_t)hi;
        red[4 * w + 3] = (uint32_t)(hi >> 32);
    }
    __syncthreads();
    for (uint32_t w = 0; w < (blockDim.x >> 6); w++) {
        const unsigned long long l = ((unsigned long long)red[4 * w + 1] << 32) | red[4 * w];
        const unsigned long long h = ((unsigned long long)red[4 * w + 3] << 32) | red[4 * w + 2];
        lo = l < lo ? l : lo;
        hi = h > hi ? h : hi;
    }
    __syncthreads();
}

// A group of records (one phase, or consecutive phases in the packed
// layout; at most TILE, held in registers) is decided with the group's LDS
// array as scratch, by a method chosen from the span of its cells (cell =
// record >> (tb + 1): the index, or phase and index):
//  table   span <= TBL_CELLS: per cell, the least tid, the least writing
//          tid and the least tid other than the first, by LDS atomics.
//          Definition 1 needs nothing else: the cell races iff a second tid
//          and a writer exist, and the witness is (least tid, least other
//          tid if the least tid writes, else least writer).
//  filter  otherwise: a seen / repeated bitmap pair (indexed by the cell's
//          offset when the span fits 2^FILTER_BITS bits, else by a hash of
//          the cell) removes every cell touched by a single record (one
//          access cannot race).  When no cell repeats the group is race
//          free; otherwise the records left are aggregated per cell as in
//          the table method, in an LDS hash table.
//  split   (LIGHT) when the survivors hold more distinct cells than the
//          hash table takes, a second hash of the cell splits them four
//          ways and each part takes a table pass of its own.
//  sort    when a table still overflows (or without LIGHT): the survivors
//          are sorted and scanned (with LIGHT by a sort whose stages all
//          go through LDS).
// Tiles run 512-thread workgroups: at most 16 records per thread stay in
// registers, and the two workgroups the LDS admits per CU give 4 waves per
// SIMD.
constexpr int TWG = 512;
constexpr uint32_t TBL_CELLS = (TILE_LDS * 2) / 3;       // three u32 per cell
constexpr uint32_t FILTER_WORDS = 1u << (FILTER_BITS - 5);
static_assert(2 * FILTER_WORDS <= 2 * TILE_LDS, "filter bitmaps exceed the group LDS");
static_assert(TILE % TWG == 0 && TILE / TWG <= 16, "tile records per thread");
static_assert(TILE / WG <= 32, "fused records per thread (one mask bit each)");
static_assert(FUSED_PACK % WG == 0, "fused group size");
constexpr uint32_t RED_WORDS = 5 * (TWG / 64) + 1;       // scan slots of the widest workgroup, then
constexpr uint32_t RED_CAND = RED_WORDS - 1;             // the filter's repeat flag / hash cell counter
constexpr uint32_t RED_OVF = 38;                         // hash table overflow flag
constexpr uint32_t RED_NC = 39;                          // survivor count
// Up to SURV_CAP survivors of the filter are also kept compact in LDS,
// below the repeated bitmap; the hash table then lies above them.
constexpr uint32_t SURV_CAP = 1024;
constexpr uint32_t SURV_WORDS = 2 * (SURV_CAP + SURV_CAP / 32);
static_assert(SURV_WORDS <= FILTER_WORDS, "compact survivors overlap the repeated bitmap");
static_assert((2 * TILE_LDS - SURV_WORDS) / 4 >= 2 * SURV_CAP, "no room for the table above the survivors");
static_assert(RED_OVF >= 4 * (TWG / 64) && RED_OVF < RED_NC && RED_NC < RED_CAND,
              "reduction slots overlap");

constexpr uint32_t HSLOTS_MAX = 4096;   // hash table slots at most
static_assert(HSLOTS_MAX * 16 <= TILE_LDS * 8, "hash table exceeds the group LDS");

constexpr uint32_t floor_log2(uint32_t x) { return x <= 1 ? 0 : 1 + floor_log2(x >> 1); }

// Sizes of the decision's methods for a scratch array of LW u64 words (a
// group of at most LW - LW / 33 records): table cells, filter bitmap bits,
// compact survivors and hash table slots all scale with the scratch.
template <uint32_t LW>
struct Scratch {
    static constexpr uint32_t words = 2 * LW;                                   // u32 words
    static constexpr uint32_t tbl_cells = words / 3;                            // three u32 per cell
    static constexpr uint32_t fbits = floor_log2(LW) + 5 < FILTER_BITS ? floor_log2(LW) + 5 : FILTER_BITS;
    static constexpr uint32_t fwords = 1u << (fbits - 5);                       // each bitmap
    static constexpr uint32_t surv_cap = (1u << floor_log2(words / 12)) < SURV_CAP ? (1u << floor_log2(words / 12))
                                                                                   : SURV_CAP;
    static constexpr uint32_t surv_words = 2 * (surv_cap + surv_cap / 32);
    static constexpr uint32_t hslots = (1u << floor_log2(words / 4)) < HSLOTS_MAX ? (1u << floor_log2(words / 4))
                                                                                  : HSLOTS_MAX;
    static_assert(2 * fwords <= words, "filter bitmaps exceed the scratch");
    static_assert(surv_words <= fwords, "compact survivors overlap the repeated bitmap");
    static_assert((words - surv_words) / 4 >= 2 * surv_cap, "no room for the table above the survivors");
    static_assert(hslots * 4 <= words, "hash table exceeds the scratch");
    static_assert(2 * fwords + 64 <= words, "no words above the filter bitmaps");
};

// One record's update of its cell's aggregate (least tid t0, least tid
// other than t0 t1, least writing tid w0), in one pass over the records:
// atomicMin on t0 returns the minimum before it, and whenever that is a
// different tid, the larger of the two is offered to t1.  Every offer is a
// tid of the cell other than the final t0, hence >= the second least tid;
// and the second least tid is always offered (whether it comes before or
// after the least one, or after a larger one), so t1 ends exact.
DEV void cell_update(uint32_t *t0, uint32_t *t1, uint32_t *w0, uint32_t tid, bool wr) {
    const uint32_t old = atomicMin(t0, tid);
    if (old != NONE32 && old != tid) atomicMin(t1, old > tid ? old : tid);
    if (wr) atomicMin(w0, tid);
}

// Exact decision of the filter's survivors by per-cell aggregation in an
// LDS hash table at mem: open addressing on the cell's offset from lo (the
// span is below 2^32), linear probing over 2^hb slots of (key, least tid,
// least writing tid, least tid other than the first), the table sized for
// twice the survivors.  Probing never takes more steps than there are
// slots; more distinct cells than three quarters of the slots is an
// overflow.  src(f) calls f(r, vm) for the survivors this thread owns,
// four at a time (r[d] is one when bit d of vm is set; the same ones on
// every call), so that the four records' atomics are in flight together.
// Returns 1 (racy cell found), 0 (none) or -1 (overflow: the caller falls
// back to another method).
template <int NT, class Src>
DEV int hash_agg(const Src &src, uint32_t nc, uint32_t ish, uint32_t tmask, unsigned long long lo, uint32_t *mem,
                 uint32_t max_slots, uint32_t *red, unsigned long long &key, uint32_t &i1, uint32_t &i2) {
    uint32_t hb = 8;
    while ((1u << hb) < 2 * nc && (2u << hb) <= max_slots) hb++;
    const uint32_t S = 1u << hb, cap = S - S / 4;
    uint32_t *K = mem, *T0 = K + S, *W0 = T0 + S, *T1 = W0 + S;
    uint4 *K4 = reinterpret_cast<uint4 *>(K);   // mem is 16-byte aligned: cleared 16 bytes at a time
    for (uint32_t k = threadIdx.x; k < S; k += NT) K4[k] = make_uint4(NONE32, NONE32, NONE32, NONE32);
    if (threadIdx.x == 0) {
        red[RED_CAND] = 0;
        red[RED_OVF] = 0;
    }
    __syncthreads();
    bool ovf = false;
    src([&](const unsigned long long (&r)[4], uint32_t vm) {
        uint32_t c[4], h[4], o[4];
#pragma unroll
        for (int d = 0; d < 4; d++) {
            c[d] = (uint32_t)((r[d] >> ish) - lo);
            h[d] = (c[d] * 0x9E3779B1u) >> (32 - hb);
            o[d] = NONE32;
            if ((vm >> d) & 1u) o[d] = atomicCAS(&K[h[d]], NONE32, c[d]);
        }
        // a slot taken by another cell: probe on, one record at a time
        uint32_t placed = 0, fresh = 0;
#pragma unroll
        for (int d = 0; d < 4; d++) {
            if (!((vm >> d) & 1u)) continue;
            uint32_t old = o[d];
            for (uint32_t st = 1; st < S && old != NONE32 && old != c[d]; st++) {
                h[d] = (h[d] + 1) & (S - 1);
                old = atomicCAS(&K[h[d]], NONE32, c[d]);
            }
            if (old == NONE32 || old == c[d]) {
                placed |= 1u << d;
                fresh += old == NONE32 ? 1u : 0u;
            } else {
                ovf = true;
            }
        }
        // new cells of the wave counted by one atomic of its first active lane
        const uint64_t b0 = ballot(fresh & 1u), b1 = ballot(fresh & 2u), b2 = ballot(fresh & 4u);
        const uint32_t nf = (uint32_t)(__builtin_popcountll(b0) + 2 * __builtin_popcountll(b1) +
                                       4 * __builtin_popcountll(b2));
        if (nf) {
            const uint32_t leader = (uint32_t)__builtin_ctzll(ballot(true));
            uint32_t base = 0;
            if (lane_id() == leader) base = atomicAdd(&red[RED_CAND], nf);
            base = readlane(base, leader);
            if (base + nf > cap) ovf = true;
        }
        // the cells' aggregates (cell_update, four records at a time)
        uint32_t t0o[4], tid[4];
#pragma unroll
        for (int d = 0; d < 4; d++) {
            tid[d] = (uint32_t)(r[d] >> 1) & tmask;
            t0o[d] = NONE32;
            if ((placed >> d) & 1u) {
                t0o[d] = atomicMin(T0 + h[d], tid[d]);
                if (r[d] & 1ull) atomicMin(W0 + h[d], tid[d]);
            }
        }
#pragma unroll
        for (int d = 0; d < 4; d++)
            if (((placed >> d) & 1u) && t0o[d] != NONE32 && t0o[d] != tid[d])
                atomicMin(T1 + h[d], t0o[d] > tid[d] ? t0o[d] : tid[d]);
    });

    if (ovf) red[RED_OVF] = 1;
    __syncthreads();
    if (red[RED_OVF]) return -1;
    // least racy cell, with its slot in the low bits (a cell has one slot)
    unsigned long long best = ~0ull, none = 0;
    // four slots a thread per step
    const uint4 *T14 = reinterpret_cast<const uint4 *>(T1), *W04 = reinterpret_cast<const uint4 *>(W0);
    for (uint32_t q = threadIdx.x; q < S / 4; q += NT) {
        const uint4 kv = K4[q], tv = T14[q], wv = W04[q];
        const uint32_t kk[4] = {kv.x, kv.y, kv.z, kv.w}, tt[4] = {tv.x, tv.y, tv.z, tv.w},
                       ww[4] = {wv.x, wv.y, wv.z, wv.w};
#pragma unroll
        for (int d = 0; d < 4; d++) {
            const unsigned long long c = ((unsigned long long)kk[d] << 32) | (4 * q + (uint32_t)d);
            if ((kk[d] != NONE32) & (tt[d] != NONE32) & (ww[d] != NONE32)) best = c < best ? c : best;
        }
    }

    block_minmax64(best, none, red);
    if (best == ~0ull) return 0;
    const uint32_t k = (uint32_t)best;
    key = lo + (best >> 32);
    i1 = T0[k];
    i2 = W0[k] == T0[k] ? T1[k] : W0[k];
    __syncthreads();   // the table is read before the caller reuses the LDS
    return 1;
}

// Bit of a cell in the filter bitmaps: its offset from the least cell when
// the span fits the bitmap, else a multiplicative hash of the cell.  Equal
// cells always share a bit, so no cell touched twice can be missed; a hash
// collision only lets a single record through to the exact aggregation.
DEV uint32_t filter_bit(unsigned long long cell, unsigned long long lo, bool hashed, uint32_t bits) {
    return hashed ? (uint32_t)((cell * 0x9E3779B97F4A7C15ull) >> (64 - bits)) : (uint32_t)(cell - lo);
}

// (a holds LW u64 words; larger sizes are never asked for: n is at most
// the group's record count)
template <int E, int NT, uint32_t LW>
DEV void sort_e(unsigned long long *a, uint32_t n) {
    if constexpr ((uint32_t)E * NT <= (uint32_t)TILE && (uint32_t)E * NT + (uint32_t)E * NT / 32 <= LW)
        block_sort_e<E, NT>(a, n);
}

// Sorts a[0..n) (n a power of two, NT <= n <= TILE) with an NT-thread
// workgroup and returns the first racy group of its cnt records.
template <int NT, uint32_t LW>
DEV bool sort_scan(unsigned long long *a, uint32_t n, uint32_t cnt, uint32_t tb, uint32_t *red,
                   unsigned long long &key, uint32_t &i1, uint32_t &i2) {
    switch (n / NT) {
    case 1: sort_e<1, NT, LW>(a, n); break;
    case 2: sort_e<2, NT, LW>(a, n); break;
    case 4: sort_e<4, NT, LW>(a, n); break;
    case 8: sort_e<8, NT, LW>(a, n); break;
    case 16: sort_e<16, NT, LW>(a, n); break;
    default: sort_e<32, NT, LW>(a, n); break;
    }
    return block_first_racy(a, cnt, tb, red, key, i1, i2);
}

// Decides the cnt records held in registers (element i = j * NT + thread;
// lanes past the end hold a copy of a real record) with the LDS array a
// (LW words) as scratch.  Returns whether a cell races, with the least racy
// cell and its witness pair.  LIGHT (the register-light fallbacks above)
// is chosen per caller by its register budget.
template <int E, int NT, uint32_t LW = TILE_LDS, bool LIGHT = false>
DEV bool decide(const unsigned long long (&u)[E], uint32_t cnt, uint32_t tb, unsigned long long *a, uint32_t *red,
                unsigned long long &key, uint32_t &i1, uint32_t &i2) {
    using SC = Scratch<LW>;
    static_assert((uint32_t)E * NT + (uint32_t)E * NT / 32 <= LW, "records exceed the scratch");
    const uint32_t ish = tb + 1;
    const uint32_t tmask = tb >= 32 ? 0xFFFFFFFFu : ((1u << tb) - 1u);
    uint32_t *w32 = reinterpret_cast<uint32_t *>(a);
    unsigned long long lo = ~0ull, hi = 0;
#pragma unroll
    for (int j = 0; j < E; j++) {
        const unsigned long long x = u[j] >> ish;
        lo = x < lo ? x : lo;
        hi = x > hi ? x : hi;
    }
    block_minmax64(lo, hi, red);
    const unsigned long long span = hi - lo + 1;   // cells are below 2^63

    if (span <= SC::tbl_cells) {
        const uint32_t sp = (uint32_t)span;
        uint32_t *t0 = w32, *w0 = w32 + sp, *t1 = w32 + 2 * sp;
        for (uint32_t k = threadIdx.x; k < 3 * sp; k += NT) w32[k] = NONE32;
        __syncthreads();
        // four rows at a time: the least-tid atomics in flight together,
        // then the second-tid offers (cell_update, reordered)
#pragma unroll
        for (int j0 = 0; j0 < E; j0 += 4) {
            if ((uint32_t)j0 * NT < cnt) {
                uint32_t bb[4], tid[4], old[4];
#pragma unroll
                for (int d = 0; d < 4 && j0 + d < E; d++) {
                    const int j = j0 + d;
                    bb[d] = (uint32_t)((u[j] >> ish) - lo);
                    tid[d] = (uint32_t)(u[j] >> 1) & tmask;
                    old[d] = NONE32;
                    if ((uint32_t)j * NT + threadIdx.x < cnt) {
                        old[d] = atomicMin(t0 + bb[d], tid[d]);
                        if (u[j] & 1ull) atomicMin(w0 + bb[d], tid[d]);
                    }
                }
#pragma unroll
                for (int d = 0; d < 4 && j0 + d < E; d++)
                    if (old[d] != NONE32 && old[d] != tid[d])
                        atomicMin(t1 + bb[d], old[d] > tid[d] ? old[d] : tid[d]);
            }
        }
        __syncthreads();
        uint32_t first = NONE32;
        for (uint32_t k = threadIdx.x; k < sp; k += NT) {
            if (t1[k] != NONE32 && w0[k] != NONE32) { first = k; break; }
        }
        first = block_min(first, red);
        bool found = false;
        if (first != NONE32) {
            found = true;
            key = lo + first;
            i1 = t0[first];
            const uint32_t aw = w0[first];
            i2 = aw == i1 ? t1[first] : aw;
        }
        __syncthreads();   // the table is read before the caller reuses the LDS
        return found;
    }

    // filter: seen / repeated bitmaps (atomicOr returns the old word: a
    // record whose cell was seen marks it repeated); when no cell repeats
    // the group is race free (most groups end there), else the survivors:
    // their mask per thread, and (up to SURV_CAP) a compact copy at
    // a[ph(0..)], below the repeated bitmap (the seen bitmap is no longer
    // read)
    uint32_t keepm = 0, nc;
    {
        const bool hashed = span > (1ull << SC::fbits);
        // bitmap words, a multiple of four: cleared 16 bytes at a time
        const uint32_t nw = hashed ? SC::fwords : (((uint32_t)((span + 31) >> 5) + 3u) & ~3u);
        uint32_t *seen = w32, *rep = w32 + SC::fwords;
        uint4 *seen4 = reinterpret_cast<uint4 *>(seen), *rep4 = reinterpret_cast<uint4 *>(rep);
        for (uint32_t q = threadIdx.x; q < nw / 4; q += NT) {
            seen4[q] = make_uint4(0u, 0u, 0u, 0u);
            rep4[q] = make_uint4(0u, 0u, 0u, 0u);
        }
        if (threadIdx.x == 0) {
            red[RED_CAND] = 0;
            red[RED_NC] = 0;
        }
        __syncthreads();
        // rows four at a time, branch free within the four (a lane past the
        // records sets a bit of a word of its own that no one reads), so
        // that the four seen atomics are in flight together
        bool again = false;
        uint32_t *const dummy = w32 + 2 * SC::fwords + lane_id();
#pragma unroll
        for (int j0 = 0; j0 < E; j0 += 4) {
            if ((uint32_t)j0 * NT < cnt) {
                uint32_t old[4], bits[4], wd[4];
#pragma unroll
                for (int d = 0; d < 4 && j0 + d < E; d++) {
                    const int j = j0 + d;
                    const uint32_t b = filter_bit(u[j] >> ish, lo, hashed, SC::fbits);
                    bits[d] = 1u << (b & 31);
                    wd[d] = b >> 5;
                    old[d] = atomicOr((uint32_t)j * NT + threadIdx.x < cnt ? &seen[wd[d]] : dummy, bits[d]);
                }
#pragma unroll
                for (int d = 0; d < 4 && j0 + d < E; d++) {
                    if ((uint32_t)(j0 + d) * NT + threadIdx.x < cnt && (old[d] & bits[d])) {
                        atomicOr(&rep[wd[d]], bits[d]);
                        again = true;
                    }
                }
            }
        }
        if (again) red[RED_CAND] = 1;
        __syncthreads();
        if (red[RED_CAND] == 0) return false;   // every cell touched once
        // the survivors (rows four at a time: their bitmap reads in flight
        // together), then one reservation per wave for all of its survivors
        // (each lane's count and prefix from its count's bits), written lane
        // by lane
#pragma unroll
        for (int j0 = 0; j0 < E; j0 += 4) {
            if ((uint32_t)j0 * NT < cnt) {
                uint32_t wv[4], bb[4];
#pragma unroll
                for (int d = 0; d < 4 && j0 + d < E; d++) {
                    const uint32_t b = filter_bit(u[j0 + d] >> ish, lo, hashed, SC::fbits);
                    bb[d] = b & 31;
                    wv[d] = rep[b >> 5];
                }
#pragma unroll
                for (int d = 0; d < 4 && j0 + d < E; d++)
                    if ((uint32_t)(j0 + d) * NT + threadIdx.x < cnt && ((wv[d] >> bb[d]) & 1u)) keepm |= 1u << (j0 + d);
            }
        }
        {
            const uint32_t mine = (uint32_t)__builtin_popcount(keepm);
            uint32_t tot = 0, excl = 0;
#pragma unroll
            for (int k = 0; k < 6; k++) {   // mine <= 32
                const uint64_t bk = ballot((mine >> k) & 1u);
                tot += (uint32_t)__builtin_popcountll(bk) << k;
                excl += mbcnt(bk) << k;
            }
            if (tot) {
                uint32_t base = 0;
                if (lane_id() == 0) base = atomicAdd(&red[RED_NC], tot);
                uint32_t pos = readlane(base, 0) + excl;
#pragma unroll
                for (int j = 0; j < E; j++) {
                    if ((keepm >> j) & 1u) {
                        if (pos < SC::surv_cap) a[ph(pos)] = u[j];
                        pos++;
                    }
                }
            }
        }
        __syncthreads();   // the bitmaps are read for the last time
        nc = red[RED_NC];
    }
    const bool compact = nc <= SC::surv_cap;
    if (span <= 0xFFFFFFFFull) {
        // one hash pass over the survivors; when its table overflows, the
        // cells are split four ways by a second hash of the cell and each
        // part takes a pass of its own (the least racy cell over the parts
        // is the least of all)
        for (uint32_t nparts = 1; nparts <= (LIGHT ? 4u : 1u); nparts *= 4) {
            bool over = false, found = false;
            unsigned long long bk = ~0ull;
            uint32_t b1 = 0, b2 = 0;
            for (uint32_t q = 0; q < nparts; q++) {
                auto part = [&](unsigned long long r) {
                    return nparts == 1 || (((uint32_t)((r >> ish) - lo) * 0x85EBCA6Bu) >> 30) == q;
                };
                unsigned long long k2 = 0;
                uint32_t j1 = 0, j2 = 0;
                int r;
                if (compact) {
                    // survivors spread over the threads, the table above them
                    auto src = [&](auto f) {
                        for (uint32_t i = threadIdx.x; i < nc; i += 4 * NT) {
                            unsigned long long x[4];
                            uint32_t vm = 0;
#pragma unroll
                            for (int d = 0; d < 4; d++) {
                                const uint32_t id = i + (uint32_t)d * NT;
                                x[d] = a[ph(id < nc ? id : i)];
                                if (id < nc && part(x[d])) vm |= 1u << d;
                            }
                            if (vm) f(x, vm);
                        }
                    };
                    r = hash_agg<NT>(src, nc, ish, tmask, lo, w32 + SC::surv_words, (SC::words - SC::surv_words) / 4,
                                     red, k2, j1, j2);
                } else {
                    auto src = [&](auto f) {
#pragma unroll
                        for (int j0 = 0; j0 < E; j0 += 4) {
                            unsigned long long x[4];
                            uint32_t vm = 0;
#pragma unroll
                            for (int d = 0; d < 4; d++) {
                                x[d] = u[j0 + d < E ? j0 + d : j0];
                                if (j0 + d < E && ((keepm >> (j0 + d)) & 1u) && part(x[d])) vm |= 1u << d;
                            }
                            if (vm) f(x, vm);
                        }
                    };
                    r = hash_agg<NT>(src, nc, ish, tmask, lo, w32, SC::hslots, red, k2, j1, j2);
                }
                if (r < 0) {
                    over = true;
                    break;
                }
                if (r == 1 && k2 < bk) {
                    found = true;
                    bk = k2;
                    b1 = j1;
                    b2 = j2;
                }
            }
            __syncthreads();   // every thread has seen the outcome
            if (!over) {
                if (found) {
                    key = bk;
                    i1 = b1;
                    i2 = b2;
                }
                return found;
            }
        }
    }
    // sort the survivors (compacted to a[ph(0..nc))), padded to a power of two
    if (!compact) {
        if (threadIdx.x == 0) red[RED_CAND] = 0;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < E; j++) {
            const bool keep = (keepm >> j) & 1u;
            const uint64_t m = ballot(keep);
            if (m) {
                uint32_t base = 0;
                if (lane_id() == 0) base = atomicAdd(&red[RED_CAND], (uint32_t)__builtin_popcountll(m));
                base = __shfl(base, 0);
                if (keep) a[ph(base + mbcnt(m))] = u[j];
            }
        }
    }
    uint32_t np = NT;
    while (np < nc) np <<= 1;
    for (uint32_t k = nc + threadIdx.x; k < np; k += NT) a[ph(k)] = ~0ull;
    __syncthreads();
    if constexpr (LIGHT) {
        block_sort_lds<NT>(a, np);
        return block_first_racy(a, nc, tb, red, key, i1, i2);
    } else {
        return sort_scan<NT, LW>(a, np, nc, tb, red, key, i1, i2);
    }
}

// =============================================================== fused path
constexpr uint32_t FN_CACHE = 16;
// One workgroup per unit: for every phase of the unit (small phases only),
// evaluate all access events of the phase straight into LDS, sort them and
// scan for the first racy group.  No record touches HBM.
struct FusedSink {
    unsigned long long *lds;
    uint32_t *lds_n;
    unsigned long long pre;     // phase-in-group prefix of the key
    uint32_t ish;               // index shift (tid bits + 1)
    uint32_t tid;
    uint32_t cap;               // records the LDS array holds
    DEV void acc(bool act, uint32_t idx, uint32_t mode) {
        const uint64_t m = ballot(act);
        if (m == 0) return;
        uint32_t off = 0;
        if (lane_id() == 0) off = atomicAdd(lds_n, (uint32_t)__builtin_popcountll(m));
        off = __shfl(off, 0);
        const uint32_t pos = off + mbcnt(m);
        if (act && pos < cap)
            lds[ph(pos)] = pre | ((unsigned long long)idx << ish) | ((unsigned long long)tid << 1) | mode;
    }
};

// Compiled leaves in the fused kernel: at the start of a unit the
// workgroup evaluates, for the iterations the unit covers of each of the
// first FN_CACHE nests (as far as STAGE_WORDS allow), the phase, the thread
// limit and every uniform slot, one iteration per lane.  Each phase then
// only runs the lanes' access chains.
constexpr uint32_t STAGE_WORDS = 2048;
// Each staged nest also gets its access headers decoded into w (HSTRIDE
// words each: the fixed-form words and op count of the compiled access,
// then the offset of its op list in the code blob), and the nests with
// iterations in the unit are listed (act_*) when all of them are staged.
constexpr uint32_t HSTRIDE = 16;
static_assert(CAL_HDR + 1 <= HSTRIDE, "decoded access header");
struct FusedStage {
    uint32_t base[FN_CACHE];            // first word of the nest's block in w, or NONE32 (not staged)
    uint32_t cnt[FN_CACHE];             // staged iterations
    uint32_t acc[FN_CACHE];             // word offset of the access blocks in the compiled leaf
    unsigned long long f0[FN_CACHE];    // first staged iteration
    uint32_t all;                       // every nest with iterations in the unit is staged
    uint32_t nact;                      // ... and how many there are
    uint32_t act_ni[FN_CACHE], act_sb[FN_CACHE], act_cs[FN_CACHE], act_nacc[FN_CACHE], act_hofs[FN_CACHE];
    uint32_t w[STAGE_WORDS];            // per nest: phase - k0, thread limit, each slot (cnt words each), headers
};

// Index of one compiled access whose header was decoded to LDS at hp, for
// a header that may differ between lanes.
DEV uint32_t cal_index_lane(const uint32_t *hp, const uint32_t *__restrict__ code, uint32_t tid, const uint32_t *U,
                            uint32_t ustride) {
    if (hp[1] == 1u) {
        const uint32_t c0 = hp[2], m0k = hp[3], m0 = hp[4], a = hp[5], us = hp[6], pk = hp[7], pa = hp[8];
        uint32_t v = fixed_op(tid + c0, m0k, m0, hp[9], hp[10]) * a;
        if (us != NONE32) v += U[us * ustride];
        return fixed_op(v, pk, pa, hp[11], hp[12]);
    }
    const uint32_t *op = code + hp[CAL_HDR];
    uint32_t v = tid;
    for (uint32_t o = 0; o < hp[CAL_HDR - 1]; o++) {
        const uint32_t opw = op[2 * o], arg = op[2 * o + 1];
        const uint32_t x = (opw & C_UNI) ? U[arg * ustride] : arg;
        switch (opw & 0xFFu) {
        case C_ADD: v += x; break;
        case C_MUL: v *= x; break;
        case C_MONUS: v = v > x ? v - x : 0u; break;
        case C_RMONUS: v = x > v ? x - v : 0u; break;
        case C_DIV: v = x ? v / x : 0u; break;
        case C_MOD: v = x ? v % x : v; break;
        case C_SHL: v = x >= 32u ? 0u : v << x; break;
        case C_SHR: v = x >= 32u ? 0u : v >> x; break;
        case C_MIN: v = v < x ? v : x; break;
        case C_MAX: v = v > x ? v : x; break;
        default: v &= x; break;   // C_AND
        }
    }
    return v;
}


// ------------------------------------------- fused path: records in registers
// When every nest with iterations in a unit is staged, the unit's records
// are known by arithmetic: iteration i of listed nest a holds
// nacc_a * min(limit_i, n) records (access-major: record e is access
// e / L of tid e mod L).  The thread limits of the staged iterations are
// replaced by the prefix sums of these counts, and each thread then
// generates the records of a group at its own positions straight into
// registers (a cursor over the prefix sums), with no LDS record writes and
// no per-phase loop.
struct FastLds {
    uint32_t ptot[FN_CACHE];          // records of each listed nest's staged iterations
    uint32_t nbase[FN_CACHE + 1];     // prefix of the flat iteration list at each nest's first
    uint32_t mag[FN_CACHE], sh[FN_CACHE];   // division by each nest's access count
    uint32_t gs[64], ge[64], gc[64];  // groups of a window: phase offsets [gs, ge), records
    uint32_t ng;
    uint32_t G[FN_CACHE], ilo[FN_CACHE], plo[FN_CACHE];   // per group and nest: first record,
                                                           // first iteration, prefix there
};

// Division magic of d >= 1 for 32-bit dividends (the same construction as
// the planner's: Granlund and Montgomery, unsigned case).
DEV void div_magic_dev(uint32_t d, uint32_t &mag, uint32_t &sh) {
    uint32_t l = 0;
    while (l < 32 && (1ull << l) < d) l++;
    mag = (uint32_t)(((((1ull << l) - d) << 32) / d) + 1);
    sh = (l < 1 ? l : 1u) | ((l > 0 ? l - 1 : 0u) << 8);
}
DEV uint32_t div_by_magic(uint32_t x, uint32_t mag, uint32_t sh) {
    const uint32_t t = __umulhi(mag, x);
    return (t + ((x - t) >> (sh & 0xFFu))) >> (sh >> 8);
}

// First position in the non-decreasing ph[0..n) holding a value >= key.
DEV uint32_t lower_bound_u32(const uint32_t *ph, uint32_t n, uint32_t key) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t m = (lo + hi) >> 1;
        if (ph[m] < key) lo = m + 1;
        else hi = m;
    }
    return lo;
}

constexpr uint32_t FAST_CAP = 1u << 31;   // unit records the prefix sums may reach
DEV uint32_t sat_add(uint32_t a, uint32_t b) { return a + b < FAST_CAP && a + b >= a ? a + b : FAST_CAP; }

// Block-wide exclusive prefix of v (saturating at FAST_CAP); *total gets the
// saturated sum.  red: at least WG / 64 words.
DEV uint32_t block_excl_sat(uint32_t v, uint32_t *red, uint32_t &total) {
    uint32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, (unsigned)o);
        if ((int)lane_id() >= o) x = sat_add(x, y);
    }
    const uint32_t w = threadIdx.x >> 6;
    if (lane_id() == 63) red[w] = x;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    for (uint32_t q = 0; q < WG / 64; q++) {
        const uint32_t r = red[q];
        if (q < w) base = sat_add(base, r);
        tot = sat_add(tot, r);
    }
    total = tot;
    __syncthreads();
    return sat_add(base, x) - v;   // exact whenever the total is below FAST_CAP
}

template <typename T, bool WIDE, uint32_t FT = TILE>
DEV void fused_body(const Unit *__restrict__ units, uint32_t nunits, const uint32_t *__restrict__ nunits_dev,
                    uint32_t *__restrict__ qhead,
                    const NestDesc *__restrict__ nests, const ProtoDesc *__restrict__ protos,
                    const FixedVal *__restrict__ fixed, const uint32_t *__restrict__ code,
                    unsigned long long *__restrict__ phase_counts, unsigned long long *__restrict__ nrec,
                    uint32_t *__restrict__ ovf_flags, Cand *__restrict__ cands, Best *__restrict__ best,
                    uint32_t tile) {
    constexpr uint32_t FT_LDS = FT + FT / 32;
    constexpr uint32_t PACK = FUSED_PACK < FT ? FUSED_PACK : FT;
    __shared__ __align__(16) unsigned long long lds_rec[FT_LDS];
    __shared__ uint32_t lds_n;
    __shared__ uint32_t lds_res[RED_WORDS];
    __shared__ uint32_t lds_unit;
    __shared__ uint32_t lds_ovf;
    // per wave: the next unprocessed iteration of each of the protocol's
    // first FN_CACHE nests (each wave reads only its own row: no barrier)
    __shared__ unsigned long long lds_nf[WG / 64][FN_CACHE];
    __shared__ FusedStage lds_st;
    __shared__ FastLds lds_fx;
    unsigned long long *nf = lds_nf[threadIdx.x >> 6];
    if (nunits_dev) nunits = *nunits_dev;   // a graph replay: the count of this run
    // persistent: workgroups pull units (largest first) from a device queue
    for (;;) {
        if (threadIdx.x == 0) {
            lds_unit = atomicAdd(qhead, 1u);
            lds_ovf = 0;
        }
        __syncthreads();
        const uint32_t ui = lds_unit;
        if (ui >= nunits) break;
        const Unit u = units[ui];
        const bool stat = (u.flags & UNIT_STATIC) != 0;
        const ProtoDesc pd = protos[u.proto];
        Cand *my = &cands[ui];
        if (threadIdx.x == 0) { my->key = ~0ull; my->pair = 0; my->proto = u.proto; }
        bool have = false;
        unsigned long long total = 0;
        bool ovf = false;
        const bool pack = pd.pack != 0;
        const uint32_t tb = pack ? pd.tb : 31u;
        const uint32_t ish = tb + 1;
        const uint32_t psh = pack ? pd.ib + tb + 1 : 64u;   // phase-in-group shift
        const uint32_t ncache = pd.nnests < FN_CACHE ? pd.nnests : FN_CACHE;
        for (uint32_t ni = lane_id(); ni < ncache; ni += 64) nf[ni] = first_iter_at(nests[pd.nest0 + ni], u.k0);
        if constexpr (!WIDE) {
            if (threadIdx.x < 64) {
                // wave 0 plans the staging, lane ni for nest ni; nests are
                // staged in order while their words fit
                const uint32_t ni = threadIdx.x;
                uint32_t need = 0, acc = 0, nacc = 0, nuni = 0;
                uint64_t fa = 0, fb = 0;
                bool active = false;
                if (ni < pd.nnests) {
                    const NestDesc &nd = nests[pd.nest0 + ni];
                    if (u.k1 > nd.phase_base && u.k0 <= nd.phase_last) {
                        fa = first_iter_at(nd, u.k0);
                        fb = first_iter_at(nd, u.k1);
                        active = fb > fa;
                        if (active && ni < ncache && nd.cal_off != NONE32) {
                            const uint32_t *cal = code + nd.cal_off;
                            nacc = cal[0];
                            nuni = cal[1];
                            const uint64_t w = (2 + (uint64_t)nuni) * (fb - fa) + (uint64_t)HSTRIDE * nacc;
                            if (w <= STAGE_WORDS) {
                                need = (uint32_t)w;
                                acc = cal[2];
                            }
                        }
                    }
                }
                uint32_t inc = need;
                for (int o = 1; o < 64; o <<= 1) {
                    const uint32_t y = __shfl_up(inc, (unsigned)o);
                    if ((int)lane_id() >= o) inc += y;
                }
                const bool staged = need && inc <= STAGE_WORDS;
                if (ni < ncache) {
                    lds_st.base[ni] = staged ? inc - need : NONE32;
                    lds_st.cnt[ni] = (uint32_t)(fb - fa);
                    lds_st.acc[ni] = acc;
                    lds_st.f0[ni] = fa;
                }
                const bool all = ballot(active && !staged) == 0 && pd.nnests <= 64;
                const uint64_t sm = ballot(staged);
                if (staged) {
                    const uint32_t a = mbcnt(sm);
                    lds_st.act_ni[a] = ni;
                    lds_st.act_sb[a] = inc - need;
                    lds_st.act_cs[a] = (uint32_t)(fb - fa);
                    lds_st.act_nacc[a] = nacc;
                    lds_st.act_hofs[a] = inc - need + (2 + nuni) * (uint32_t)(fb - fa);
                }
                if (ni == 0) {
                    lds_st.all = all ? 1u : 0u;
                    lds_st.nact = (uint32_t)__builtin_popcountll(sm);
                }
            }
            __syncthreads();
            // staging in blocks of (nest, value): the phase and thread limit,
            // then each uniform slot, for all of the nest's staged iterations
            // (a lane per iteration); the waves take the blocks in turn, so a
            // block's program is the same on all lanes of its wave
            {
                const uint32_t wv = threadIdx.x >> 6;
                uint32_t blk = 0;
                for (uint32_t ni = 0; ni < ncache; ni++) {
                    const uint32_t sb = lds_st.base[ni];
                    if (sb == NONE32) continue;
                    const NestDesc &nd = nests[pd.nest0 + ni];
                    const uint32_t cs = lds_st.cnt[ni];
                    const uint32_t *cal = code + nd.cal_off;
                    const uint32_t nuni = rfl(cal[1]);
                    const uint32_t *up = cal + 3;
                    for (uint32_t z = 0; z <= nuni; z++) {   // z = 0: phase and limit; z > 0: slot z - 1
                        const uint32_t *prog = up;
                        if (z > 0) up += 1 + rfl(up[0]);
                        if ((blk++ & (WG / 64 - 1)) != wv) continue;
                        for (uint32_t fi = lane_id(); fi < cs; fi += 64) {
                            T vars[MAXSLOTS];
                            for (int y = 0; y < MAXSLOTS; y++) vars[y] = 0;
                            load_fixed<T>(nd, fixed, vars);
                            Odo<T> odo;
                            odo.start(nd, lds_st.f0[ni] + fi, vars);
                            if (z == 0) {
                                lds_st.w[sb + fi] = (uint32_t)(odo.phase - u.k0);
                                lds_st.w[sb + cs + fi] = tid_limit<T>(nd, code, vars, pd.n);
                            } else {
                                bool o = false;
                                lds_st.w[sb + (1 + z) * cs + fi] =
                                    (uint32_t)eval_expr<T, false>(prog + 1, rfl(prog[0]), vars, (T)0, o);
                            }
                        }
                    }
                }
            }
            // decoded access headers of the staged nests, a thread per nest
            if (threadIdx.x < lds_st.nact) {
                const uint32_t a = threadIdx.x;
                const uint32_t *cal = code + nests[pd.nest0 + lds_st.act_ni[a]].cal_off;
                const uint32_t *ap = cal + cal[2];
                uint32_t *hp = lds_st.w + lds_st.act_hofs[a];
                for (uint32_t j = 0; j < lds_st.act_nacc[a]; j++) {
                    for (uint32_t q = 0; q < CAL_HDR; q++) hp[q] = ap[q];
                    hp[CAL_HDR] = (uint32_t)(ap + CAL_HDR - code);
                    ap += CAL_HDR + 2 * ap[CAL_HDR - 1];
                    hp += HSTRIDE;
                }
            }
            __syncthreads();
        }
        // Records of a unit are produced group by group into LDS, by one of
        // two producers, then decided by the same code.  The arithmetic
        // producer runs when every nest with iterations in the unit is staged
        // and the unit's records stay below 2^31; the other one evaluates
        // the nests phase by phase.
        bool done = false;   // the arithmetic producer is used
        if constexpr (!WIDE) {
            if (lds_st.all != 0) {
                const uint32_t nact = lds_st.nact;
                // per-iteration record counts, their prefix sums over the flat
                // list of staged iterations (nest after nest), four a thread
                uint32_t nflat = 0;
                for (uint32_t a = 0; a < nact; a++) nflat += lds_st.act_cs[a];
                uint32_t rr[4], loc = 0, fa[4], fi[4];
                {
                    uint32_t a = 0, F = 0;
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        const uint32_t f = 4 * threadIdx.x + (uint32_t)q;
                        rr[q] = 0;
                        fa[q] = NONE32;
                        fi[q] = 0;
                        if (f < nflat) {
                            while (f >= F + lds_st.act_cs[a]) F += lds_st.act_cs[a++];
                            const uint32_t cs = lds_st.act_cs[a], i = f - F;
                            const uint32_t lim = lds_st.w[lds_st.act_sb[a] + cs + i];
                            const uint64_t r = (uint64_t)lds_st.act_nacc[a] * (lim < pd.n ? lim : pd.n);
                            rr[q] = r < FAST_CAP ? (uint32_t)r : FAST_CAP;
                            fa[q] = a;
                            fi[q] = i;
                        }
                        loc = sat_add(loc, rr[q]);
                    }
                }
                uint32_t tot = 0;
                const uint32_t excl = block_excl_sat(loc, lds_res, tot);
                if (tot < FAST_CAP) {
                    done = true;
                    uint32_t pf[4];
                    {
                        uint32_t run = excl;
#pragma unroll
                        for (int q = 0; q < 4; q++) {
                            pf[q] = run;
                            run += rr[q];
                            if (fa[q] != NONE32 && fi[q] == 0) lds_fx.nbase[fa[q]] = pf[q];
                        }
                    }
                    if (threadIdx.x == 0) lds_fx.nbase[nact] = tot;
                    __syncthreads();
                    // the thread limits become the prefix sums within each nest
#pragma unroll
                    for (int q = 0; q < 4; q++)
                        if (fa[q] != NONE32)
                            lds_st.w[lds_st.act_sb[fa[q]] + lds_st.act_cs[fa[q]] + fi[q]] = pf[q] - lds_fx.nbase[fa[q]];
                    if (threadIdx.x < nact) {
                        const uint32_t a = threadIdx.x;
                        lds_fx.ptot[a] = lds_fx.nbase[a + 1] - lds_fx.nbase[a];
                        div_magic_dev(lds_st.act_nacc[a], lds_fx.mag[a], lds_fx.sh[a]);
                    }
                    __syncthreads();
                }
            }
        }
        // prefix of listed nest a at staged iteration i (i <= cs)
        auto pref = [&](uint32_t a, uint32_t i) -> uint32_t {
            const uint32_t cs = lds_st.act_cs[a];
            return i < cs ? lds_st.w[lds_st.act_sb[a] + cs + i] : lds_fx.ptot[a];
        };
        uint64_t k = u.k0;                 // next phase (evaluating producer)
        uint64_t kw = u.k0, kwc = u.k0;    // next window / current window (arithmetic producer)
        uint32_t g = 0, ngr = 0;           // next group of the current window, groups in it
        for (;;) {
            uint64_t gk0;
            uint32_t cnt;
            if (done) {
                const uint32_t nact = lds_st.nact;
                if (g == ngr) {
                    if (kw >= u.k1) break;
                    // the next window of up to 64 phases: records of each phase
                    // (a lane per phase), then phases packed into groups
                    const uint32_t nw = (uint32_t)(u.k1 - kw < 64 ? u.k1 - kw : 64);
                    const uint32_t krw = (uint32_t)(kw - u.k0);
                    if (threadIdx.x < 64) {
                        const uint32_t l = threadIdx.x;
                        uint32_t c = 0;
                        if (l < nw) {
                            for (uint32_t a = 0; a < nact; a++) {
                                const uint32_t *phs = lds_st.w + lds_st.act_sb[a];
                                const uint32_t cs = lds_st.act_cs[a];
                                const uint32_t lo = lower_bound_u32(phs, cs, krw + l);
                                const uint32_t hi = lower_bound_u32(phs, cs, krw + l + 1);
                                c += pref(a, hi) - pref(a, lo);
                            }
                            if (stat && c != 0) phase_counts[kw + l] = c;
                        }
                        // the same scalar loop on every lane: empty phases are
                        // passed over, a phase above the tile (in HBM) ends a group
                        uint32_t ng = 0, est = 0, gs = NONE32;
                        for (uint32_t q = 0; q < nw; q++) {
                            const uint32_t cq = readlane(c, q);
                            if (cq == 0) continue;
                            const bool big = cq > tile;
                            if (gs != NONE32 &&
                                (big || !pack || est + cq > PACK || ((uint64_t)(q - gs) >> (64 - psh)) != 0)) {
                                if (l == 0) {
                                    lds_fx.gs[ng] = gs;
                                    lds_fx.ge[ng] = q;
                                    lds_fx.gc[ng] = est;
                                }
                                ng++;
                                gs = NONE32;
                            }
                            if (big) continue;
                            if (gs == NONE32) {
                                gs = q;
                                est = 0;
                            }
                            est += cq;
                        }
                        if (gs != NONE32) {
                            if (l == 0) {
                                lds_fx.gs[ng] = gs;
                                lds_fx.ge[ng] = nw;
                                lds_fx.gc[ng] = est;
                            }
                            ng++;
                        }
                        if (l == 0) lds_fx.ng = ng;
                    }
                    __syncthreads();
                    ngr = lds_fx.ng;
                    g = 0;
                    kwc = kw;
                    kw += 64;
                    __syncthreads();   // lds_fx.ng is read before the next window writes it
                    continue;
                }
                const uint32_t gs = lds_fx.gs[g], ge = lds_fx.ge[g];
                cnt = lds_fx.gc[g];
                g++;
                gk0 = kwc + gs;
                const uint32_t krw = (uint32_t)(kwc - u.k0);
                if (threadIdx.x < 64) {
                    // each nest's first record, first iteration and prefix there
                    const uint32_t a = threadIdx.x;
                    uint32_t q = 0, ilo = 0, plo = 0;
                    if (a < nact) {
                        const uint32_t *phs = lds_st.w + lds_st.act_sb[a];
                        const uint32_t cs = lds_st.act_cs[a];
                        ilo = lower_bound_u32(phs, cs, krw + gs);
                        const uint32_t ihi = lower_bound_u32(phs, cs, krw + ge);
                        plo = pref(a, ilo);
                        q = pref(a, ihi) - plo;
                    }
                    uint32_t inc = q;
                    for (int o = 1; o < 64; o <<= 1) {
                        const uint32_t y = __shfl_up(inc, (unsigned)o);
                        if ((int)lane_id() >= o) inc += y;
                    }
                    if (a < nact) {
                        lds_fx.G[a] = inc - q;
                        lds_fx.ilo[a] = ilo;
                        lds_fx.plo[a] = plo;
                    }
                }
                __syncthreads();
                // each thread writes a contiguous block of the group's records;
                // it locates its first record (nest by the group bases,
                // iteration by a binary search over the prefix sums), then
                // walks tid, access and iteration forward (access-major:
                // record e of an iteration is access e / L of tid e mod L)
                {
                    const uint32_t per = (cnt + WG - 1) / WG;
                    uint32_t p = threadIdx.x * per;
                    const uint32_t pend = p + per < cnt ? p + per : cnt;
                    while (p < pend) {
                        uint32_t a = 0;
                        for (uint32_t b = 1; b < nact; b++)
                            if (lds_fx.G[b] <= p) a = b;
                        const uint32_t sb = lds_st.act_sb[a], cs = lds_st.act_cs[a], na = lds_st.act_nacc[a];
                        const uint32_t ptot = lds_fx.ptot[a];
                        const uint32_t *P = lds_st.w + sb + cs;        // prefix sums of nest a
                        const uint32_t qq = p - lds_fx.G[a] + lds_fx.plo[a];
                        // the largest i in [ilo, cs) with P[i] <= qq (P[cs] = ptot > qq)
                        uint32_t lo = lds_fx.ilo[a], hi = cs - 1;
                        while (lo < hi) {
                            const uint32_t m = (lo + hi + 1) >> 1;
                            if (P[m] <= qq) lo = m;
                            else hi = m - 1;
                        }
                        const uint32_t i = lo;
                        const uint32_t p0 = P[i], pn = i + 1 < cs ? P[i + 1] : ptot;
                        const uint32_t L = div_by_magic(pn - p0, lds_fx.mag[a], lds_fx.sh[a]);
                        uint32_t tid = qq - p0, j = 0;
                        while (tid >= L && j + 1 < na) {   // j < na: the iteration holds na * L records
                            tid -= L;
                            j++;
                        }
                        if (tid >= L) break;   // cannot happen (qq < pn = p0 + na * L); ends the block
                        const uint32_t *U = lds_st.w + sb + 2 * cs + i;
                        const unsigned long long pre =
                            pack ? ((unsigned long long)(lds_st.w[sb + i] + u.k0 - gk0) << psh) : 0ull;
                        // the rest of this iteration, access by access
                        for (; j < na && p < pend; j++) {
                            const uint32_t *hp = lds_st.w + lds_st.act_hofs[a] + j * HSTRIDE;
                            const uint32_t mode = hp[0];
                            const uint32_t t1 = tid + (pend - p < L - tid ? pend - p : L - tid);
                            if (hp[1] == 1u && hp[3] != CAL_K_AND && hp[7] != CAL_K_AND) {
                                // fixed form v = ((tid + c0) m0-op m0) * a + U, then pk-op pa,
                                // advanced tid by tid: x = (tid + c0) mod m0 steps by one
                                // (back to 0 at m0), v by a (mod pa: one conditional
                                // subtraction of pa); every value stays below 2^32 (32-bit plan)
                                const uint32_t c0 = hp[2], m0k = hp[3], m0 = hp[4], am = hp[5], us = hp[6];
                                const uint32_t pk = hp[7], pa = hp[8], m0mag = hp[9], m0sh = hp[10];
                                const uint32_t pamag = hp[11], pash = hp[12];
                                const uint32_t uv = us != NONE32 ? U[us * cs] : 0u;
                                const bool pmod = pk == CAL_K_MOD, xmod = m0k == CAL_K_MOD;
                                const uint32_t astep = pmod ? fixed_op(am, CAL_K_MOD, pa, pamag, pash) : am;
                                const uint32_t v0 = fixed_op(uv, pk, pa, pamag, pash);   // v at x = 0
                                uint32_t x = fixed_op(tid + c0, m0k, m0, m0mag, m0sh);
                                uint32_t v = fixed_op(x * am + uv, pk, pa, pamag, pash);
                                for (; tid < t1; tid++, p++) {
                                    lds_rec[ph(p)] = pre | ((unsigned long long)v << ish) |
                                                     ((unsigned long long)tid << 1) | mode;
                                    x++;
                                    if (xmod && x == m0) {
                                        x = 0;
                                        v = v0;
                                    } else if (pmod) {
                                        v = v >= pa - astep ? v - (pa - astep) : v + astep;
                                    } else {
                                        v += astep;
                                    }
                                }
                            } else if (hp[1] == 1u) {
                                const uint32_t c0 = hp[2], m0k = hp[3], m0 = hp[4], am = hp[5], us = hp[6];
                                const uint32_t pk = hp[7], pa = hp[8], m0mag = hp[9], m0sh = hp[10];
                                const uint32_t pamag = hp[11], pash = hp[12];
                                const uint32_t uv = us != NONE32 ? U[us * cs] : 0u;
                                for (; tid < t1; tid++, p++) {
                                    const uint32_t v = fixed_op(fixed_op(tid + c0, m0k, m0, m0mag, m0sh) * am + uv, pk, pa,
                                                                pamag, pash);
                                    lds_rec[ph(p)] = pre | ((unsigned long long)v << ish) |
                                                     ((unsigned long long)tid << 1) | mode;
                                }
                            } else {
                                for (; tid < t1; tid++, p++) {
                                    const uint32_t v = cal_index_lane(hp, code, tid, U, cs);
                                    lds_rec[ph(p)] = pre | ((unsigned long long)v << ish) |
                                                     ((unsigned long long)tid << 1) | mode;
                                }
                            }
                            tid = 0;
                        }
                    }
                }
                __syncthreads();
            } else {
                // one group of consecutive phases whose events fit one tile
                gk0 = k;
                if (threadIdx.x == 0) lds_n = 0;
                __syncthreads();
                if (threadIdx.x == 0) lds_n = 0;
                __syncthreads();
                uint32_t est = 0, before = 0;
                bool any = false;
                while (k < u.k1) {
                    uint32_t c;
                    if (!stat) {
                        const unsigned long long ck = phase_counts[k];
                        if (ck == 0 || ck > (unsigned long long)tile) {   // empty or in HBM
                            k++;
                            if (!any) gk0 = k;
                            continue;
                        }
                        c = (uint32_t)ck;
                    } else {
                        c = pd.phase_bound;
                    }
                    // a packed group's phases must fit the key bits above the index
                    if (any && (!pack || est + c > PACK || ((k - gk0) >> (64 - psh)) != 0)) break;
                    const unsigned long long pre = pack ? ((unsigned long long)(k - gk0) << psh) : 0ull;
                    for (uint32_t ni = 0; ni < pd.nnests; ni++) {
                        const NestDesc &nd = nests[pd.nest0 + ni];
                        if (k < nd.phase_base || k > nd.phase_last) continue;
                        if constexpr (!WIDE) {
                            const uint32_t sb = ni < ncache ? lds_st.base[ni] : NONE32;
                            if (sb != NONE32) {
                                const uint32_t cs = lds_st.cnt[ni];
                                const uint32_t kr = (uint32_t)(k - u.k0);
                                uint32_t i = (uint32_t)(nf[ni] - lds_st.f0[ni]);
                                while (i < cs && rfl(lds_st.w[sb + i]) < kr) i++;   // phases skipped since
                                const uint32_t *cal = code + nd.cal_off;
                                const uint32_t nacc = rfl(cal[0]);
                                const uint32_t *acc0 = cal + rfl(lds_st.acc[ni]);
                                for (; i < cs && rfl(lds_st.w[sb + i]) == kr; i++) {
                                    const uint32_t lim = rfl(lds_st.w[sb + cs + i]);
                                    const uint32_t *U = lds_st.w + sb + 2 * cs + i;
                                    for (uint32_t t0 = 0; t0 < lim; t0 += WG) {
                                        const uint32_t tid = t0 + threadIdx.x;
                                        const bool act = tid < pd.n && tid < lim;
                                        // one reservation per wave for all accesses (no branches)
                                        const uint64_t m = ballot(act);
                                        if (m == 0) continue;
                                        const uint32_t na = (uint32_t)__builtin_popcountll(m);
                                        uint32_t r0 = 0;
                                        if (lane_id() == 0) r0 = atomicAdd(&lds_n, na * nacc);
                                        const uint32_t p0 = readlane(r0, 0) + mbcnt(m);
                                        const uint32_t *ap = acc0;
                                        for (uint32_t j = 0; j < nacc; j++) {
                                            const uint32_t mode = rfl(ap[0]);
                                            const uint32_t v = cal_index(ap, tid, U, cs);
                                            const uint32_t pos = p0 + j * na;
                                            if (act && pos < FT)
                                                lds_rec[ph(pos)] = pre | ((unsigned long long)v << ish) |
                                                                   ((unsigned long long)tid << 1) | mode;
                                            ap += CAL_HDR + 2 * rfl(ap[CAL_HDR - 1]);
                                        }
                                    }
                                }
                                nf[ni] = lds_st.f0[ni] + i;
                                continue;
                            }
                        }
                        // the cached iteration is the first of phase k unless
                        // phases were skipped since (then search again)
                        uint64_t fa = ni < ncache ? nf[ni] : first_iter_at(nd, k);
                        if (fa < nd.iters && phase_of(nd, fa) < k) fa = first_iter_at(nd, k);
                        if (fa >= nd.iters) continue;
                        T vars[MAXSLOTS];
                        for (int s = 0; s < MAXSLOTS; s++) vars[s] = 0;
                        load_fixed<T>(nd, fixed, vars);
                        Odo<T> odo;
                        odo.start(nd, fa, vars);
                        const uint32_t *leaf = code + nd.code_off;
                        uint64_t f = fa;
                        for (; f < nd.iters && odo.phase == k; f++) {
                            const uint32_t lim = tid_limit<T>(nd, code, vars, pd.n);
                            for (uint32_t t0 = 0; t0 < lim; t0 += WG) {
                                const uint32_t tid = t0 + threadIdx.x;
                                FusedSink sink{lds_rec, &lds_n, pre, ish, tid, FT};
                                run_leaf<T, WIDE>(leaf, vars, (T)tid, tid < pd.n, ovf, sink);
                            }
                            odo.next(nd, vars);
                        }
                        if (ni < ncache) nf[ni] = f;
                    }
                    if (stat) {
                        __syncthreads();
                        const uint32_t now = lds_n;
                        if (threadIdx.x == 0) phase_counts[k] = now - before;
                        before = now;
                        __syncthreads();
                    }
                    est += c;
                    any = true;
                    k++;
                }
                if (!any) break;
                __syncthreads();
                cnt = lds_n;
            }
            total += cnt;
            if (cnt > FT) {
                // more events than the count or the plan bounded: the records
                // past the tile were dropped, so the protocol gets an error
                // status instead of a verdict
                if (threadIdx.x == 0) atomicOr(&ovf_flags[u.proto], OVF_LIMIT);
                cnt = FT;
            }
            if (cnt == 0) {
                __syncthreads();
                continue;
            }
            // the records move to registers (lanes past the end copy a real
            // one) and the whole LDS array becomes the decision's scratch
            constexpr int FE = FT / WG;
            unsigned long long v[FE];
#pragma unroll
            for (int jj = 0; jj < FE; jj++) {
                const uint32_t i = (uint32_t)jj * WG + threadIdx.x;
                if ((uint32_t)jj * WG < cnt) v[jj] = lds_rec[ph(i < cnt ? i : cnt - 1)];
                else v[jj] = v[0];
            }
            __syncthreads();
            unsigned long long key = 0;
            uint32_t r1 = 0, r2 = 0;
            const bool f = decide<FE, WG, FT_LDS, true>(v, cnt, tb, lds_rec, lds_res, key, r1, r2);
            if (f && !have) {
                have = true;
                const uint64_t kk = gk0 + (pack ? (key >> pd.ib) : 0ull);
                const uint32_t idx = pack ? (uint32_t)(key & ((1ull << pd.ib) - 1)) : (uint32_t)key;
                if (threadIdx.x == 0) offer(best, my, u.proto, (uint32_t)(kk - pd.phase_off), idx, r1, r2);
            }
            __syncthreads();
        }
        if (stat) {
            if (ballot(ovf) != 0 && lane_id() == 0) atomicOr(&lds_ovf, 1u);
            __syncthreads();
            if (threadIdx.x == 0) {
                atomicAdd(&nrec[u.proto], total);
                if (lds_ovf) atomicOr(&ovf_flags[u.proto], OVF_RANGE);
            }
        }
        __syncthreads();
    }
}

#define FUSED_PARAMS                                                                                    \
    const Unit *__restrict__ units, uint32_t nunits, const uint32_t *__restrict__ nunits_dev,            \
        uint32_t *__restrict__ qhead,                                                                   \
        const NestDesc *__restrict__ nests, const ProtoDesc *__restrict__ protos,                       \
        const FixedVal *__restrict__ fixed, const uint32_t *__restrict__ code,                          \
        unsigned long long *__restrict__ phase_counts, unsigned long long *__restrict__ nrec,           \
        uint32_t *__restrict__ ovf_flags, Cand *__restrict__ cands, Best *__restrict__ best, uint32_t tile
#define FUSED_ARGS \
    units, nunits, nunits_dev, qhead, nests, protos, fixed, code, phase_counts, nrec, ovf_flags, cands, best, tile
// 32-bit evaluator: two workgroups per CU fit the LDS, so ask for the
// registers of two waves per SIMD.  The 64-bit one keeps its natural
// allocation (bounding it would spill).
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(2))) void k_fused32(FUSED_PARAMS) {
    fused_body<uint32_t, false>(FUSED_ARGS);
}
__global__ __launch_bounds__(WG) void k_fused64(FUSED_PARAMS) { fused_body<uint64_t, true>(FUSED_ARGS); }
#undef FUSED_PARAMS
#undef FUSED_ARGS

// =============================================================== partition
// Runs of equal digits in consecutive lanes of a wave whose valid lanes are
// [0, nv): whether this lane heads a run, the run's length (on its head)
// and the run's head lane (on every lane).  Records arrive in emission
// order, so neighbouring lanes often share a digit: one atomic per run then
// replaces one per lane (atomics on one address serialize).
DEV void digit_runs(uint32_t d, uint32_t nv, bool &head, uint32_t &len, uint32_t &hl) {
    const uint32_t l = lane_id();
    const uint32_t dp = __shfl_up(d, 1u);
    head = l < nv && (l == 0 || dp != d);
    const uint64_t H = ballot(head);
    const uint64_t after = H & bits_from(l + 1);
    const uint32_t nh = after ? ctz64(after) : 64u;
    len = (nh < nv ? nh : nv) - l;
    const uint64_t upto = H & ~bits_from(l + 1);
    hl = upto ? 63u - (uint32_t)__builtin_clzll(upto) : 0u;
}

__global__ __launch_bounds__(WG) void k_hist(const Seg *__restrict__ segs, const Chunk *__restrict__ chunks,
                                              const unsigned long long *__restrict__ in,
                                              unsigned long long *__restrict__ hist) {
    __shared__ uint32_t h[RADIX];
    const Chunk ch = chunks[blockIdx.x];
    const Seg sg = segs[ch.seg];
    for (uint32_t i = threadIdx.x; i < RADIX; i += WG) h[i] = 0;
    __syncthreads();
    const uint64_t b = sg.start + (uint64_t)ch.c * CHUNK;
    const uint32_t n = (uint32_t)((sg.start + sg.len < b + CHUNK) ? sg.start + sg.len - b : CHUNK);
    const uint32_t mask = (1u << sg.dbits) - 1;
    // all loads of a thread are issued before its first atomic
    unsigned long long r[CHUNK / WG];
#pragma unroll
    for (int j = 0; j < CHUNK / WG; j++) {
        const uint32_t i = (uint32_t)j * WG + threadIdx.x;
        r[j] = in[b + (i < n ? i : n - 1)];
    }
    // one atomic per run of equal digits
#pragma unroll
    for (int j = 0; j < CHUNK / WG; j++) {
        const bool v = (uint32_t)j * WG + threadIdx.x < n;   // the valid lanes are a prefix
        const uint32_t d = (rec_idx(r[j]) >> sg.shift) & mask;
        const uint32_t nv = (uint32_t)__builtin_popcountll(ballot(v));
        bool head;
        uint32_t len, hl;
        digit_runs(d, nv, head, len, hl);
        if (head) atomicAdd(&h[d], len);
    }
    __syncthreads();
    const uint32_t nd = 1u << sg.dbits;
    for (uint32_t d = threadIdx.x; d < nd; d += WG) hist[sg.hbase + (uint64_t)ch.c * nd + d] = h[d];
}

// Per segment: each digit's count in every chunk becomes the output
// position of that chunk's first record of the digit (digit bases in digit
// order, chunks in order within a digit); starts[sbase + d] = first output
// position of digit d.  One workgroup per segment; each thread walks the
// chunks for its digits (reads coalesced across digits).
__global__ __launch_bounds__(WG) void k_offsets(const Seg *__restrict__ segs, uint32_t nsegs,
                                                 unsigned long long *__restrict__ hist,
                                                 unsigned long long *__restrict__ starts) {
    __shared__ unsigned long long tot[RADIX];
    const uint32_t s = blockIdx.x;
    if (s >= nsegs) return;
    const Seg sg = segs[s];
    const uint32_t nd = 1u << sg.dbits;
    unsigned long long *H = hist + sg.hbase;
    for (uint32_t d = threadIdx.x; d < nd; d += WG) {
        unsigned long long t = 0;
#pragma unroll 8
        for (uint32_t c = 0; c < sg.nchunks; c++) t += H[(uint64_t)c * nd + d];
        tot[d] = t;
    }
    __syncthreads();
    {
        // exclusive scan of the digit totals: each thread takes nd / WG
        // consecutive digits, then a wave and a cross-wave scan
        __shared__ unsigned long long wsum[WG / 64];
        const uint32_t per = (nd + WG - 1) / WG;
        const uint32_t d0 = threadIdx.x * per;
        unsigned long long loc = 0;
        for (uint32_t k = 0; k < per; k++)
            if (d0 + k < nd) loc += tot[d0 + k];
        unsigned long long inc = loc;
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned long long y = __shfl_up(inc, (unsigned)o);
            if ((int)lane_id() >= o) inc += y;
        }
        if (lane_id() == 63) wsum[threadIdx.x >> 6] = inc;
        __syncthreads();
        unsigned long long run = sg.obase + inc - loc;
        for (uint32_t w = 0; w < (threadIdx.x >> 6); w++) run += wsum[w];
        for (uint32_t k = 0; k < per; k++) {
            if (d0 + k < nd) {
                const unsigned long long t = tot[d0 + k];
                tot[d0 + k] = run;
                run += t;
            }
        }
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < nd; d += WG) {
        unsigned long long run = tot[d];
        starts[(uint64_t)sg.sbase + d] = run;
#pragma unroll 8
        for (uint32_t c = 0; c < sg.nchunks; c++) {
            const unsigned long long x = H[(uint64_t)c * nd + d];
            H[(uint64_t)c * nd + d] = run;
            run += x;
        }
    }
}

__global__ __launch_bounds__(WG) void k_scatter(const Seg *__restrict__ segs, const Chunk *__restrict__ chunks,
                                                 const unsigned long long *__restrict__ in,
                                                 const unsigned long long *__restrict__ offs,
                                                 unsigned long long *__restrict__ out, unsigned long long cap) {
    __shared__ uint32_t cur[RADIX];
    __shared__ unsigned long long base[RADIX];
    const Chunk ch = chunks[blockIdx.x];
    const Seg sg = segs[ch.seg];
    const uint32_t nd = 1u << sg.dbits;
    for (uint32_t d = threadIdx.x; d < nd; d += WG) {
        cur[d] = 0;
        base[d] = offs[sg.hbase + (uint64_t)ch.c * nd + d];
    }
    __syncthreads();
    const uint64_t b = sg.start + (uint64_t)ch.c * CHUNK;
    const uint32_t n = (uint32_t)((sg.start + sg.len < b + CHUNK) ? sg.start + sg.len - b : CHUNK);
    const uint32_t mask = nd - 1;
    unsigned long long r[CHUNK / WG];
#pragma unroll
    for (int j = 0; j < CHUNK / WG; j++) {
        const uint32_t i = (uint32_t)j * WG + threadIdx.x;
        r[j] = in[b + (i < n ? i : n - 1)];
    }
    // one reservation per run of equal digits; a run's records go to
    // consecutive positions
#pragma unroll
    for (int j = 0; j < CHUNK / WG; j++) {
        const bool v = (uint32_t)j * WG + threadIdx.x < n;   // the valid lanes are a prefix
        const uint32_t d = (rec_idx(r[j]) >> sg.shift) & mask;
        const uint32_t nv = (uint32_t)__builtin_popcountll(ballot(v));
        bool head;
        uint32_t len, hl;
        digit_runs(d, nv, head, len, hl);
        uint32_t b0 = 0;
        if (head) b0 = atomicAdd(&cur[d], len);
        const uint32_t o = (uint32_t)__shfl((int)b0, (int)hl) + (lane_id() - hl);
        if (v && base[d] + o < cap) out[base[d] + o] = r[j];
    }
}

// ================================================================== tiles
// Tile records are read straight into registers (all loads issued before
// any use; lanes past the end re-read the last record, so no branch sits
// between the loads).
template <int E>
DEV void tile_run(const Tile &t, const unsigned long long *__restrict__ src, unsigned long long *a, uint32_t *red,
                  Cand *my, Best *best) {
    const uint32_t cnt = t.len;
    unsigned long long u[E];
    const uint32_t last = cnt - 1;
#pragma unroll
    for (int j = 0; j < E; j++) {
        const uint32_t i = (uint32_t)j * TWG + threadIdx.x;
        u[j] = src[i < cnt ? i : last];
    }
    unsigned long long key;
    uint32_t r1, r2;
    const bool f = decide<E, TWG>(u, cnt, 31, a, red, key, r1, r2);
    if (f && threadIdx.x == 0) offer(best, my, t.proto, t.phase, (uint32_t)key, r1, r2);
}

// two workgroups per CU fit the LDS: ask for the registers of four waves per SIMD
__global__ __launch_bounds__(TWG) __attribute__((amdgpu_waves_per_eu(4))) void k_tile(
    const Tile *__restrict__ tiles, const unsigned long long *__restrict__ recs, Cand *__restrict__ cands,
    Best *__restrict__ best) {
    __shared__ __align__(16) unsigned long long lds_rec[TILE_LDS];
    __shared__ uint32_t lds_res[RED_WORDS];
    const Tile t = tiles[blockIdx.x];
    Cand *my = &cands[blockIdx.x];
    if (threadIdx.x == 0) { my->key = ~0ull; my->pair = 0; my->proto = t.proto; }
    const uint32_t cnt = t.len;
    if (cnt == 0) return;
    uint32_t npow = TWG;
    while (npow < cnt) npow <<= 1;
    const unsigned long long *src = recs + t.start;
    switch (npow / TWG) {
    case 1: tile_run<1>(t, src, lds_rec, lds_res, my, best); break;
    case 2: tile_run<2>(t, src, lds_rec, lds_res, my, best); break;
    case 4: tile_run<4>(t, src, lds_rec, lds_res, my, best); break;
    case 8: tile_run<8>(t, src, lds_rec, lds_res, my, best); break;
    default: tile_run<16>(t, src, lds_rec, lds_res, my, best); break;
    }
}

// ============================================= single-index large groups
// All records of a group share one index.  Pass 1: least tid, least writer,
// largest tid.  Pass 2 (when the least tid writes): least tid != t0.

__global__ __launch_bounds__(WG) void k_single1(const Group *__restrict__ groups, uint32_t ngroups,
                                                 const unsigned long long *__restrict__ recs, SingleAcc *__restrict__ acc) {
    const Group g = groups[blockIdx.y];
    uint32_t t0 = NONE32, w0 = NONE32, tm = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * WG + threadIdx.x; i < g.len; i += (uint64_t)gridDim.x * WG) {
        const unsigned long long r = recs[g.start + i];
        const uint32_t t = rec_tid(r);
        t0 = t < t0 ? t : t0;
        tm = t > tm ? t : tm;
        if (r & 1ull) w0 = t < w0 ? t : w0;
    }
    t0 = wave_min(t0);
    w0 = wave_min(w0);
    tm = wave_max(tm);
    if (lane_id() == 0) {
        atomicMin(&acc[blockIdx.y].t0, t0);
        atomicMin(&acc[blockIdx.y].w0, w0);
        atomicMax(&acc[blockIdx.y].tmax, tm);
    }
}

__global__ __launch_bounds__(WG) void k_single2(const Group *__restrict__ groups, uint32_t ngroups,
                                                 const unsigned long long *__restrict__ recs, SingleAcc *__restrict__ acc) {
    const Group g = groups[blockIdx.y];
    const uint32_t t0 = acc[blockIdx.y].t0;
    uint32_t t1 = NONE32;
    for (uint64_t i = (uint64_t)blockIdx.x * WG + threadIdx.x; i < g.len; i += (uint64_t)gridDim.x * WG) {
        const uint32_t t = rec_tid(recs[g.start + i]);
        if (t != t0 && t < t1) t1 = t;
    }
    t1 = wave_min(t1);
    if (lane_id() == 0) atomicMin(&acc[blockIdx.y].t1, t1);
}

__global__ void k_single3(const Group *__restrict__ groups, uint32_t ngroups, const unsigned long long *__restrict__ recs,
                          const SingleAcc *__restrict__ acc, Cand *__restrict__ cands, Best *__restrict__ best) {
    const uint32_t gi = blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= ngroups) return;
    const Group g = groups[gi];
    const SingleAcc a = acc[gi];
    Cand *my = &cands[gi];
    my->key = ~0ull;
    my->pair = 0;
    my->proto = g.proto;
    if (a.w0 != NONE32 && a.tmax != a.t0) {
        const uint32_t idx = rec_idx(recs[g.start]);
        offer(best, my, g.proto, g.phase, idx, a.t0, a.w0 == a.t0 ? a.t1 : a.w0);
    }
}

// ==================================================== witness pair pick
__global__ void k_pick(const Cand *__restrict__ cands, uint64_t n, const uint32_t *__restrict__ n_dev,
                       Best *__restrict__ best) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n_dev) n = *n_dev;
    if (i >= n) return;
    const Cand c = cands[i];
    if (c.key != ~0ull && c.key == best[c.proto].key) best[c.proto].pair = c.pair;
}

// ================================================================ results
// Least racy cell of each table phase (a second tid and a writer): blocks
// of a table scan strided slices of its cells; each thread's first racy
// cell is the least of its slice, and the minimum reaches tmin by
// atomicMin.
__global__ void k_table_scan(const TablePhase *__restrict__ tp, const uint32_t *__restrict__ tabs,
                             uint32_t *__restrict__ tmin) {
    const TablePhase t = tp[blockIdx.y];
    const uint32_t *t1 = tabs + t.off + t.cells, *w0 = t1 + t.cells;
    uint32_t first = NONE32;
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < t.cells; c += gridDim.x * blockDim.x)
        if (t1[c] != NONE32 && w0[c] != NONE32) {
            first = c;
            break;
        }
    first = wave_min(first);
    if (lane_id() == 0 && first != NONE32) atomicMin(&tmin[blockIdx.y], first);
}

// The witness candidate of each table phase: its least racy cell with the
// pair (t0, t1) if t0 writes, else (t0, w0).
__global__ void k_table_offer(const TablePhase *__restrict__ tp, uint32_t ntp, const uint32_t *__restrict__ tabs,
                              const uint32_t *__restrict__ tmin, Cand *__restrict__ cands, Best *__restrict__ best) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ntp) return;
    const TablePhase t = tp[j];
    Cand *my = &cands[j];
    my->key = ~0ull;
    my->pair = 0;
    my->proto = t.proto;
    const uint32_t c = tmin[j];
    if (c == NONE32) return;
    const uint32_t *t0 = tabs + t.off;
    const uint32_t a = t0[c], b = t0[t.cells + c], w = t0[2 * t.cells + c];
    offer(best, my, t.proto, t.phase, c, a, w == a ? b : w);
}

__global__ void k_result(uint32_t count, const uint32_t *__restrict__ count_dev, const ResultIn *__restrict__ rin,
                         const Best *__restrict__ best, const unsigned long long *__restrict__ nrec,
                         const uint32_t *__restrict__ ovf_flags, drf_result_dev *__restrict__ out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (count_dev) count = *count_dev;
    if (i >= count) return;
    ResultIn r = rin[i];
    if (r.flags & RESULT_FROM_DEVICE) {
        r.num_records = nrec[i];
        if (ovf_flags[i] & OVF_RANGE) r.status = -7;   // range overflow found while evaluating
    }
    if (r.status == 0 && (ovf_flags[i] & OVF_LIMIT)) r.status = -10;
    drf_result_dev o;
    o.status = r.status;
    o.racy = 0;
    o.phase = o.index = o.tid_i = o.tid_j = NONE32;
    o.num_records = 0;
    o.num_phases = 0;
    o.reserved = 0;
    if (r.status == 0) {
        const Best b = best[i];
        o.num_records = r.num_records;
        o.num_phases = r.num_phases;
        if (b.key != ~0ull) {
            o.racy = 1;
            o.phase = (uint32_t)(b.key >> 32);
            o.index = (uint32_t)b.key;
            o.tid_i = (uint32_t)(b.pair >> 32);
            o.tid_j = (uint32_t)b.pair;
        }
    }
    out[i] = o;
}

// ================================================================== fills
// (graph-safe replacements for memset: kernels, never memset nodes)
__global__ void k_fill_u32(uint32_t *__restrict__ p, uint32_t v, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Block b fills part of the fill whose block range holds b.
__global__ void k_fill_multi(FillList L) {
    const uint32_t b = blockIdx.x;
    uint32_t f = 0;
    while (f + 1 < L.count && b >= L.b0[f + 1]) f++;
    const uint64_t nb = (f + 1 < L.count ? L.b0[f + 1] : gridDim.x) - L.b0[f];
    uint32_t *__restrict__ p = L.p[f];
    const uint32_t v = L.v[f];
    const uint64_t n = L.n[f];
    for (uint64_t i = (uint64_t)(b - L.b0[f]) * 256 + threadIdx.x; i < n; i += nb * 256) p[i] = v;
}

__global__ void k_init_acc(SingleAcc *__restrict__ a, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = SingleAcc{NONE32, NONE32, 0u, NONE32};
}

// ============================================================== wrappers
template <typename K, typename... A>
static hipError_t launch(K kern, dim3 grid, dim3 block, hipStream_t s, A... args) {
    if (grid.x == 0 || grid.y == 0) return hipSuccess;
    hipLaunchKernelGGL(kern, grid, block, 0, s, args...);
    return hipGetLastError();
}

hipError_t launch_count(const Item *items, uint32_t nitems, bool wide, const NestDesc *nests,
                        const ProtoDesc *protos, const FixedVal *fixed, const uint32_t *code,
                        unsigned long long *phase_counts, uint32_t *item_cnt, uint32_t *proto_ovf,
                        hipStream_t s) {
    if (wide)
        return launch(k_count<uint64_t, true>, dim3(nitems), dim3(WG), s, items, nests, protos, fixed, code,
                      phase_counts, item_cnt, proto_ovf);
    return launch(k_count<uint32_t, false>, dim3(nitems), dim3(WG), s, items, nests, protos, fixed, code,
                  phase_counts, item_cnt, proto_ovf);
}

hipError_t launch_emit(const Item *items, uint32_t nitems, bool wide, const NestDesc *nests,
                       const ProtoDesc *protos, const FixedVal *fixed, const uint32_t *code,
                       const uint32_t *item_cnt, const unsigned long long *big_base,
                       unsigned long long *cursor, uint64_t win_lo, uint64_t win_n, unsigned long long *recs,
                       unsigned long long cap, hipStream_t s, bool table) {
    if (table) {
        if (wide)
            return launch(k_emit<uint64_t, true, true>, dim3(nitems), dim3(WG), s, items, nests, protos, fixed, code,
                          item_cnt, big_base, cursor, win_lo, win_n, recs, cap);
        return launch(k_emit<uint32_t, false, true>, dim3(nitems), dim3(WG), s, items, nests, protos, fixed, code,
                      item_cnt, big_base, cursor, win_lo, win_n, recs, cap);
    }
    if (wide)
        return launch(k_emit<uint64_t, true, false>, dim3(nitems), dim3(WG), s, items, nests, protos, fixed, code,
                      item_cnt, big_base, cursor, win_lo, win_n, recs, cap);
    return launch(k_emit<uint32_t, false, false>, dim3(nitems), dim3(WG), s, items, nests, protos, fixed, code,
                  item_cnt, big_base, cursor, win_lo, win_n, recs, cap);
}

hipError_t launch_table_scan(const TablePhase *tp, uint32_t ntp, const uint32_t *tabs, uint32_t *tmin,
                             uint32_t blocks_per_table, hipStream_t s) {
    if (ntp == 0) return hipSuccess;
    return launch(k_table_scan, dim3(blocks_per_table, ntp), dim3(WG), s, tp, tabs, tmin);
}

hipError_t launch_table_offer(const TablePhase *tp, uint32_t ntp, const uint32_t *tabs, const uint32_t *tmin,
                              Cand *cands, Best *best, hipStream_t s) {
    if (ntp == 0) return hipSuccess;
    return launch(k_table_offer, dim3((ntp + 255) / 256), dim3(256), s, tp, ntp, tabs, tmin, cands, best);
}

hipError_t launch_fused(const Unit *units, uint32_t nunits, uint32_t *qhead, bool wide, const NestDesc *nests,
                        const ProtoDesc *protos, const FixedVal *fixed, const uint32_t *code,
                        unsigned long long *phase_counts, unsigned long long *nrec, uint32_t *ovf_flags,
                        Cand *cands, Best *best, uint32_t grid, uint32_t tile, hipStream_t s,
                        const uint32_t *nunits_dev) {
    // with nunits_dev the count is read on the device and nunits bounds it
    const uint32_t g = nunits < grid ? nunits : grid;
    if (g == 0) return hipSuccess;
    if (wide)
        return launch(k_fused64, dim3(g), dim3(WG), s, units, nunits, nunits_dev, qhead, nests, protos, fixed, code,
                      phase_counts, nrec, ovf_flags, cands, best, tile);
    return launch(k_fused32, dim3(g), dim3(WG), s, units, nunits, nunits_dev, qhead, nests, protos, fixed, code,
                  phase_counts, nrec, ovf_flags, cands, best, tile);
}

hipError_t launch_hist(const Seg *segs, const Chunk *chunks, uint32_t nchunks, const unsigned long long *in,
                       unsigned long long *hist, hipStream_t s) {
    return launch(k_hist, dim3(nchunks), dim3(WG), s, segs, chunks, in, hist);
}

hipError_t launch_scatter(const Seg *segs, const Chunk *chunks, uint32_t nchunks, const unsigned long long *in,
                          const unsigned long long *offs, unsigned long long *out, unsigned long long cap,
                          hipStream_t s) {
    return launch(k_scatter, dim3(nchunks), dim3(WG), s, segs, chunks, in, offs, out, cap);
}

hipError_t launch_offsets(const Seg *segs, uint32_t nsegs, unsigned long long *hist, unsigned long long *starts,
                          hipStream_t s) {
    return launch(k_offsets, dim3(nsegs), dim3(WG), s, segs, nsegs, hist, starts);
}

hipError_t launch_tiles(const Tile *tiles, uint32_t ntiles, const unsigned long long *recs, Cand *cands, Best *best,
                        hipStream_t s) {
    return launch(k_tile, dim3(ntiles), dim3(TWG), s, tiles, recs, cands, best);
}

hipError_t launch_single(const Group *groups, uint32_t ngroups, const unsigned long long *recs, SingleAcc *acc,
                         Cand *cands, Best *best, hipStream_t s) {
    if (ngroups == 0) return hipSuccess;
    hipError_t e = launch(k_single1, dim3(64, ngroups), dim3(WG), s, groups, ngroups, recs, acc);
    if (e != hipSuccess) return e;
    e = launch(k_single2, dim3(64, ngroups), dim3(WG), s, groups, ngroups, recs, acc);
    if (e != hipSuccess) return e;
    return launch(k_single3, dim3((ngroups + 255) / 256), dim3(256), s, groups, ngroups, recs,
                  (const SingleAcc *)acc, cands, best);
}

hipError_t launch_result(uint32_t count, const ResultIn *rin, const Best *best, const unsigned long long *nrec,
                         const uint32_t *ovf_flags, drf_result_dev *out, hipStream_t s, const uint32_t *count_dev) {
    if (count == 0) return hipSuccess;
    return launch(k_result, dim3((count + 255) / 256), dim3(256), s, count, count_dev, rin, best, nrec, ovf_flags,
                  out);
}

__global__ __launch_bounds__(WG) void k_best_min(Best *__restrict__ best, const Best *__restrict__ best2,
                                                  uint32_t count) {
    const uint32_t p = blockIdx.x * WG + threadIdx.x;
    if (p < count && best2[p].key < best[p].key) best[p] = best2[p];
}

hipError_t launch_best_min(Best *best, const Best *best2, uint32_t count, hipStream_t s) {
    if (count == 0) return hipSuccess;
    return launch(k_best_min, dim3((count + WG - 1) / WG), dim3(WG), s, best, best2, count);
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, uint64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint64_t blocks = (n + 255) / 256;
    return launch(k_fill_u32, dim3((uint32_t)(blocks < 4096 ? blocks : 4096)), dim3(256), s, p, v, n);
}

hipError_t launch_fill_multi(FillList L, hipStream_t s) {
    // empty fills are dropped; each remaining one gets its own blocks
    FillList M{};
    uint32_t blocks = 0;
    for (uint32_t i = 0; i < L.count && i < (uint32_t)FILL_MAX; i++) {
        if (L.n[i] == 0) continue;
        const uint32_t k = M.count++;
        M.p[k] = L.p[i];
        M.n[k] = L.n[i];
        M.v[k] = L.v[i];
        M.b0[k] = blocks;
        const uint64_t nb = (L.n[i] + 255) / 256;
        blocks += (uint32_t)(nb < 1024 ? nb : 1024);
    }
    if (M.count == 0) return hipSuccess;
    return launch(k_fill_multi, dim3(blocks), dim3(256), s, M);
}

hipError_t launch_init_acc(SingleAcc *a, uint32_t n, hipStream_t s) {
    return launch(k_init_acc, dim3((n + 255) / 256), dim3(256), s, a, n);
}

hipError_t launch_pick(const Cand *cands, uint64_t ncands, Best *best, hipStream_t s, const uint32_t *n_dev) {
    if (ncands == 0) return hipSuccess;
    return launch(k_pick, dim3((uint32_t)((ncands + 255) / 256)), dim3(256), s, cands, ncands, n_dev, best);
}

// ------------------------------------------------ fixed scratch array
// Scratch of the allocation-free checking call: one array per device, part
// of the code object, so it exists from module load until the process
// ends and no call allocates it.  Host code must not pass `scratch` itself
// to a kernel (on the host the name is only a stand-in); it passes the
// device address hipGetSymbolAddress returns with that device current.
static __device__ __align__(256) unsigned char scratch[FIXED_SCRATCH_BYTES];

constexpr int FIXED_MAX_DEVICES = 64;

hipError_t fixed_scratch_address(int device, void **ptr) {
    static std::mutex mu;
    static void *addr[FIXED_MAX_DEVICES] = {};
    if (device < 0 || device >= FIXED_MAX_DEVICES || !ptr) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> g(mu);
    if (!addr[device]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

}  // namespace drf
