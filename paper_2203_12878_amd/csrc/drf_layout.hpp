// Layouts shared by the host planner and the gfx950 kernels.
//
// A planned protocol is a set of "leaf nests": one unsynchronized leaf
// (a sync-free statement at the synchronized level) together with the
// for^S loops around it that are kept symbolic.  Iteration f of a nest has
// mixed-radix digits d_l (loop 0 outermost, d_l in [0, trip_l)); the loop
// variable of loop l is lo_l + d_l and the phase of every access the leaf
// performs in that iteration is phase_base + sum_l d_l * stride_l, where
// stride_l is the number of syncs one iteration of loop l executes.  This
// is exact because sync closes a phase for all threads and for^S bounds
// are tid-free, so every thread executes the same barriers.
#pragma once
#include <stdint.h>

namespace drf {

constexpr int MAXSLOTS = 16;     // loop variable slots per protocol
constexpr int MAXLOOPS = 8;      // symbolic for^S loops around one leaf
constexpr int MAXSTACK = 16;     // expression evaluation stack
constexpr int MAXDEPTH = 30;     // if / for^U nesting inside one leaf
constexpr uint32_t NONE32 = 0xFFFFFFFFu;
constexpr uint64_t NONE64 = ~0ull;

// Leaf code executed by every lane (uniform program counter, per-lane
// activity masks).  Offsets are word offsets from the start of the leaf.
enum : uint32_t {
    U_ACC = 1,     // mode len <expr>
    U_IF = 2,      // len <cond> else_pc
    U_ELSE = 3,    // endif_pc
    U_ENDIF = 4,   //
    U_FOR = 5,     // slot lolen <lo> hilen <hi> end_pc
    U_ENDFOR = 6,  // slot body_pc
    U_END = 7,
};

// Postfix expression ops of leaf code.
enum : uint32_t {
    X_CONST = 1,   // lo hi
    X_TID,         //
    X_VAR,         // slot
    X_ADD, X_MONUS, X_MUL, X_DIV, X_MOD, X_SHL, X_SHR, X_MIN, X_MAX,
    X_TRUE, X_FALSE, X_LT, X_LE, X_EQ, X_NE, X_GT, X_GE, X_AND, X_OR, X_NOT,
    // immediate-operand forms (constant right operand below 2^32)
    X_ADDC,        // c
    X_MULC,        // c
    X_DIVC,        // c (c > 0)
    X_MODC,        // c (c > 0)
    X_ANDC,        // mask: mod by a power of two
    X_SHRC,        // k: div by a power of two
    X_AFF,         // nterms c_lo c_hi {var c} * nterms  (var: slot, or NONE32 for tid)
};

// Compiled access leaf: a leaf that is a straight-line sequence of
// accesses (possibly inside a thread-limit guard) whose index expressions
// are a chain of operations applied to tid, each with a tid-free operand.
// The tid-free operands ("uniform slots") are evaluated once per iteration;
// each lane then runs its short chain.  Layout (words, from cal_off):
//   nacc nuni acc_off (offset of the first access block from cal_off)
//   nuni x { len <postfix X_* code over loop variables> }
//   nacc x { mode form c0 m0k m0 a us pk pa m0mag m0sh pamag pash nops
//            { opw arg } * nops }
// opw = C_* | (C_UNI if arg is a uniform slot, else arg is the immediate).
// form 1: the chain is ((tid + c0) m0-op m0) * a + U[us] then pk-op pa, with
// op kinds CAL_K_NONE / CAL_K_AND / CAL_K_MOD, us NONE32 when there is no
// uniform term (the same operations as the chain, in the same order).  A
// modulus d of the fixed form is >= 1 (mod 0 is the identity: kind NONE)
// and comes with the multiplier and shifts of exact division by the
// invariant d (mag, sh1 | sh2 << 8: Granlund and Montgomery, "Division by
// invariant integers using multiplication", 1994, unsigned case):
// x / d = (t + ((x - t) >> sh1)) >> sh2 with t = mulhi(mag, x), for every
// 32-bit x.  form 0: only the chain applies.
enum : uint32_t {
    C_ADD = 1, C_MUL, C_MONUS, C_RMONUS, C_DIV, C_MOD, C_SHL, C_SHR, C_MIN, C_MAX, C_AND,
    C_UNI = 0x100,
};
constexpr uint32_t CAL_K_NONE = 0, CAL_K_AND = 1, CAL_K_MOD = 2;
constexpr uint32_t CAL_HDR = 14;     // words before an access's chain ops
constexpr uint32_t CAL_MAXU = 32;    // uniform slots of one leaf (a chunk then stages >= 64 iterations)
constexpr uint32_t CAL_MAXOPS = 16;  // chain operations of one access

struct ProtoDesc {
    uint32_t n;          // threads
    uint32_t wide;       // 64-bit evaluator with overflow checks
    uint32_t nest0;      // first nest of this protocol
    uint32_t nnests;
    uint64_t phase_off;  // global id of phase 0
    uint64_t nphases;
    // LDS key layout of the fused path: with `pack`, a record of phase
    // k0 + r is (r << (ib + tb + 1)) | index << (tb + 1) | tid << 1 | write,
    // so several phases share one sort; otherwise index << 32 | tid << 1 | w
    uint32_t tb;         // bits of the largest tid
    uint32_t ib;         // bits of the largest index
    uint32_t pack;
    uint32_t phase_bound;  // static bound on the events of one phase (clipped)
};

struct NestDesc {
    uint32_t proto;
    uint32_t code_off;     // word offset of the leaf code in the code blob
    uint32_t nloops;
    uint32_t nfixed;       // host-unrolled enclosing loops: fixed slot values
    uint32_t fixed_off;    // into the fixed (slot, value) table
    uint32_t rec_bound;    // per-lane access events per iteration (upper bound, saturated)
    uint32_t guard_off;    // thread-limit expression (word offset) or NONE32: only tids below
                           // its value can access memory in an iteration
    uint32_t cal_off;      // compiled access leaf (word offset) or NONE32
    uint64_t iters;        // product of trips (>= 1)
    uint64_t phase_base;   // global phase id of iteration 0
    uint64_t phase_last;   // global phase id of the last iteration
    uint32_t slot[MAXLOOPS];
    uint64_t lo[MAXLOOPS];
    uint64_t trip[MAXLOOPS];
    uint64_t stride[MAXLOOPS];
};

struct FixedVal {
    uint32_t slot;
    uint32_t pad;
    uint64_t value;
};

// Count / emit work item: one workgroup, iterations [f0, f1) of one nest
// for nblk consecutive blocks of 256 tids from tid0 (one block at a time,
// lanes = tids); k_lo = global phase of f0, span = phases covered.
struct Item {
    uint32_t nest;
    uint32_t tid0;
    uint64_t f0, f1;
    uint64_t k_lo;
    uint64_t cnt_off;      // per-(item, phase) counts at cnt_off + (k - k_lo)
    uint32_t span;
    uint32_t nblk;         // blocks of 256 tids (>= 1)
};

// Fused work unit: phases [k0, k1) (global ids) of one protocol, each with
// at most the LDS tile capacity of access events.  With UNIT_STATIC the
// planner proved the bound (no count pass ran): the unit writes the phase
// counts, adds its events to the protocol total and flags range overflow.
// Otherwise the count pass ran and phases above the tile are skipped.
constexpr uint32_t UNIT_STATIC = 1;

struct Unit {
    uint32_t proto;
    uint32_t flags;
    uint64_t k0, k1;
};

// Candidate witness of a tile / unit: key = phase << 32 | index (global
// phase id), pair = tid_i << 32 | tid_j.
struct Cand {
    uint64_t key;
    uint64_t pair;
    uint32_t proto;
    uint32_t pad;
};

}  // namespace drf
