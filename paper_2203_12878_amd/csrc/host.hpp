// Host side of libdrf: text compiler, bytecode decoder, static checks,
// planner and leaf-code generation.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "drf_layout.hpp"

namespace drf {

// Bytecode opcodes (see include/drf.h).
enum : uint32_t {
    B_SKIP = 0x01, B_ACC = 0x02, B_SEQ = 0x03, B_IF = 0x04, B_FORU = 0x05, B_SYNC = 0x06, B_FORS = 0x07,
    B_CONST32 = 0x20, B_CONST64 = 0x21, B_TID = 0x22, B_VAR = 0x23,
    B_ADD = 0x30, B_MONUS = 0x31, B_MUL = 0x32, B_DIV = 0x33, B_MOD = 0x34, B_SHL = 0x35, B_SHR = 0x36,
    B_MIN = 0x37, B_MAX = 0x38,
    B_TRUE = 0x40, B_FALSE = 0x41, B_LT = 0x42, B_LE = 0x43, B_EQ = 0x44, B_NE = 0x45, B_GT = 0x46,
    B_GE = 0x47, B_AND = 0x48, B_OR = 0x49, B_NOT = 0x4A,
};

// Decoded protocol.
struct XNode {          // expression node
    uint32_t op;        // B_* expression opcode
    uint64_t val;       // constants
    uint32_t slot;      // B_VAR
    int a = -1, b = -1;
};

struct SNode {          // statement node
    uint32_t kind;      // B_SKIP .. B_FORS
    uint32_t mode = 0;  // B_ACC: 0 read, 1 write
    uint32_t array = 0; // B_ACC: shared array accessed (0 in a one-array protocol)
    uint32_t slot = 0;  // loops
    int e = -1;         // B_ACC index / B_IF condition
    int lo = -1, hi = -1;
    std::vector<int> kids;
    bool has_s = false; // contains sync or for^S
};

struct IR {
    std::vector<XNode> x;
    std::vector<SNode> s;
    int root = -1;
    uint32_t nslots = 0;
};

struct Loop {
    uint32_t slot;
    uint64_t lo, trip, stride;
};

struct Nest {
    int leaf = -1;               // statement index of the leaf
    std::vector<Loop> loops;     // symbolic for^S loops, outermost first
    std::vector<std::pair<uint32_t, uint64_t>> fixed;  // host-unrolled loop values
    uint64_t phase_base = 0;     // local phase of iteration 0
    uint64_t iters = 0;
    uint64_t phase_last = 0;
    uint32_t rec_bound = 0;      // per-lane events per iteration (saturated)
    uint32_t tid_bound = 0;      // tids below this may access memory (thread-limit guard bound, else n)
};

struct Plan {
    int status = 0;
    uint32_t n = 0;
    uint64_t num_phases = 0;
    uint32_t index_bits = 0;
    bool wide = false;
    uint64_t max_records = 0;
    uint64_t max_phase_records = 0;   // static bound on the events of one phase
    std::vector<Nest> nests;
    // leaf code: leaf statement index -> words
    std::vector<int> leaf_ids;
    std::vector<std::vector<uint32_t>> leaf_code;
    std::vector<int> nest_leaf_code;   // per nest: index into leaf_code
    std::vector<int> leaf_guard;       // per leaf code: offset of its thread-limit block, or -1
    std::vector<int> leaf_cal;         // per leaf code: offset of its compiled access leaf, or -1
};

// Arrays of one access word: bit 0 write, bits 1.. the array id.
constexpr uint32_t MAX_ARRAYS = 1u << 16;

int compile_text(const char *text, size_t len, std::vector<uint32_t> &out);
// Slot the text compiler gives `name` (names get slots in order of first
// appearance); -1 when the text does not mention it or does not compile.
int text_slot(const char *text, size_t len, const char *name);
int decode(const uint32_t *code, uint32_t words, IR &ir);     // 0 or E_BYTECODE
int static_check(const IR &ir);                               // first violation or 0
int plan_protocol(const uint32_t *code, uint32_t words, uint32_t n, Plan &plan);

// Memory access protocol (text form) of a BabyCUDA program under the
// typing context {tid} + params (space-separated names, may be null):
// 0, a typing status (DRF_E_ILLTYPED, DRF_E_UNBOUND, DRF_E_SHADOW) or
// DRF_E_ARG when the text is not a BabyCUDA program.
int babycuda_infer(const char *text, size_t len, const char *params, std::string &map_text);

// Bytecode of a decoded protocol (the inverse of decode).
void encode(const IR &ir, std::vector<uint32_t> &out);
// Arrays a protocol accesses: 1 + the largest array id (1 without accesses).
uint32_t ir_arrays(const IR &ir);
// The protocol of one array: its accesses become array-0 accesses, every
// access to another array becomes skip (one protocol per array).
void ir_project(IR &ir, uint32_t array);
// Replaces every occurrence of variable `slot` by the constant v; false
// when a loop binds the slot (it is then not a free parameter).
bool ir_bind(IR &ir, uint32_t slot, uint64_t v);

}  // namespace drf
