// Host side of libdrf: text compiler, bytecode decoder, static checks,
// planner (leaf nests with affine phase maps, interval analysis) and leaf
// code generation for the gfx950 evaluator.
#include "host.hpp"

#include <string.h>

#include <algorithm>
#include <string>
#include <unordered_map>

#include "../../include/drf.h"

namespace drf {

// Multiplier and shifts for exact unsigned division of 32-bit values by
// the invariant d >= 1 (Granlund and Montgomery, "Division by invariant
// integers using multiplication", 1994, unsigned case with N = 32):
// l = ceil(log2 d), mag = floor(2^32 (2^l - d) / d) + 1, sh1 = min(l, 1),
// sh2 = max(l - 1, 0); then x / d = (t + ((x - t) >> sh1)) >> sh2 with
// t = floor(mag * x / 2^32).
static void div_magic(uint32_t d, uint32_t &mag, uint32_t &sh) {
    uint32_t l = 0;
    while (l < 32 && (1ull << l) < d) l++;
    mag = (uint32_t)(((((1ull << l) - d) << 32) / d) + 1);
    const uint32_t sh1 = l < 1 ? l : 1, sh2 = l > 0 ? l - 1 : 0;
    sh = sh1 | (sh2 << 8);
}

typedef unsigned __int128 u128;
static const u128 SAT = (u128)1 << 64;                 // saturation point of intervals
static const uint64_t VALUE_LIMIT = 1ull << 63;
static const uint64_t MAX_EVENTS = 1ull << 40;
static const uint64_t MAX_UNROLLED = 1ull << 22;

// ================================================================ text form
namespace {

struct TextCompiler {
    const char *s;
    size_t n, pos = 0;
    bool err = false;
    std::unordered_map<std::string, uint32_t> slots;
    std::unordered_map<std::string, uint32_t> arrays;   // "" is the unnamed array
    std::vector<uint32_t> out;

    static bool is_space(char c) { return c == ' ' || c == '\t' || c == '\n' || c == '\r'; }

    bool next(std::string &tok) {
        while (pos < n && is_space(s[pos])) pos++;
        if (pos >= n) return false;
        if (s[pos] == '(' || s[pos] == ')') { tok.assign(1, s[pos++]); return true; }
        size_t b = pos;
        while (pos < n && !is_space(s[pos]) && s[pos] != '(' && s[pos] != ')') pos++;
        tok.assign(s + b, pos - b);
        return true;
    }
    bool peek(std::string &tok) { size_t p = pos; bool r = next(tok); pos = p; return r; }
    void expect(const char *want) { std::string t; if (!next(t) || t != want) err = true; }

    static bool keyword(const std::string &t) {
        static const char *kw[] = {"+", "-", "*", "/", "mod", "<<", ">>", "min", "max", "<", "<=", "=", "!=", ">",
                                   ">=", "and", "or", "not", "true", "false", "skip", "rd", "wr", "seq", "if",
                                   "foru", "fors", "sync", nullptr};
        for (int i = 0; kw[i]; i++) if (t == kw[i]) return true;
        return false;
    }
    static bool ident(const std::string &t) {
        if (t.empty()) return false;
        char c = t[0];
        if (!((c >= 'a' && c <= 'z') || (c >= 'A' && c <= 'Z') || c == '_')) return false;
        for (char ch : t)
            if (!((ch >= 'a' && ch <= 'z') || (ch >= 'A' && ch <= 'Z') || (ch >= '0' && ch <= '9') || ch == '_'))
                return false;
        return !keyword(t);
    }
    uint32_t slot_of(const std::string &name) {
        auto it = slots.find(name);
        if (it != slots.end()) return it->second;
        uint32_t s2 = (uint32_t)slots.size();
        slots.emplace(name, s2);
        return s2;
    }

    // arithmetic expression, postfix into `w`
    void nexp(std::vector<uint32_t> &w) {
        std::string t;
        if (!next(t)) { err = true; return; }
        if (t == "(") {
            std::string op;
            if (!next(op)) { err = true; return; }
            static const char *ops[] = {"+", "-", "*", "/", "mod", "<<", ">>", "min", "max"};
            static const uint32_t codes[] = {B_ADD, B_MONUS, B_MUL, B_DIV, B_MOD, B_SHL, B_SHR, B_MIN, B_MAX};
            int k = -1;
            for (int i = 0; i < 9; i++) if (op == ops[i]) k = i;
            if (k < 0) { err = true; return; }
            nexp(w);
            if (err) return;
            nexp(w);
            if (err) return;
            expect(")");
            w.push_back(codes[k]);
            return;
        }
        if (t[0] >= '0' && t[0] <= '9') {
            u128 v = 0;
            for (char c : t) {
                if (c < '0' || c > '9') { err = true; return; }
                v = v * 10 + (uint32_t)(c - '0');
                if (v >= SAT) { err = true; return; }
            }
            uint64_t x = (uint64_t)v;
            if (x < (1ull << 32)) { w.push_back(B_CONST32); w.push_back((uint32_t)x); }
            else { w.push_back(B_CONST64); w.push_back((uint32_t)x); w.push_back((uint32_t)(x >> 32)); }
            return;
        }
        if (t == "tid") { w.push_back(B_TID); return; }
        if (ident(t)) { w.push_back(B_VAR); w.push_back(slot_of(t)); return; }
        err = true;
    }

    void bexp(std::vector<uint32_t> &w) {
        std::string t;
        if (!next(t)) { err = true; return; }
        if (t == "true") { w.push_back(B_TRUE); return; }
        if (t == "false") { w.push_back(B_FALSE); return; }
        if (t != "(") { err = true; return; }
        std::string op;
        if (!next(op)) { err = true; return; }
        static const char *rels[] = {"<", "<=", "=", "!=", ">", ">="};
        static const uint32_t rcodes[] = {B_LT, B_LE, B_EQ, B_NE, B_GT, B_GE};
        for (int i = 0; i < 6; i++)
            if (op == rels[i]) {
                nexp(w);
                if (!err) nexp(w);
                if (!err) expect(")");
                w.push_back(rcodes[i]);
                return;
            }
        if (op == "and" || op == "or") {
            bexp(w);
            if (!err) bexp(w);
            if (!err) expect(")");
            w.push_back(op == "and" ? B_AND : B_OR);
            return;
        }
        if (op == "not") {
            bexp(w);
            if (!err) expect(")");
            w.push_back(B_NOT);
            return;
        }
        err = true;
    }

    void block(bool boolean) {
        std::vector<uint32_t> w;
        if (boolean) bexp(w); else nexp(w);
        out.push_back((uint32_t)w.size());
        out.insert(out.end(), w.begin(), w.end());
    }

    void stmt() {
        expect("(");
        if (err) return;
        std::string h;
        if (!next(h)) { err = true; return; }
        if (h == "skip") out.push_back(B_SKIP);
        else if (h == "sync") out.push_back(B_SYNC);
        else if (h == "rd" || h == "wr" || h.compare(0, 3, "rd:") == 0 || h.compare(0, 3, "wr:") == 0) {
            // rd / wr access "the" array; rd:A / wr:A name one of several
            // arrays (ids in order of first appearance, the unnamed one too)
            const std::string name = h.size() > 2 ? h.substr(3) : std::string();
            if (h.size() > 2 && !ident(name)) { err = true; return; }
            auto it = arrays.find(name);
            const uint32_t id = it != arrays.end() ? it->second : (uint32_t)arrays.size();
            if (it == arrays.end()) arrays.emplace(name, id);
            if (id >= MAX_ARRAYS) { err = true; return; }
            out.push_back(B_ACC);
            out.push_back((h[0] == 'w' ? 1u : 0u) | id << 1);
            block(false);
        } else if (h == "seq") {
            out.push_back(B_SEQ);
            size_t at = out.size();
            out.push_back(0);
            uint32_t cnt = 0;
            std::string p;
            while (!err && peek(p) && p != ")") { stmt(); cnt++; }
            out[at] = cnt;
        } else if (h == "if") {
            out.push_back(B_IF);
            block(true);
            if (!err) stmt();
            if (!err) stmt();
        } else if (h == "foru" || h == "fors") {
            out.push_back(h == "foru" ? B_FORU : B_FORS);
            std::string x;
            if (!next(x)) { err = true; return; }
            if (x == "tid") out.push_back(DRF_TID_SLOT);
            else if (ident(x)) out.push_back(slot_of(x));
            else { err = true; return; }
            block(false);
            if (!err) block(false);
            if (!err) stmt();
        } else {
            err = true;
            return;
        }
        if (!err) expect(")");
    }
};

}  // namespace

int text_slot(const char *text, size_t len, const char *name) {
    TextCompiler c;
    c.s = text;
    c.n = len;
    c.stmt();
    std::string t;
    if (c.err || c.next(t)) return -1;
    auto it = c.slots.find(name);
    return it == c.slots.end() ? -1 : (int)it->second;
}

int compile_text(const char *text, size_t len, std::vector<uint32_t> &words) {
    TextCompiler c;
    c.s = text;
    c.n = len;
    c.stmt();
    std::string t;
    if (!c.err && c.next(t)) c.err = true;
    if (c.err) return DRF_E_ARG;
    words.clear();
    words.push_back(DRF_MAGIC);
    words.push_back(1);
    words.push_back((uint32_t)c.slots.size());
    words.push_back((uint32_t)c.out.size());
    words.insert(words.end(), c.out.begin(), c.out.end());
    return DRF_OK;
}

// ================================================================ decoding
namespace {

struct Decoder {
    const uint32_t *w;
    uint32_t n, pos = 0;
    IR &ir;
    int status = 0;
    int depth = 0;
    explicit Decoder(IR &r) : ir(r) {}

    void bad(int st = DRF_E_BYTECODE) { if (!status) status = st; }

    // expression block; wants_bool selects the expected result type
    int expr(bool wants_bool) {
        if (pos >= n) { bad(); return -1; }
        uint32_t len = w[pos++];
        if (len > n - pos) { bad(); return -1; }
        if (len > 16384) { bad(DRF_E_LIMIT); return -1; }
        uint32_t end = pos + len;
        std::vector<std::pair<int, bool>> st;   // (node, is_bool)
        while (pos < end && !status) {
            uint32_t op = w[pos++];
            XNode x{};
            x.op = op;
            bool is_bool = false;
            switch (op) {
            case B_CONST32:
                if (pos >= end) { bad(); break; }
                x.val = w[pos++];
                break;
            case B_CONST64:
                if (end - pos < 2) { bad(); break; }
                x.val = (uint64_t)w[pos] | ((uint64_t)w[pos + 1] << 32);
                pos += 2;
                break;
            case B_TID: break;
            case B_VAR:
                if (pos >= end) { bad(); break; }
                x.slot = w[pos++];
                if (x.slot >= ir.nslots) bad();
                break;
            case B_ADD: case B_MONUS: case B_MUL: case B_DIV: case B_MOD: case B_SHL: case B_SHR:
            case B_MIN: case B_MAX:
            case B_LT: case B_LE: case B_EQ: case B_NE: case B_GT: case B_GE:
            case B_AND: case B_OR: {
                bool boolean_args = (op == B_AND || op == B_OR);
                if (st.size() < 2 || st[st.size() - 1].second != boolean_args || st[st.size() - 2].second != boolean_args) {
                    bad();
                    break;
                }
                x.b = st.back().first; st.pop_back();
                x.a = st.back().first; st.pop_back();
                is_bool = (op >= B_LT);
                break;
            }
            case B_NOT:
                if (st.empty() || !st.back().second) { bad(); break; }
                x.a = st.back().first; st.pop_back();
                is_bool = true;
                break;
            case B_TRUE: case B_FALSE: is_bool = true; break;
            default: bad(); break;
            }
            if (status) return -1;
            ir.x.push_back(x);
            st.push_back({(int)ir.x.size() - 1, is_bool});
        }
        if (status) return -1;
        if (st.size() != 1 || st[0].second != wants_bool) { bad(); return -1; }
        return st[0].first;
    }

    int stmt() {
        if (status) return -1;
        if (++depth > 4096) { bad(DRF_E_LIMIT); return -1; }
        if (pos >= n) { bad(); return -1; }
        SNode s;
        s.kind = w[pos++];
        switch (s.kind) {
        case B_SKIP: case B_SYNC: break;
        case B_ACC:
            if (pos >= n) { bad(); break; }
            s.mode = w[pos] & 1u;
            s.array = w[pos++] >> 1;
            if (s.array >= MAX_ARRAYS) { bad(); break; }
            s.e = expr(false);
            break;
        case B_SEQ: {
            if (pos >= n) { bad(); break; }
            uint32_t cnt = w[pos++];
            if (cnt > n - pos) { bad(); break; }
            for (uint32_t i = 0; i < cnt && !status; i++) s.kids.push_back(stmt());
            break;
        }
        case B_IF:
            s.e = expr(true);
            s.kids.push_back(stmt());
            s.kids.push_back(stmt());
            break;
        case B_FORU: case B_FORS:
            if (pos >= n) { bad(); break; }
            s.slot = w[pos++];
            if (s.slot >= ir.nslots && s.slot != DRF_TID_SLOT) { bad(); break; }
            s.lo = expr(false);
            s.hi = expr(false);
            s.kids.push_back(stmt());
            break;
        default: bad(); break;
        }
        depth--;
        if (status) return -1;
        ir.s.push_back(s);
        return (int)ir.s.size() - 1;
    }
};

}  // namespace

int decode(const uint32_t *code, uint32_t words, IR &ir) {
    ir = IR();
    if (!code || words < 4 || code[0] != DRF_MAGIC || code[1] != 1 || code[3] != words - 4 || code[2] > (1u << 20))
        return DRF_E_BYTECODE;
    ir.nslots = code[2];
    Decoder d(ir);
    d.w = code + 4;
    d.n = words - 4;
    ir.root = d.stmt();
    if (!d.status && d.pos != d.n) d.bad();
    return d.status;
}

// ============================================================ static checks
namespace {

bool any_unbound(const IR &ir, int e, const std::vector<char> &bound) {
    if (e < 0) return false;
    const XNode &x = ir.x[e];
    if (x.op == B_VAR && !bound[x.slot]) return true;
    return any_unbound(ir, x.a, bound) || any_unbound(ir, x.b, bound);
}

bool mentions_tid(const IR &ir, int e) {
    if (e < 0) return false;
    const XNode &x = ir.x[e];
    return x.op == B_TID || mentions_tid(ir, x.a) || mentions_tid(ir, x.b);
}

int check_stmt(const IR &ir, int si, std::vector<char> &bound, bool in_u) {
    const SNode &s = ir.s[si];
    switch (s.kind) {
    case B_SKIP: return 0;
    case B_ACC: return any_unbound(ir, s.e, bound) ? DRF_E_UNBOUND : 0;
    case B_SEQ:
        for (int k : s.kids) { int st = check_stmt(ir, k, bound, in_u); if (st) return st; }
        return 0;
    case B_IF: {
        if (any_unbound(ir, s.e, bound)) return DRF_E_UNBOUND;
        int st = check_stmt(ir, s.kids[0], bound, true);
        return st ? st : check_stmt(ir, s.kids[1], bound, true);
    }
    case B_SYNC: return in_u ? DRF_E_SYNC_IN_U : 0;
    case B_FORU: case B_FORS: {
        if (s.kind == B_FORS && in_u) return DRF_E_SYNC_IN_U;
        if (any_unbound(ir, s.lo, bound) || any_unbound(ir, s.hi, bound)) return DRF_E_UNBOUND;
        if (s.kind == B_FORS && (mentions_tid(ir, s.lo) || mentions_tid(ir, s.hi))) return DRF_E_DIVERGENT;
        if (s.slot == DRF_TID_SLOT || bound[s.slot]) return DRF_E_SHADOW;
        bound[s.slot] = 1;
        int st = check_stmt(ir, s.kids[0], bound, in_u || s.kind == B_FORU);
        bound[s.slot] = 0;
        return st;
    }
    }
    return DRF_E_BYTECODE;
}

}  // namespace

int static_check(const IR &ir) {
    std::vector<char> bound(ir.nslots + 1, 0);
    return check_stmt(ir, ir.root, bound, false);
}

// ================================================================ planning
namespace {

struct Iv { u128 lo, hi; };

static u128 sat(u128 v) { return v > SAT ? SAT : v; }
static u128 smul(u128 a, u128 b) {
    if (a == 0 || b == 0) return 0;
    if (a >= SAT || b >= SAT) return SAT;
    return sat(a * b);   // both < 2^64: product < 2^128
}

struct Planner {
    IR &ir;
    uint32_t n;
    Plan &plan;
    int status = 0;
    // renumbered slots: loop statement -> depth; slot -> depth during walks
    std::vector<uint32_t> depth_of_slot;
    std::vector<char> unroll;          // per statement: for^S unrolled on host
    uint64_t unrolled = 0;
    // current binding of slot depths to values (host-unrolled loops)
    std::vector<std::pair<uint32_t, uint64_t>> fixed;
    std::vector<Loop> loops;
    uint32_t max_depth = 0;
    std::unordered_map<int, int> code_of_leaf;
    u128 events = 0;
    u128 phase_events = 0;   // sum over nests of their per-phase maxima
    u128 total_work = 0;
    uint64_t max_index = 0;

    Planner(IR &r, uint32_t nn, Plan &p) : ir(r), n(nn), plan(p) {}
    void fail(int st) { if (!status) status = st; }

    // ---- renumber loop slots by nesting depth (binders along a path are
    // distinct, so the depth identifies a variable uniquely in scope)
    void renumber_expr(int e, const std::vector<uint32_t> &map) {
        if (e < 0) return;
        XNode &x = ir.x[e];
        if (x.op == B_VAR) x.slot = map[x.slot];
        renumber_expr(x.a, map);
        renumber_expr(x.b, map);
    }
    void renumber(int si, std::vector<uint32_t> &map, uint32_t depth) {
        SNode &s = ir.s[si];
        if (s.kind == B_ACC || s.kind == B_IF) renumber_expr(s.e, map);
        if (s.kind == B_FORU || s.kind == B_FORS) {
            renumber_expr(s.lo, map);
            renumber_expr(s.hi, map);
            uint32_t old = s.slot, prev = map[old];
            map[old] = depth;
            s.slot = depth;
            max_depth = std::max(max_depth, depth + 1);
            renumber(s.kids[0], map, depth + 1);
            map[old] = prev;
            return;
        }
        for (int k : s.kids) renumber(k, map, depth);
    }

    // has_s: the statement contains sync or for^S (if / for^U cannot,
    // after the static checks)
    bool mark_s(int si) {
        SNode &s = ir.s[si];
        bool h = (s.kind == B_SYNC || s.kind == B_FORS);
        for (int k : s.kids) if (mark_s(k)) h = true;
        s.has_s = h;
        return h;
    }

    // slots mentioned by bounds of for^S loops nested inside si
    void nested_bound_slots(int si, std::vector<char> &out) {
        const SNode &s = ir.s[si];
        for (int k : s.kids) {
            const SNode &c = ir.s[k];
            if (c.kind == B_FORS) { collect_slots(c.lo, out); collect_slots(c.hi, out); }
            nested_bound_slots(k, out);
        }
    }
    void collect_slots(int e, std::vector<char> &out) {
        if (e < 0) return;
        const XNode &x = ir.x[e];
        if (x.op == B_VAR) out[x.slot] = 1;
        collect_slots(x.a, out);
        collect_slots(x.b, out);
    }
    void decide_unroll() {
        unroll.assign(ir.s.size(), 0);
        for (size_t i = 0; i < ir.s.size(); i++) {
            if (ir.s[i].kind != B_FORS) continue;
            std::vector<char> m(MAXSLOTS + 1, 0);
            nested_bound_slots((int)i, m);
            unroll[i] = m[ir.s[i].slot];
        }
    }

    // ---- exact host evaluation of for^S bounds
    bool lookup(uint32_t slot, uint64_t &v) {
        for (auto it = fixed.rbegin(); it != fixed.rend(); ++it) if (it->first == slot) { v = it->second; return true; }
        return false;
    }
    uint64_t eval(int e, bool &ovf) {
        const XNode &x = ir.x[e];
        switch (x.op) {
        case B_CONST32: case B_CONST64: if (x.val >= VALUE_LIMIT) ovf = true; return x.val;
        case B_TID: fail(DRF_E_DIVERGENT); return 0;
        case B_VAR: { uint64_t v = 0; if (!lookup(x.slot, v)) fail(DRF_E_BYTECODE); return v; }
        }
        uint64_t a = eval(x.a, ovf), b = eval(x.b, ovf);
        if (ovf) return 0;
        u128 r;
        switch (x.op) {
        case B_ADD: r = (u128)a + b; break;
        case B_MONUS: r = a > b ? a - b : 0; break;
        case B_MUL: r = (u128)a * b; break;
        case B_DIV: r = b ? a / b : 0; break;
        case B_MOD: r = b ? a % b : a; break;
        case B_SHL: r = a == 0 ? 0 : (b >= 63 ? (u128)VALUE_LIMIT : (u128)a << b); break;
        case B_SHR: r = b >= 64 ? 0 : a >> b; break;
        case B_MIN: r = std::min(a, b); break;
        case B_MAX: r = std::max(a, b); break;
        default: fail(DRF_E_BYTECODE); return 0;
        }
        if (r >= VALUE_LIMIT) { ovf = true; return 0; }
        return (uint64_t)r;
    }

    // ---- interval analysis of a leaf (for one nest's variable ranges)
    Iv var_iv[MAXSLOTS + 1];
    u128 iv_max = 0;
    Iv ivx(int e) {
        const XNode &x = ir.x[e];
        Iv r;
        switch (x.op) {
        case B_CONST32: case B_CONST64: r = {x.val, x.val}; break;
        case B_TID: r = {0, n ? (u128)(n - 1) : 0}; break;
        case B_VAR: r = var_iv[x.slot]; break;
        case B_TRUE: case B_FALSE: return {0, 1};
        case B_NOT: ivx(x.a); return {0, 1};
        case B_AND: case B_OR: ivx(x.a); ivx(x.b); return {0, 1};
        case B_LT: case B_LE: case B_EQ: case B_NE: case B_GT: case B_GE: ivx(x.a); ivx(x.b); return {0, 1};
        default: {
            Iv a = ivx(x.a), b = ivx(x.b);
            switch (x.op) {
            case B_ADD: r = {sat(a.lo + b.lo), sat(a.hi + b.hi)}; break;
            case B_MONUS: r = {a.lo > b.hi ? a.lo - b.hi : 0, a.hi > b.lo ? a.hi - b.lo : 0}; break;
            case B_MUL: r = {smul(a.lo, b.lo), smul(a.hi, b.hi)}; break;
            case B_DIV:
                r.lo = (b.lo == 0 || b.hi == 0) ? 0 : a.lo / b.hi;
                r.hi = (b.lo == 0) ? (b.hi >= 1 ? a.hi : 0) : a.hi / b.lo;
                break;
            case B_MOD:
                if (b.lo == 0) r = {0, std::max(a.hi, b.hi)};
                else if (a.hi < b.lo) r = a;
                else r = {0, std::min(a.hi, b.hi - 1)};
                break;
            case B_SHL:
                // a <= 2^64 and b < 64: the shifted value fits in 128 bits
                r.lo = (a.lo == 0) ? 0 : (b.lo >= 64 ? SAT : sat(a.lo << (unsigned)b.lo));
                r.hi = (a.hi == 0) ? 0 : (b.hi >= 64 ? SAT : sat(a.hi << (unsigned)b.hi));
                break;
            case B_SHR:
                r.lo = b.hi >= 64 ? 0 : a.lo >> (unsigned)b.hi;
                r.hi = b.lo >= 64 ? 0 : a.hi >> (unsigned)b.lo;
                break;
            case B_MIN: r = {std::min(a.lo, b.lo), std::min(a.hi, b.hi)}; break;
            case B_MAX: r = {std::max(a.lo, b.lo), std::max(a.hi, b.hi)}; break;
            default: r = {0, SAT}; break;
            }
        }
        }
        iv_max = std::max(iv_max, r.hi);
        return r;
    }
    // per-lane bound of executed leaf instructions (loop iterations count)
    u128 work = 0;
    // returns per-lane event bound of statement si (saturated)
    u128 iv_stmt(int si) {
        const SNode &s = ir.s[si];
        switch (s.kind) {
        case B_SKIP: return 0;
        case B_ACC: {
            Iv v = ivx(s.e);
            if (v.hi < SAT) max_index = std::max<uint64_t>(max_index, (uint64_t)std::min<u128>(v.hi, ~0ull));
            else max_index = ~0ull;
            return 1;
        }
        case B_SEQ: { u128 t = 0; for (int k : s.kids) t = sat(t + iv_stmt(k)); return t; }
        case B_IF: { ivx(s.e); u128 a = iv_stmt(s.kids[0]); u128 b = iv_stmt(s.kids[1]); return std::max(a, b); }
        case B_FORU: {
            Iv lo = ivx(s.lo), hi = ivx(s.hi);
            Iv saved = var_iv[s.slot];
            var_iv[s.slot] = {lo.lo, hi.hi > 0 ? hi.hi - 1 : 0};
            u128 w0 = work;
            work = 0;
            u128 body = iv_stmt(s.kids[0]);
            var_iv[s.slot] = saved;
            u128 trips = hi.hi > lo.lo ? hi.hi - lo.lo : 0;
            work = sat(w0 + smul(trips, sat(work + 1)) + 1);
            return smul(trips, body);
        }
        }
        return 0;
    }

    // ---- the synchronized walk: leaf nests with affine phase maps
    void walk(int si, uint64_t &cursor) {
        if (status) return;
        const SNode &s = ir.s[si];
        if (s.kind == B_SYNC) {
            if (++cursor >= 0xFFFFFFFFull) fail(DRF_E_LIMIT);
            return;
        }
        if (s.kind == B_SEQ && s.has_s) {
            for (int k : s.kids) walk(k, cursor);
            return;
        }
        if (s.kind == B_FORS) {
            bool ovf = false;
            uint64_t lo = eval(s.lo, ovf);
            uint64_t hi = eval(s.hi, ovf);
            if (ovf) { fail(DRF_E_RANGE); return; }
            if (status) return;
            uint64_t trip = hi > lo ? hi - lo : 0;
            if (unroll[si]) {
                for (uint64_t v = lo; v < hi && !status; v++) {
                    if (++unrolled > MAX_UNROLLED) { fail(DRF_E_LIMIT); return; }
                    fixed.push_back({s.slot, v});
                    walk(s.kids[0], cursor);
                    fixed.pop_back();
                }
                return;
            }
            if (trip == 0) return;
            if (loops.size() >= (size_t)MAXLOOPS) { fail(DRF_E_LIMIT); return; }
            loops.push_back({s.slot, lo, trip, 0});
            size_t nest_first = plan.nests.size();
            uint64_t c0 = cursor;
            walk(s.kids[0], cursor);
            if (status) return;
            uint64_t stride = cursor - c0;
            loops.pop_back();
            // stride is known only now: patch the nests created inside
            size_t depth = loops.size();
            for (size_t i = nest_first; i < plan.nests.size(); i++) plan.nests[i].loops[depth].stride = stride;
            u128 total = (u128)c0 + (u128)trip * stride;
            if (total >= 0xFFFFFFFFull) { fail(DRF_E_LIMIT); return; }
            cursor = (uint64_t)total;
            return;
        }
        // an unsynchronized leaf
        if (n == 0) return;
        Nest ne;
        ne.leaf = si;
        ne.loops = loops;
        ne.fixed = fixed;
        ne.phase_base = cursor;
        plan.nests.push_back(ne);
    }

    // ---- leaf code generation
    std::vector<uint32_t> *code = nullptr;
    int stack_depth = 0, stack_max = 0;
    int nest_depth = 0;
    void push_depth(int d) { stack_depth += d; stack_max = std::max(stack_max, stack_depth); }

    static bool is_const(const XNode &x) { return x.op == B_CONST32 || x.op == B_CONST64; }

    // Affine flattening: e = c0 + sum coef * leaf over tid and loop
    // variables, through + and multiplication by constants.  With 64-bit
    // overflow checks every multiplier must be >= 1, so that every
    // intermediate value of the original tree is at most the final sum and
    // checking the sum alone is exact.
    bool affine(int e, u128 mult, std::vector<std::pair<uint32_t, u128>> &terms, u128 &c0, bool wide) {
        const XNode &x = ir.x[e];
        switch (x.op) {
        case B_CONST32: case B_CONST64:
            if (x.val >= VALUE_LIMIT) return false;
            c0 = sat(c0 + smul(mult, x.val));
            return true;
        case B_TID: case B_VAR: {
            const uint32_t v = x.op == B_TID ? NONE32 : x.slot;
            for (auto &t : terms) if (t.first == v) { t.second = sat(t.second + mult); return true; }
            terms.push_back({v, mult});
            return true;
        }
        case B_ADD: return affine(x.a, mult, terms, c0, wide) && affine(x.b, mult, terms, c0, wide);
        case B_MUL: {
            const XNode &A = ir.x[x.a], &B = ir.x[x.b];
            if (is_const(B) && B.val < VALUE_LIMIT && (!wide || B.val >= 1))
                return affine(x.a, smul(mult, B.val), terms, c0, wide);
            if (is_const(A) && A.val < VALUE_LIMIT && (!wide || A.val >= 1))
                return affine(x.b, smul(mult, A.val), terms, c0, wide);
            return false;
        }
        }
        return false;
    }

    bool gen_affine(int e) {
        const XNode &x = ir.x[e];
        if (x.op != B_ADD && x.op != B_MUL) return false;
        std::vector<std::pair<uint32_t, u128>> terms;
        u128 c0 = 0;
        if (!affine(e, 1, terms, c0, plan.wide)) return false;
        if (!plan.wide) {
            std::vector<std::pair<uint32_t, u128>> nz;
            for (auto &t : terms) if (t.second) nz.push_back(t);
            terms.swap(nz);
        }
        const u128 climit = plan.wide ? (u128)VALUE_LIMIT : (u128)1 << 32;
        if (c0 >= climit || terms.size() > 8) return false;
        for (auto &t : terms) if (t.second >= ((u128)1 << 32)) return false;
        auto &c = *code;
        c.push_back(X_AFF);
        c.push_back((uint32_t)terms.size());
        c.push_back((uint32_t)(uint64_t)c0);
        c.push_back((uint32_t)((uint64_t)c0 >> 32));
        for (auto &t : terms) { c.push_back(t.first); c.push_back((uint32_t)t.second); }
        push_depth(1);
        return true;
    }

    void gen_x(int e) {
        const XNode &x = ir.x[e];
        auto &c = *code;
        if (gen_affine(e)) return;
        switch (x.op) {
        case B_CONST32: case B_CONST64:
            c.push_back(X_CONST); c.push_back((uint32_t)x.val); c.push_back((uint32_t)(x.val >> 32));
            push_depth(1);
            return;
        case B_TID: c.push_back(X_TID); push_depth(1); return;
        case B_VAR: c.push_back(X_VAR); c.push_back(x.slot); push_depth(1); return;
        case B_TRUE: c.push_back(X_TRUE); push_depth(1); return;
        case B_FALSE: c.push_back(X_FALSE); push_depth(1); return;
        case B_NOT: gen_x(x.a); c.push_back(X_NOT); return;
        }
        // immediate forms: constant right operand (or left for + and *) below 2^32
        const XNode &A = ir.x[x.a], &B = ir.x[x.b];
        int var_side = -1;
        uint64_t k = 0;
        if (is_const(B) && B.val < (1ull << 32)) { var_side = x.a; k = B.val; }
        else if ((x.op == B_ADD || x.op == B_MUL) && is_const(A) && A.val < (1ull << 32)) { var_side = x.b; k = A.val; }
        if (var_side >= 0) {
            uint32_t op = 0, arg = (uint32_t)k;
            bool pow2 = k && !(k & (k - 1));
            switch (x.op) {
            case B_ADD: op = X_ADDC; break;
            case B_MUL: op = X_MULC; break;
            case B_DIV: if (k) { if (pow2) { op = X_SHRC; arg = (uint32_t)__builtin_ctzll(k); } else op = X_DIVC; } break;
            case B_MOD: if (k) { if (pow2) { op = X_ANDC; arg = (uint32_t)(k - 1); } else op = X_MODC; } break;
            }
            if (op) {
                gen_x(var_side);
                c.push_back(op);
                c.push_back(arg);
                return;
            }
        }
        gen_x(x.a);
        gen_x(x.b);
        static const uint32_t map[][2] = {{B_ADD, X_ADD}, {B_MONUS, X_MONUS}, {B_MUL, X_MUL}, {B_DIV, X_DIV},
                                          {B_MOD, X_MOD}, {B_SHL, X_SHL}, {B_SHR, X_SHR}, {B_MIN, X_MIN},
                                          {B_MAX, X_MAX}, {B_LT, X_LT}, {B_LE, X_LE}, {B_EQ, X_EQ},
                                          {B_NE, X_NE}, {B_GT, X_GT}, {B_GE, X_GE}, {B_AND, X_AND}, {B_OR, X_OR}};
        for (auto &m : map) if (m[0] == x.op) { c.push_back(m[1]); push_depth(-1); return; }
        fail(DRF_E_BYTECODE);
    }

    void gen_block(int e) {
        auto &c = *code;
        size_t at = c.size();
        c.push_back(0);
        stack_depth = 0;
        gen_x(e);
        c[at] = (uint32_t)(c.size() - at - 1);
        if (stack_max > MAXSTACK) fail(DRF_E_LIMIT);
    }

    void gen_s(int si) {
        const SNode &s = ir.s[si];
        auto &c = *code;
        switch (s.kind) {
        case B_SKIP: return;
        case B_ACC: c.push_back(U_ACC); c.push_back(s.mode); gen_block(s.e); return;
        case B_SEQ: for (int k : s.kids) gen_s(k); return;
        case B_IF: {
            if (++nest_depth > MAXDEPTH) fail(DRF_E_LIMIT);
            c.push_back(U_IF);
            gen_block(s.e);
            size_t else_slot = c.size();
            c.push_back(0);
            gen_s(s.kids[0]);
            c[else_slot] = (uint32_t)c.size();
            c.push_back(U_ELSE);
            size_t end_slot = c.size();
            c.push_back(0);
            gen_s(s.kids[1]);
            c[end_slot] = (uint32_t)c.size();
            c.push_back(U_ENDIF);
            nest_depth--;
            return;
        }
        case B_FORU: {
            if (++nest_depth > MAXDEPTH) fail(DRF_E_LIMIT);
            c.push_back(U_FOR);
            c.push_back(s.slot);
            gen_block(s.lo);
            gen_block(s.hi);
            size_t end_slot = c.size();
            c.push_back(0);
            uint32_t body = (uint32_t)c.size();
            gen_s(s.kids[0]);
            c.push_back(U_ENDFOR);
            c.push_back(s.slot);
            c.push_back(body);
            c[end_slot] = (uint32_t)c.size();
            nest_depth--;
            return;
        }
        default: fail(DRF_E_BYTECODE); return;
        }
    }

    // ---- compiled access leaf (see drf_layout.hpp)
    struct COp {
        uint32_t op;
        uint64_t imm;              // constant part of the operand
        std::vector<int> adds;     // tid-free expression nodes added to it
    };

    // e as a chain of operations on tid with tid-free operands
    bool chain(int e, std::vector<COp> &ops) {
        const XNode &x = ir.x[e];
        if (x.op == B_TID) return true;
        if (x.a < 0 || x.b < 0) return false;
        const bool ta = mentions_tid(ir, x.a), tbv = mentions_tid(ir, x.b);
        if (ta == tbv) return false;
        const int v = ta ? x.a : x.b, u = ta ? x.b : x.a;
        uint32_t op = 0;
        switch (x.op) {
        case B_ADD: op = C_ADD; break;
        case B_MUL: op = C_MUL; break;
        case B_MIN: op = C_MIN; break;
        case B_MAX: op = C_MAX; break;
        case B_MONUS: op = ta ? C_MONUS : C_RMONUS; break;
        case B_DIV: op = ta ? C_DIV : 0; break;
        case B_MOD: op = ta ? C_MOD : 0; break;
        case B_SHL: op = ta ? C_SHL : 0; break;
        case B_SHR: op = ta ? C_SHR : 0; break;
        default: break;
        }
        if (!op || !chain(v, ops)) return false;
        COp c{op, 0, {}};
        const XNode &U = ir.x[u];
        if (is_const(U)) c.imm = U.val; else c.adds.push_back(u);
        // consecutive additions share one operand: with every value of the
        // original expression below 2^32 the regrouped sum is too
        if (op == C_ADD && !ops.empty() && ops.back().op == C_ADD) {
            ops.back().imm += c.imm;
            ops.back().adds.insert(ops.back().adds.end(), c.adds.begin(), c.adds.end());
            return true;
        }
        ops.push_back(std::move(c));
        return true;
    }

    bool straight(int si, std::vector<int> &accs) const {
        const SNode &s = ir.s[si];
        if (s.kind == B_SKIP) return true;
        if (s.kind == B_ACC) { accs.push_back(si); return true; }
        if (s.kind != B_SEQ) return false;
        for (int k : s.kids) if (!straight(k, accs)) return false;
        return true;
    }

    // Appends the compiled access leaf of `leaf` to the current code and
    // returns its offset, or -1 when the leaf has another shape.  `guarded`:
    // the leaf is a thread-limit if whose accesses are all in its then part.
    int gen_cal(int leaf, bool guarded) {
        if (plan.wide) return -1;
        std::vector<int> accs;
        if (!straight(guarded ? ir.s[leaf].kids[0] : leaf, accs) || accs.empty()) return -1;
        std::vector<std::vector<COp>> chains(accs.size());
        for (size_t j = 0; j < accs.size(); j++) {
            if (!chain(ir.s[accs[j]].e, chains[j]) || chains[j].size() > CAL_MAXOPS) return -1;
            for (auto &c : chains[j]) if (c.imm >= (1ull << 32)) return -1;
        }
        // uniform slots (identical operands share one)
        std::vector<std::pair<std::vector<int>, uint64_t>> slots;
        auto slot_of = [&](const COp &c) -> int {
            for (size_t i = 0; i < slots.size(); i++)
                if (slots[i].first == c.adds && slots[i].second == c.imm) return (int)i;
            slots.push_back({c.adds, c.imm});
            return (int)slots.size() - 1;
        };
        std::vector<std::vector<std::pair<uint32_t, uint32_t>>> enc(accs.size());
        for (size_t j = 0; j < accs.size(); j++) {
            for (auto &c : chains[j]) {
                if (!c.adds.empty()) {
                    enc[j].push_back({c.op | C_UNI, (uint32_t)slot_of(c)});
                    continue;
                }
                const uint64_t k = c.imm;
                const bool pow2 = k && !(k & (k - 1));
                if (c.op == C_MOD && pow2) enc[j].push_back({C_AND, (uint32_t)(k - 1)});
                else if (c.op == C_DIV && pow2) enc[j].push_back({C_SHR, (uint32_t)__builtin_ctzll(k)});
                else enc[j].push_back({c.op, (uint32_t)k});
            }
        }
        if (slots.size() > CAL_MAXU) return -1;
        auto &c = *code;
        const int at = (int)c.size();
        c.push_back((uint32_t)accs.size());
        c.push_back((uint32_t)slots.size());
        const size_t acc_at = c.size();
        c.push_back(0);   // word offset of the first access block, set below
        for (auto &sl : slots) {
            const size_t len_at = c.size();
            c.push_back(0);
            stack_depth = 0;
            stack_max = 0;
            for (size_t i = 0; i < sl.first.size(); i++) {
                gen_x(sl.first[i]);
                if (i) { c.push_back(X_ADD); push_depth(-1); }
            }
            if (sl.second) { c.push_back(X_ADDC); c.push_back((uint32_t)sl.second); }
            c[len_at] = (uint32_t)(c.size() - len_at - 1);
            if (stack_max > MAXSTACK) {
                c.resize((size_t)at);
                return -1;
            }
        }
        c[acc_at] = (uint32_t)(c.size() - (size_t)at);
        for (size_t j = 0; j < accs.size(); j++) {
            // the fixed form: [ADD c0] [AND|MOD m0] [MUL a] [ADD uniform] [AND|MOD pa]
            // form c0 m0k m0 a us pk pa m0mag m0sh pamag pash (mode before,
            // nops after: CAL_HDR words in all)
            uint32_t hdr[CAL_HDR - 2] = {0, 0, CAL_K_NONE, 0, 1, NONE32, CAL_K_NONE, 0, 0, 0, 0, 0};
            size_t q = 0;
            const auto &e = enc[j];
            auto kind = [](uint32_t op) { return op == C_AND ? CAL_K_AND : op == C_MOD ? CAL_K_MOD : CAL_K_NONE; };
            if (q < e.size() && e[q].first == C_ADD) { hdr[1] = e[q].second; q++; }
            if (q < e.size() && (e[q].first == C_AND || e[q].first == C_MOD)) { hdr[2] = kind(e[q].first); hdr[3] = e[q].second; q++; }
            if (q < e.size() && e[q].first == C_MUL) { hdr[4] = e[q].second; q++; }
            if (q < e.size() && e[q].first == (C_ADD | C_UNI)) { hdr[5] = e[q].second; q++; }
            if (q < e.size() && (e[q].first == C_AND || e[q].first == C_MOD)) { hdr[6] = kind(e[q].first); hdr[7] = e[q].second; q++; }
            hdr[0] = q == e.size() ? 1u : 0u;
            // moduli of the fixed form: mod 0 is the identity, any other
            // gets its division magic
            for (int m = 0; m < 2; m++) {
                uint32_t &k = hdr[m ? 6 : 2];
                const uint32_t d = hdr[m ? 7 : 3];
                if (k != CAL_K_MOD) continue;
                if (d == 0) { k = CAL_K_NONE; continue; }
                div_magic(d, hdr[m ? 10 : 8], hdr[m ? 11 : 9]);
            }
            c.push_back(ir.s[accs[j]].mode);
            for (uint32_t w : hdr) c.push_back(w);
            c.push_back((uint32_t)e.size());
            for (auto &o : e) { c.push_back(o.first); c.push_back(o.second); }
        }
        return at;
    }

    bool has_access(int si) const {
        const SNode &s = ir.s[si];
        if (s.kind == B_ACC) return true;
        for (int k : s.kids) if (has_access(k)) return true;
        return false;
    }

    // A leaf `if (tid < e) {..} else {no access}` (or <=, >, >= with tid on
    // the matching side) with e free of tid: only tids below e (or e + 1)
    // can access memory.  Returns the expression and whether to add 1.
    int thread_limit(int si, bool &plus1) const {
        const SNode &s = ir.s[si];
        if (s.kind != B_IF || has_access(s.kids[1])) return -1;
        const XNode &c = ir.x[s.e];
        const XNode *A = c.a >= 0 ? &ir.x[c.a] : nullptr, *B = c.b >= 0 ? &ir.x[c.b] : nullptr;
        if (!A || !B) return -1;
        if ((c.op == B_LT || c.op == B_LE) && A->op == B_TID && !mentions_tid(ir, c.b)) {
            plus1 = c.op == B_LE;
            return c.b;
        }
        if ((c.op == B_GT || c.op == B_GE) && B->op == B_TID && !mentions_tid(ir, c.a)) {
            plus1 = c.op == B_GE;
            return c.a;
        }
        return -1;
    }

    void run() {
        std::vector<uint32_t> map(ir.nslots + 1, 0);
        renumber(ir.root, map, 0);
        if (max_depth > (uint32_t)MAXSLOTS) { fail(DRF_E_LIMIT); return; }
        if (n > (1u << 31)) { fail(DRF_E_LIMIT); return; }
        mark_s(ir.root);
        decide_unroll();
        uint64_t cursor = 0;
        walk(ir.root, cursor);
        if (status) return;
        plan.num_phases = cursor + 1;
        // per nest: iterations, last phase, intervals, event bound
        for (Nest &ne : plan.nests) {
            u128 it = 1;
            u128 last = ne.phase_base;
            for (auto &l : ne.loops) { it = smul(it, l.trip); last += (u128)(l.trip - 1) * l.stride; }
            if (it >= MAX_EVENTS) { fail(DRF_E_LIMIT); return; }
            ne.iters = (uint64_t)it;
            ne.phase_last = (uint64_t)last;
            for (int i = 0; i <= MAXSLOTS; i++) var_iv[i] = {0, 0};
            for (auto &l : ne.loops) var_iv[l.slot] = {l.lo, (u128)l.lo + l.trip - 1};
            for (auto &f : ne.fixed) var_iv[f.first] = {f.second, f.second};
            work = 0;
            u128 per = iv_stmt(ne.leaf);
            ne.rec_bound = (uint32_t)std::min<u128>(per, 0xFFFFFFFFu);
            // a thread-limit guard bounds the tids that can access memory
            ne.tid_bound = n;
            {
                bool plus1 = false;
                const int lim = thread_limit(ne.leaf, plus1);
                if (lim >= 0) {
                    const u128 hi = sat(ivx(lim).hi + (plus1 ? 1 : 0));
                    if (hi < (u128)n) ne.tid_bound = (uint32_t)hi;
                }
            }
            const u128 tids = ne.tid_bound;
            events = sat(events + smul(smul(per, tids), it));
            total_work = sat(total_work + smul(smul(sat(work + per + 1), n), it));
            // iterations sharing one phase: the loops whose body holds no sync
            u128 same = 1;
            for (auto &l : ne.loops) if (l.stride == 0) same = smul(same, l.trip);
            phase_events = sat(phase_events + smul(smul(per, tids), same));
        }
        plan.max_phase_records = (uint64_t)std::min<u128>(phase_events, ~0ull);
        if (events >= MAX_EVENTS || total_work >= MAX_EVENTS * 4) { fail(DRF_E_LIMIT); return; }
        plan.max_records = (uint64_t)events;
        plan.wide = iv_max >= (u128)(1ull << 32);
        // leaf code (the 32- or 64-bit evaluator decides what may be folded)
        for (Nest &ne : plan.nests) {
            auto f = code_of_leaf.find(ne.leaf);
            if (f == code_of_leaf.end()) {
                plan.leaf_code.emplace_back();
                code = &plan.leaf_code.back();
                stack_max = 0;
                nest_depth = 0;
                gen_s(ne.leaf);
                code->push_back(U_END);
                // thread limit (32-bit evaluator only: no overflow to detect)
                bool plus1 = false;
                const int lim = plan.wide ? -1 : thread_limit(ne.leaf, plus1);
                if (lim >= 0) {
                    plan.leaf_guard.push_back((int)code->size());
                    stack_max = 0;
                    gen_block(lim);
                    if (plus1) {
                        // the block's postfix code grows by one immediate op
                        (*code)[plan.leaf_guard.back()] += 2;
                        code->push_back(X_ADDC);
                        code->push_back(1);
                    }
                } else {
                    plan.leaf_guard.push_back(-1);
                }
                plan.leaf_cal.push_back(gen_cal(ne.leaf, lim >= 0));
                int id = (int)plan.leaf_code.size() - 1;
                code_of_leaf[ne.leaf] = id;
                plan.nest_leaf_code.push_back(id);
            } else {
                plan.nest_leaf_code.push_back(f->second);
            }
            if (status) return;
        }
        uint32_t bits = 0;
        while (bits < 32 && (max_index >> bits) != 0) bits++;
        plan.index_bits = bits;
    }
};

}  // namespace

int plan_protocol(const uint32_t *code, uint32_t words, uint32_t n, Plan &plan) {
    plan = Plan();
    plan.n = n;
    IR ir;
    int st = decode(code, words, ir);
    if (!st) st = static_check(ir);
    // several arrays: one protocol per array (drf_check_arrays)
    if (!st && ir_arrays(ir) > 1) st = DRF_E_MULTI;
    if (st) { plan.status = st; return 0; }
    Planner p(ir, n, plan);
    p.run();
    if (p.status) {
        int s2 = p.status;
        plan = Plan();
        plan.n = n;
        plan.status = s2;
    }
    return 0;
}

// ================================================== rewriting of protocols
namespace {

void enc_expr(const IR &ir, int e, std::vector<uint32_t> &w) {
    const XNode &x = ir.x[e];
    if (x.a >= 0) enc_expr(ir, x.a, w);
    if (x.b >= 0) enc_expr(ir, x.b, w);
    switch (x.op) {
    case B_CONST32: case B_CONST64:
        if (x.val < (1ull << 32)) {
            w.push_back(B_CONST32);
            w.push_back((uint32_t)x.val);
        } else {
            w.push_back(B_CONST64);
            w.push_back((uint32_t)x.val);
            w.push_back((uint32_t)(x.val >> 32));
        }
        break;
    case B_VAR:
        w.push_back(B_VAR);
        w.push_back(x.slot);
        break;
    default: w.push_back(x.op); break;
    }
}

void enc_block(const IR &ir, int e, std::vector<uint32_t> &out) {
    std::vector<uint32_t> w;
    enc_expr(ir, e, w);
    out.push_back((uint32_t)w.size());
    out.insert(out.end(), w.begin(), w.end());
}

void enc_stmt(const IR &ir, int si, std::vector<uint32_t> &out) {
    const SNode &s = ir.s[si];
    out.push_back(s.kind);
    switch (s.kind) {
    case B_ACC:
        out.push_back(s.mode | s.array << 1);
        enc_block(ir, s.e, out);
        break;
    case B_SEQ:
        out.push_back((uint32_t)s.kids.size());
        for (int k : s.kids) enc_stmt(ir, k, out);
        break;
    case B_IF:
        enc_block(ir, s.e, out);
        enc_stmt(ir, s.kids[0], out);
        enc_stmt(ir, s.kids[1], out);
        break;
    case B_FORU: case B_FORS:
        out.push_back(s.slot);
        enc_block(ir, s.lo, out);
        enc_block(ir, s.hi, out);
        enc_stmt(ir, s.kids[0], out);
        break;
    default: break;   // skip, sync
    }
}

}  // namespace

void encode(const IR &ir, std::vector<uint32_t> &out) {
    std::vector<uint32_t> body;
    if (ir.root >= 0) enc_stmt(ir, ir.root, body);
    out.clear();
    out.push_back(DRF_MAGIC);
    out.push_back(1);
    out.push_back(ir.nslots);
    out.push_back((uint32_t)body.size());
    out.insert(out.end(), body.begin(), body.end());
}

uint32_t ir_arrays(const IR &ir) {
    uint32_t a = 0;
    for (const SNode &s : ir.s)
        if (s.kind == B_ACC && s.array > a) a = s.array;
    return a + 1;
}

void ir_project(IR &ir, uint32_t array) {
    for (SNode &s : ir.s) {
        if (s.kind != B_ACC) continue;
        if (s.array == array) {
            s.array = 0;
        } else {
            s.kind = B_SKIP;
            s.e = -1;
        }
    }
}

bool ir_bind(IR &ir, uint32_t slot, uint64_t v) {
    for (const SNode &s : ir.s)
        if ((s.kind == B_FORU || s.kind == B_FORS) && s.slot == slot) return false;
    for (XNode &x : ir.x)
        if (x.op == B_VAR && x.slot == slot) {
            x.op = v < (1ull << 32) ? B_CONST32 : B_CONST64;
            x.val = v;
        }
    return true;
}

}  // namespace drf
