// BabyCUDA front end of libdrf: parser of the s-expression text form of
// BabyCUDA programs and the behavioural type system that gives a program
// its memory access protocol (Section 4, Fig. "Behavioral type system",
// judgement V |- b |> u), with the synchronized fragment added as for
// protocols (sync passes through; a loop whose body synchronizes becomes
// for^S).
//
// Text form (Section 3, Fig. "Syntax and semantics of BabyCUDA"):
//   b ::= (skip) | (sync) | (wr n n') | (rd y n b) | (seq b ...)
//       | (if c b b) | (for x n n b)
// (wr n n') writes payload n' at index n; (rd y n b) reads index n into y
// and continues with b; wr:A / rd:A name one of several shared arrays.
// n and c are the protocol language's arithmetic and boolean expressions.
//
// Typing (all rules of the figure):
//   t-n / t-b   an index, guard or loop bound mentions only variables of V
//               (V starts as {tid} plus the caller's parameters); a variable
//               bound by a read there is a data-dependent access: ill-typed
//   t-write     wr[n] := n'  has type wr[n]; the payload may use any
//               variable in scope (read data included) and is dropped
//   t-read      let y = rd[n] in b  has type rd[n]; u where b : u under the
//               same V (y is not added: data never reaches control flow or
//               indices); y is a fresh binder
//   t-for       bounds typed under V, x fresh, body under V + {x}
//   t-seq, t-if, t-skip   follow the shape of the program
// Nested binders are distinct (the side condition x, y not in V).
#include <string.h>

#include <set>
#include <string>
#include <vector>

#include "../../include/drf.h"
#include "host.hpp"

namespace drf {
namespace {

struct SNodeB {
    bool list = false;
    std::string atom;
    std::vector<SNodeB> kids;
};

struct Reader {
    const char *s;
    size_t n, pos = 0;
    bool err = false;
    static bool space(char c) { return c == ' ' || c == '\t' || c == '\n' || c == '\r'; }
    bool token(std::string &t) {
        while (pos < n && space(s[pos])) pos++;
        if (pos >= n) return false;
        if (s[pos] == '(' || s[pos] == ')') {
            t.assign(1, s[pos++]);
            return true;
        }
        const size_t b = pos;
        while (pos < n && !space(s[pos]) && s[pos] != '(' && s[pos] != ')') pos++;
        t.assign(s + b, pos - b);
        return true;
    }
    bool read(SNodeB &out, int depth = 0) {
        std::string t;
        if (depth > 4096 || !token(t) || t == ")") return false;
        if (t != "(") {
            out.atom = t;
            return true;
        }
        out.list = true;
        for (;;) {
            const size_t save = pos;
            std::string u;
            if (!token(u)) return false;
            if (u == ")") return true;
            pos = save;
            SNodeB k;
            if (!read(k, depth + 1)) return false;
            out.kids.push_back(std::move(k));
        }
    }
};

const char *const KEYWORDS[] = {"+",   "-",    "*",    "/",    "mod",  "<<",   ">>",   "min",  "max", "<",
                                "<=",  "=",    "!=",   ">",    ">=",   "and",  "or",   "not",  "true", "false",
                                "skip", "rd",  "wr",   "seq",  "if",   "foru", "fors", "sync", "for",  "tid",
                                nullptr};

bool ident(const std::string &t) {
    if (t.empty()) return false;
    const char c = t[0];
    if (!((c >= 'a' && c <= 'z') || (c >= 'A' && c <= 'Z') || c == '_')) return false;
    for (char ch : t)
        if (!((ch >= 'a' && ch <= 'z') || (ch >= 'A' && ch <= 'Z') || (ch >= '0' && ch <= '9') || ch == '_'))
            return false;
    for (int i = 0; KEYWORDS[i]; i++)
        if (t == KEYWORDS[i]) return false;
    return true;
}

bool numeral(const std::string &t) {
    if (t.empty() || t.size() > 20) return false;
    for (char c : t)
        if (c < '0' || c > '9') return false;
    return true;
}

struct Infer {
    int status = 0;                  // first typing violation (pre-order)
    bool syntax = false;             // not a BabyCUDA program at all
    std::set<std::string> V;         // variables usable in indices, guards, bounds
    std::set<std::string> D;         // read-bound variables in scope (payloads only)

    void fail(int st) {
        if (!status) status = st;
    }

    // A variable occurrence in an index, guard or bound (t-n / t-b).
    void typed_var(const std::string &v) {
        if (V.count(v)) return;
        fail(D.count(v) ? DRF_E_ILLTYPED : DRF_E_UNBOUND);
    }
    // A variable occurrence in a payload (any variable in scope).
    void scoped_var(const std::string &v) {
        if (!V.count(v) && !D.count(v)) fail(DRF_E_UNBOUND);
    }

    // Arithmetic expression: validates, applies `use` to each variable and
    // prints it back.
    template <class Use>
    std::string nexp(const SNodeB &e, Use use) {
        if (!e.list) {
            if (numeral(e.atom)) return e.atom;
            if (e.atom == "tid") {
                use(std::string("tid"));
                return e.atom;
            }
            if (ident(e.atom)) {
                use(e.atom);
                return e.atom;
            }
            syntax = true;
            return "";
        }
        static const char *ops[] = {"+", "-", "*", "/", "mod", "<<", ">>", "min", "max", nullptr};
        if (e.kids.size() == 3 && !e.kids[0].list) {
            for (int i = 0; ops[i]; i++)
                if (e.kids[0].atom == ops[i]) {
                    std::string a = nexp(e.kids[1], use), b = nexp(e.kids[2], use);
                    return "(" + e.kids[0].atom + " " + a + " " + b + ")";
                }
        }
        syntax = true;
        return "";
    }

    template <class Use>
    std::string bexp(const SNodeB &c, Use use) {
        if (!c.list) {
            if (c.atom == "true" || c.atom == "false") return c.atom;
            syntax = true;
            return "";
        }
        static const char *rels[] = {"<", "<=", "=", "!=", ">", ">=", nullptr};
        if (c.kids.size() == 3 && !c.kids[0].list) {
            const std::string &h = c.kids[0].atom;
            for (int i = 0; rels[i]; i++)
                if (h == rels[i]) {
                    std::string a = nexp(c.kids[1], use), b = nexp(c.kids[2], use);
                    return "(" + h + " " + a + " " + b + ")";
                }
            if (h == "and" || h == "or") {
                std::string a = bexp(c.kids[1], use), b = bexp(c.kids[2], use);
                return "(" + h + " " + a + " " + b + ")";
            }
        }
        if (c.kids.size() == 2 && !c.kids[0].list && c.kids[0].atom == "not")
            return "(not " + bexp(c.kids[1], use) + ")";
        syntax = true;
        return "";
    }

    std::string typed_n(const SNodeB &e) {
        return nexp(e, [&](const std::string &v) { typed_var(v); });
    }

    // A fresh binder: not tid, not any variable in scope (nested binders
    // are distinct, and a read's variable is no loop's).
    void binder(const std::string &x) {
        if (x == "tid" || V.count(x) || D.count(x)) fail(DRF_E_SHADOW);
    }

    static bool access_head(const std::string &h, const char *mode, std::string &array) {
        const size_t m = strlen(mode);
        if (h.compare(0, m, mode) != 0) return false;
        if (h.size() == m) {
            array.clear();
            return true;
        }
        if (h[m] != ':') return false;
        array = h.substr(m + 1);
        return ident(array);
    }

    // V |- b |> u: returns the protocol text of b; *sync tells whether it
    // holds a barrier.
    std::string stmt(const SNodeB &b, bool &sync) {
        if (!b.list || b.kids.empty() || b.kids[0].list) {
            syntax = true;
            return "";
        }
        const std::string &h = b.kids[0].atom;
        const size_t k = b.kids.size();
        std::string arr;
        if (h == "skip" && k == 1) return "(skip)";                                 // t-skip
        if (h == "sync" && k == 1) {
            sync = true;
            return "(sync)";
        }
        if (access_head(h, "wr", arr) && k == 3) {                                  // t-write
            std::string idx = typed_n(b.kids[1]);
            nexp(b.kids[2], [&](const std::string &v) { if (v != "tid") scoped_var(v); });
            return "(wr" + (arr.empty() ? std::string() : ":" + arr) + " " + idx + ")";
        }
        if (access_head(h, "rd", arr) && k == 4) {                                  // t-read
            if (b.kids[1].list || !ident(b.kids[1].atom)) {
                syntax = true;
                return "";
            }
            const std::string y = b.kids[1].atom;
            std::string idx = typed_n(b.kids[2]);
            binder(y);
            const bool fresh = !D.count(y);
            D.insert(y);
            std::string u = stmt(b.kids[3], sync);
            if (fresh) D.erase(y);
            return "(seq (rd" + (arr.empty() ? std::string() : ":" + arr) + " " + idx + ") " + u + ")";
        }
        if (h == "seq") {                                                           // t-seq
            std::string out = "(seq";
            for (size_t i = 1; i < k; i++) out += " " + stmt(b.kids[i], sync);
            return out + ")";
        }
        if (h == "if" && k == 4) {                                                  // t-if
            std::string c = bexp(b.kids[1], [&](const std::string &v) { typed_var(v); });
            std::string u1 = stmt(b.kids[2], sync);
            std::string u2 = stmt(b.kids[3], sync);
            return "(if " + c + " " + u1 + " " + u2 + ")";
        }
        if (h == "for" && k == 5) {                                                 // t-for
            if (b.kids[1].list || !(ident(b.kids[1].atom) || b.kids[1].atom == "tid")) {
                syntax = true;
                return "";
            }
            const std::string x = b.kids[1].atom;
            std::string lo = typed_n(b.kids[2]);
            std::string hi = typed_n(b.kids[3]);
            binder(x);
            const bool fresh = !V.count(x);
            V.insert(x);
            bool inner = false;
            std::string u = stmt(b.kids[4], inner);
            if (fresh) V.erase(x);
            sync |= inner;
            return std::string(inner ? "(fors " : "(foru ") + x + " " + lo + " " + hi + " " + u + ")";
        }
        syntax = true;
        return "";
    }
};

}  // namespace

int babycuda_infer(const char *text, size_t len, const char *params, std::string &map_text) {
    Reader r{text, len};
    SNodeB root;
    if (!r.read(root)) return DRF_E_ARG;
    std::string extra;
    if (r.token(extra)) return DRF_E_ARG;
    Infer inf;
    inf.V.insert("tid");
    if (params) {
        Reader p{params, strlen(params)};
        std::string name;
        while (p.token(name)) {
            if (!ident(name)) return DRF_E_ARG;
            inf.V.insert(name);
        }
    }
    bool sync = false;
    map_text = inf.stmt(root, sync);
    if (inf.syntax) return DRF_E_ARG;
    return inf.status;
}

}  // namespace drf
