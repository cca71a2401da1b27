/*
 * O2: plain C oracle for data-race freedom of memory access protocols.
 * Test infrastructure only (tests, smoke check and the CPU baseline of the
 * bench run it); the HIP product path never links or runs it.
 *
 * Same definition as the Python oracle (ref.py), written independently:
 *   - protocol syntax: Fig. "Syntax of MAPs", with a U leaf inside S;
 *   - thread-level rules seq / if-t / if-f / for-1 / for-2 / skip and the
 *     parallel rule par of Fig. "Syntax and semantics of BabyCUDA";
 *   - sync closes the current phase for all of T and opens an empty one;
 *     for^S bounds are evaluated once per loop entry and are tid-free;
 *   - Definition 1: a phase is racy iff some index is written by a thread
 *     and read or written by another thread in that phase.
 *
 * Per phase it keeps, for every index touched, an aggregate cell
 *   t0 = least tid touching it, t1 = least tid different from t0,
 *   w0 = least tid writing it.
 * The index is racy iff w0 and t1 both exist, and the least pair (i1 < i2)
 * with at least one writer is (t0, w0 == t0 ? t1 : w0): i1 = t0 always
 * works (if t0 writes, pair it with t1; otherwise w0 > t0 writes).
 *
 * Input  (stdin or argv[1]): one protocol per line, "<n> <s-expression>".
 * Output (stdout): one line per protocol, in input order:
 *   <status> <racy> <phase> <index> <tid_i> <tid_j> <num_records> <num_phases> <count_0> ... <count_K>
 * (witness fields are 4294967295 when there is no race; counts are omitted
 * when status != 0).  Options: -j N worker threads over protocols (default
 * 1), -t print per-protocol wall time to stderr.
 */
#define _GNU_SOURCE
#include <errno.h>
#include <pthread.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

enum { OK = 0, E_UNBOUND = -3, E_SHADOW = -4, E_SYNC_IN_U = -5, E_DIVERGENT = -6, E_RANGE = -7 };
#define VALUE_LIMIT (UINT64_C(1) << 63)
#define INDEX_LIMIT (UINT64_C(1) << 32)
#define NONE32 0xFFFFFFFFu

/* ------------------------------------------------------------- AST ----- */
typedef enum {
    N_CONST, N_TID, N_VAR, N_BIN,           /* arithmetic */
    B_TRUE, B_FALSE, B_REL, B_AND, B_OR, B_NOT, /* boolean */
    S_SKIP, S_RD, S_WR, S_SEQ, S_IF, S_FORU, S_SYNC, S_FORS
} Kind;

typedef enum { OP_ADD, OP_SUB, OP_MUL, OP_DIV, OP_MOD, OP_SHL, OP_SHR, OP_MIN, OP_MAX } Op;
typedef enum { R_LT, R_LE, R_EQ, R_NE, R_GT, R_GE } Rel;

typedef struct Node {
    Kind kind;
    int op;                 /* Op or Rel */
    uint64_t value;         /* N_CONST */
    char name[80];          /* N_VAR and loop binder name */
    int slot;               /* resolved variable slot (N_VAR / loop binder) */
    int has_s;              /* statement contains sync or for^S */
    struct Node **kids;     /* children */
    int nkids;
} Node;

typedef struct { const char *s; size_t pos, len; int err; } Lexer;

static void skip_ws(Lexer *L) { while (L->pos < L->len && (L->s[L->pos] == ' ' || L->s[L->pos] == '\t' || L->s[L->pos] == '\n' || L->s[L->pos] == '\r')) L->pos++; }

/* next token into buf; returns 0 at end */
static int next_tok(Lexer *L, char *buf, size_t cap) {
    skip_ws(L);
    if (L->pos >= L->len) return 0;
    char c = L->s[L->pos];
    if (c == '(' || c == ')') { buf[0] = c; buf[1] = 0; L->pos++; return 1; }
    size_t k = 0;
    while (L->pos < L->len) {
        c = L->s[L->pos];
        if (c == ' ' || c == '\t' || c == '\n' || c == '\r' || c == '(' || c == ')') break;
        if (k + 1 < cap) buf[k++] = c; else L->err = 1;
        L->pos++;
    }
    buf[k] = 0;
    return 1;
}

static int peek_tok(Lexer *L, char *buf, size_t cap) { size_t p = L->pos; int r = next_tok(L, buf, cap); L->pos = p; return r; }

static Node *mk(Kind k) { Node *n = calloc(1, sizeof(Node)); n->kind = k; n->slot = -1; return n; }
static void add_kid(Node *p, Node *c) { p->kids = realloc(p->kids, sizeof(Node *) * (p->nkids + 1)); p->kids[p->nkids++] = c; }
static void free_node(Node *n) { if (!n) return; for (int i = 0; i < n->nkids; i++) free_node(n->kids[i]); free(n->kids); free(n); }

static const char *KEYW[] = {"+","-","*","/","mod","<<",">>","min","max","<","<=","=","!=",">",">=",
                             "and","or","not","true","false","skip","rd","wr","seq","if","foru","fors","sync",0};
static int is_keyword(const char *t) { for (int i = 0; KEYW[i]; i++) if (!strcmp(KEYW[i], t)) return 1; return 0; }
static int is_ident(const char *t) {
    if (!((t[0] >= 'a' && t[0] <= 'z') || (t[0] >= 'A' && t[0] <= 'Z') || t[0] == '_')) return 0;
    for (const char *p = t; *p; p++)
        if (!((*p >= 'a' && *p <= 'z') || (*p >= 'A' && *p <= 'Z') || (*p >= '0' && *p <= '9') || *p == '_')) return 0;
    return !is_keyword(t);
}
static int arith_op(const char *t) {
    static const char *ops[] = {"+","-","*","/","mod","<<",">>","min","max"};
    for (int i = 0; i < 9; i++) if (!strcmp(ops[i], t)) return i;
    return -1;
}
static int rel_op(const char *t) {
    static const char *ops[] = {"<","<=","=","!=",">",">="};
    for (int i = 0; i < 6; i++) if (!strcmp(ops[i], t)) return i;
    return -1;
}

static int expect(Lexer *L, const char *want) { char b[80]; if (!next_tok(L, b, sizeof b) || strcmp(b, want)) { L->err = 1; return 0; } return 1; }

static Node *p_nexp(Lexer *L) {
    char b[80];
    if (!next_tok(L, b, sizeof b)) { L->err = 1; return NULL; }
    if (!strcmp(b, "(")) {
        char op[80];
        if (!next_tok(L, op, sizeof op)) { L->err = 1; return NULL; }
        int o = arith_op(op);
        if (o < 0) { L->err = 1; return NULL; }
        Node *n = mk(N_BIN); n->op = o;
        add_kid(n, p_nexp(L)); if (L->err) return n;
        add_kid(n, p_nexp(L)); if (L->err) return n;
        expect(L, ")");
        return n;
    }
    if (b[0] >= '0' && b[0] <= '9') {
        for (char *p = b; *p; p++) if (*p < '0' || *p > '9') { L->err = 1; return NULL; }
        errno = 0;
        unsigned long long v = strtoull(b, NULL, 10);
        if (errno == ERANGE) { L->err = 1; return NULL; }
        Node *n = mk(N_CONST); n->value = v; return n;
    }
    if (!strcmp(b, "tid")) return mk(N_TID);
    if (is_ident(b)) { Node *n = mk(N_VAR); snprintf(n->name, sizeof n->name, "%s", b); return n; }
    L->err = 1; return NULL;
}

static Node *p_bexp(Lexer *L) {
    char b[80];
    if (!next_tok(L, b, sizeof b)) { L->err = 1; return NULL; }
    if (!strcmp(b, "true")) return mk(B_TRUE);
    if (!strcmp(b, "false")) return mk(B_FALSE);
    if (strcmp(b, "(")) { L->err = 1; return NULL; }
    char op[80];
    if (!next_tok(L, op, sizeof op)) { L->err = 1; return NULL; }
    Node *n;
    int r = rel_op(op);
    if (r >= 0) { n = mk(B_REL); n->op = r; add_kid(n, p_nexp(L)); if (!L->err) add_kid(n, p_nexp(L)); }
    else if (!strcmp(op, "and") || !strcmp(op, "or")) { n = mk(op[0] == 'a' ? B_AND : B_OR); add_kid(n, p_bexp(L)); if (!L->err) add_kid(n, p_bexp(L)); }
    else if (!strcmp(op, "not")) { n = mk(B_NOT); add_kid(n, p_bexp(L)); }
    else { L->err = 1; return NULL; }
    if (!L->err) expect(L, ")");
    return n;
}

static Node *p_stmt(Lexer *L) {
    char b[80];
    if (!expect(L, "(")) return NULL;
    if (!next_tok(L, b, sizeof b)) { L->err = 1; return NULL; }
    Node *n = NULL;
    if (!strcmp(b, "skip")) n = mk(S_SKIP);
    else if (!strcmp(b, "sync")) n = mk(S_SYNC);
    else if (!strcmp(b, "rd") || !strcmp(b, "wr")) { n = mk(b[0] == 'r' ? S_RD : S_WR); add_kid(n, p_nexp(L)); }
    else if (!strcmp(b, "seq")) {
        n = mk(S_SEQ);
        char pk[80];
        while (!L->err && peek_tok(L, pk, sizeof pk) && strcmp(pk, ")")) add_kid(n, p_stmt(L));
    } else if (!strcmp(b, "if")) {
        n = mk(S_IF); add_kid(n, p_bexp(L));
        if (!L->err) add_kid(n, p_stmt(L));
        if (!L->err) add_kid(n, p_stmt(L));
    } else if (!strcmp(b, "foru") || !strcmp(b, "fors")) {
        n = mk(b[3] == 'u' ? S_FORU : S_FORS);
        char x[80];
        if (!next_tok(L, x, sizeof x) || !(is_ident(x) || !strcmp(x, "tid"))) { L->err = 1; return n; }
        snprintf(n->name, sizeof n->name, "%s", x);
        add_kid(n, p_nexp(L));
        if (!L->err) add_kid(n, p_nexp(L));
        if (!L->err) add_kid(n, p_stmt(L));
    } else { L->err = 1; return NULL; }
    if (!L->err) expect(L, ")");
    return n;
}

/* ------------------------------------------------------ static checks -- */
#define MAXSCOPE 64
typedef struct { const char *names[MAXSCOPE]; int n; } Scope;

static int scope_find(const Scope *s, const char *name) { for (int i = s->n - 1; i >= 0; i--) if (!strcmp(s->names[i], name)) return i; return -1; }

/* 1 if expression mentions a variable not in scope; resolves slots */
static int unbound_in(Node *e, const Scope *s) {
    if (!e) return 0;
    if (e->kind == N_VAR) { e->slot = scope_find(s, e->name); return e->slot < 0; }
    int u = 0;
    for (int i = 0; i < e->nkids; i++) u |= unbound_in(e->kids[i], s);
    return u;
}
static int mentions_tid(const Node *e) {
    if (e->kind == N_TID) return 1;
    for (int i = 0; i < e->nkids; i++) if (mentions_tid(e->kids[i])) return 1;
    return 0;
}

/* pre-order, left to right; first violation wins */
static int check(Node *s, Scope *sc, int in_u) {
    switch (s->kind) {
    case S_SKIP: return OK;
    case S_RD: case S_WR: return unbound_in(s->kids[0], sc) ? E_UNBOUND : OK;
    case S_SEQ:
        for (int i = 0; i < s->nkids; i++) { int st = check(s->kids[i], sc, in_u); if (st) return st; }
        return OK;
    case S_IF: {
        if (unbound_in(s->kids[0], sc)) return E_UNBOUND;
        int st = check(s->kids[1], sc, 1);
        return st ? st : check(s->kids[2], sc, 1);
    }
    case S_SYNC: return in_u ? E_SYNC_IN_U : OK;
    case S_FORU: case S_FORS: {
        if (s->kind == S_FORS && in_u) return E_SYNC_IN_U;
        int u1 = unbound_in(s->kids[0], sc), u2 = unbound_in(s->kids[1], sc);
        if (u1 || u2) return E_UNBOUND;
        if (s->kind == S_FORS && (mentions_tid(s->kids[0]) || mentions_tid(s->kids[1]))) return E_DIVERGENT;
        if (!strcmp(s->name, "tid") || scope_find(sc, s->name) >= 0) return E_SHADOW;
        if (sc->n >= MAXSCOPE) return E_SHADOW;
        sc->names[sc->n] = s->name; s->slot = sc->n; sc->n++;
        int st = check(s->kids[2], sc, in_u || s->kind == S_FORU);
        sc->n--;
        return st;
    }
    default: return OK;
    }
}

static int mark_s(Node *s) {
    if (s->kind == S_SYNC || s->kind == S_FORS) { s->has_s = 1; if (s->kind == S_FORS) mark_s(s->kids[2]); return 1; }
    if (s->kind == S_SEQ) { int h = 0; for (int i = 0; i < s->nkids; i++) h |= mark_s(s->kids[i]); s->has_s = h; return h; }
    return 0;
}

/* --------------------------------------------------------- evaluation -- */
typedef struct {
    uint64_t env[MAXSCOPE];
    uint64_t tid;
    int overflow;
} Env;

static uint64_t chk(Env *E, uint64_t v) { if (v >= VALUE_LIMIT) E->overflow = 1; return v; }

static uint64_t eval_n(const Node *e, Env *E) {
    switch (e->kind) {
    case N_CONST: return chk(E, e->value);
    case N_TID: return E->tid;
    case N_VAR: return E->env[e->slot];
    case N_BIN: {
        uint64_t a = eval_n(e->kids[0], E), b = eval_n(e->kids[1], E);
        if (E->overflow) return 0;
        switch ((Op)e->op) {
        case OP_ADD: return chk(E, a + b); /* both < 2^63: no wrap */
        case OP_SUB: return a > b ? a - b : 0;
        case OP_MUL: { unsigned __int128 r = (unsigned __int128)a * b; if (r >= VALUE_LIMIT) { E->overflow = 1; return 0; } return (uint64_t)r; }
        case OP_DIV: return b ? a / b : 0;
        case OP_MOD: return b ? a % b : a;
        case OP_SHL: {
            if (a == 0) return 0;
            if (b >= 63) { E->overflow = 1; return 0; }
            unsigned __int128 r = (unsigned __int128)a << b;
            if (r >= VALUE_LIMIT) { E->overflow = 1; return 0; }
            return (uint64_t)r;
        }
        case OP_SHR: return b >= 64 ? 0 : a >> b;
        case OP_MIN: return a < b ? a : b;
        case OP_MAX: return a > b ? a : b;
        }
    }
    default: return 0;
    }
}

static int eval_b(const Node *c, Env *E) {
    switch (c->kind) {
    case B_TRUE: return 1;
    case B_FALSE: return 0;
    case B_REL: {
        uint64_t a = eval_n(c->kids[0], E), b = eval_n(c->kids[1], E);
        switch ((Rel)c->op) {
        case R_LT: return a < b; case R_LE: return a <= b; case R_EQ: return a == b;
        case R_NE: return a != b; case R_GT: return a > b; case R_GE: return a >= b;
        }
        return 0;
    }
    case B_NOT: return !eval_b(c->kids[0], E);
    case B_AND: { int a = eval_b(c->kids[0], E), b = eval_b(c->kids[1], E); return a && b; }
    case B_OR:  { int a = eval_b(c->kids[0], E), b = eval_b(c->kids[1], E); return a || b; }
    default: return 0;
    }
}

/* ------------------------------------------- per-phase aggregate table -- */
typedef struct { uint64_t key; uint32_t t0, t1, w0; } Cell;   /* key = index+1, 0 = empty */
typedef struct { Cell *c; size_t cap, used; } Table;

static void tab_init(Table *t) { t->cap = 1024; t->used = 0; t->c = calloc(t->cap, sizeof(Cell)); }
static void tab_free(Table *t) { free(t->c); t->c = NULL; }
static void tab_clear(Table *t) { if (t->used) memset(t->c, 0, t->cap * sizeof(Cell)); t->used = 0; }
static size_t hash64(uint64_t k) { k ^= k >> 33; k *= UINT64_C(0xff51afd7ed558ccd); k ^= k >> 33; return (size_t)k; }

static Cell *tab_get(Table *t, uint64_t index) {
    if (2 * (t->used + 1) > t->cap) {
        Table n; n.cap = t->cap * 2; n.used = 0; n.c = calloc(n.cap, sizeof(Cell));
        for (size_t i = 0; i < t->cap; i++) if (t->c[i].key) {
            size_t h = hash64(t->c[i].key) & (n.cap - 1);
            while (n.c[h].key) h = (h + 1) & (n.cap - 1);
            n.c[h] = t->c[i]; n.used++;
        }
        free(t->c); *t = n;
    }
    uint64_t key = index + 1;
    size_t h = hash64(key) & (t->cap - 1);
    while (t->c[h].key && t->c[h].key != key) h = (h + 1) & (t->cap - 1);
    if (!t->c[h].key) { t->c[h].key = key; t->c[h].t0 = t->c[h].t1 = t->c[h].w0 = NONE32; t->used++; }
    return &t->c[h];
}

/* ----------------------------------------------------------- checker --- */
typedef struct {
    int status, racy;
    uint32_t wk, wj, wi1, wi2;
    uint64_t num_records;
    uint64_t *counts; size_t nphases, capphases;
} Out;

typedef struct { Table tab; Out *out; uint64_t cur_count; int found; } Run;

static void record(Run *R, uint32_t tid, int is_write, uint64_t index) {
    Cell *c = tab_get(&R->tab, index);
    if (tid < c->t0) { if (c->t0 != NONE32) c->t1 = c->t0; c->t0 = tid; }
    else if (tid != c->t0 && tid < c->t1) c->t1 = tid;
    if (is_write && tid < c->w0) c->w0 = tid;
    R->cur_count++;
}

static void close_phase(Run *R) {
    Out *o = R->out;
    if (!R->found) {
        int have = 0; uint64_t best = 0; uint32_t bi = 0, bj = 0;
        for (size_t i = 0; i < R->tab.cap; i++) {
            Cell *c = &R->tab.c[i];
            if (!c->key || c->w0 == NONE32 || c->t1 == NONE32) continue;
            uint64_t idx = c->key - 1;
            if (!have || idx < best) { have = 1; best = idx; bi = c->t0; bj = (c->w0 == c->t0) ? c->t1 : c->w0; }
        }
        if (have) { R->found = 1; o->racy = 1; o->wk = (uint32_t)o->nphases; o->wj = (uint32_t)best; o->wi1 = bi; o->wi2 = bj; }
    }
    if (o->nphases == o->capphases) { o->capphases = o->capphases ? 2 * o->capphases : 64; o->counts = realloc(o->counts, o->capphases * sizeof(uint64_t)); }
    o->counts[o->nphases++] = R->cur_count;
    o->num_records += R->cur_count;
    R->cur_count = 0;
    tab_clear(&R->tab);
}

/* thread-level rules for one thread on an unsynchronized leaf */
static void run_u(const Node *s, Env *E, Run *R) {
    if (E->overflow) return;
    switch (s->kind) {
    case S_SKIP: return;
    case S_RD: case S_WR: {
        uint64_t j = eval_n(s->kids[0], E);
        if (E->overflow) return;
        if (j >= INDEX_LIMIT) { E->overflow = 1; return; }
        record(R, (uint32_t)E->tid, s->kind == S_WR, j);
        return;
    }
    case S_SEQ: for (int i = 0; i < s->nkids && !E->overflow; i++) run_u(s->kids[i], E, R); return;
    case S_IF: { int c = eval_b(s->kids[0], E); if (E->overflow) return; run_u(s->kids[c ? 1 : 2], E, R); return; }
    case S_FORU: {
        uint64_t lo = eval_n(s->kids[0], E), hi = eval_n(s->kids[1], E);
        for (uint64_t v = lo; v < hi && !E->overflow; v++) { E->env[s->slot] = v; run_u(s->kids[2], E, R); }
        return;
    }
    default: return;
    }
}

/* synchronized walk: phase counter, for^S bounds once, leaves for all tids */
static void walk_s(const Node *s, Env *E, Run *R, uint64_t n) {
    if (E->overflow) return;
    if (s->kind == S_SYNC) { close_phase(R); return; }
    if (s->kind == S_SEQ && s->has_s) { for (int i = 0; i < s->nkids && !E->overflow; i++) walk_s(s->kids[i], E, R, n); return; }
    if (s->kind == S_FORS) {
        uint64_t lo = eval_n(s->kids[0], E), hi = eval_n(s->kids[1], E);
        for (uint64_t v = lo; v < hi && !E->overflow; v++) { E->env[s->slot] = v; walk_s(s->kids[2], E, R, n); }
        return;
    }
    for (uint64_t i = 0; i < n && !E->overflow; i++) { E->tid = i; run_u(s, E, R); }
}

static void check_protocol(const char *text, uint64_t n, Out *o) {
    memset(o, 0, sizeof *o);
    o->wk = o->wj = o->wi1 = o->wi2 = NONE32;
    Lexer L = {text, 0, strlen(text), 0};
    Node *root = p_stmt(&L);
    char b[8];
    if (!L.err && next_tok(&L, b, sizeof b)) L.err = 1;
    if (L.err || !root) { o->status = -100; free_node(root); return; }  /* parse error */
    Scope sc = {{0}, 0};
    int st = check(root, &sc, 0);
    if (st) { o->status = st; free_node(root); return; }
    mark_s(root);
    Env *E = calloc(1, sizeof(Env));
    Run R; tab_init(&R.tab); R.out = o; R.cur_count = 0; R.found = 0;
    walk_s(root, E, &R, n);
    if (E->overflow) {
        o->status = E_RANGE; o->racy = 0; o->wk = o->wj = o->wi1 = o->wi2 = NONE32;
        o->num_records = 0; o->nphases = 0;
    } else {
        close_phase(&R);   /* the phase after the last sync */
    }
    tab_free(&R.tab); free(E); free_node(root);
}

/* --------------------------------------------------------------- main -- */
typedef struct { char **texts; uint64_t *ns; Out *outs; double *secs; size_t count; size_t next; pthread_mutex_t mu; } Work;

static double now(void) { struct timespec ts; clock_gettime(CLOCK_MONOTONIC, &ts); return ts.tv_sec + ts.tv_nsec * 1e-9; }

static void *worker(void *arg) {
    Work *w = arg;
    for (;;) {
        pthread_mutex_lock(&w->mu); size_t i = w->next++; pthread_mutex_unlock(&w->mu);
        if (i >= w->count) return NULL;
        double t0 = now();
        check_protocol(w->texts[i], w->ns[i], &w->outs[i]);
        w->secs[i] = now() - t0;
    }
}

int main(int argc, char **argv) {
    int jobs = 1, timing = 0;
    const char *path = NULL;
    for (int i = 1; i < argc; i++) {
        if (!strcmp(argv[i], "-j") && i + 1 < argc) jobs = atoi(argv[++i]);
        else if (!strcmp(argv[i], "-t")) timing = 1;
        else path = argv[i];
    }
    FILE *f = path ? fopen(path, "r") : stdin;
    if (!f) { perror("open"); return 2; }
    Work w; memset(&w, 0, sizeof w); pthread_mutex_init(&w.mu, NULL);
    size_t cap = 0; char *line = NULL; size_t lcap = 0; ssize_t len;
    while ((len = getline(&line, &lcap, f)) > 0) {
        char *p = line; while (*p == ' ') p++;
        if (*p == '\n' || *p == 0) continue;
        char *end; unsigned long long n = strtoull(p, &end, 10);
        if (w.count == cap) { cap = cap ? 2 * cap : 256; w.texts = realloc(w.texts, cap * sizeof(char *)); w.ns = realloc(w.ns, cap * sizeof(uint64_t)); }
        w.texts[w.count] = strdup(end); w.ns[w.count] = n; w.count++;
    }
    free(line);
    if (path) fclose(f);
    w.outs = calloc(w.count ? w.count : 1, sizeof(Out));
    w.secs = calloc(w.count ? w.count : 1, sizeof(double));
    if (jobs < 1) jobs = 1;
    pthread_t *th = calloc(jobs, sizeof(pthread_t));
    for (int i = 0; i < jobs; i++) pthread_create(&th[i], NULL, worker, &w);
    for (int i = 0; i < jobs; i++) pthread_join(th[i], NULL);
    for (size_t i = 0; i < w.count; i++) {
        Out *o = &w.outs[i];
        printf("%d %d %u %u %u %u %llu %zu", o->status, o->racy, o->wk, o->wj, o->wi1, o->wi2,
               (unsigned long long)o->num_records, o->status ? (size_t)0 : o->nphases);
        if (!o->status) for (size_t k = 0; k < o->nphases; k++) printf(" %llu", (unsigned long long)o->counts[k]);
        printf("\n");
        if (timing) fprintf(stderr, "%zu %.6f\n", i, w.secs[i]);
        free(o->counts); free(w.texts[i]);
    }
    free(w.outs); free(w.secs); free(w.texts); free(w.ns); free(th);
    return 0;
}
