/*
 * drf.h -- C ABI of libdrf: data-race-freedom checking of memory access
 * protocols (MAPs) on an AMD Instinct MI355X (gfx950).
 *
 * What is decided.  A protocol (the MAP syntax of Liew, Cogumbreiro and
 * Lange, "Provable GPU Data-Races in Static Race Detection", Fig. "Syntax of
 * MAPs": accesses rd[n] / wr[n] at index expressions over tid and loop
 * variables, skip, sequencing, if, for^U, sync and for^S) is run by the
 * threads T = {0..n-1}.  Every thread evaluates it independently (rule par
 * of Fig. "Syntax and semantics of BabyCUDA"); sync is a barrier for all of
 * T that closes the current phase.  A phase is racy when some index is
 * written by one thread and read or written by another thread in that phase
 * (Definition 1); the protocol is data-race free (DRF) when no phase is.
 *
 * Results (all exact integers):
 *   racy          0 or 1
 *   witness       the lexicographically least (phase, index, tid_i, tid_j)
 *                 with tid_i < tid_j, both threads accessing index in that
 *                 phase and at least one of them writing it; phases are
 *                 numbered from 0 in execution order
 *   phase counts  number of executed access events per phase
 *                 (num_phases = syncs executed + 1; empty phases count 0)
 *   num_records   sum of the phase counts
 *
 * Conventions of the protocol language (points the paper leaves open):
 *   arithmetic is on naturals: a - b = 0 when b > a, a / 0 = 0, a mod 0 = a,
 *   a << b = a * 2^b, a >> b = floor(a / 2^b); both operands of and / or are
 *   evaluated; loops run over the half-open range lo..hi with stride 1,
 *   bounds evaluated once at loop entry; for^S bounds may not mention tid.
 *   Any evaluated value >= 2^63 or accessed index >= 2^32 makes the status
 *   DRF_E_RANGE.
 *
 * Bytecode (input of every checking call).  A little-endian stream of u32
 * words, statements in prefix order:
 *   header      'MAP1' (0x3150414D), version (1), num_slots, code_words
 *   SKIP  0x01
 *   ACC   0x02 mode(0 rd, 1 wr) <expr>
 *   SEQ   0x03 count <stmt>*count
 *   IF    0x04 <cond> <stmt then> <stmt else>
 *   FORU  0x05 slot <expr lo> <expr hi> <stmt body>
 *   SYNC  0x06
 *   FORS  0x07 slot <expr lo> <expr hi> <stmt body>
 * An <expr> / <cond> is a word count followed by that many words of
 * postfix code:
 *   0x20 CONST32 v | 0x21 CONST64 lo hi | 0x22 TID | 0x23 VAR slot
 *   0x30 ADD 0x31 MONUS 0x32 MUL 0x33 DIV 0x34 MOD 0x35 SHL 0x36 SHR
 *   0x37 MIN 0x38 MAX
 *   0x40 TRUE 0x41 FALSE 0x42 LT 0x43 LE 0x44 EQ 0x45 NE 0x46 GT 0x47 GE
 *   0x48 AND 0x49 OR 0x4A NOT
 * Loop variables are slots 0..num_slots-1; slot 0xFFFFFFFF names tid (so a
 * loop binding it is rejected).  drf_compile_text produces this bytecode
 * from the s-expression text form.
 *
 * Errors.  Every function returns DRF_OK or a negative call-level code
 * (DRF_E_ARG, DRF_E_NOMEM, DRF_E_HIP).  Problems of one protocol go in its
 * status field instead, so a batch continues past a bad protocol:
 *   DRF_E_BYTECODE   malformed bytecode
 *   DRF_E_UNBOUND    an index, guard or bound mentions a variable that no
 *                    enclosing loop binds (typing rules t-n / t-b)
 *   DRF_E_SHADOW     a loop rebinds tid or a variable of an enclosing loop
 *                    (nested binders are distinct)
 *   DRF_E_SYNC_IN_U  sync or for^S under if or for^U
 *   DRF_E_DIVERGENT  for^S bounds mention tid
 *   DRF_E_RANGE      an evaluated value >= 2^63 or index >= 2^32
 *   DRF_E_LIMIT      outside this implementation's limits (more than 16
 *                    loop slots, more than 8 nested for^S, expression stack
 *                    deeper than 16, if/for^U nesting deeper than 30,
 *                    more than 2^40 access events or 2^32 - 1 phases,
 *                    n > 2^31)
 * When status != 0 the other result fields are zero and the witness fields
 * are 0xFFFFFFFF.  Nothing throws or aborts across this ABI.
 *
 * Memory and streams.  Device pointers (prefix d_) are caller-owned device
 * memory; host pointers (h_ or none) are read during the call only.  The
 * context owns a device scratch pool that grows on demand up to the limit
 * given at creation and is reused across calls; it never holds caller
 * memory.  A context is used by one host thread at a time; use one context
 * per thread (and stream) for concurrent checking.  The checking calls
 * enqueue work on `stream` (a hipStream_t) and return once the work is
 * enqueued; they wait on the stream internally once, after counting, to
 * size the rest.  Results are valid after the caller synchronizes `stream`.
 */
#ifndef DRF_H
#define DRF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DRF_OK 0
#define DRF_E_ARG (-1)
#define DRF_E_BYTECODE (-2)
#define DRF_E_UNBOUND (-3)
#define DRF_E_SHADOW (-4)
#define DRF_E_SYNC_IN_U (-5)
#define DRF_E_DIVERGENT (-6)
#define DRF_E_RANGE (-7)
#define DRF_E_NOMEM (-8)
#define DRF_E_HIP (-9)
#define DRF_E_LIMIT (-10)

#define DRF_MAGIC 0x3150414Du
#define DRF_TID_SLOT 0xFFFFFFFFu
#define DRF_NONE 0xFFFFFFFFu

typedef struct drf_ctx drf_ctx;

/* Static plan of one protocol (host only, no device work). */
typedef struct {
    int32_t status;        /* 0 or a per-protocol status code */
    uint32_t num_phases;   /* syncs executed + 1 (0 when status != 0) */
    uint32_t index_bits;   /* bits of the largest index the protocol can reach */
    uint32_t wide;         /* 1 when values may reach 2^32 (64-bit evaluator) */
    uint64_t max_records;  /* upper bound on executed access events */
    uint64_t nests;        /* unsynchronized leaves times host-unrolled iterations */
    uint64_t max_phase_records;  /* upper bound on the events of any one phase */
} drf_plan;                /* 40 bytes */

/* Result of one protocol. */
typedef struct {
    int32_t status;
    uint32_t racy;
    uint32_t phase, index, tid_i, tid_j;   /* witness, DRF_NONE when DRF */
    uint64_t num_records;
    uint32_t num_phases;
    uint32_t reserved;
} drf_result;              /* 40 bytes */

/* Compile the s-expression text form of one protocol into bytecode.
 * text/len: the text (need not be NUL terminated).  out/cap: output words.
 * *nwords receives the number of words written (or needed, when cap is too
 * small: then DRF_E_NOMEM).  DRF_E_ARG for text that is not a protocol.
 * Unbound names, shadowing and misplaced sync still compile: they are
 * reported as statuses by the planning and checking calls. Host only. */
int drf_compile_text(const char *text, size_t len, uint32_t *out, uint32_t cap, uint32_t *nwords);

/* Validate and plan one protocol run by num_threads threads (host only).
 * code/words: bytecode.  Writes *out; returns DRF_OK unless arguments are
 * invalid (the protocol's own problems go in out->status). */
int drf_plan_protocol(const uint32_t *code, uint32_t words, uint32_t num_threads, drf_plan *out);

/* Create a context on HIP device `hip_device`; scratch_limit_bytes bounds
 * the device scratch pool (0 = 3/4 of the free device memory). */
int drf_ctx_create(int hip_device, uint64_t scratch_limit_bytes, drf_ctx **out);
int drf_ctx_destroy(drf_ctx *ctx);

/* Check one protocol.  d_result: one drf_result in device memory.
 * d_phase_counts: device array of phase_cap u64 (needs plan.num_phases).
 * stream: hipStream_t (NULL = default stream). */
int drf_check_protocol(drf_ctx *ctx, const uint32_t *code, uint32_t words, uint32_t num_threads,
                       drf_result *d_result, uint64_t *d_phase_counts, uint64_t phase_cap,
                       void *stream);

/* Check `count` protocols in one launch sequence.  Protocol i's bytecode is
 * code[code_off[i] .. code_off[i+1]) (code_off has count+1 entries), run by
 * nthreads[i] threads.  d_results: count drf_result (device).
 * d_phase_counts: device array of phase_cap u64; protocol i's counts start
 * at the sum of num_phases of protocols 0..i-1 (its plan's num_phases;
 * protocols with status != 0 take none). */
int drf_check_batch(drf_ctx *ctx, const uint32_t *code, const uint64_t *code_off,
                    const uint32_t *nthreads, uint32_t count,
                    drf_result *d_results, uint64_t *d_phase_counts, uint64_t phase_cap,
                    void *stream);

/* Per-kernel timing of a context (for measurement).  When enabled, every
 * kernel launch is bracketed by HIP events recorded on the call's stream;
 * elapsed times are added up per kernel class once the call's work is
 * complete.  `records` counts the access events the class processed and
 * `bytes` its algorithmic HBM traffic (records written or read once at
 * 8 bytes each; 0 for classes that keep records in LDS).  Classes:
 * count, fused, emit, hist, scan, scatter, tile, single, other. */
typedef struct {
    char name[16];
    uint64_t launches;
    double ms;
    uint64_t records;
    uint64_t bytes;
} drf_kernel_stat;         /* 48 bytes */

int drf_ctx_set_profiling(drf_ctx *ctx, int on);
/* Copies up to cap entries into out, sets *n to the number of classes and
 * resets the totals when reset != 0. */
int drf_ctx_kernel_stats(drf_ctx *ctx, drf_kernel_stat *out, uint32_t cap, uint32_t *n, int reset);

/* Prepared batch: checks the batch once (like drf_check_batch, with the
 * same outputs in the same caller buffers) while recording every device
 * operation, then captures that sequence into one hipGraph.  Each
 * drf_run_prepared replays the whole device work of the check (count,
 * fused, emit, partition, tiles, witness, results) as one graph launch on
 * `stream` and rewrites the same outputs; the host plan and partition lists
 * of the first run are reused.  The prepared batch owns its scratch memory
 * (not the context's pools) and keeps d_results / d_phase_counts pointers:
 * they must stay valid until drf_prepared_destroy.  Replays of one prepared
 * batch must not overlap (run them on one stream). */
typedef struct drf_prepared drf_prepared;

int drf_prepare_batch(drf_ctx *ctx, const uint32_t *code, const uint64_t *code_off, const uint32_t *nthreads,
                      uint32_t count, drf_result *d_results, uint64_t *d_phase_counts, uint64_t phase_cap,
                      void *stream, drf_prepared **out);
int drf_run_prepared(drf_prepared *p, void *stream);
int drf_prepared_destroy(drf_prepared *p);
/* Number of device operations in the prepared graph. */
uint64_t drf_prepared_launches(const drf_prepared *p);

/* Tuning of a context (what the autotuner sets).  tile_events: most access
 * events of one phase (or bucket) sorted in one LDS tile, a power of two in
 * [256, 8192]; digit_bits: the most index bits of one MSD partition level,
 * 4..10 (a level takes fewer for a short segment);
 * unit_events / item_events: target events per fused unit / per count and
 * emit work item.  Zero fields keep their value; DRF_E_ARG when out of
 * range (nothing changes then). */
typedef struct {
    uint32_t tile_events;
    uint32_t digit_bits;
    uint32_t unit_events;
    uint32_t item_events;
} drf_tuning;

int drf_ctx_set_tuning(drf_ctx *ctx, const drf_tuning *t);
int drf_ctx_get_tuning(drf_ctx *ctx, drf_tuning *t);

/* Library version string. */
const char *drf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DRF_H */
