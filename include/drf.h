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
 *   ACC   0x02 mode(0 rd, 1 wr; | array << 1) <expr>
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
 *   DRF_E_MULTI      the protocol accesses several arrays (drf_check_arrays)
 *   DRF_E_LIMIT      outside this implementation's limits (more than 16
 *                    loop slots, more than 8 nested for^S, expression stack
 *                    deeper than 16, if/for^U nesting deeper than 30,
 *                    more than 2^40 access events or 2^32 - 1 phases,
 *                    n > 2^31)
 * When status != 0 the other result fields are zero and the witness fields
 * are 0xFFFFFFFF.  Nothing throws or aborts across this ABI.
 *
 * Memory and streams.  Device pointers (prefix d_) are caller-owned device
 * memory; host pointers (h_ or none) are read during the call only (the
 * caller may free them on return).  Device scratch is not caller-owned:
 * each context keeps two scratch pools that grow on demand in stream order
 * (hipMallocAsync on the call's stream), never beyond the limit given at
 * creation (DRF_E_NOMEM when a call cannot fit even after splitting its
 * big phases into waves), are reused across calls and can be handed back
 * with drf_ctx_release.  The sizes come from the per-phase counts that the
 * count pass finds on the device, which a caller cannot know in advance;
 * drf_plan.scratch_bytes gives an upper bound for admission control.  A
 * context is used by one host thread at a time; use one context per thread
 * (and stream) for concurrent checking.
 *
 * Asynchrony.  The checking calls enqueue their work on `stream` (a
 * hipStream_t; NULL = the default stream) and return without waiting for
 * its completion: results and counts are valid after the caller
 * synchronizes `stream`.  The host does wait inside a call where it needs
 * device data to plan further work: once for the per-phase counts of the
 * protocols whose phases the planner cannot prove small (statically small
 * protocols need no wait at all), once per partition level of phases
 * above one tile (the host packs the next tiles from the bucket starts
 * while the scatter runs), and, at the start of a call, for the same
 * context's previous call (its pinned staging is reused).  Part of a
 * call's work may run on a second stream that the context owns (the fused
 * decision of counted small phases, beside the partition of the big ones);
 * the call's stream waits for it before the results are written, so
 * synchronizing `stream` covers it.  `stream` must be
 * a live stream of the context's device (HIP does not validate handles: a
 * stale or made-up one is undefined behaviour, as in HIP itself).
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
#define DRF_E_MULTI (-11)
#define DRF_E_ILLTYPED (-12)

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
    uint64_t scratch_bytes;      /* upper bound on the device scratch a check of this
                                    protocol alone takes (a limit below it splits the
                                    big phases into waves; see drf_ctx_create) */
} drf_plan;                /* 48 bytes */

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
 * Defines: the MAP syntax (Section 2, Fig. "Syntax of MAPs"), with the
 * operators and relations of the index language spelled out above.
 * text/len: the text (need not be NUL terminated).  out/cap: output words.
 * *nwords receives the number of words written (or needed, when cap is too
 * small: then DRF_E_NOMEM).  DRF_E_ARG for text that is not a protocol.
 * Unbound names, shadowing and misplaced sync still compile: they are
 * reported as statuses by the planning and checking calls. Host only. */
int drf_compile_text(const char *text, size_t len, uint32_t *out, uint32_t cap, uint32_t *nwords);

/* Validate and plan one protocol run by num_threads threads (host only).
 * Defines: the well-formedness side conditions of the typing rules
 * (Section 4, Fig. "Behavioral type system": variables in scope for rules
 * t-n / t-b, distinct binders) and the split of a synchronized protocol
 * into barrier-separated phases (Section 2, synchronized protocols).
 * code/words: bytecode.  Writes *out (scratch_bytes for the default
 * tuning); returns DRF_OK unless arguments are invalid (the protocol's own
 * problems go in out->status). */
int drf_plan_protocol(const uint32_t *code, uint32_t words, uint32_t num_threads, drf_plan *out);

/* Plan `count` protocols laid out as for drf_check_batch (host only).
 * plans: count drf_plan (host), each as drf_plan_protocol gives it.
 * *scratch_bytes_total (may be NULL): upper bound on the device scratch
 * one drf_check_batch of all of them takes.  ctx (may be NULL) supplies
 * the tuning the sizes are computed for (the library default when NULL);
 * it is only read.  DRF_E_ARG for missing arrays. */
int drf_plan_batch(const drf_ctx *ctx, const uint32_t *code, const uint64_t *code_off, const uint32_t *nthreads,
                   uint32_t count, drf_plan *plans, uint64_t *scratch_bytes_total);

/* Create a context on HIP device `hip_device`; scratch_limit_bytes bounds
 * the two device scratch pools together (0 = 3/4 of the free device
 * memory).  DRF_E_HIP when the device does not exist or HIP fails. */
int drf_ctx_create(int hip_device, uint64_t scratch_limit_bytes, drf_ctx **out);
/* Waits for the context's work, frees its pools and staging. */
int drf_ctx_destroy(drf_ctx *ctx);
/* Hands the context's scratch pools back to the device's stream-ordered
 * allocator when they hold more than keep_bytes together (pool A is kept
 * when it alone fits).  The memory is released after the context's last
 * call completes, without waiting for it on the host or on other streams;
 * the next call grows the pools again. */
int drf_ctx_release(drf_ctx *ctx, uint64_t keep_bytes);

/* Check one protocol.  Defines: Definition 1 (a phase is racy when two
 * distinct threads access one index in it and one of them writes), applied
 * to every phase of the protocol's synchronized execution (Section 2;
 * threads run independently, rule par of Fig. "Syntax and semantics of
 * BabyCUDA").
 * d_result: one drf_result in device memory.  d_phase_counts: device array
 * of phase_cap u64 (needs plan.num_phases).  stream: hipStream_t (NULL =
 * default stream).  Returns DRF_OK once the work is enqueued (see
 * Asynchrony), DRF_E_ARG for missing pointers or phase_cap too small,
 * DRF_E_NOMEM when the scratch limit cannot hold the call's metadata,
 * DRF_E_HIP for a HIP failure.  After a call-level
 * error nothing has been written to d_result / d_phase_counts (DRF_E_HIP
 * from a failed launch excepted) and the context stays usable. */
int drf_check_protocol(drf_ctx *ctx, const uint32_t *code, uint32_t words, uint32_t num_threads,
                       drf_result *d_result, uint64_t *d_phase_counts, uint64_t phase_cap,
                       void *stream);

/* Check `count` protocols in one launch sequence (same definition as
 * drf_check_protocol, per protocol).  Protocol i's bytecode is
 * code[code_off[i] .. code_off[i+1]) (code_off has count+1 entries), run by
 * nthreads[i] threads.  d_results: count drf_result (device).
 * d_phase_counts: device array of phase_cap u64; protocol i's counts start
 * at the sum of num_phases of protocols 0..i-1 (its plan's num_phases;
 * protocols with status != 0 take none).  A protocol whose single phase
 * cannot fit the scratch limit gets status DRF_E_NOMEM; the others are
 * still checked.  Return codes as for drf_check_protocol. */
int drf_check_batch(drf_ctx *ctx, const uint32_t *code, const uint64_t *code_off,
                    const uint32_t *nthreads, uint32_t count,
                    drf_result *d_results, uint64_t *d_phase_counts, uint64_t phase_cap,
                    void *stream);

/* Allocation-free variant of drf_check_batch, for callers that cannot
 * allocate device memory (code being captured into a HIP graph, tight
 * serving loops, hosts that forbid it).  Same arguments, results, layout
 * and per-protocol statuses as drf_check_batch.  It calls no hipMalloc,
 * hipMallocAsync, hipHostMalloc or hipFree and grows no context pool: its
 * device scratch is a fixed array of DRF_FIXED_SCRATCH_BYTES per device
 * (part of the library's code object, held from load until the process
 * ends; drf_ctx_create looks up its address), and its host staging and
 * read-backs use ordinary host heap memory instead of pinned memory.
 * Limits: the call's metadata (pool A) must fit the array, else the call
 * returns DRF_E_NOMEM and writes nothing; the records of phases above one
 * LDS tile use the rest of it, in waves, and a protocol with a single
 * phase too large for that gets status DRF_E_NOMEM while the others are
 * still checked.  Unlike the other checking calls it returns only after
 * its work on `stream` has completed (its heap staging must outlive the
 * copies).  Every allocation-free call on one device shares that device's
 * array, which keeps the previous call's contents (the call clears what it
 * needs): allocation-free calls that overlap on one device (other threads,
 * other contexts or streams) race and must be serialized by the caller.
 * Calls of the other entry points do not touch the array.  Profiling
 * (drf_ctx_set_profiling) does not cover these calls. */
#define DRF_FIXED_SCRATCH_BYTES (64ull << 20)
int drf_check_batch_noalloc(drf_ctx *ctx, const uint32_t *code, const uint64_t *code_off,
                            const uint32_t *nthreads, uint32_t count, drf_result *d_results,
                            uint64_t *d_phase_counts, uint64_t phase_cap, void *stream);

/* ---------------------------------------------------- parameter sweeps
 * A protocol may mention a free parameter (the racy example of Section 2
 * loops up to a symbolic M, typed under the context {M, tid} in Section 4).
 * The paper reasons about every M symbolically; these calls check the
 * concrete instances p[M := v] for v = first .. first + count - 1 as one
 * batch.  The parameter is a variable slot that no loop binds. */

/* Slot the text compiler gives variable `name` in `text` (names get slots
 * in order of first appearance).  DRF_E_ARG when the text does not compile
 * or never mentions the name.  Host only. */
int drf_text_slot(const char *text, size_t len, const char *name, uint32_t *slot);

/* Bytecode of the protocol with every occurrence of variable `slot`
 * replaced by the constant `value` (out/cap/nwords as drf_compile_text).
 * DRF_E_ARG when a loop binds the slot; the bytecode's own problems as
 * DRF_E_BYTECODE.  Host only. */
int drf_bind_param(const uint32_t *code, uint32_t words, uint32_t slot, uint64_t value, uint32_t *out,
                   uint32_t cap, uint32_t *nwords);

/* Plans of the count instances (as drf_plan_batch); instance i's phase
 * counts start at the sum of num_phases of instances 0..i-1. */
int drf_plan_sweep(const uint32_t *code, uint32_t words, uint32_t num_threads, uint32_t slot, uint64_t first,
                   uint32_t count, drf_plan *plans, uint64_t *scratch_bytes_total);

/* Check the count instances in one launch sequence: d_results[i] is the
 * result of p[slot := first + i] (layout and return codes as
 * drf_check_batch). */
int drf_check_sweep(drf_ctx *ctx, const uint32_t *code, uint32_t words, uint32_t num_threads, uint32_t slot,
                    uint64_t first, uint32_t count, drf_result *d_results, uint64_t *d_phase_counts,
                    uint64_t phase_cap, void *stream);

/* ------------------------------------------------ several shared arrays
 * The analysis gives one behavioural type per shared array (Section 3,
 * Syntax): accesses to different arrays never race.  In the bytecode the
 * ACC mode word carries the array in its upper bits (write | array << 1;
 * text form rd:A / wr:A, arrays numbered in order of first appearance, the
 * plain rd / wr counting as one of them).  The planning and checking calls
 * above give such a protocol the status DRF_E_MULTI; these calls check one
 * protocol per array. */

/* Number of arrays the protocol accesses (1 + the largest array id; 1 for
 * a protocol without accesses).  Host only. */
int drf_protocol_arrays(const uint32_t *code, uint32_t words, uint32_t *num_arrays);

/* Plans of every array's protocol (cap: entries of plans; DRF_E_ARG when
 * the protocol has more arrays). */
int drf_plan_arrays(const uint32_t *code, uint32_t words, uint32_t num_threads, drf_plan *plans, uint32_t cap,
                    uint64_t *scratch_bytes_total);

/* Check every array's protocol (the protocol with the other arrays'
 * accesses replaced by skip) in one launch sequence: d_results[a] and the
 * phase counts of array a (num_phases u64 each, array after array) as
 * drf_check_batch lays them out.  Defined by Definition 1 per array. */
int drf_check_arrays(drf_ctx *ctx, const uint32_t *code, uint32_t words, uint32_t num_threads,
                     drf_result *d_results, uint64_t *d_phase_counts, uint64_t phase_cap, void *stream);

/* ------------------------------------------------- BabyCUDA front end
 * Infers the memory access protocol of a BabyCUDA program (Section 3, Fig.
 * "Syntax and semantics of BabyCUDA") with the behavioural type system of
 * Section 4 (Fig. "Behavioral type system": V |- b |> u, rules t-n, t-b,
 * t-write, t-read, t-seq, t-if, t-for, t-skip), V = {tid} plus `params`
 * (space-separated parameter names, e.g. "M"; NULL for none).  By Theorem 1
 * a well-typed program is DRF exactly when its protocol is, so the
 * protocol can be checked in its place.  Text form of programs:
 *   (skip) (sync) (wr n n') (rd y n b) (seq b ...) (if c b b) (for x n n b)
 * with wr:A / rd:A for several arrays; the protocol comes out in the text
 * form of drf_compile_text (loops holding a sync become for^S).
 * Returns DRF_E_ARG when the text is not a BabyCUDA program, else DRF_OK
 * with *status 0 (out holds the NUL-terminated protocol; *needed its size
 * with the NUL; DRF_E_NOMEM when cap is smaller) or a typing status:
 *   DRF_E_ILLTYPED  a variable bound by a read reaches an index, guard or
 *                   loop bound (data-dependent access, the ill-typed
 *                   example of Section 4)
 *   DRF_E_UNBOUND   a variable no binder or parameter introduces
 *   DRF_E_SHADOW    a binder that is not fresh (nested binders distinct)
 * Host only. */
int drf_babycuda_infer(const char *text, size_t len, const char *params, char *out, size_t cap, size_t *needed,
                       int32_t *status);

/* Per-kernel timing of a context (for measurement).  When enabled, every
 * kernel launch is bracketed by HIP events recorded on the stream it runs on
 * (the call's, or the context's second stream);
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
/* Waits on the host for the context's last call, then copies up to cap
 * entries into out, sets *n to the number of classes and resets the totals
 * when reset != 0. */
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

/* Shape-class graph: one hipGraph captured over fixed device buffers for
 * batches up to the capacities below whose protocols are all statically
 * small (the planner proves every phase fits one LDS tile, so the check is
 * device work only: fills, the fused launches, witness picks, results; see
 * drf_plan.max_phase_records and drf_ctx_get_tuning's tile_events), and
 * replayed for each new batch of the class.  Same definition and results
 * as drf_check_batch (Definition 1 per protocol).  The graph is created on
 * ctx's device with ctx's tuning and owns its buffers (hipMalloc and pinned
 * staging at creation; none per check). */
typedef struct {
    uint32_t max_protocols;   /* protocols of one batch */
    uint32_t max_nests;       /* unsynchronized leaves times host-unrolled iterations, whole batch */
    uint32_t max_code_words;  /* compiled leaf code of the whole batch */
    uint32_t max_fixed;       /* host-unrolled loop values of the whole batch */
    uint64_t max_phases;      /* phases of the whole batch */
    uint32_t max_units;       /* fused work units of each evaluator width (at most 2^20) */
    uint32_t reserved;
} drf_graph_caps;             /* 32 bytes */
typedef struct drf_graph drf_graph;

/* DRF_E_ARG for zero or out-of-range capacities, DRF_E_NOMEM, DRF_E_HIP.
 * stream is unused (reserved). */
int drf_graph_create(drf_ctx *ctx, const drf_graph_caps *caps, void *stream, drf_graph **out);
/* Check a batch of the class (arguments, layout and results as
 * drf_check_batch): plans it on the host, uploads it, replays the graph on
 * `stream` and copies results and phase counts into the caller's buffers;
 * returns once that is enqueued (the host waits only for the previous
 * check's upload).  DRF_E_LIMIT, with nothing written, when the batch is
 * outside the class (a protocol not statically small, or a capacity
 * exceeded): use drf_check_batch for it.  Checks of one graph must not
 * overlap (one host thread, one stream at a time). */
int drf_graph_check(drf_graph *g, const uint32_t *code, const uint64_t *code_off, const uint32_t *nthreads,
                    uint32_t count, drf_result *d_results, uint64_t *d_phase_counts, uint64_t phase_cap,
                    void *stream);
int drf_graph_destroy(drf_graph *g);

/* Tuning of a context (what the autotuner sets).  tile_events: most access
 * events of one phase (or bucket) sorted in one LDS tile, a power of two in
 * [256, 8192]; digit_bits: the most index bits of one MSD partition level,
 * 4..10 (a level takes fewer for a short segment);
 * unit_events / item_events: target events per fused unit / per count and
 * emit work item; table_bits: phases above one tile whose protocol indexes
 * at most 2^table_bits cells (1..24) and that hold at least as many events
 * as cells are decided by a table of the cells in device memory instead of
 * emitting records and partitioning them (the sort-free conflict table of
 * Definition 1: per cell the least tid, the second least and the least
 * writer); DRF_TABLE_OFF turns this off (the default).  Zero fields keep
 * their value; DRF_E_ARG when out of range (nothing changes then). */
#define DRF_TABLE_OFF 255u
typedef struct {
    uint32_t tile_events;
    uint32_t digit_bits;
    uint32_t unit_events;
    uint32_t item_events;
    uint32_t table_bits;   /* 0 in drf_ctx_get_tuning: off */
} drf_tuning;

int drf_ctx_set_tuning(drf_ctx *ctx, const drf_tuning *t);
int drf_ctx_get_tuning(drf_ctx *ctx, drf_tuning *t);

/* Library version string. */
const char *drf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DRF_H */
