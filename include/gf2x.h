/*
 * gf2x.h -- C ABI of the MI355X (gfx950) library for products of dense
 * binary polynomials in F2[X] and in the ring F2[X]/(X^n - 1).
 *
 * Operation (Robert & Veron, "Faster Multiplication over F2[X] using AVX512
 * instruction set and VPCLMULQDQ instruction"):
 *   - Section 2.1: two binary polynomials of degree at most n-1, each packed
 *     into ceil(n/64) 64-bit words, are multiplied; the product has degree at
 *     most 2n-2.
 *   - Section 1 (circulant matrices and the ring F2[X]/(X^N - 1)): the
 *     code-based KEMs need that product reduced modulo X^n - 1, i.e. bit k+n
 *     of the full product is added to bit k.
 *   - Appendix A (Karatsuba 2-, 3- and 5-way splits), Section 3 with
 *     Appendix D (word-aligned Toom-Cook 3 with evaluation points 0, 1, x,
 *     x+1, infinity and exact divisions by x and x+1) and the Toom-Cook 4
 *     and 5 splits of Section 3 (7 and 9 products) are the recursions the GPU kernels
 *     implement; a measured per-size table picks among them, and the result
 *     does not depend on the choice.
 *   - Section 1 (sparse-dense products of HQC and BIKE): a dense operand
 *     times a sparse one given by its positions (GF2X_SPARSE_KIND below).
 *
 * Layout.  A polynomial of n coefficients occupies W(n) = ceil(n/64)
 * uint64 words, little-endian: coefficient i is bit (i mod 64) of word
 * floor(i/64).  Input bits at positions >= n are ignored (masked on load).
 * Output bits beyond the result's degree bound are written as zero: bits >= n
 * for ring products, bits >= 2n-1 for full products.
 *
 * Pointers.  Every operand and result pointer is a DEVICE pointer (memory
 * from hipMalloc or equivalent on the context's device), 8-byte aligned.
 * Items and options passed by pointer are HOST memory unless a flag says
 * otherwise.  The caller owns every buffer and keeps it alive until the
 * stream has passed the call.
 *
 * Streams and synchronisation.  Calls enqueue work on the given HIP stream
 * (NULL = the default stream) and return; they do not wait for the device,
 * except where a call says so (the tuner, plan creation and destruction,
 * gf2x_device_item_errors, the server's drain, and the growth of a
 * workspace, which waits for its previous user).  One context may be used
 * from one host thread at a time.
 *
 * Constant time.  Control flow, loop bounds and every memory address inside
 * the kernels depend only on n (public) and, for dense x sparse items, on the
 * weight w (public); never on operand bits or sparse positions.
 *
 * Errors.  Every entry point returns 0 on success or a negative GF2X_E* code;
 * no exception crosses the ABI.  On error nothing has been enqueued.
 */
#ifndef GF2X_H
#define GF2X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

struct ihipStream_t;                       /* hipStream_t is a pointer to this */
typedef struct ihipStream_t *gf2x_stream_t;

#define GF2X_OK 0
#define GF2X_EINVAL (-1)  /* bad argument: null pointer, n out of range, misaligned or overlapping buffers */
#define GF2X_ENOMEM (-2)  /* a device workspace could not be allocated                                     */
#define GF2X_EDEVICE (-3) /* a HIP runtime call failed; gf2x_last_device_error() names it                   */
#define GF2X_EAGAIN (-4)  /* serving: the host queue is full, submit again later (backpressure)            */
#define GF2X_ENOTSUP (-5) /* the request is valid but this build cannot serve it (see gf2x_mul_batched)    */

/* Largest supported n, in bits (the paper's largest operand size, Table perfKaratRec). */
#define GF2X_MAX_BITS 131072u

/* Item kinds for gf2x_mul_batched. */
#define GF2X_KIND_CYCLIC 0u /* c: W(n) words, c = a*b mod (X^n - 1) */
#define GF2X_KIND_FULL 1u   /* c: 2*W(n) words, c = a*b in F2[X]    */
/* Dense x sparse ring product (Section 1: the sparse-dense products of the
 * code-based KEMs), constant time in the positions: c (W(n) words) =
 * a * (X^p_1 + ... + X^p_w) mod (X^n - 1), where the w positions are uint32
 * values at b_base + b_off (read as uint32 words from that uint64 offset),
 * each taken modulo n (equal positions cancel, as in F2).  The weight w is
 * public and is carried in the kind: GF2X_SPARSE_KIND(w), 0 <= w < 2^24.
 * n <= GF2X_SPARSE_MAX_BITS.  Host items only (device-resident descriptors
 * of this kind are skipped). */
#define GF2X_KIND_SPARSE 2u
#define GF2X_SPARSE_KIND(w) (GF2X_KIND_SPARSE | ((uint32_t)(w) << 8))
#define GF2X_SPARSE_MAX_BITS 65504u

/* Flags for gf2x_mul_batched. */
#define GF2X_ITEMS_ON_DEVICE 0x1u  /* `items` is a device pointer (not validated on the host; see below)     */
#define GF2X_SHARED_A 0x2u         /* every item has the same a_off and n (one operand shared by the batch) */
#define GF2X_FORCE_PACKED 0x4u     /* use the bit-packed Karatsuba/Toom path even when GF2X_SHARED_A is set */
#define GF2X_FORCE_TOEPLITZ 0x8u   /* with GF2X_SHARED_A: use the Toeplitz int8-MFMA path                   */
#define GF2X_USE_GRAPH 0x10u       /* replay a cached HIP graph of the launch (host items only)             */
#define GF2X_FUSED 0x20u           /* one persistent launch, each item in its one-workgroup class (below)   */

typedef struct gf2x_ctx gf2x_ctx;

typedef struct gf2x_opts {
    int device;              /* HIP device ordinal the context's work runs on                         */
    size_t hbm_budget_bytes; /* cap on the context's own device workspace (0 = 1 GiB)                 */
    const char *tune_cache;  /* path of the schedule table written by the tuner, or NULL for defaults */
    uint32_t flags;          /* reserved, must be 0                                                   */
} gf2x_opts;

/* One product of a batch.  Offsets count uint64 words from the base pointers
 * given to gf2x_mul_batched; operands hold W(n_bits) words. */
typedef struct gf2x_item {
    uint32_t n_bits; /* 1 <= n_bits <= GF2X_MAX_BITS */
    uint32_t kind;   /* GF2X_KIND_CYCLIC, GF2X_KIND_FULL or GF2X_SPARSE_KIND(w) */
    uint64_t a_off, b_off, c_off;
} gf2x_item;

/* Create a context on opts->device (opts may be NULL: device 0, defaults).
 * *out receives the context.  Errors: GF2X_EINVAL, GF2X_EDEVICE. */
int gf2x_create(gf2x_ctx **out, const gf2x_opts *opts);

/* Release a context and its device workspace.  The caller must make sure no
 * enqueued work still uses it.  NULL is accepted. */
void gf2x_destroy(gf2x_ctx *ctx);

/* Full product c = a*b in F2[X] (Section 2.1).
 * a, b: W(n) words each; c: 2*W(n) words (bits >= 2n-1 written zero).
 * c must not overlap a or b.  Errors: GF2X_EINVAL, GF2X_EDEVICE, GF2X_ENOMEM.
 * The product runs in the class with the lowest measured single-product
 * latency for its size: one workgroup, or a staged class spread over several
 * workgroups (then the context's workspace is used, ordered by its event, and
 * the first call for a given (n, kind) writes a small descriptor to the device
 * synchronously).  On a stream under capture it is always one launch. */
int gf2x_mul(gf2x_ctx *ctx, uint64_t *c, const uint64_t *a, const uint64_t *b,
             uint32_t n_bits, gf2x_stream_t stream);

/* Ring product c = a*b mod (X^n - 1) (Section 1).  a, b, c: W(n) words each;
 * bits >= n of c written zero.  c must not overlap a or b.  Scheduled as
 * gf2x_mul.  Errors: GF2X_EINVAL, GF2X_EDEVICE, GF2X_ENOMEM. */
int gf2x_mul_cyclic(gf2x_ctx *ctx, uint64_t *c, const uint64_t *a, const uint64_t *b,
                    uint32_t n_bits, gf2x_stream_t stream);

/* `count` independent products (persistent kernels).  Item i reads
 * a_base + items[i].a_off and b_base + items[i].b_off and writes
 * c_base + items[i].c_off (sizes per its kind).  Items may mix sizes and
 * kinds.  With host items (default) the library validates n and kind, sorts
 * the work by decreasing n and copies the descriptors to its workspace;
 * with GF2X_ITEMS_ON_DEVICE the descriptors are used as given and must be
 * valid.  Output ranges of different items must not overlap each other or
 * any operand range (operand ranges may be shared); with host items the
 * library checks this and returns GF2X_EINVAL.
 * GF2X_SHARED_A (all items share a_off, n and kind == CYCLIC) lets the
 * library pick the Toeplitz MFMA path for that batch; the FORCE flags pin
 * the choice.  GF2X_USE_GRAPH captures the launch sequence in a HIP graph the
 * first time a given (items, count, bases, flags, stream) is seen and
 * replays it afterwards.  A replay reads the host descriptors once to notice
 * an edited array (then the batch is recorded again); the context keeps at
 * most 64 such graphs and releases the least recently used one first.  Each
 * graph holds its own descriptors and staged workspace within the budget.
 * gf2x_plan_create records a batch without the per-call check.
 * GF2X_FUSED runs the whole batch as one persistent launch: every workgroup
 * takes the next item from a device work queue (most expensive first) and
 * computes it in the size's fastest one-workgroup class.  Only sizes whose
 * one-workgroup class is one of the classes the schedule table gives the six
 * ring sizes 12323 ... 57637 are accepted (else GF2X_ENOTSUP), ring and full
 * kinds; not with GF2X_ITEMS_ON_DEVICE or GF2X_SHARED_A.  Without the flag, a
 * batch of several size classes runs one launch (or, for a size that spreads
 * its top Karatsuba/Toom level over workgroups, four) per class, the classes
 * on up to four internal streams.
 * count == 0 is a no-op.
 * A stream under capture is refused with GF2X_ENOTSUP: the call orders the
 * context's workspace with the context's event and writes descriptors to
 * context-owned buffers, which a graph recorded from it could not replay
 * safely.  GF2X_USE_GRAPH records and replays a graph that owns its own
 * descriptors and workspace.
 * Errors: GF2X_EINVAL, GF2X_ENOMEM, GF2X_EDEVICE, GF2X_ENOTSUP (FORCE_TOEPLITZ
 * without SHARED_A, device items with GF2X_USE_GRAPH, or a capturing stream). */
int gf2x_mul_batched(gf2x_ctx *ctx, const gf2x_item *items, uint32_t count,
                     uint64_t *c_base, const uint64_t *a_base, const uint64_t *b_base,
                     uint32_t flags, gf2x_stream_t stream);

/* For callers that cannot allocate device memory (tight serving loops, code
 * that must not call hipMalloc): gf2x_mul_batched with host items, without
 * any allocation.  The descriptors and the staged workspace of the call live
 * in a static device array of GF2X_NOALLOC_SCRATCH_BYTES per device (held
 * until the process ends): descriptors of at most GF2X_NOALLOC_MAX_ITEMS
 * items (2.5 MiB), the rest of the array as workspace; a size class whose staged workspace does not fit runs its
 * one-workgroup form (same result).  Items, operands and results are those
 * of gf2x_mul_batched without flags (ring and full kinds, mixed sizes); the
 * class groups run one after another on `stream`, and the descriptors are
 * copied from `items` during the call.  Every call on a device shares
 * that device's array and overwrites it: calls that overlap on one device
 * (different streams, or other host threads) race; calls ordered on one
 * stream are safe.  A stream under capture is refused (GF2X_ENOTSUP).
 * Errors: GF2X_EINVAL, GF2X_ENOMEM (count above GF2X_NOALLOC_MAX_ITEMS),
 * GF2X_EDEVICE, GF2X_ENOTSUP. */
#define GF2X_NOALLOC_SCRATCH_BYTES (32u << 20)
#define GF2X_NOALLOC_MAX_ITEMS 65536u
int gf2x_mul_batched_noalloc(gf2x_ctx *ctx, const gf2x_item *items, uint32_t count, uint64_t *c_base,
                             const uint64_t *a_base, const uint64_t *b_base, gf2x_stream_t stream);

/* ------------------------------------------------------------------ plans
 * A batch recorded once and replayed many times with constant host work.
 * gf2x_plan_create validates the host items (as gf2x_mul_batched does), groups
 * them by size class, copies the descriptors to device memory owned by the
 * plan (synchronously), allocates the plan's staged workspace, and records the
 * launch sequence (the same kernels as gf2x_mul_batched) in a HIP graph.  Its
 * device memory counts against the context's budget until the plan is
 * destroyed.  The items array may be freed or reused after the call; the
 * base pointers are baked into the plan and must stay valid while it is used.
 * flags: 0 or GF2X_FUSED (as in gf2x_mul_batched).  count == 0 gives a plan
 * that launches nothing.
 * Errors: GF2X_EINVAL, GF2X_ENOMEM, GF2X_EDEVICE. */
typedef struct gf2x_plan gf2x_plan;
int gf2x_plan_create(gf2x_plan **out, gf2x_ctx *ctx, const gf2x_item *items, uint32_t count, uint64_t *c_base,
                     const uint64_t *a_base, const uint64_t *b_base, uint32_t flags);

/* Enqueue one replay of the plan on `stream`, with host work independent of
 * the number of items: for a batch of one size class its kernels are
 * launched directly (one, or four for a class whose top level is spread over
 * workgroups), otherwise the graph is launched; then one event record.
 * Replays on different streams must not overlap (they share the plan's
 * workspace).
 * Errors: GF2X_EINVAL, GF2X_EDEVICE. */
int gf2x_plan_launch(gf2x_plan *plan, gf2x_stream_t stream);

/* Wait for the plan's last replay, then free it and return its device memory
 * to the context's budget.  NULL is accepted.  The context must outlive it. */
void gf2x_plan_destroy(gf2x_plan *plan);

/* Device-resident descriptors (GF2X_ITEMS_ON_DEVICE) are not validated on the
 * host; one with n == 0, n > GF2X_MAX_BITS or a kind other than
 * GF2X_KIND_CYCLIC / GF2X_KIND_FULL is skipped (its output is not written)
 * and counted on the device.  This call waits for the context's device to
 * finish its work, returns the number of descriptors skipped since the last
 * call, and clears the count.  Errors: GF2X_EINVAL, GF2X_EDEVICE. */
int gf2x_device_item_errors(gf2x_ctx *ctx, uint64_t *count);

/* Schedule the library uses for n: the padded operand size in 32-bit words,
 * the number of 32x32-bit word products computed by the base case, the
 * algorithmic VALU lane-op count of one product (per-schedule cost model:
 * base-case bit operations plus one op per word of every XOR pass), and the
 * schedule's name.  ctx may be NULL (then the built-in default table is used;
 * no device is touched).  Any output pointer may be NULL.  Host only.
 * Errors: GF2X_EINVAL. */
int gf2x_schedule_info(gf2x_ctx *ctx, uint32_t n_bits, uint32_t *padded_words32,
                       uint64_t *base_products, uint64_t *lane_ops, char *name, size_t name_len);

/* Inverses in F2[X]/(X^n - 1) for the BIKE rings: c_i = a_i^(2^(n-1) - 2) for
 * the `count` items (all with the same n_bits = n and kind GF2X_KIND_CYCLIC;
 * b_off is ignored).  n must be an odd prime (as the BIKE block lengths
 * 12323, 24659 and 40973 are; there 2 is moreover primitive modulo n, so the
 * units are exactly the elements of odd weight).  X^n - 1 is then X + 1 times
 * irreducibles of degree ord_n(2), which divides n - 1, so c_i is the inverse
 * of a_i whenever a_i is invertible (for other a_i, c_i is that power, not an
 * inverse; nothing is checked, since checking would depend on the operand).
 * The sequence of operations depends only on n and count: about log2(n)
 * batched products (the same kernels as gf2x_mul_batched) and as many
 * repeated squarings, each a public bit permutation.  c_base + c_off[i] may
 * overlap a_base + a_off[i].  Uses a context workspace of about 4 * count *
 * W(n) words (within the budget), ordered by the context's event; for that
 * reason a stream under capture is refused (GF2X_ENOTSUP), as in
 * gf2x_mul_batched.
 * Errors: GF2X_EINVAL (arguments, or n not an odd prime), GF2X_ENOMEM,
 * GF2X_EDEVICE, GF2X_ENOTSUP. */
int gf2x_inv_cyclic_batched(gf2x_ctx *ctx, const gf2x_item *items, uint32_t count, uint64_t *c_base,
                            const uint64_t *a_base, uint32_t flags, gf2x_stream_t stream);

/* Autotuner.  For each n in sizes[0..nsizes), time every size class whose
 * padded size holds n (up to 1.6x padding) on a batch of `batch` ring
 * products of synthetic operands in a temporary device buffer (contents do
 * not matter: the kernels are constant time), and the latency of one product
 * through the gf2x_mul_cyclic path in each class.  The context's tables keep,
 * per size, the fastest class for batches, the fastest direct (one workgroup
 * per product) class, and the lowest-latency class for single products.  If
 * out_path is not NULL the tuned sizes are written to that file, one line
 * "w32 batch_class direct_class single_class" each, the format
 * opts->tune_cache reads (lines with only the first one or two classes are
 * accepted too).  This call is synchronous: it waits for the device on a
 * private stream.  Errors: GF2X_EINVAL, GF2X_ENOMEM, GF2X_EDEVICE. */
int gf2x_tune(gf2x_ctx *ctx, const uint32_t *sizes, uint32_t nsizes, uint32_t batch, const char *out_path);

/* ------------------------------------------------------------------ serving
 * Continuous batching of ring products (Section 1's products, arriving as a
 * stream of requests) on one context.  A scheduler thread keeps `streams`
 * slots; each slot holds up to max_batch requests of at most max_bits bits in
 * its own device and pinned host buffers, and the device buffers together
 * stay within hbm_budget_bytes.  Requests whose arrival time has passed are
 * admitted into free slots in submission order; while a slot's batch runs,
 * later arrivals form the next batch on another slot, so their work overlaps
 * on the device.  A batch of at most 256 requests runs each product in its
 * size's lowest-latency class (possibly staged, using a per-slot workspace
 * within half of the budget; with many streams or a small budget the limit
 * is halved until the workspaces fit, down to none); larger batches run
 * each product in its size's fastest one-workgroup class.  A batch whose
 * classes the phase kernels hold runs as three launches for all of its sizes
 * (evaluations, one-workgroup products, interpolations), else one launch per
 * size class.  Operands and descriptors reach the device, and results the
 * pinned buffer, through copy kernels (no DMA copy call per batch).  Results
 * are identical to gf2x_mul_cyclic of the same operands (every class
 * computes the same exact product). */
typedef struct gf2x_srv gf2x_srv;

typedef struct gf2x_srv_opts {
    size_t hbm_budget_bytes; /* device memory for in-flight requests (0 = 256 MiB)          */
    uint32_t streams;        /* concurrent batches, 1..16 (0 = 4)                           */
    uint32_t max_bits;       /* largest n that will be submitted (0 = 57637)                */
    uint32_t max_batch;      /* cap on requests per batch (0 = as many as the budget allows) */
    uint32_t max_pending;    /* host queue length before GF2X_EAGAIN (0 = 4M)               */
    uint32_t flags;          /* reserved, must be 0                                         */
} gf2x_srv_opts;

typedef struct gf2x_srv_stats {
    uint64_t submitted, admitted, completed, refused, pending;
    uint64_t batches, launches;
    uint32_t max_batch, max_batch_seen, max_slots_busy;
    uint64_t hbm_bytes;        /* device memory held by the slots                                     */
    uint64_t phased_batches;   /* batches run as three phase kernels                                  */
    /* Host time of the scheduler per batch, in ns (totals and maxima): packing
     * the operands and descriptors into the pinned buffer, issuing the copies
     * and launches, handing the results back.  device_max_ns is the longest
     * time from a batch's last HIP call to its completion being seen (device
     * work plus polling), batch_max_ns the longest from admission to the
     * results handed back, loop_busy_max_ns the longest scheduler iteration
     * without its idle wait, wake_late_max_ns the longest overshoot of an
     * idle wait.  Together they place a slow batch in host or device time. */
    uint64_t host_pack_ns, host_issue_ns, host_retire_ns;
    uint64_t host_pack_max_ns, host_issue_max_ns, host_retire_max_ns;
    uint64_t device_max_ns, batch_max_ns, loop_busy_max_ns, wake_late_max_ns;
    uint64_t loop_busy_max_at_ns; /* steady-clock start of the longest scheduler iteration */
    /* The issue time split by HIP call (maxima over batches): the copy in
     * (a kernel that reads the descriptors and operands out of the pinned
     * buffer), the product kernel launches (with any sub-stream fork and
     * join events), the copy back (a kernel that writes the results into the
     * pinned buffer) and the completion event. */
    uint64_t host_issue_copy_max_ns, host_issue_launch_max_ns, host_issue_tail_max_ns;
} gf2x_srv_stats;

/* Start a server on ctx (which must outlive it).  Errors: GF2X_EINVAL,
 * GF2X_ENOMEM (budget below one request per stream, or allocation failed),
 * GF2X_EDEVICE. */
int gf2x_srv_create(gf2x_srv **out, gf2x_ctx *ctx, const gf2x_srv_opts *opts);

/* Submit `count` requests.  Request i multiplies the HOST polynomials at
 * a_base + a_off[i] and b_base + b_off[i] (W(n_bits[i]) words each, read when
 * the request is admitted) and writes the ring product to the HOST words at
 * c_base + c_off[i] when it completes; the caller keeps all three alive until
 * then.  arrival_ns[i] (steady clock, gf2x_srv_now_ns; NULL = now) is the
 * earliest admission time.  Tickets first_ticket .. first_ticket+count-1 are
 * assigned in order.  Errors: GF2X_EINVAL (n above max_bits, null pointers),
 * GF2X_EAGAIN (host queue full: nothing was queued), a pending device error. */
int gf2x_srv_submit(gf2x_srv *srv, uint32_t count, const uint32_t *n_bits, const uint64_t *a_base,
                    const uint64_t *a_off, const uint64_t *b_base, const uint64_t *b_off, uint64_t *c_base,
                    const uint64_t *c_off, const uint64_t *arrival_ns, uint64_t *first_ticket);

/* Completion stamps (steady clock ns; 0 = not yet complete) of tickets
 * first_ticket .. first_ticket+count-1.  The server keeps a stamp until it has
 * been returned here and every earlier ticket's stamp has been returned too;
 * after that, reading the ticket again gives 1 (completed, stamp no longer
 * kept).  So the memory held for stamps is bounded by the tickets not yet
 * read.  Errors: GF2X_EINVAL (a ticket not yet issued), or the device error
 * the scheduler hit. */
int gf2x_srv_completion(gf2x_srv *srv, uint64_t first_ticket, uint32_t count, uint64_t *done_ns);

/* Wait until every submitted request has completed (timeout_ms 0 = 1 hour).
 * Returns GF2X_EAGAIN on timeout. */
int gf2x_srv_drain(gf2x_srv *srv, uint64_t timeout_ms);

/* Counters of the server.  Errors: GF2X_EINVAL. */
int gf2x_srv_get_stats(gf2x_srv *srv, gf2x_srv_stats *stats);

/* Steady-clock time in ns, the time base of arrival and completion stamps. */
uint64_t gf2x_srv_now_ns(void);

/* Stop the server after the queued requests complete, and free it.  NULL is
 * accepted. */
void gf2x_srv_destroy(gf2x_srv *srv);

/* Static message for a GF2X_E* code. */
const char *gf2x_strerror(int code);

/* Name of the last HIP error seen by this thread's calls ("" if none). */
const char *gf2x_last_device_error(void);

/* Library version, as 10000*major + 100*minor + patch. */
int gf2x_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GF2X_H */
