/*
 * iqcc.h -- C ABI of the MI355X (gfx950) iQCC hot-path library, libiqcc.so.
 *
 * What the library computes (the parallel iQCC paper, arXiv 2603.08883):
 *   H = sum_k C_k P_k                                   (Sec. II, Eq. 2)
 *   H' = e^{i tau P/2} H e^{-i tau P/2}                 (Sec. II, Eq. 5, closed form)
 *      = merge of the raw terms D = H + I                (App. D, sortless dressing)
 *      followed by dropping terms with |c| < eps         (App. A, iterative procedure,
 *                                                         optional compression step)
 *   E = <Omega| H |Omega>, QMF product state            (Sec. II, Eq. 3)
 *   g_a = Im <Omega| H P_a |Omega>                      (Sec. II, Eq. 7; App. A DIS)
 *   dE/dtheta_j, dE/dphi_j                              (derivative of Eq. 3 energy)
 *
 * Pauli words.  A word on n qubits is W = ceil(n/64) uint64 "x" words and W
 * "z" words; qubit j is bit j%64 of word j/64.  The local operator is
 * I (x=0,z=0), X (1,0), Z (0,1), Y (1,1) with Y the Hermitian Pauli-Y; no phase
 * is stored and coefficients are real FP64.  Bits at qubits >= n must be 0.
 * Device arrays of words are word-major planes: word w of row i lives at
 * x[w*ld + i] (ld >= number of rows).
 *
 * Term store.  Terms live in an opaque device-resident iqcc_store: word planes
 * plus coefficients, partitioned into 2^m buckets by a GF(2)-linear 32-bit hash
 * of the key (the one-device form of the paper's bit-wise partitioning,
 * App. B): hash(K xor P) = hash(K) xor hash(P), so the new term K xor P of a
 * term in bucket b lands in bucket b xor (hash(P) mod 2^m) and every merge is
 * local to one bucket pair.  Keys in a store are unique.  The order of terms
 * inside a store is unspecified; export returns them grouped by bucket.
 *
 * Conventions for every call:
 *   - return value: IQCC_OK (0) or a negative IQCC_ERR_* code; a message is
 *     available from iqcc_last_error(ctx).  No C++ exception crosses the ABI.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).  Calls
 *     are asynchronous and stream-ordered unless documented as synchronising.
 *   - device pointers are owned by the caller unless stated; the library
 *     never frees caller memory.  Outputs never alias inputs.
 *   - argument validation happens on the host before any device work; invalid
 *     arguments leave every output untouched.
 *   - a context is bound to one device and must not be used by two threads
 *     at once.  Stores belong to the context that created them.
 */
#ifndef IQCC_H
#define IQCC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IQCC_OK 0
#define IQCC_ERR_INVALID_ARG (-1) /* null pointer, bad size, padding bits, non-finite tau, eps < 0 */
#define IQCC_ERR_CAPACITY (-2)    /* a store's arena or bucket table is too small */
#define IQCC_ERR_HIP (-3)         /* a HIP runtime call failed */
#define IQCC_ERR_UNSUPPORTED (-4) /* e.g. more than 256 qubits */

#define IQCC_MAX_WORDS 4 /* up to 256 qubits */

typedef struct iqcc_ctx iqcc_ctx;
typedef struct iqcc_store iqcc_store;
typedef struct iqcc_batch iqcc_batch;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device`.  Allocates small device scratch. */
int iqcc_ctx_create(iqcc_ctx **ctx, int device);
/* Destroy a context (NULL is allowed).  Stores must be destroyed first. */
int iqcc_ctx_destroy(iqcc_ctx *ctx);
/* Last error message of this context ("" if none).  Valid until the next call. */
const char *iqcc_last_error(const iqcc_ctx *ctx);
/* Library version string. */
const char *iqcc_version(void);

/* Tuning knobs (the autotuner and tests set them).  Names:
 *   "load_bucket_terms"  target mean bucket size when a store is loaded
 *                        (1 .. 16384; a load ranks each bucket's terms, at a
 *                        cost that grows with the square of the bucket size)
 *   "split_bucket_terms" a dressing step doubles the bucket count when the
 *                        mean input bucket exceeds this many terms (>= 1)
 *   "anti_cap"           LDS capacity, in anticommuting terms, of one bucket
 *                        pair; larger pairs are processed in hash rounds
 *                        (16 .. 8192)
 *   "grid_per_cu"        persistent workgroups per compute unit (1 .. 16)
 *   "batch_split_bucket_terms", "batch_anti_cap"
 *                        the same two settings for batched dressing of many
 *                        small Hamiltonians (iqcc_dress_batched, iqcc_batch_*)
 *   "batch_unit_pairs"   consecutive bucket pairs of one Hamiltonian per work
 *                        unit of a batch (1 .. 65536); read when the batch is
 *                        created
 *   "energy_grid_per_cu" workgroups per compute unit of the stand-alone energy
 *                        kernel (1 .. 32)
 *   "fuse_energy"        1: dressing evaluates the energy of its output in the
 *                        same pass when angles are given; 0: separate pass
 *   "dis_tile"           DIS candidates held per workgroup tile (1 .. 256)
 *   "dis_bucket_ranges"  bucket ranges (workgroups along the terms) of the
 *                        batched DIS launch; 0 = about 8 workgroups per CU
 *                        in total (0 .. 4096)
 *   "inplace_bucket_terms" mean bucket size of an IQCC_STORE_INPLACE store
 *                        when it holds max_terms terms (1 .. 16384)
 *   "inplace_item_terms" input terms per work item of iqcc_dress_inplace
 *                        while buckets are small; 0 = 1.5 x the stash
 *   "inplace_cap"        anticommuting terms a wavefront of iqcc_dress_inplace
 *                        stages in LDS; 0 = as many as fit (0 .. 512);
 *                        larger sets go to the pool in hash rounds
 *   "inplace_region_rows" smallest region of a bucket when an in-place store
 *                        is loaded or copied (a bucket with c terms gets at
 *                        least 2c rows); 0 = the arena minus the pool,
 *                        divided evenly (0 .. 2^24)
 * Returns IQCC_ERR_INVALID_ARG for an unknown name or out-of-range value. */
int iqcc_set_param(iqcc_ctx *ctx, const char *name, int64_t value);
int iqcc_get_param(const iqcc_ctx *ctx, const char *name, int64_t *value);

/* ---- term stores ---------------------------------------------------------- */

/* Store flags.  IQCC_STORE_INPLACE: a store that can be dressed in place
 * (iqcc_dress_inplace).  Its contents, once written by iqcc_store_load,
 * iqcc_store_copy or iqcc_dress_inplace, are laid out in bucket regions: about
 * max_terms / "inplace_bucket_terms" buckets (fixed for the store's life),
 * each owning a region of rows with free rows after its live ones, and a pool
 * of max_terms / 2 rows for buckets that outgrow their region.  Device memory
 * about 3.5*max_terms*(16*W + 8) bytes; rows below 2^31 (max_terms up to
 * about 6e8).  Every other call accepts such a store like any other; when
 * an out-of-place call writes it, the region layout is gone until the next
 * load or copy. */
#define IQCC_STORE_INPLACE 1u

/* Create an empty store for `n_qubits` (1..256) qubits able to hold up to
 * `max_terms` terms as the output of a dressing step (the device arena holds
 * 2*max_terms rows because a step reserves, per bucket pair, the worst-case
 * output size 2*(n_b + n_b')).  Device memory: about
 * 2*max_terms*(16*W + 8) bytes plus the bucket table, allocated by the
 * library (synchronising). */
int iqcc_store_create(iqcc_ctx *ctx, int n_qubits, int64_t max_terms, iqcc_store **store);
/* As iqcc_store_create with store flags (0 or IQCC_STORE_INPLACE). */
int iqcc_store_create_ex(iqcc_ctx *ctx, int n_qubits, int64_t max_terms, uint32_t flags,
                         iqcc_store **store);
/* HOST only: *bytes = device memory a store of these parameters needs
 * (header, bucket table and arena in one block).  IQCC_ERR_INVALID_ARG for
 * n_qubits < 1, max_terms outside 1..2^38 or unknown flags. */
int iqcc_store_bytes(int n_qubits, int64_t max_terms, uint32_t flags, int64_t *bytes);
/* Create a store inside caller-owned DEVICE memory `mem` of `bytes` bytes
 * (256-byte aligned, at least iqcc_store_bytes; e.g. a torch tensor).  The
 * library never frees it; destroy the store before releasing the memory.
 * The empty-store initialisation is enqueued on `stream` (no synchronisation).
 * IQCC_ERR_CAPACITY if `bytes` is too small. */
int iqcc_store_wrap(iqcc_ctx *ctx, int n_qubits, int64_t max_terms, uint32_t flags, void *mem,
                    int64_t bytes, iqcc_store **store, void *stream);
/* Destroy a store (NULL is allowed); frees its memory only when the library
 * allocated it (iqcc_store_create*). */
int iqcc_store_destroy(iqcc_ctx *ctx, iqcc_store *store);
/* Copy the live terms of `src` into `dst`, an IQCC_STORE_INPLACE store of the
 * same n_qubits, laid out in bucket regions (the previous contents of dst
 * are discarded).  Each bucket of dst takes its terms in the order they have
 * in src, so a copy of the same store gives the same rows every time.
 * Asynchronous; IQCC_ERR_CAPACITY is reported by the next iqcc_store_count on
 * dst if the regions do not fit its arena, and an invalid src makes dst
 * invalid. */
int iqcc_store_copy(iqcc_ctx *ctx, const iqcc_store *src, iqcc_store *dst, void *stream);
/* Number of qubits / words of a store. */
int iqcc_store_shape(const iqcc_store *store, int *n_qubits, int *n_words);

/* Replace the contents of `store` with n rows of device arrays x, z (word
 * planes, leading dimension ld >= n) and c.  Keys must be unique and bits at
 * qubits >= n_qubits zero; this is not checked unless the IQCC_DEBUG_VALIDATE
 * environment variable is set, which adds a synchronising host-side check of
 * both (IQCC_ERR_INVALID_ARG, store unchanged, on a duplicate key or a set
 * padding bit).  Chooses the bucket count from "load_bucket_terms".  Each
 * bucket receives its terms in ascending key order, so loading the same terms
 * (in any input order) gives the same rows, and every later step and sum
 * over the store repeats bit for bit.  Uses library working memory of about
 * 8 bytes per row (the context's scratch, grown on demand). */
int iqcc_store_load(iqcc_ctx *ctx, iqcc_store *store, const uint64_t *x, const uint64_t *z,
                    const double *c, int64_t n, int64_t ld, void *stream);

/* Synchronising: number of live terms of the store.  Returns IQCC_ERR_CAPACITY
 * if the dressing step that produced the store ran out of arena or bucket
 * table (its contents are then undefined). */
int iqcc_store_count(iqcc_ctx *ctx, const iqcc_store *store, int64_t *n, void *stream);

/* *out (DEVICE scalar) = sum of c^2 over the live terms of the store.  By
 * Eq. 5 a dressing step keeps this sum (cos^2 + sin^2 = 1 on every rotated
 * pair) and compression (App. A) lowers it by the squares it drops, so it is a
 * per-step check of a chain.  Asynchronous; the per-workgroup sums are reduced
 * in a fixed order. */
int iqcc_store_sum_squares(iqcc_ctx *ctx, const iqcc_store *store, double *out, void *stream);

/* Synchronising: counters of the dressing step that produced `store`:
 * *n_anti = input terms that anticommuted with the entangler, *n_new = output
 * terms whose key was not in the input (both 0 after iqcc_store_load). */
int iqcc_store_stats(iqcc_ctx *ctx, const iqcc_store *store, int64_t *n_anti, int64_t *n_new,
                     void *stream);

/* Point lookup of n keys (DEVICE word planes qx, qz, leading dimension ld):
 * found[i] = 1 and val[i] = coefficient if key i is in the store, else 0 and
 * 0.0 (DEVICE int8 / double arrays).  One wave scans the key's bucket. */
int iqcc_store_lookup(iqcc_ctx *ctx, const iqcc_store *store, const uint64_t *qx,
                      const uint64_t *qz, int64_t n, int64_t ld, int8_t *found, double *val,
                      void *stream);

/* Synchronising: copy the live terms to device arrays x, z (planes, leading
 * dimension ld) and c with room for `cap` rows; *n receives the row count.
 * IQCC_ERR_CAPACITY (outputs untouched, *n set) if cap is too small. */
int iqcc_store_export(iqcc_ctx *ctx, const iqcc_store *store, uint64_t *x, uint64_t *z,
                      double *c, int64_t cap, int64_t ld, int64_t *n, void *stream);

/* ---- dressing, merge, compression (Eq. 5, App. D, App. A) ---------------- */

/* One fused dressing step out = compress_eps(merge(e^{i tau P/2} in e^{-i tau P/2})).
 * px, pz: HOST arrays of n_words words (the entangler; identity is a no-op).
 * For a term A of `in` that anticommutes with P, with P*A = i^e Q:
 *   out[A]  += RN(cos(tau) * c_A)
 *   out[Q]  += s * RN(sin(tau) * c_A),   s = +1 if e == 3, -1 if e == 1;
 * terms that commute are copied unchanged.  Every key receives at most two
 * contributions; their sum is one IEEE addition, so the result does not depend
 * on order.  cos/sin are evaluated once on the host with the C library.  A term
 * is dropped when |c| < eps (eps >= 0; eps = 0 keeps exact zeros).
 * theta, phi (DEVICE, n_qubits each) and energy (DEVICE scalar) are optional
 * (all NULL or all set): when set, *energy receives <Omega|out|Omega>.
 * `out` must be a different store with the same n_qubits; its previous
 * contents are discarded.  Asynchronous: a capacity failure is reported by the
 * next iqcc_store_count / iqcc_store_export on `out`. */
int iqcc_dress(iqcc_ctx *ctx, const iqcc_store *in, const uint64_t *px, const uint64_t *pz,
               double tau, double eps, const double *theta, const double *phi, double *energy,
               iqcc_store *out, void *stream);

/* iqcc_dress with the energy carried forward: energy_in (DEVICE scalar) holds
 * <Omega|in|Omega> for the same theta, phi; *energy_out (DEVICE scalar, may be
 * the same address) receives <Omega|out|Omega>.  By Eq. 5 the terms that commute
 * with P keep their coefficients, and the energy is linear in the coefficients
 * (Eq. 3), so the pass evaluates <Omega|K|Omega> only for anticommuting terms,
 * their images K*P and commuting terms removed by compression, and adds that
 * change to *energy_in.  The result equals the full sum up to rounding order.
 * All four energy arguments are required; otherwise as iqcc_dress. */
int iqcc_dress_energy_update(iqcc_ctx *ctx, const iqcc_store *in, const uint64_t *px,
                             const uint64_t *pz, double tau, double eps, const double *theta,
                             const double *phi, const double *energy_in, double *energy_out,
                             iqcc_store *out, void *stream);

/* In-place form of iqcc_dress / iqcc_dress_energy_update (Sec. II Eq. 5,
 * App. D merge, App. A compression): `store` becomes the dressed, merged and
 * compressed Hamiltonian, with the same terms and coefficients bit for bit
 * as iqcc_dress would write.  Terms that commute with P keep their rows and
 * are not rewritten; an anticommuting term's new coefficient is written into
 * its own row; new keys are appended after the live rows of their bucket;
 * rows freed by compression are refilled from the end of the bucket.  A
 * bucket that outgrows its region moves to the store's pool.
 * `store` must be an IQCC_STORE_INPLACE store in the region layout
 * (IQCC_ERR_INVALID_ARG otherwise).  theta, phi, energy_out (DEVICE) are
 * optional, all NULL or all set: *energy_out receives <Omega|store|Omega>
 * after the step.  energy_in (DEVICE, optional, needs the other three) holds
 * the energy before the step; then only the change is evaluated, as in
 * iqcc_dress_energy_update (energy_out may equal energy_in).  Row positions,
 * coefficients and the energy are the same on every run for the same input
 * layout (one wavefront per work item, items dealt out in a fixed order).
 * Asynchronous; if the pool runs out the store becomes invalid, which the next
 * iqcc_store_count reports as IQCC_ERR_CAPACITY. */
int iqcc_dress_inplace(iqcc_ctx *ctx, iqcc_store *store, const uint64_t *px, const uint64_t *pz,
                       double tau, double eps, const double *theta, const double *phi,
                       const double *energy_in, double *energy_out, void *stream);

/* Synchronising diagnostics of the last iqcc_dress_inplace on `store` (each
 * pointer may be NULL): work items moved to the pool, rows freed by
 * compression, rows per bucket region, pool rows in use. */
int iqcc_store_inplace_stats(iqcc_ctx *ctx, const iqcc_store *store, int64_t *relocated, int64_t *freed,
                             int64_t *region_rows, int64_t *pool_used, void *stream);

/* Synchronising sizing call for a dressing step of `in` by P (HOST words px,
 * pz; Eq. 5): *n_anti = number of terms of `in` that anticommute with P.
 * The raw output of the step (before the merge D = H + I of App. D) has
 * count + n_anti rows, and the merged output at most that many. */
int iqcc_dress_count(iqcc_ctx *ctx, const iqcc_store *in, const uint64_t *px, const uint64_t *pz,
                     int64_t *n_anti, void *stream);

/* Pauli products P1 P2 = i^e P3 of n pairs of words (DEVICE word planes with
 * leading dimension ld >= n, n_qubits qubits): x3 = x1 ^ x2, z3 = z1 ^ z2 and
 * e[i] in 0..3 (DEVICE int8) with the Hermitian-Y encoding.  Exported for
 * tests of the phase rule that dressing and DIS gradients use (Eqs. 5, 7). */
int iqcc_pauli_products(iqcc_ctx *ctx, int n_qubits, const uint64_t *x1, const uint64_t *z1,
                        const uint64_t *x2, const uint64_t *z2, int64_t n, int64_t ld,
                        uint64_t *x3, uint64_t *z3, int8_t *e, void *stream);

/* Raw dressing (no merge, no compression) of flat device rows: for each input
 * row i (in order) emits row 2i = (A, c or RN(cos*c)) and, for anticommuting
 * rows only, row 2i+1 = (Q, s*RN(sin*c)).  Rows 2i+1 of commuting inputs are
 * written with c = NaN and flag[i] = 0; flag[i] = 1 marks anticommuting input
 * rows.  Outputs: ox, oz planes with leading dimension ld_out >= 2n, oc, flag
 * (int8, n entries).  Stream-ordered, no synchronisation. */
int iqcc_dress_raw(iqcc_ctx *ctx, int n_qubits, const uint64_t *x, const uint64_t *z,
                   const double *c, int64_t n, int64_t ld, const uint64_t *px,
                   const uint64_t *pz, double tau, uint64_t *ox, uint64_t *oz, double *oc,
                   int8_t *flag, int64_t ld_out, void *stream);

/* Merge of an arbitrary multiset of rows (D = H + I of App. D) followed by
 * compression: equal keys are summed in increasing row order (left to right),
 * then rows with |sum| < eps are dropped; the unique result replaces the
 * contents of `out` (which needs room for n rows).  x, z are device word planes
 * with leading dimension ld >= n, c device coefficients.  Asynchronous; uses
 * about (16*W + 24) * n bytes of context scratch. */
int iqcc_merge_truncate(iqcc_ctx *ctx, const uint64_t *x, const uint64_t *z, const double *c,
                        int64_t n, int64_t ld, double eps, iqcc_store *out, void *stream);

/* ---- many Hamiltonians at once (one entangler each) --------------------- */

/* Dress n_ham independent Hamiltonians, item i: outs[i] = compress_eps(dress(
 * ins[i], P_i, taus[i])) with the same rules as iqcc_dress (no energy).  All
 * stores share n_words; px, pz are HOST arrays [n_ham][n_words], taus HOST
 * [n_ham].  One persistent launch takes (Hamiltonian, bucket pair) items from
 * a device queue, the single-device analogue of over-partitioning with dynamic
 * reassignment (App. C).  Outputs must be distinct from each other and from
 * every input.  Synchronises the stream before returning. */
int iqcc_dress_batched(iqcc_ctx *ctx, int n_ham, const iqcc_store *const *ins,
                       iqcc_store *const *outs, const uint64_t *px, const uint64_t *pz,
                       const double *taus, double eps, void *stream);

/* The same batch captured once into a HIP graph (plan kernel + persistent
 * kernel; every size is computed on the device, no memset nodes).
 * iqcc_batch_launch replays it asynchronously on `stream`; the stores are
 * referenced, not copied, so replays see their current contents. */
int iqcc_batch_create(iqcc_ctx *ctx, int n_ham, const iqcc_store *const *ins,
                      iqcc_store *const *outs, const uint64_t *px, const uint64_t *pz,
                      const double *taus, double eps, iqcc_batch **batch);
int iqcc_batch_launch(iqcc_ctx *ctx, iqcc_batch *batch, void *stream);
int iqcc_batch_destroy(iqcc_ctx *ctx, iqcc_batch *batch);

/* ---- reverse mode through the dressing chain (Eqs. 4 and 6) -------------- */

/* Host value: rows of the store's arena (the length of per-row arrays such as
 * tapes and cotangents indexed by arena row). */
int iqcc_store_rows(const iqcc_store *store, int64_t *rows);

/* iqcc_dress without energy that also records a tape for the backward pass:
 * for every live row r of `in`, tape_self[r] = output row of its key (-1 if
 * compression dropped it); tape_partner[r] = -1 for a commuting row, and for
 * an anticommuting row 2 * (t + 1) + b, where t is the output row of key ^ P
 * (-1 if absent or dropped) and b = 1 when P K = i^3 (K ^ P) (the sign s_K of
 * Eq. 5's new term is +1), else 0.  Both are DEVICE int32 arrays of
 * iqcc_store_rows(in) entries (caller-owned); the tape stays valid while `in`
 * and `out` are unchanged.  The arena of `out` must hold fewer than 2^30 rows
 * (IQCC_ERR_INVALID_ARG otherwise). */
int iqcc_dress_taped(iqcc_ctx *ctx, const iqcc_store *in, const uint64_t *px, const uint64_t *pz,
                     double tau, double eps, iqcc_store *out, int32_t *tape_self,
                     int32_t *tape_partner, void *stream);

/* Backward of one taped dressing step with the compression decisions of the
 * forward pass held fixed.  lambda_out: DEVICE cotangent dE/dc per row of
 * `out` (iqcc_store_rows(out) entries, read at live rows only); lambda_in:
 * DEVICE output per row of `in`; *dtau (DEVICE scalar) = dE/dtau of this step:
 *   lambda_in[A] = cos(t) lambda_out[A] + s_A sin(t) lambda_out[A^P]  (anticommuting A)
 *   lambda_in[A] = lambda_out[A]                                      (commuting A)
 *   dtau = sum_A -sin(t) c_A lambda_out[A] + s_A cos(t) c_A lambda_out[A^P].
 * The rows of A^P and the signs s_A come from the tape of iqcc_dress_taped;
 * px, pz name the step's entangler and are only checked against n_qubits.
 * dtau is an exact fixed-point sum (resolution 2^-60) of the per-row terms, so
 * it has the same bits for any order of the rows; it is NaN if a term is not
 * finite or the terms' magnitudes add up to 2^31 or more. */
int iqcc_dress_backward(iqcc_ctx *ctx, const iqcc_store *in, const uint64_t *px,
                        const uint64_t *pz, double tau, const int32_t *tape_self,
                        const int32_t *tape_partner, const double *lambda_out,
                        double *lambda_in, double *dtau, void *stream);

/* The whole taped chain of Eq. 6 in one call: outs[j] = step j applied to
 * outs[j-1] (outs[-1] = h0) with entangler j (HOST px, pz [n_steps][n_words]),
 * amplitude taus[j] (HOST) and compression eps, recording the tapes of
 * iqcc_dress_taped in tape_self[j], tape_partner[j] (DEVICE int32 arrays of
 * iqcc_store_rows of the step's input).  outs: n_steps distinct stores, none
 * equal to h0, each large enough for its step.  Asynchronous. */
int iqcc_chain_forward(iqcc_ctx *ctx, const iqcc_store *h0, int n_steps, const uint64_t *px,
                       const uint64_t *pz, const double *taus, double eps,
                       iqcc_store *const *outs, int32_t *const *tape_self,
                       int32_t *const *tape_partner, void *stream);

/* Reverse sweep of iqcc_chain_forward (same h0, entanglers, taus, outs and
 * tapes; compression decisions held fixed).  lambda_final: DEVICE dE/dc per
 * row of outs[n_steps-1]; dtau: DEVICE [n_steps] receives dE/dtau_j;
 * lambda_h0 (DEVICE, iqcc_store_rows(h0) entries, or NULL) receives dE/dc per
 * row of h0; work0, work1: DEVICE buffers of at least the largest
 * iqcc_store_rows among h0 and outs.  Asynchronous. */
int iqcc_chain_backward(iqcc_ctx *ctx, const iqcc_store *h0, int n_steps, const uint64_t *px,
                        const uint64_t *pz, const double *taus, iqcc_store *const *outs,
                        int32_t *const *tape_self, int32_t *const *tape_partner,
                        const double *lambda_final, double *work0, double *work1,
                        double *lambda_h0, double *dtau, void *stream);

/* out[r] = scale * <Omega| P_r |Omega> for every live row r of the store
 * (DEVICE array of iqcc_store_rows entries; scale a DEVICE scalar or NULL = 1):
 * the cotangent of the energy with respect to each coefficient. */
int iqcc_expectations(iqcc_ctx *ctx, const iqcc_store *h, const double *theta, const double *phi,
                      const double *scale, double *out, void *stream);

/* ---- QMF energy and its gradient (Eq. 3) ---------------------------------- */

/* *energy (DEVICE scalar) = sum_k c_k prod_j <sigma_kj>, with <X> = sin t cos f,
 * <Y> = sin t sin f, <Z> = cos t per qubit (theta, phi DEVICE arrays). */
int iqcc_qmf_energy(iqcc_ctx *ctx, const iqcc_store *h, const double *theta,
                    const double *phi, double *energy, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * energy as iqcc_qmf_energy, from the same kernels, with no allocation of any
 * kind.  Its scratch (the QMF group table and the per-workgroup partial sums)
 * is a fixed array of device memory inside the library, 128 KB per
 * device, held until the process ends.  The grid (n_cu * energy_grid_per_cu
 * workgroups) may use at most 8192 partial sums; a larger one is refused with
 * IQCC_ERR_CAPACITY before any launch.  All calls on one device share that
 * scratch, so calls that overlap on a device (other streams, other contexts
 * or threads) race; calls in one stream are ordered.  Each call rewrites all
 * the scratch it reads. */
int iqcc_qmf_energy_noalloc(iqcc_ctx *ctx, const iqcc_store *h, const double *theta,
                            const double *phi, double *energy, void *stream);

/* Backward of iqcc_qmf_energy: dtheta[j] = dE_scale * dE/dtheta_j and
 * dphi[j] = dE_scale * dE/dphi_j (DEVICE arrays of n_qubits), where dE_scale
 * is the DEVICE scalar upstream gradient (NULL means 1).  lambda (NULL, or a
 * DEVICE array of iqcc_store_rows entries) receives, for every live row r,
 * dE_scale * <Omega| P_r |Omega>: the cotangent of each coefficient, as
 * iqcc_expectations computes it (same values up to the rounding of the
 * product; rows that hold no term are left untouched).  dtheta and dphi are
 * the same bits on every run and for any order of the rows within the
 * buckets: every per-term contribution is added as an exact 120-bit fixed-
 * point integer (resolution 2^-60), and the per-workgroup sums are reduced
 * in a fixed order.  The exact sums need every |c| < 2^31 and, per workgroup,
 * (largest |c|) * (terms) < 2^42; past those bounds, or with a non-finite
 * coefficient or angle, dtheta and dphi come out NaN. */
int iqcc_qmf_energy_backward(iqcc_ctx *ctx, const iqcc_store *h, const double *theta,
                             const double *phi, const double *dE_scale, double *dtheta,
                             double *dphi, double *lambda, void *stream);

/* ---- DIS gradient screening (Eq. 7, App. A) ------------------------------- */

#define IQCC_DIS_BATCHED 0 /* one persistent launch over candidate tiles */
#define IQCC_DIS_PLAIN 1   /* one launch per candidate (reference form) */

/* g[a] = Im <Omega| H P_a |Omega> = sum_k c_k Im(i^e) <Q_k>, P_k P_a = i^e Q_k,
 * for n_cand candidates given as DEVICE word planes cx, cz (leading dimension
 * ld_cand >= n_cand).  g is a DEVICE array of n_cand doubles. */
int iqcc_dis_gradients(iqcc_ctx *ctx, const iqcc_store *h, const double *theta,
                       const double *phi, const uint64_t *cx, const uint64_t *cz,
                       int64_t n_cand, int64_t ld_cand, int mode, double *g, void *stream);

/* ---- sortless dressing (App. D): the comparison path ---------------------- */

/* Synchronising: the same dressing step as iqcc_dress (Eq. 5, merge D = H + I,
 * compression |c| < eps) on a flat Hamiltonian that is globally sorted in
 * canonical order (x words, then z words, most significant word first) and has
 * unique keys, following the paper's sortless dressing: partition H by the key
 * bits P flips (each partition stays sorted), dress each partition, merge the
 * images into the partition they land in, and restore the global order by a
 * multiway merge.  x, z: DEVICE word planes (leading dimension ld >= n), c:
 * DEVICE coefficients; the result (sorted, unique) goes to the DEVICE arrays
 * ox, oz (leading dimension ld_out >= cap), oc, and *n_out (HOST) receives its
 * size (IQCC_ERR_CAPACITY when it exceeds cap).  The entangler may flip at
 * most 20 key bits (popcount of its x and z words).  Working memory is
 * allocated per call. */
int iqcc_sortless_dress(iqcc_ctx *ctx, int n_qubits, const uint64_t *x, const uint64_t *z,
                        const double *c, int64_t n, int64_t ld, const uint64_t *px,
                        const uint64_t *pz, double tau, double eps, uint64_t *ox, uint64_t *oz,
                        double *oc, int64_t cap, int64_t ld_out, int64_t *n_out, void *stream);

/* ---- term-limit compression ---------------------------------------------- */

/* Synchronising: out = the max_terms terms of `in` with the largest |c|; when
 * several terms share the |c| at the boundary, those with the smaller canonical
 * key (x words, then z words, most significant word first) are kept, so the
 * result is unique.  All terms are kept when `in` has at most max_terms.  This
 * is the maximum-terms limit of the Ru-catalyst runs (Results, the run tables
 * and the discussion of the coefficient cutoff and the term limit), applied
 * next to the coefficient cutoff of iqcc_dress.
 * out keeps in's bucket table and arena rows (each bucket's kept terms in
 * input order), so it must be a different store at least as large as `in`. */
int iqcc_truncate_top(iqcc_ctx *ctx, const iqcc_store *in, int64_t max_terms, iqcc_store *out,
                      void *stream);

/* ---- one iQCC iteration (Sec. II, iterative procedure) -------------------- */

/* *energy_anti (DEVICE scalar) = sum over the terms K of h that anticommute with
 * P (HOST words px, pz) of c_K <Omega|K|Omega>.  With a = E - energy_anti,
 * b = energy_anti and c = the DIS gradient of P (Eq. 7), dressing h with P at
 * amplitude tau (Eq. 5) gives exactly E(tau) = a + b cos(tau) + c sin(tau). */
int iqcc_qmf_energy_anti(iqcc_ctx *ctx, const iqcc_store *h, const uint64_t *px,
                         const uint64_t *pz, const double *theta, const double *phi,
                         double *energy_anti, void *stream);

/* Synchronising: the distinct flip sets F (x parts, the positions of X or Y)
 * of the terms of h with 1 <= |F| <= w_max, in ascending order of their words
 * (most significant word first), written to the HOST array fx as rows of
 * n_words words.  *n receives the count; IQCC_ERR_CAPACITY (fx untouched) when
 * it exceeds cap.  Matching a flip set of H is the second DIS condition of
 * App. A. */
int iqcc_flip_sets(iqcc_ctx *ctx, const iqcc_store *h, int w_max, uint64_t *fx, int64_t cap,
                   int64_t *n);

/* Synchronising: one iteration of the iQCC procedure on the Hamiltonian *h.
 *  1. candidates: for every flip set F of *h (iqcc_flip_sets order, |F| <= w_max)
 *     and every qubit q of F in ascending order, the generator with Y on q and
 *     X on the rest of F (one Y: odd Y parity; flip set of a term: App. A);
 *  2. DIS gradients of all candidates in one batched launch (Eq. 7);
 *  3. the n_select candidates of largest |g| (ties: ascending canonical key,
 *     x words then z words, most significant first; zero gradients are never
 *     taken), in that order;
 *  4. for each of them on the current Hamiltonian: b = iqcc_qmf_energy_anti,
 *     c = its DIS gradient, tau = atan2(-c, -b) (0 when b = c = 0), which
 *     minimises E(tau) = a + b cos(tau) + c sin(tau); dress with (P, tau) and
 *     compress with eps (as iqcc_dress).
 * *h and *spare (distinct stores of the same n_qubits, *spare at least as
 * large) are swapped as the steps ping-pong; on return *h holds the result.
 * HOST outputs: sel_x, sel_z [n_select][n_words] (applied generators), sel_g
 * [n_select] (their screening gradients), sel_tau [n_select], energy
 * [n_select + 1] (energy before the first step and after each), the number of
 * candidates and the number of generators applied (<= n_select). */
int iqcc_qcc_iteration(iqcc_ctx *ctx, iqcc_store **h, iqcc_store **spare, const double *theta,
                       const double *phi, int w_max, int n_select, double eps, uint64_t *sel_x,
                       uint64_t *sel_z, double *sel_g, double *sel_tau, double *energy,
                       int64_t *n_candidates, int *n_applied);

/* ---- several generators at once (Eqs. 5 and 6) ----------------------------- */

/* Synchronising.  Dressing h with P_1 at tau_1, then P_2 at tau_2, ..., P_n at
 * tau_n (Eq. 6, no compression) turns every term into a sum over branches in
 * which each generator contributes 1, cos(tau_k) or sin(tau_k) (Eq. 5), so the
 * QMF energy is exactly the trigonometric polynomial
 *   E(tau) = sum_s coef[s] prod_k f_{s_k}(tau_k),  f_0 = 1, f_1 = cos, f_2 = sin,
 *   s = s_0 + 3 s_1 + ... + 3^(n-1) s_(n-1).
 * The 3^n coefficients (HOST array, 1 <= n <= 8) are obtained from the energies
 * of the dressed Hamiltonians on the grid tau_k in {0, pi/2, pi} (3^n chains,
 * sharing prefixes) and one 3x3 inverse per axis.  px, pz: HOST [n][n_words];
 * work: n distinct stores (same n_qubits, large enough for each prefix of the
 * chain), overwritten. */
int iqcc_energy_trig_poly(iqcc_ctx *ctx, const iqcc_store *h, int n, const uint64_t *px,
                          const uint64_t *pz, const double *theta, const double *phi,
                          iqcc_store *const *work, double *coef);

/* HOST only: value of that polynomial at tau[0..n) (NaN for n outside 1..8 or
 * a null array). */
double iqcc_trig_poly_eval(int n, const double *coef, const double *tau);

/* HOST only: coordinate descent on the polynomial; each coordinate update is
 * the exact minimiser of a + b cos(tau_k) + c sin(tau_k) with the other
 * amplitudes fixed.  tau (in: start, out: result); stops after `sweeps` sweeps
 * or when a sweep does not lower the energy; *energy receives E(tau). */
int iqcc_trig_poly_minimize(int n, const double *coef, double *tau, int sweeps, double *energy);

#ifdef __cplusplus
}
#endif

#endif /* IQCC_H */
