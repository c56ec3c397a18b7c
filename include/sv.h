/*
 * libsv -- single-GPU (MI355X, gfx950) state-vector engine for ordered fused
 * k-qubit gates on a 2^N complex64 state, resolved through a
 * logical-to-physical layout map.
 *
 * Semantics follow the paper's fused-operator interface (Section III, R2:
 * apply(L, Psi, G, V) -> (L', Psi')), its little-endian target convention
 * (Section II, "Fused gates and requests": target q_j supplies bit j of the
 * row and column index of G), its layout map (Section II, "State and layout
 * notation"; Section IV-D: physical index y has y_{L(q)} = x_q for logical
 * index x), decode-on-output (Section IV-D, after Theorem 1) and
 * strict-upper-bound hierarchical-CDF sampling (Section IV-E, "Sampling").
 *
 * Conventions for every call:
 *   - every function returns SV_OK (0) or a negative SV_ERR_* code; the text
 *     of the last error of the calling thread is sv_last_error();
 *   - no C++ exception crosses this interface;
 *   - device work is enqueued on the stream given to sv_alloc and is
 *     asynchronous unless the call says it synchronises;
 *   - calls on one handle are not thread-safe; distinct handles are
 *     independent;
 *   - the library never allocates device memory: the state and the workspace
 *     belong to the caller (for instance PyTorch tensors).  It allocates only
 *     the handle, a small pinned host staging ring and HIP events.
 */
#ifndef SV_H_
#define SV_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SV_OK 0
#define SV_ERR_ARG (-1)         /* invalid argument: range, null pointer, size, duplicate target */
#define SV_ERR_DEVICE (-2)      /* a HIP runtime call failed */
#define SV_ERR_UNSUPPORTED (-3) /* valid request that this build has no kernel for */
#define SV_ERR_STATE (-4)       /* call not valid in the handle's current state */

#define SV_MIN_QUBITS 1
#define SV_MAX_QUBITS 35 /* the paper's GPU engine range tops out at 35 (Appendix C-A) */
#define SV_MAX_K 8       /* widest fused gate accepted (the paper's largest fusion cap is 7) */

typedef struct sv_state sv_state;
typedef struct sv_plan sv_plan;

/* ------------------------------------------------------------------ state */

/* Bytes of device workspace sv_alloc needs for an n-qubit state. */
size_t sv_workspace_bytes(int n_qubits);

/*
 * Bind a handle to caller-owned device memory and initialise |0...0> with the
 * identity layout L(q) = q (the paper's initial invariant, Theorem 1).
 *   out        receives the handle (owned by the library until sv_free)
 *   n_qubits   N in [1, 35]
 *   amps_dev   device pointer, >= 8 * 2^N bytes, 256-byte aligned; complex64
 *              amplitudes interleaved (re, im) in PHYSICAL order
 *   ws_dev     device workspace of >= sv_workspace_bytes(N) bytes, 256-byte aligned
 *   stream     hipStream_t (NULL = default stream) on which all work is enqueued
 * Errors: SV_ERR_ARG (range, null, size, alignment), SV_ERR_DEVICE.
 */
int sv_alloc(sv_state **out, int n_qubits, void *amps_dev, size_t amps_bytes, void *ws_dev,
             size_t ws_bytes, void *stream);

/* Release the handle (not the caller's buffers).  Synchronises the stream. */
int sv_free(sv_state *s);

/* Re-initialise |0...0> and the identity layout. */
int sv_reset(sv_state *s);

/*
 * Apply one fused gate (Algorithm 2 semantics: A = (L(q_0), ..., L(q_{k-1}))
 * is resolved from the current layout, then G acts on the ordered physical
 * targets; output amplitude r of each group = sum_c G[r][c] * input c).
 *   matrix   host pointer, complex128 row-major interleaved (re, im),
 *            2^k x 2^k; row/column bit j <-> targets[j]; copied before return
 *   targets  host pointer, k distinct LOGICAL qubits in [0, N)
 *   k        1 <= k <= min(N, SV_MAX_K)
 * The call may change the layout map (lazy relabel, L' = alpha o L); read it
 * with sv_get_layout.  A matrix whose off-diagonal entries are all exactly
 * zero takes the streaming diagonal lowering (Algorithm 2, diag branch):
 * one pass multiplying each amplitude by the entry its target bits select,
 * layout unchanged.  A matrix that only permutes the target qubits (entries
 * exactly 0 and 1, |c> -> |pi(c)> for a permutation of the bits) moves no
 * data: the layout map absorbs it (SV_VARIANT_AUTO only).  Unitarity is not
 * checked.
 * Errors: SV_ERR_ARG, SV_ERR_UNSUPPORTED, SV_ERR_DEVICE.
 */
int sv_apply_fused(sv_state *s, const double *matrix, const int32_t *targets, int k);

/*
 * Physically move amplitudes so that the layout map becomes new_layout
 * (a bijection logical -> physical bit, host int32[N]).  The identity
 * canonicalises the state (the "request materialisation" consumer of
 * Section IV-D).  Errors: SV_ERR_ARG (not a bijection).
 */
int sv_permute_layout(sv_state *s, const int32_t *new_layout);

/* Copy the current layout map L (logical -> physical) into host int32[N]. */
int sv_get_layout(const sv_state *s, int32_t *out);

/*
 * p_x = |psi_x|^2 in FP64 ((double)re^2 + (double)im^2) into device
 * out_dev[2^N].  logical_order = 1: index is the logical basis index decoded
 * through L; 0: physical order (pair with sv_get_layout).
 */
int sv_probs(sv_state *s, double *out_dev, int logical_order);

/* ||psi||^2 accumulated in FP64 into *out_host.  Synchronises the stream. */
int sv_norm(sv_state *s, double *out_host);

/*
 * Draw `shots` computational-basis samples (Section IV-E, "Sampling"):
 * hierarchical CDF over 2^10-entry blocks with exact integer block totals
 * (q_x = floor(p_x * 2^62) as uint64), per shot the 64-bit Philox4x32-10 draw
 * r (key = seed, counter = shot index) gives t = floor(r * T / 2^64) and the
 * outcome is the smallest physical index y with C(y) > t (strict upper bound:
 * a zero-probability outcome is never drawn).  Each outcome is decoded through
 * L (Section IV-D): bit q of out_host[s] = logical qubit q.  Deterministic for
 * (state, seed, shots).  Synchronises the stream.
 * Errors: SV_ERR_ARG (shots < 0, null), SV_ERR_STATE (zero total probability;
 * an amplitude that is not finite; ||psi||^2 of 4 or more, whose fixed-point
 * total T would not fit in 64 bits -- unitarity is not checked elsewhere).
 */
int sv_sample(sv_state *s, uint64_t seed, int64_t shots, uint64_t *out_host);

/*
 * The same sampler on a caller-supplied FP64 probability array
 * (device, 2^n entries), outcome = array index.  Every entry must be finite
 * and in [0, 4), and the entries must sum to less than 4 (so that the
 * fixed-point total fits in 64 bits); they need not be normalised.
 * ws_dev >= sv_workspace_bytes(n).  Synchronises `stream`.
 * Errors: SV_ERR_ARG (null, n out of range, small workspace, an entry that
 * is negative, not finite or 4 or more, or a total of 4 or more -- found on
 * the GPU during the CDF build, before any shot is drawn), SV_ERR_STATE (all
 * entries zero).
 */
int sv_sample_probs(const double *probs_dev, int n, uint64_t seed, int64_t shots, uint64_t *out_host,
                    void *ws_dev, size_t ws_bytes, void *stream);

/*
 * For callers that cannot allocate device memory (code that may not call
 * hipMalloc or an allocating library routine: tight serving loops,
 * harnesses that forbid allocation): sv_sample_probs without a workspace.
 * The sampler's scratch -- CDF block totals, their chunk totals, a chunk of
 * SV_NOALLOC_SHOT_CHUNK outcomes and a flag, SV_NOALLOC_SCRATCH_BYTES in all
 * -- is a fixed device array inside the library; each GPU holds its own copy
 * from the first call on it until the process ends, and the call allocates
 * nothing.  Arguments, outcomes and errors are those of sv_sample_probs
 * (outcomes are bit-identical for the same inputs), with n limited to
 * [1, SV_NOALLOC_MAX_QUBITS].  `stream` must belong to the calling thread's
 * current device, whose copy of the array is used.  The array keeps the last
 * call's contents (every call rewrites what it reads).  Calls that overlap on
 * one GPU -- from several host threads, or on several streams -- share the
 * array and race: serialise them.  Synchronises `stream`.
 * Errors: SV_ERR_ARG (as sv_sample_probs, or n > SV_NOALLOC_MAX_QUBITS),
 * SV_ERR_STATE, SV_ERR_DEVICE.
 */
#define SV_NOALLOC_MAX_QUBITS 26
#define SV_NOALLOC_SHOT_CHUNK 65536
#define SV_NOALLOC_SCRATCH_BYTES 1049600
int sv_sample_probs_noalloc(const double *probs_dev, int n, uint64_t seed, int64_t shots, uint64_t *out_host,
                            void *stream);

/*
 * Copy the state to caller-owned host memory (out_host >= 8 * 2^N bytes,
 * complex64 interleaved).  logical_order = 0: physical order, as stored;
 * 1: logical basis order, out[x] = amps[y] with y_{L(q)} = x_q (decoded on the
 * host through a 32 MiB staging buffer: the layout and the device state are
 * left as they are).  Waits for the handle's stream first.  Errors:
 * SV_ERR_ARG (null), SV_ERR_DEVICE (a HIP call or the staging allocation
 * failed).
 */
int sv_copy_out(sv_state *s, void *out_host, int logical_order);

/* Wait for all work enqueued by this handle. */
int sv_sync(sv_state *s);

/* Text of the calling thread's last error ("" if none).  Valid until the next call. */
const char *sv_last_error(void);

/* ------------------------------------------------------------------ options */

/* Kernel selector override (tests and measurements force every lowering). */
#define SV_OPT_VARIANT 1
#define SV_VARIANT_AUTO 0
#define SV_VARIANT_VALU 1    /* per-thread group gather / FMA / scatter, k <= 4 */
#define SV_VARIANT_SHUFFLE 2 /* k = 1 on a physical bit < 7, wavefront shuffle */
#define SV_VARIANT_MFMA 3    /* LDS-tiled real-embedded complex GEMM on MFMA, 4 <= k <= 7 */
#define SV_VARIANT_GENERIC 4 /* one group per workgroup, any k <= 8 */
#define SV_VARIANT_DIAG 5    /* diagonal matrices only: streaming elementwise multiply, any k <= 8 */

/* Arithmetic of the MFMA lowering. */
#define SV_OPT_PRECISION 2
#define SV_PREC_FP32 0   /* FP32 MFMA, FP32 accumulate */
#define SV_PREC_BF16X3 1 /* x = hi + lo in bf16, hi*hi + hi*lo + lo*hi, FP32 accumulate */

/* Smallest k routed to MFMA when SV_OPT_VARIANT is AUTO (default 4). */
#define SV_OPT_MFMA_MIN_K 3

/* Lazy relabel (the single-GPU analogue of on-demand promotion, Section IV-D):
 * 1 = when a fused gate has targets at physical bits >= SV_OPT_LOW_BITS, the
 * MFMA sweep writes its tile back with those targets exchanged with low
 * non-target bits of the same tile (L' = alpha o L, no extra traffic); the
 * victims are chosen by SV_OPT_POLICY.  0 = never (default). */
#define SV_OPT_LAZY_RELABEL 4

/* Physical bits below this count are the "frames" of the relabel policy (default 12). */
#define SV_OPT_LOW_BITS 5

/* Victim policy among eligible low bits (Corollary 1: farthest next use
 * minimises promotions when the future is known). */
#define SV_OPT_POLICY 7
#define SV_POLICY_BELADY 0     /* farthest next use (hints from sv_hint_next_use), else LRU */
#define SV_POLICY_FIRST_FREE 1 /* lowest-indexed eligible bit */
#define SV_POLICY_LRU 2        /* least recently used qubit */

/* Where the waves of an MFMA sweep read the gate operand: their own
 * registers (k <= 5), once per workgroup in LDS (k <= 7), or from global
 * memory through the caches (k >= 5).  AUTO (default) takes the placement
 * measured fastest for each width and precision (LDS);
 * kernels without the requested placement use their AUTO choice. */
#define SV_OPT_MFMA_OPERAND 6
#define SV_MFMA_OPERAND_REGS 0
#define SV_MFMA_OPERAND_LDS 1
#define SV_MFMA_OPERAND_GLOBAL 2
#define SV_MFMA_OPERAND_AUTO 3

/* Order in which the workgroups of an LDS-tiled sweep (MFMA gates, layout
 * permutations) take tiles.  Consecutive workgroups go to the eight XCDs in
 * turn; with value x > 0 the three lowest workgroup-index bits move to
 * tile-index bits x..x+2, so each XCD walks runs of 2^x consecutive tiles
 * (states with fewer than 2^(x+3) tiles keep the plain order).  0 = plain
 * order (workgroup i takes tile i); -1 (default) = the order measured
 * fastest on MI355X: plain for gate sweeps, x = 9 for layout permutations. */
#define SV_OPT_TILE_ORDER 8

int sv_set_option(sv_state *s, int key, int value);
int sv_get_option(const sv_state *s, int key, int *value);

/* Counters since sv_alloc/sv_reset. */
typedef struct sv_stats {
  int64_t gate_sweeps;      /* fused-gate applications */
  int64_t swap_half_sweeps; /* single bit-transposition passes (half of the state moves) */
  int64_t relabels;         /* target bits moved down by the lazy relabel */
  int64_t launches;         /* kernels launched by gate and layout calls */
  int64_t by_variant[6];    /* gate applications per SV_VARIANT_* */
  int64_t permute_sweeps;   /* full-sweep tile permutation passes */
  int64_t layout_only;      /* fused gates that only permute their qubits: applied to the layout map, no sweep */
  int64_t diag_chunks;      /* 16-byte chunks the diagonal blocks' sweeps read and wrote (a full sweep is
                               2^(N-1); entries exactly 1 need no visit, so a block may sweep less) */
} sv_stats;
int sv_get_stats(const sv_state *s, sv_stats *out);

/*
 * Planner hint for the relabel policy: next_use[q] = position in the caller's
 * gate stream of the next gate that targets logical qubit q (INT64_MAX: none).
 * Positions only need to be comparable between qubits.  Host int64[N],
 * copied.  Without hints the BELADY policy behaves as LRU.
 */
int sv_hint_next_use(sv_state *s, const int64_t *next_use);

/*
 * Host-only simulation of the promotion policy in the all-frame demand model
 * of Corollary 1: `frames` low positions hold logical qubits 0..frames-1
 * initially; for each target tuple (concatenated, sizes ks[i] <= frames),
 * every target not in a frame is promoted by evicting an eligible frame (one
 * whose qubit is not in the current tuple) chosen by `policy`.  Returns the
 * total number of promotions in *out.  No GPU involved.
 */
int sv_policy_simulate(int n_qubits, int frames, int policy, int n_tuples, const int32_t *ks,
                       const int32_t *targets, int64_t *out);

#ifdef __cplusplus
}
#endif
#endif /* SV_H_ */
