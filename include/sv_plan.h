/*
 * libsv fusion planning: turn an ordered gate list into fused blocks.
 *
 * A fused block is the matrix product of a run of consecutive gates (Section IV-C),
 * taken in circuit order with each later gate's matrix multiplying from the
 * left; a block counts as diagonal when all of its gates do.  The products
 * are computed on the host in FP64.
 *
 * Gate lists are passed flat:
 *   ks[i]        width of gate i (1..8)
 *   targets      concatenated ordered logical targets (sum ks entries)
 *   mats         concatenated complex128 row-major interleaved matrices
 *                (2 * 4^ks[i] doubles each), little-endian in the targets
 *   diag         optional (may be NULL) per-gate flag: 1 if the matrix is diagonal.
 *                The planner marks a gate diagonal when its matrix is exactly
 *                diagonal; a flag of 1 on a non-diagonal matrix is SV_ERR_ARG.
 * Plans are host objects owned by the library until sv_plan_free.
 */
#ifndef SV_PLAN_H_
#define SV_PLAN_H_

#include "sv.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Greedy fusion (the paper's planner is a windowed dynamic program; this
 * fallback follows its cross-window greedy merge in its simplest form): walk
 * the gates in circuit order and absorb the next gate while the union of
 * targets has at most k_max qubits, otherwise emit the block and start a new
 * one.  A gate wider than k_max is kept as a singleton.  No reordering.  The
 * block tuple is its distinct qubits in ascending order.
 * Errors: SV_ERR_ARG (k_max not in [1, 8], bad gate).
 */
int sv_plan_greedy(int n_qubits, int n_gates, const int32_t *ks, const int32_t *targets, const double *mats,
                   const int8_t *diag, int k_max, sv_plan **out);

/*
 * Dynamic-programming fusion (Section IV-C, Eq. dp-recurrence): the gate list
 * is cut into consecutive windows of `window` gates; inside a window
 *   D_0 = 0,  D_i = min_{j in J_i} { D_j + Gamma(B(j, i)) },
 * where B(j, i) is the block of gates j..i-1, J_i holds every j whose block
 * width (distinct qubits) is within the cap for its mode (k_max for dense,
 * diag_max for all-diagonal blocks) and always i-1 (an over-cap gate stays a
 * singleton).  Backtracking gives the boundaries; a greedy pass then merges
 * adjacent blocks across window boundaries when the merged block is within
 * the cap and scores lower than the two apart.  Gates keep circuit order
 * unless SV_PLAN_REORDER is set.
 *   score = SV_SCORE_PAPER:   Gamma = 4^k (dense), 1 (diagonal)
 *   score = SV_SCORE_LEARNED: Gamma = exp(MLP(features) + (N - 30) ln 2), the
 *           cost model's predicted sweep time in ms (the network predicts it
 *           at N=30 scale; sv_mlp.h), params host FP32 (nin, hid)
 *   score = SV_SCORE_ROOFLINE: Gamma = the analytic time of the sweep at
 *           MI355X's peaks in ms, max(bytes / 8 TB/s, flops / peak) with
 *           16 B per amplitude visited and the flops of the kernel that runs
 *           the block (8 * 2^k per amplitude at 78.6 TFLOP/s for k <= 3, the
 *           same on 157.3 TFLOP/s FP32 MFMA for k = 4, 6 * 2^k there for
 *           5 <= k <= 7); no parameters
 * For a diagonal block the learned and analytic scores use what the
 * streaming lowering sweeps: the block's diagonal (the FP64 product of its
 * gates' diagonals) is covered by subcubes exactly as sv_apply_fused covers
 * it (entries exactly 1 need no visit), giving the swept fraction and the
 * number of launches (sv_diag_sweep_cost); the analytic score charges
 * fraction + launches / 256 sweeps.
 * Physical positions for the features are the logical qubits (identity
 * layout at planning time).
 */
#define SV_SCORE_PAPER 0
#define SV_SCORE_LEARNED 1
#define SV_SCORE_ROOFLINE 2
/* flags: SV_PLAN_REORDER first applies a commute-aware reorder (Section
 * IV-C): a gate moves only across gates on disjoint qubits, so each qubit's
 * gate sequence is kept; clusters are grown from the dependency front,
 * taking at each step the ready gate that enlarges the cluster's qubit set
 * least (earliest on ties) while it stays within max(k_max, diag_max). */
#define SV_PLAN_REORDER 1
/* flags: SV_PLAN_SEARCH_CAP (learned and analytic scores) plans with every dense
 * width cap c from 4 to k_max, each with diagonal cap min(c, diag_max) and
 * diag_max, and keeps the plan of least predicted total time. */
#define SV_PLAN_SEARCH_CAP 2
/* flags: SV_PLAN_REPEAT runs the reorder-and-fuse pipeline again on the
 * emitted blocks, at most four rounds in all, stopping when the block count
 * no longer decreases (Section IV-C). */
#define SV_PLAN_REPEAT 4
int sv_plan_dp(int n_qubits, int n_gates, const int32_t *ks, const int32_t *targets, const double *mats,
               const int8_t *diag, int k_max, int diag_max, int window, int score, const float *mlp_params_host,
               int mlp_nin, int mlp_hid, int flags, sv_plan **out);

/*
 * Cost-model features of one fused sweep (SV_MLP_FEATURES floats): N/35,
 * k/8, the k physical target positions sorted ascending divided by 35 and
 * padded with -0.25 to seven slots, 1 if the block is diagonal (it then
 * takes the streaming diagonal lowering) else 0, and for a diagonal block
 * the fraction of the state its sweeps visit and its launch count / 16
 * (dense blocks: 1 and 1/16).  swept_fraction in [0, 1], launches in
 * [0, 64] (see sv_diag_sweep_cost).  Errors: SV_ERR_ARG (k outside [1, 7],
 * ranges).
 */
int sv_cost_features(int n_qubits, int k, const int32_t *phys_targets, int diagonal, double swept_fraction,
                     int launches, float *out);

/*
 * What the streaming diagonal lowering sweeps for a diagonal operator (host
 * only, no GPU): diag = its 2^k entries, complex128 interleaved, entry r for
 * the basis state whose bit j is the bit at physical position
 * phys_targets[j].  Entries exactly 1 + 0i need no visit; the exact minimum
 * cover by subcubes (target bits at position 4 or above held fixed, at most
 * 16 sweeps) gives *fraction, the share of the state visited, and
 * *launches, the partial sweeps run (0 and 0 for the identity).  The same
 * cover sv_apply_fused uses.  Errors: SV_ERR_ARG (k outside [1, 8],
 * positions outside [0, 64) or repeated).
 */
int sv_diag_sweep_cost(int k, const double *diag, const int32_t *phys_targets, double *fraction, int *launches);

/* Number of fused blocks. */
int sv_plan_num_blocks(const sv_plan *p, int *out);

/* Block i: width k, ordered logical targets (host int32[k]: k <= 8 for a fused
 * block, up to 14 for a layout-swap block; pass targets = null to read k
 * first), gate count, diagonal flag. */
int sv_plan_block_info(const sv_plan *p, int i, int *k, int32_t *targets, int *n_gates, int *diag);

/* Block i's FP64 fused matrix (2 * 4^k doubles, complex128 row-major
 * interleaved).  SV_ERR_ARG for a layout-swap block, which has none. */
int sv_plan_block_matrix(const sv_plan *p, int i, double *out);

/*
 * Layout swaps chosen by the learned cost model (an addition to the paper:
 * its placement policy, Corollary 1 and Eq. lazy-vol, decides where qubits
 * go by next use; here the model decides whether moving them pays).  The
 * pass walks the plan with the layout a run from the identity layout would
 * have (blocks that only permute qubits update it, as in sv_apply_fused).
 * Before each dense, non-permutation block it considers moving the block's
 * targets onto every window of k consecutive physical bits (each target that
 * is outside the window exchanged with the qubit on a free window bit) and
 * predicts, with the model, the time the next `horizon` blocks gain at their
 * new physical positions.  It inserts the best move as a layout-swap block
 * when that gain exceeds the predicted cost of the permutation sweeps
 * (the in-place tile passes sv_permute_layout runs for the move: up to five
 * disjoint exchanges per pass while the tile keeps physical bits 0..3; each
 * priced as a streaming sweep times SV_PLAN_SWAP_SWEEP_FACTOR) by more than
 * the factor
 * (1 + margin).  A swap block changes only where qubits are stored, never
 * the logical state.  States under SV_PLAN_SWAP_MIN_QUBITS qubits get no
 * swaps: the model was trained from 24 qubits up, and smaller states stay in
 * the caches, where the placement of target bits matters little.
 * mlp_params_host: the cost model as in sv_plan_dp.  *inserted (may be null):
 * swap blocks added.  Errors: SV_ERR_ARG.
 */
#define SV_PLAN_SWAP_SWEEP_FACTOR 1.15
#define SV_PLAN_SWAP_MIN_QUBITS 24
int sv_plan_swaps(sv_plan *p, const float *mlp_params_host, int mlp_nin, int mlp_hid, int horizon, double margin,
                  int *inserted);

/* Block i a layout-swap block?  *is_swap = 1 and dest (host int32[k], may be
 * null) holds the physical bit each of its logical targets goes to; else
 * *is_swap = 0. */
int sv_plan_block_swap(const sv_plan *p, int i, int *is_swap, int32_t *dest);

/* Apply every block in order: fused blocks through sv_apply_fused, layout-
 * swap blocks through sv_permute_layout (each listed logical qubit moved to
 * its physical bit, the qubit found there taking its old place). */
int sv_run_plan(sv_state *s, const sv_plan *p);

int sv_plan_free(sv_plan *p);

/*
 * Bound plan: every block of a plan lowered once for one state handle (its
 * current layout, options and precision), with all device operands uploaded
 * into caller memory.  A run is then a sequence of kernel launches on the
 * handle's stream with no host work or copy per block, so it can be captured
 * into a HIP graph and replayed (launch-bound circuits: small states, many
 * narrow gates).  Lazy relabel must be off; a run requires the layout map to
 * be the one the plan was bound with, and leaves it as sv_run_plan would
 * (blocks that only permute qubits go to the layout map, as in
 * sv_apply_fused), so a second run needs a reset or the original layout.
 *   sv_bound_bytes      device bytes the operands need (*out; 0 if all by value)
 *   sv_plan_bind        lower every block, copy the operands into op_dev
 *                       (caller-owned device memory, >= sv_bound_bytes,
 *                       256-B aligned; the copy completes before return)
 *   sv_bound_run        launch every block in order (asynchronous)
 *   sv_bound_graph_run  first call: capture the launches into a HIP graph on
 *                       the handle's stream and instantiate it; every call:
 *                       launch the graph (asynchronous).  The graph holds
 *                       kernel nodes only.
 *   sv_bound_free       release the host object (and the graph)
 * The bound plan keeps pointers to the handle and to op_dev: free it before
 * either.  Errors: SV_ERR_ARG (relabel on, buffer too small or misaligned,
 * layout changed since binding), SV_ERR_UNSUPPORTED (a plan with layout-swap
 * blocks: run it with sv_run_plan), SV_ERR_DEVICE.
 */
typedef struct sv_bound sv_bound;
int sv_bound_bytes(sv_state *s, const sv_plan *p, size_t *out);
int sv_plan_bind(sv_state *s, const sv_plan *p, void *op_dev, size_t op_bytes, sv_bound **out);
int sv_bound_run(sv_bound *b);
int sv_bound_graph_run(sv_bound *b);
int sv_bound_free(sv_bound *b);

#ifdef __cplusplus
}
#endif
#endif /* SV_PLAN_H_ */
