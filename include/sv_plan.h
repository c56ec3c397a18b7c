/*
 * libsv fusion planning: turn an ordered gate list into fused blocks.
 *
 * Fusion replaces consecutive gates by their matrix product (Section IV-C):
 * within a block matrices stay in circuit order with later gates multiplied
 * on the left; a block is diagonal when every constituent gate is.  Products
 * are formed on the host in FP64.
 *
 * Gate lists are passed flat:
 *   ks[i]        width of gate i (1..8)
 *   targets      concatenated ordered logical targets (sum ks entries)
 *   mats         concatenated complex128 row-major interleaved matrices
 *                (2 * 4^ks[i] doubles each), little-endian in the targets
 *   diag         optional (may be NULL) per-gate flag: 1 if the matrix is diagonal
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

/* Number of fused blocks. */
int sv_plan_num_blocks(const sv_plan *p, int *out);

/* Block i: width, ordered logical targets (host int32[8]), gate count, diagonal flag. */
int sv_plan_block_info(const sv_plan *p, int i, int *k, int32_t *targets, int *n_gates, int *diag);

/* Block i's FP64 fused matrix (2 * 4^k doubles, complex128 row-major interleaved). */
int sv_plan_block_matrix(const sv_plan *p, int i, double *out);

/* Apply every block in order through sv_apply_fused. */
int sv_run_plan(sv_state *s, const sv_plan *p);

int sv_plan_free(sv_plan *p);

#ifdef __cplusplus
}
#endif
#endif /* SV_PLAN_H_ */
