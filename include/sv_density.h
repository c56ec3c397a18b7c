/*
 * libsv density matrices: the paper's density-matrix wrapper over the same
 * fused-operator interface (Section IV-B, the vectorised density matrix).
 *
 * An N-qubit density matrix rho (2^N x 2^N) is held as the complex64 vector
 * vec(rho) of 2N logical qubits, stacked column by column: vector index
 * x = row + 2^N * column, so logical qubits 0..N-1 select the row and
 * N..2N-1 the column.  A channel with Kraus operators E_1..E_R on the ordered
 * targets V = (q_0..q_{k-1}) maps rho to sum_i E_i rho E_i^dagger; on the
 * vector that is the 2k-target operator S = sum_i conj(E_i) (x) E_i applied
 * with sv_apply_fused to the targets (q_0..q_{k-1}, q_0+N..q_{k-1}+N): row
 * copies first, each group in target order, E_i on the lower (row) bits and
 * its conjugate on the higher (column) bits.  S is built once per channel on
 * the host in FP64 (Theta(R * 16^k)).
 *
 * A density-matrix handle is an sv_state of 2N qubits, so every call of
 * sv.h applies to it as well: sv_apply_fused (a raw 2N-qubit operator),
 * sv_permute_layout and sv_get_layout (the layout of the 2N vector qubits),
 * sv_run_plan of a plan built over superoperators on 2N qubits, and sv_norm,
 * which returns sum |rho_ij|^2 = Tr(rho^dagger rho) (the purity for a
 * Hermitian rho).  sv_probs and sv_sample on it would treat vec(rho) as a
 * pure state; the calls below give the measurement distribution instead.
 *
 * The paper's engine range for density matrices is 2 <= N <= 17 (Appendix C-A, engine table); a
 * 17-qubit density matrix takes 8 * 4^17 B = 128 GiB.
 */
#ifndef SV_DENSITY_H_
#define SV_DENSITY_H_

#include "sv.h"

#ifdef __cplusplus
extern "C" {
#endif

#define SV_DM_MIN_QUBITS 2
#define SV_DM_MAX_QUBITS 17
#define SV_DM_MAX_K 4 /* a channel's 2k-target superoperator must fit a fused gate (2k <= SV_MAX_K) */

/* Bytes of vec(rho) (8 * 4^N) and of the workspace for an N-qubit density matrix; 0 outside the range. */
size_t sv_dm_state_bytes(int n_qubits);
size_t sv_dm_workspace_bytes(int n_qubits);

/*
 * A density-matrix handle for N qubits over caller-owned device memory
 * (amps_dev >= sv_dm_state_bytes(N), ws_dev >= sv_dm_workspace_bytes(N),
 * both 256-byte aligned), initialised to rho = |0..0><0..0| with the identity
 * layout.  Release with sv_free.  Errors: SV_ERR_ARG (N outside
 * [SV_DM_MIN_QUBITS, SV_DM_MAX_QUBITS], null or small buffers), SV_ERR_DEVICE.
 */
int sv_dm_alloc(sv_state **out, int n_qubits, void *amps_dev, size_t amps_bytes, void *ws_dev, size_t ws_bytes,
                void *stream);

/* N for a density-matrix handle, 0 for a plain state vector, negative on a null handle. */
int sv_dm_qubits(const sv_state *s);

/*
 * Host only: the superoperator S = sum_i conj(E_i) (x) E_i of a k-qubit
 * channel, 4^k x 4^k complex128 row-major interleaved into out (caller-owned,
 * 2 * 16^k doubles).  kraus: n_kraus matrices of 2^k x 2^k complex128,
 * row-major interleaved, back to back.  Row index r = r_row + 2^k r_col:
 * S[r][c] = sum_i E_i[r_row][c_row] * conj(E_i[r_col][c_col]).
 * Errors: SV_ERR_ARG (k outside [1, SV_DM_MAX_K], n_kraus < 1, null).
 */
int sv_dm_superop(const double *kraus, int n_kraus, int k, double *out);

/*
 * rho <- sum_i E_i rho E_i^dagger on the ordered logical targets (k distinct
 * qubits in [0, N)).  The Kraus operators are copied before return; the
 * sweep is asynchronous on the handle's stream.  Completeness
 * (sum E_i^dagger E_i = I) is not checked: any operator sum is applied as
 * given.  Errors: SV_ERR_ARG (not a density-matrix handle, k, targets,
 * n_kraus, null), and those of sv_apply_fused.
 */
int sv_dm_apply_channel(sv_state *s, const double *kraus, int n_kraus, const int32_t *targets, int k);

/*
 * Outcome probabilities of a computational-basis measurement, p_x = Re rho_xx
 * in FP64, into device out_dev[2^N], indexed by the logical basis index x
 * (the diagonal entries are read through the layout map).  A negative entry
 * (FP32 rounding of a zero population) is returned as 0.  Asynchronous.
 */
int sv_dm_probs(sv_state *s, double *out_dev);

/* Tr(rho) = sum_x Re rho_xx accumulated in FP64 into *out_host.  Synchronises the stream. */
int sv_dm_trace(sv_state *s, double *out_host);

/*
 * Draw `shots` measurement outcomes from the diagonal of rho with the
 * sampler of sv_sample (exact integer CDF, Philox4x32-10 with key = seed and
 * counter = shot index, strict upper bound).  probs_dev: caller-owned device
 * scratch of 2^N doubles that receives sv_dm_probs.  Bit q of out_host[s] is
 * qubit q.  Synchronises the stream.  Errors: as sv_sample; SV_ERR_STATE if
 * the diagonal has no positive entry.
 */
int sv_dm_sample(sv_state *s, uint64_t seed, int64_t shots, uint64_t *out_host, double *probs_dev);

#ifdef __cplusplus
}
#endif

#endif /* SV_DENSITY_H_ */
