/*
 * libsv batched path: many small independent circuits in one persistent
 * kernel launch (an addition to the paper's method, which applies one state
 * at a time through the fused-operator interface of Section III R2; the gate
 * semantics are the same).
 *
 * A circuit is a list of single-qubit gates (2x2 complex128 matrix, row-major
 * interleaved) and CNOT gates (control, target) on n <= 18 qubits, applied to
 * |0...0>.  Consecutive single-qubit gates on the same qubit are multiplied
 * on the host in FP64 (later gate on the left, Section IV-C) before launch.
 * Circuits with the same qubit count and the same gate structure (kinds and
 * qubits, angles free) are grouped into packs of P that one workgroup runs in
 * lockstep; P per qubit count comes from sv_batch_autotune or the caller.
 * States of at most 2^14 amplitudes per pack slice stay in LDS for the whole
 * circuit.  Larger states live in the caller's state buffer and run as
 * passes: each pass streams every 2^14-amplitude slice of a chosen set of 14
 * qubits through LDS and applies there every gate that acts only on them.
 * Workgroups take packs from an atomic queue ordered by decreasing cost and
 * exit when the queue is empty.
 */
#ifndef SV_BATCH_H_
#define SV_BATCH_H_

#include "sv.h"

#ifdef __cplusplus
extern "C" {
#endif

#define SV_BATCH_MAX_QUBITS 18
#define SV_BATCH_GATE_1Q 0
#define SV_BATCH_GATE_CNOT 1

typedef struct sv_batch_circuit {
  int32_t n_qubits;     /* 1 .. SV_BATCH_MAX_QUBITS */
  int32_t n_gates;
  const int32_t *kinds;  /* n_gates entries: SV_BATCH_GATE_* */
  const int32_t *qubits; /* 2 * n_gates entries: (q, unused) or (control, target) */
  const double *mats;    /* 8 * n_gates doubles: 2x2 complex128 for 1q gates (ignored for CNOT) */
} sv_batch_circuit;

/* Per-qubit-count pack sizes: config[n] = circuits per workgroup for n qubits
 * (a power of two, 1 <= config[n] <= 16, and config[n] * 2^n <= 2^14 when the
 * state is to stay in LDS; larger n must use 1).  Index 0 is unused. */
#define SV_BATCH_CONFIG_LEN (SV_BATCH_MAX_QUBITS + 1)

/* Device workspace bytes for a batch (gate records, pack table, queue). */
size_t sv_batch_workspace_bytes(int count, const sv_batch_circuit *circs);

/*
 * Run `count` circuits.  states_dev: device complex64 buffer of states_bytes
 * bytes receiving every final state (circuit i at byte offset
 * state_offsets[i], a host int64 array of multiples of 8; its 8 * 2^n_i bytes
 * must lie inside the buffer; slices must not overlap).  z0_host:
 * receives <Z_0> = sum_x |psi_x|^2 (1 - 2 x_0) per circuit, accumulated in
 * FP64.  config: pack sizes (NULL = defaults).  Synchronises `stream`.
 * The host pass over the circuits (validation, fusion of single-qubit runs,
 * slice passes) runs on up to 16 threads of the calling process; the first
 * bad circuit by index is the one reported.  Errors: SV_ERR_ARG (bad circuit
 * or config, workspace too small), SV_ERR_DEVICE.
 */
int sv_batch_run(int count, const sv_batch_circuit *circs, void *states_dev, size_t states_bytes,
                 const int64_t *state_offsets, double *z0_host, const int32_t *config, void *ws_dev, size_t ws_bytes,
                 void *stream);

/*
 * The same launch split in two, so that repeated runs of one batch (new
 * states each time, same circuits) do no host work: sv_batch_prepare packs
 * the circuits on the host and copies the records into ws_dev (complete
 * before return); sv_batch_launch resets the queue, runs the persistent
 * kernel on `stream` and, if z0_host is not NULL, copies <Z_0> per circuit
 * there and synchronises.  The prepared object refers to ws_dev and the
 * state offsets given at preparation: keep ws_dev alive and unchanged.
 */
typedef struct sv_batch_prepared sv_batch_prepared;
int sv_batch_prepare(int count, const sv_batch_circuit *circs, size_t states_bytes, const int64_t *state_offsets,
                     const int32_t *config, void *ws_dev, size_t ws_bytes, void *stream, sv_batch_prepared **out);
int sv_batch_launch(sv_batch_prepared *p, void *states_dev, double *z0_host, void *stream);
int sv_batch_prepared_free(sv_batch_prepared *p);

/*
 * Host only (no GPU): the gate records the batched kernel runs for one
 * circuit, after the host fuses adjacent single-qubit gates and, for more
 * than 2^14 amplitudes, cuts the circuit into LDS slice passes.  Each record
 * is 4 int32 (kind, q0, q1, unused) plus 8 floats:
 *   kind SV_BATCH_GATE_1Q   q0 = qubit, floats = 2x2 complex64 row-major
 *   kind SV_BATCH_GATE_CNOT q0 = control, q1 = target
 *   kind SV_BATCH_PASS      q0 = bit mask of the 14 slice qubits, q1 = number
 *                           of following records in the pass; their qubit
 *                           numbers are slice bit positions (rank of the qubit
 *                           in the mask)
 *   kind SV_BATCH_GATE_GROUP q0 = c (2..5): the next c records are
 *                           single-qubit gates on distinct qubits that the
 *                           kernel applies in one sweep (runs of consecutive
 *                           single-qubit records, grouped by the host)
 *   kind SV_BATCH_GATE_LINEAR (only inside passes) a run of q0 >= 3
 *                           consecutive CNOTs as one linear map f on the 14
 *                           slice bits: the slice becomes new[y] = old[f(y)],
 *                           f(y) the XOR of mask[b] over the set bits b of y;
 *                           masks 0..7 are the 8 float slots of this record
 *                           and masks 8..13 the first 6 of the next record
 *                           (kind SV_BATCH_GATE_LINEAR, q0 = -1), as int32
 *                           bit patterns
 * records: int32[4 * cap], mats: float[8 * cap]; *n_out = records written.
 * cap >= 3 * c->n_gates always suffices.  Errors: SV_ERR_ARG (bad circuit,
 * cap too small).
 */
#define SV_BATCH_PASS 2
#define SV_BATCH_GATE_GROUP 3
#define SV_BATCH_GATE_LINEAR 4
int sv_batch_records(const sv_batch_circuit *c, int cap, int32_t *records, float *mats, int *n_out);

/*
 * Pick config[n] for every qubit count present in the batch: a tuning subset
 * of up to `sample_per_size` circuits of every size is run as one launch
 * (hipEvent timing after one warm-up), starting from the default pack sizes,
 * and each size's pack size is varied in turn over the powers of two that
 * fit in LDS, keeping a change when the whole launch gets faster
 * (coordinate descent).  Writes SV_BATCH_CONFIG_LEN entries to config_out
 * and, if times_out is not NULL, the subset's launch time in seconds after
 * each size was tuned.  Uses states_dev / ws_dev like sv_batch_run.
 */
int sv_batch_autotune(int count, const sv_batch_circuit *circs, void *states_dev, size_t states_bytes,
                      const int64_t *state_offsets, int sample_per_size, int32_t *config_out, double *times_out,
                      void *ws_dev, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SV_BATCH_H_ */
