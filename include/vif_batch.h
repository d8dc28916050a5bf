/* vif_batch.h -- many likelihood evaluations in one enqueue (C ABI of libvif.so).
 *
 * The paper's estimator evaluates the Vecchia / VIF likelihood many times, for
 * many hyperparameter settings (Sec. "Estimation and prediction"); this
 * interface evaluates a set of independent problems -- uneven n, ragged early
 * neighbor rows, different m, k and kernels -- as one device workload:
 *
 *   * vif_batch_create plans the batch: it validates every problem (reading
 *     each problem's bounding box and time span, so it synchronises the
 *     stream), fixes each problem's slice of one caller-owned workspace, and
 *     precomputes every host-side quantity of the evaluation;
 *   * vif_batch_enqueue then enqueues all evaluations with no host
 *     synchronisation, no allocation and no host-to-device copy, so it can be
 *     captured in a HIP graph; problems are spread over `streams` forked
 *     streams joined back to the caller's stream;
 *   * vif_batch_graph_launch captures that enqueue once into a HIP graph (for a
 *     given workspace and output pointer) and launches the graph;
 *   * vif_batch_autotune times the candidate schedules (number of streams, and
 *     rows per FP32 partial of the Woodbury Gram) on the batch itself, keeps
 *     the fastest and drops any captured graph.
 *
 * Arrays are DEVICE pointers owned by the caller and must stay valid while the
 * batch (or its graph) is used. Results are written to nll [count] (device);
 * failures (non-positive-definite blocks, invalid neighbor rows) are recorded
 * on the device and read back by vif_batch_status.
 */
#ifndef VIF_BATCH_H
#define VIF_BATCH_H

#include <stddef.h>
#include <stdint.h>

#include "vif.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  vif_points points;    /* n points, SoA, time-ordered as for vif_nll */
  const double* y;      /* [n] */
  vif_kernel kern;      /* hyperparameters (host struct, copied at creation) */
  int32_t m;            /* neighbors per point (<= VIF_MAX_M) */
  const int32_t* nbr;   /* [n, m] neighbor rows, e.g. from vif_neighbors */
  vif_points ind;       /* inducing points; ind.n = 0 for plain Vecchia */
} vif_problem;

typedef struct vif_batch vif_batch; /* opaque plan (host memory) */

/* Plans `count` problems evaluated in precision `prec` (VIF_PREC_*). scratch:
 * device buffer of at least VIF_BATCH_PLAN_SCRATCH bytes, 256-byte aligned,
 * used only during the call (bounding boxes and time checks of problems with
 * inducing points). Returns NULL on error (vif_last_error() says why).
 * Synchronises the stream; creates the side streams (default priority) and
 * events that vif_batch_destroy releases. */
#define VIF_BATCH_PLAN_SCRATCH 16384
vif_batch* vif_batch_create(const vif_problem* problems, int32_t count, int32_t prec,
                            void* scratch, size_t scratch_bytes, void* hip_stream);

/* Workspace bytes the batch needs (one caller-owned device buffer, 256-byte
 * aligned); each problem owns a slice, so problems can run concurrently. */
size_t vif_batch_workspace_bytes(const vif_batch* batch);

/* Enqueues every problem's NLL on the caller's stream; nll: device [count].
 * Problems are taken in the order given and dealt round-robin to the forked
 * streams when the schedule has more than one. Two enqueues of one batch on
 * different streams, or overlapping in time, race on the workspace. */
int32_t vif_batch_enqueue(vif_batch* batch, void* ws, size_t ws_bytes, double* nll,
                          void* hip_stream);

/* As vif_batch_enqueue, through a HIP graph captured on the first call (and
 * again whenever ws, nll or the schedule change). Capture runs on a stream the
 * batch owns, so the caller's stream may be the null stream; the graph is
 * launched on the caller's stream. */
int32_t vif_batch_graph_launch(vif_batch* batch, void* ws, size_t ws_bytes, double* nll,
                               void* hip_stream);

/* Picks the fastest schedule by timing `reps` graph launches of each candidate;
 * *best_ms (HOST, may be NULL) receives its time per batch. */
int32_t vif_batch_autotune(vif_batch* batch, void* ws, size_t ws_bytes, double* nll, int32_t reps,
                           double* best_ms, void* hip_stream);

/* Current schedule: *streams and *chunk_rows (HOST). */
int32_t vif_batch_schedule(const vif_batch* batch, int32_t* streams, int32_t* chunk_rows);

/* Sets the schedule: streams in 1 .. 4; chunk_rows, the rows summed in FP32
 * per partial of the split-BF16 Woodbury Gram (FP64 and FP32 evaluations
 * ignore it), a multiple of 8 in 1024 .. 65536. Drops any captured graph. The
 * default is one stream and 4096 rows, the schedule of vif_nll, whose results
 * it reproduces bit for bit. */
int32_t vif_batch_set_schedule(vif_batch* batch, int32_t streams, int32_t chunk_rows);

/* Per-problem status of the last evaluation (VIF_OK or VIF_E_*), HOST [count].
 * Synchronises the stream. Returns the first failing status, or VIF_OK. */
int32_t vif_batch_status(vif_batch* batch, void* ws, int32_t* status, void* hip_stream);

void vif_batch_destroy(vif_batch* batch);

#ifdef __cplusplus
}
#endif

#endif /* VIF_BATCH_H */
