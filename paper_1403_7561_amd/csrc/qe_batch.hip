// Batched sweep entry points (persistent-kernel implementation pending).
#include "qe_runtime.h"

extern "C" {

size_t qe_batch_workspace_bytes(int32_t n_inst, const qe_problem* probs, const qe_options* o) {
  (void)n_inst;
  (void)probs;
  (void)o;
  return 0;
}

qe_status qe_solve_batch(int32_t n_inst, const qe_problem* probs, const qe_physics* ph, const qe_options* o,
                         double* const* phi, int32_t n_boxes, const double* boxes, double* counts,
                         const char* tune_cache, void* ws, size_t ws_bytes, void* stream, qe_report* reps) {
  (void)n_inst; (void)probs; (void)ph; (void)o; (void)phi; (void)n_boxes; (void)boxes; (void)counts;
  (void)tune_cache; (void)ws; (void)ws_bytes; (void)stream; (void)reps;
  return qe::fail(QE_ERR_INVALID_ARG, "batched solve not available in this build");
}
}
