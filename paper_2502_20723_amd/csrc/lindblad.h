// Device-side model description and launchers for the Lindbladian rows,
// the local estimator and the FP64 sample reductions.
#pragma once

#include "common.h"

namespace tdo {

struct ModelDev {
  int kind, n, nslots, has_fields;
  int gamma_ok, hmove_eq, hmove_ne;
  int rows, cols;  // rows = 1: chain; otherwise an M x C periodic lattice, row-major
  double gam, gam2, V4, g2, Jz, jm, jp, Bx, By, Bz;
  // lattice masks: sites in the last column, the other sites, the first column,
  // and the first row
  uint64_t h_last, h_keep, h_first, low_cols;
};

int32_t make_model(const tdo_model_t* m, ModelDev* out);

int32_t launch_connected(const ModelDev& m, const uint64_t* cfg, int64_t B, int kmax, uint64_t* conn,
                         float* mel, int32_t* n_conn, hipStream_t st);
int32_t launch_eval_list(const ModelDev& m, const uint64_t* cfg, int64_t B, int32_t* cnt, int64_t* off,
                         int64_t* total, uint64_t* ecfg, float* ecoef, int32_t* eowner, hipStream_t st);
int32_t launch_lloc_fixed(int64_t B, const float* lrx, const float* mel, const int32_t* ncon, int kmax,
                          const float* lrc, float* out, hipStream_t st);
int32_t launch_lloc_eval(int64_t B, const int64_t* off, const int32_t* cnt, const float* ecoef,
                         const float* elr, float* out, hipStream_t st);
// acc[0] += sum_b w_b |L_b|^2, acc[1] += sum_b w_b (w may be NULL = 1); part: >= 2*512 doubles.
int32_t launch_loss_accum(int64_t B, const float* L, const double* w, double* part, double* acc,
                          hipStream_t st);

constexpr int LOSS_PARTS = 512;

}  // namespace tdo
