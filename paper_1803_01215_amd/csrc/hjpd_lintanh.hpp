// Linear-tanh family with quadratic initial cost (differentiation workload):
// forward PDHG with the dense linear terms A x_j and A^T p_j evaluated as
// matrix-core GEMMs over (points x nodes), and the reverse sweep for
// hjpd_value_grad.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/hjpd.h"

namespace hjpd {

constexpr int kLtMaxD = 128;
constexpr int kLtMaxN = 64;

struct LtState;

int lt_create(LtState** out, const hjpd_desc& d);
void lt_destroy(LtState* s);
int lt_solve(LtState* st, const hjpd_desc& d, int64_t n, const void* x, const void* t, const int32_t* N,
             const void* hp, const void* gp, void* phi, void* xtraj, void* ptraj, int32_t* iters, int32_t* status,
             hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, int* launches, bool* timing_valid);
int lt_value_grad(LtState* st, const hjpd_desc& d, int64_t n, const void* x, const void* t, const int32_t* N,
                  const void* hp, const void* gp, const void* grad_phi, int K_iters, int ckpt_every, void* phi,
                  void* dphi_dx, void* dh, void* dg, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, int* launches,
                  bool* timing_valid);

}  // namespace hjpd

int hjpd_fail(int code, const char* msg);
