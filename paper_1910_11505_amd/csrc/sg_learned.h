// Pieces of the learned stage's own training objective shared by the CNN
// (sg_cnn.hip) and the C ABI entry that evaluates it (sg_api.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

struct sg_cnn;

namespace sg {

// batch slot of the last forward's output as an SG vector (no scaling)
void cnn_slot_to_sg(sg_cnn* C, hipStream_t s, int slot, double* c);
// a stored pair's bf16 residual as an FP64 SG vector
void cnn_pair_to_sg(sg_cnn* C, hipStream_t s, const uint16_t* R, int64_t pair, double* r);
// a slot's output gradient scale[0] g (g an SG vector) written into the network
void cnn_slot_grad_from_sg(sg_cnn* C, hipStream_t s, int slot, const double* g,
                           const double* scale);
int cnn_max_batch(const sg_cnn* C);
// dots = (a, b, rho) = (r.Kc, Kc.Kc, r.r) -> dots[3] = a / b, dots[4] =
// 2 a / (rho b batch), dots[5] = 1 - a^2 / (rho b) (all zero when b or rho is
// zero), then v = dots[3] Kc - r
void launch_stage_objective(hipStream_t s, double* dots, int batch, const double* Kc,
                            const double* r, double* v, int64_t N);

}  // namespace sg
