// Learned preconditioner (kc_nn.hip): network state and launchers.
#pragma once

#include "kc_state.h"

namespace kc {

constexpr int NN_CIN = 15;   // 9 inverse-permittivity channels, log E0 (3), k/pi (3)
constexpr int NN_CH = 32;    // hidden channels
constexpr int NN_COUT = 3;   // log-multipliers of the three components of E0

struct Net {
  DevBuf params, grads, adam_m, adam_v;  // FP32 master, [W1 b1 W2 b2 W3 b3], W[co][ci][27]
  DevBuf wt[3], wb[3], bpad[3];          // BF16 packed forward / backward-data weights, biases
  DevBuf h1, h2, out, g1, g2, g3, gpad, wpart, lpart;
  DevBuf feat;
  int step = 0;
};

size_t nn_param_count();
int nn_init(Net* net, uint64_t seed);
int nn_pack(Net* net, hipStream_t s);
int nn_forward(Net* net, int N, int batch, const uint16_t* in, float* out, hipStream_t s);
// MSE loss against target (f32 [batch][N^3][16]) and its parameter gradients (in net->grads)
int nn_gradients(Net* net, int N, int batch, const uint16_t* in, const float* target, double* loss_host,
                 hipStream_t s);
// parameter gradients (in net->grads) for a given gradient of the output (f32 [batch][N^3][16])
int nn_backward(Net* net, int N, int batch, const uint16_t* in, const float* gout, hipStream_t s);
int nn_adam(Net* net, float lr, float b1, float b2, float eps, hipStream_t s);
int nn_features(kc_op* op, int ik0, int nk, uint16_t* F, hipStream_t s);
// learned fields E (f32 [nk][3][N^3]) and, with Et != nullptr, their x-major copy ([nk][3][x][z][y])
int nn_efield(kc_op* op, int ik0, int nk, float* E, hipStream_t s, float* Et = nullptr);
// the learned fields of k-points ik0 .. ik0+nk-1 into op->efield_k and op->efield_kt
int learned_fields(kc_op* op, int ik0, int nk, hipStream_t s);
int nn_build_eps_features(kc_op* op);

}  // namespace kc
