// ffmg_learned.hpp -- layout of the learned smoother's weights and the
// launchers of its kernels (ffmg_learned.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "ffmg_device.hpp"

namespace ffmg {

// Complex weights, (tap, out, in) with the input channel fastest:
// W1 [9][16][2], W2 [9][16][16], W3 [9][1][16].
constexpr int NET_W1 = 0;
constexpr int NET_W2 = NET_W1 + 9 * 16 * 2;
constexpr int NET_W3 = NET_W2 + 9 * 16 * 16;
constexpr int NET_NW = NET_W3 + 9 * 16;   // 2736

size_t train_lds_bytes();
void launch_train_patches(const float2 *rt, const float2 *kt, const float2 *et, const float2 *Wq, float2 *dW_part,
                          float *loss_part, int count, int border, hipStream_t s);
void launch_reduce_grads(const float2 *dW_part, int count, float2 *grad, const float *loss_part, float *loss,
                         hipStream_t s);
void launch_adam(float2 *Wm, float2 *Wq, const float2 *grad, float2 *m, float2 *v, float lr, float b1, float b2,
                 float eps, int step, hipStream_t s);
void launch_round_weights(const float2 *Wm, float2 *Wq, hipStream_t s);

// inference: u += h^2 N(r, kappa h^2)  (= s h^2 N(r / s, kappa h^2), N being linear in r)
void pack_net_mfma(const float *w, unsigned short *out);      // w: interleaved complex weights
size_t net_mfma_frag_count();                                  // BF16 values written by pack_net_mfma
void launch_kappa_h2(const cx<double> *q, double k02, double h2, size_t N, unsigned *out, hipStream_t s);
void launch_net_apply(const cx<double> *r, const unsigned *kh2, cx<double> *u, int mx, int my,
                      const unsigned short *wfrag, double h2, hipStream_t st, const int *stop);

}  // namespace ffmg
