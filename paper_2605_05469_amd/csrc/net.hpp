// net.hpp -- the learned preconditioner's network: kernel launchers and the
// host-side network object (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pic {
namespace net {

// ---- kernel launchers (net_kernels.hip) ---------------------------------
size_t frag_elems(int cin, int cout);
hipError_t pack(const float* W, int ci, int co, int bwd, uint16_t* frag, hipStream_t s);
hipError_t conv_fwd(int n, int ci, int co, const uint16_t* X, const uint16_t* frag,
                    const float* bias, const uint16_t* skip, int relu, uint16_t* Y, hipStream_t s);
// Y = conv(up(Xc)) with Xc on the n/2 grid, up = nearest-neighbour 2x
// up-sampling applied while staging (z-marching kernel only).
bool conv_up_fused(int n, int ci, int co);
// Y = relu(conv(X) + b) and Yp = avgpool2(Y) (BF16) in one pass (z-marching
// kernel, 32->32, grids that are multiples of 64).
bool conv_pool_fused(int n, int ci, int co);
hipError_t conv_fwd_pool(int n, int ci, int co, const uint16_t* X, const uint16_t* frag,
                         const float* bias, uint16_t* Y, uint16_t* Yp, hipStream_t s);
hipError_t conv_fwd_up(int n, int ci, int co, const uint16_t* Xc, const uint16_t* frag,
                       const float* bias, const uint16_t* skip, int relu, uint16_t* Y,
                       hipStream_t s);
hipError_t conv_bwd_data(int n, int ci, int co, const uint16_t* G, const uint16_t* frag_bwd,
                         float* dX, int accumulate, hipStream_t s);
hipError_t conv_dw(int n, int ci, int co, const uint16_t* X, const uint16_t* G, float* part,
                   float* grad, hipStream_t s);
size_t dw_part_elems(int n, int ci, int co);
hipError_t conv_in_fwd(int n, const uint16_t* x, const float* W, const float* b, uint16_t* y,
                       hipStream_t s);
hipError_t conv_out_fwd(int n, const uint16_t* a, const float* W, const float* b, float* o,
                        hipStream_t s);
hipError_t conv_out_bwd(int n, const uint16_t* g, const float* W, float* da, int accumulate,
                        hipStream_t s);
hipError_t conv_dw_small(int n, int ci, int co, const uint16_t* X, const uint16_t* G, float* part,
                         float* grad, hipStream_t s);
hipError_t pool_fwd(int m, int C, const uint16_t* x, uint16_t* y, hipStream_t s);
hipError_t pool_bwd(int n, int C, const float* gy, float* gx, int accumulate, hipStream_t s);
hipError_t up_fwd(int n, int C, const uint16_t* x, uint16_t* y, hipStream_t s);
hipError_t up_bwd(int m, int C, const float* gy, float* gx, hipStream_t s);
hipError_t grad_round(int64_t count, const float* g, const uint16_t* act, uint16_t* out,
                      hipStream_t s);
hipError_t add_bf16(int64_t count, const uint16_t* a, float* g, hipStream_t s);
hipError_t to_bf16(int64_t count, const float* a, uint16_t* out, hipStream_t s);
int loss_parts(int n);
// Scale-free training pair: u = h2 (b - bp), e = phi - pp (bp, pp may be NULL),
// rhs = u / rms(u), tgt = e / rms(u) in FP32; s_out = rms(u) (device).
hipError_t scale_pair(int64_t n3, const double* b, const double* bp, const double* phi,
                      const double* pp, double h2, double* part, double* s_out, float* rhs,
                      float* tgt, hipStream_t s);
hipError_t loss_norms(int n, const float* t, const float* r, double* part, hipStream_t s);
hipError_t loss_pass1(int n, const float* o, const float* t, const float* r, float* d2,
                      double* part, hipStream_t s);
hipError_t loss_pass2(int n, const float* o, const float* t, const float* d2,
                      const double* norm_part, double lam, uint16_t* gout, hipStream_t s);
hipError_t adam(int64_t len, float* th, float* m, float* v, const float* g, float lr, float b1,
                float b2, float eps, int step, hipStream_t s);
int pre_parts(int64_t n3);
hipError_t prep_input(int64_t n3, const double* r, double h2, double* part, double* s_out,
                      uint16_t* x, hipStream_t s);
hipError_t post_output(int64_t n3, const float* o, const double* s_in, double* z, double* part,
                       hipStream_t s);

// ---- the network -----------------------------------------------------------
// Three levels, channels c1 = 16, c2 = 32, c3 = 64; layer order and canonical
// parameter layout ([co][ci][27] weights then [co] bias per layer):
//   e1a 1->16, e1b 16->16, e2a 16->32, e2b 32->32, b3a 32->64, b3b 64->32,
//   d2a 32->32, d2b 32->16, d1a 16->16, out 16->1.
constexpr int kLayers = 10;
int64_t param_count();

struct Net;
// Buffers for grid size n (n a multiple of 16); training adds gradients.
int create(Net** out, int n, bool training);
void destroy(Net* net);
const char* last_error();
int grid(const Net* net);
// Load FP32 parameters (device, canonical layout) and pack BF16 fragments.
int set_params(Net* net, const float* params, hipStream_t s);
int get_params(const Net* net, float* params, hipStream_t s);
// out (FP32, n^3) = NN(x) for x (FP32, n^3, rounded to BF16 on entry).
int forward_f32(Net* net, const float* x, float* out, hipStream_t s);
// Gradients (FP32, canonical layout) of sum(out * dout) after forward_f32.
int backward(Net* net, const float* dout, float* grads, hipStream_t s);
// z = s * NN(h^2 r / s) - mean, s = rms(h^2 r): the preconditioner.
int precondition(Net* net, const double* r, double h2, double* z, hipStream_t s);
// Loss of one (rhs, target) pair without an update (training buffers needed).
int eval_loss(Net* net, const float* rhs, const float* target, double lam, double* loss,
              hipStream_t s);
// A scale-free training pair from (b, phi) or from differences to (bp, pp).
int make_pair(Net* net, const double* b, const double* bp, const double* phi, const double* pp,
              double h2, float* rhs, float* tgt, double* scale, hipStream_t s);
// One Adam step on the loss of one (rhs, target) pair; loss (host) optional.
int train_step(Net* net, const float* rhs, const float* target, double lam, double lr,
               double* loss, hipStream_t s);

}  // namespace net
}  // namespace pic
