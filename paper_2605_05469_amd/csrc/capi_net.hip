// capi_net.hip -- C ABI of the network pieces: standalone network (training,
// single use) and the single-layer convolution / Adam primitives.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <string>

#include "../../include/pic.h"
#include "net.hpp"

using namespace pic;

extern "C" int pic_set_error_(int code, const char* msg);  // defined in capi.hip

struct pic_net {
    net::Net* n = nullptr;
};

static int nfail(int code) { return pic_set_error_(code, net::last_error()); }

static bool pair_ok(int ci, int co) {
    return (ci == 16 && co == 16) || (ci == 16 && co == 32) || (ci == 32 && co == 32) ||
           (ci == 32 && co == 64) || (ci == 64 && co == 32) || (ci == 32 && co == 16);
}

static int hchk(hipError_t e, const char* what) {
    if (e == hipSuccess) return PIC_OK;
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return pic_set_error_(PIC_ERR_HIP, m.c_str());
}

extern "C" {

int64_t pic_unet_param_count(void) { return net::param_count(); }

int pic_net_create(int32_t n, int32_t training, pic_net** out) {
    if (!out) return pic_set_error_(PIC_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (n < 16 || n > 1024 || n % 16 != 0)
        return pic_set_error_(PIC_ERR_INVALID, "network grid must be a multiple of 16 in [16, 1024]");
    pic_net* w = new pic_net();
    const int rc = net::create(&w->n, n, training != 0);
    if (rc) {
        delete w;
        return nfail(rc == -3 ? PIC_ERR_NOMEM : PIC_ERR_HIP);
    }
    *out = w;
    return PIC_OK;
}

int pic_net_destroy(pic_net* w) {
    if (!w) return PIC_OK;
    net::destroy(w->n);
    delete w;
    return PIC_OK;
}

#define NEEDNET(w) \
    if (!(w) || !(w)->n) return pic_set_error_(PIC_ERR_INVALID, "net is NULL")

int pic_net_set_params(pic_net* w, const float* params, void* stream) {
    NEEDNET(w);
    if (!params) return pic_set_error_(PIC_ERR_INVALID, "params is NULL");
    return net::set_params(w->n, params, (hipStream_t)stream) ? nfail(PIC_ERR_HIP) : PIC_OK;
}

int pic_net_get_params(pic_net* w, float* params, void* stream) {
    NEEDNET(w);
    if (!params) return pic_set_error_(PIC_ERR_INVALID, "params is NULL");
    return net::get_params(w->n, params, (hipStream_t)stream) ? nfail(PIC_ERR_HIP) : PIC_OK;
}

int pic_net_forward(pic_net* w, const float* x, float* out, void* stream) {
    NEEDNET(w);
    if (!x || !out) return pic_set_error_(PIC_ERR_INVALID, "x/out is NULL");
    return net::forward_f32(w->n, x, out, (hipStream_t)stream) ? nfail(PIC_ERR_HIP) : PIC_OK;
}

int pic_net_backward(pic_net* w, const float* dout, float* grads, void* stream) {
    NEEDNET(w);
    if (!dout || !grads) return pic_set_error_(PIC_ERR_INVALID, "dout/grads is NULL");
    const int rc = net::backward(w->n, dout, grads, (hipStream_t)stream);
    if (rc == -4) return nfail(PIC_ERR_STATE);
    return rc ? nfail(PIC_ERR_HIP) : PIC_OK;
}

int pic_net_train_step(pic_net* w, const float* rhs, const float* target, double lam, double lr,
                       double* loss, void* stream) {
    NEEDNET(w);
    if (!rhs || !target) return pic_set_error_(PIC_ERR_INVALID, "rhs/target is NULL");
    if (!(lr > 0.0) || !(lam >= 0.0)) return pic_set_error_(PIC_ERR_INVALID, "lr must be > 0, lam >= 0");
    const int rc = net::train_step(w->n, rhs, target, lam, lr, loss, (hipStream_t)stream);
    if (rc == -4) return nfail(PIC_ERR_STATE);
    return rc ? nfail(PIC_ERR_HIP) : PIC_OK;
}

int pic_net_loss(pic_net* w, const float* rhs, const float* target, double lam, double* loss,
                 void* stream) {
    NEEDNET(w);
    if (!rhs || !target || !loss) return pic_set_error_(PIC_ERR_INVALID, "rhs/target/loss is NULL");
    if (!(lam >= 0.0)) return pic_set_error_(PIC_ERR_INVALID, "lam must be >= 0");
    const int rc = net::eval_loss(w->n, rhs, target, lam, loss, (hipStream_t)stream);
    if (rc == -4) return nfail(PIC_ERR_STATE);
    return rc ? nfail(PIC_ERR_HIP) : PIC_OK;
}

int pic_net_make_pair(pic_net* w, const double* rho, const double* phi, const double* rho_prev,
                      const double* phi_prev, double h, float* rhs, float* target, double* scale,
                      void* stream) {
    NEEDNET(w);
    if (!rho || !phi || !rhs || !target)
        return pic_set_error_(PIC_ERR_INVALID, "rho/phi/rhs/target is NULL");
    if ((rho_prev == nullptr) != (phi_prev == nullptr))
        return pic_set_error_(PIC_ERR_INVALID, "rho_prev and phi_prev: both or neither");
    if (!(h > 0.0)) return pic_set_error_(PIC_ERR_INVALID, "h must be > 0");
    const int rc = net::make_pair(w->n, rho, rho_prev, phi, phi_prev, h * h, rhs, target, scale,
                                  (hipStream_t)stream);
    return rc ? nfail(PIC_ERR_HIP) : PIC_OK;
}

int pic_net_precondition(pic_net* w, const double* r, double h, double* z, void* stream) {
    NEEDNET(w);
    if (!r || !z) return pic_set_error_(PIC_ERR_INVALID, "r/z is NULL");
    return net::precondition(w->n, r, h * h, z, (hipStream_t)stream) ? nfail(PIC_ERR_HIP) : PIC_OK;
}

size_t pic_conv3d_frag_elems(int32_t ci, int32_t co) {
    if (!pair_ok(ci, co)) return 0;
    return net::frag_elems(ci, co);
}

int pic_conv3d_pack(int32_t ci, int32_t co, const float* w, uint16_t* ff, uint16_t* fb,
                    void* stream) {
    if (!pair_ok(ci, co)) return pic_set_error_(PIC_ERR_INVALID, "unsupported channel pair");
    if (!w) return pic_set_error_(PIC_ERR_INVALID, "w is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (ff) {
        const int rc = hchk(net::pack(w, ci, co, 0, ff, s), "pack");
        if (rc) return rc;
    }
    if (fb) return hchk(net::pack(w, ci, co, 1, fb, s), "pack");
    return PIC_OK;
}

int pic_conv3d_fwd(int32_t n, int32_t ci, int32_t co, const uint16_t* x, const uint16_t* ff,
                   const float* bias, const uint16_t* skip, int32_t relu, uint16_t* y,
                   void* stream) {
    if (!pair_ok(ci, co)) return pic_set_error_(PIC_ERR_INVALID, "unsupported channel pair");
    if (n < 4 || n % 2 || (int64_t)n * n * n % 16) return pic_set_error_(PIC_ERR_INVALID, "bad n");
    if (!x || !ff || !bias || !y) return pic_set_error_(PIC_ERR_INVALID, "NULL argument");
    return hchk(net::conv_fwd(n, ci, co, x, ff, bias, skip, relu, y, (hipStream_t)stream), "conv_fwd");
}

int pic_conv3d_bwd_data(int32_t n, int32_t ci, int32_t co, const uint16_t* gy, const uint16_t* fb,
                        float* gx, int32_t accumulate, void* stream) {
    if (!pair_ok(ci, co)) return pic_set_error_(PIC_ERR_INVALID, "unsupported channel pair");
    if (n < 4 || n % 2 || (int64_t)n * n * n % 16) return pic_set_error_(PIC_ERR_INVALID, "bad n");
    if (!gy || !fb || !gx) return pic_set_error_(PIC_ERR_INVALID, "NULL argument");
    return hchk(net::conv_bwd_data(n, ci, co, gy, fb, gx, accumulate, (hipStream_t)stream),
                "conv_bwd_data");
}

size_t pic_conv3d_wgrad_scratch_elems(int32_t n, int32_t ci, int32_t co) {
    if (!pair_ok(ci, co) || n < 4 || (int64_t)n * n * n % 32) return 0;
    return net::dw_part_elems(n, ci, co);
}

int pic_conv3d_bwd_weight(int32_t n, int32_t ci, int32_t co, const uint16_t* x, const uint16_t* gy,
                          float* scratch, float* grad, void* stream) {
    if (!pair_ok(ci, co)) return pic_set_error_(PIC_ERR_INVALID, "unsupported channel pair");
    if (n < 4 || (int64_t)n * n * n % 32) return pic_set_error_(PIC_ERR_INVALID, "bad n");
    if (!x || !gy || !scratch || !grad) return pic_set_error_(PIC_ERR_INVALID, "NULL argument");
    return hchk(net::conv_dw(n, ci, co, x, gy, scratch, grad, (hipStream_t)stream), "conv_dw");
}

int pic_adam_step(int64_t len, float* theta, float* m, float* v, const float* g, double lr,
                  double beta1, double beta2, double eps, int32_t step, void* stream) {
    if (len < 0 || step < 1) return pic_set_error_(PIC_ERR_INVALID, "bad len/step");
    if (len == 0) return PIC_OK;
    if (!theta || !m || !v || !g) return pic_set_error_(PIC_ERR_INVALID, "NULL argument");
    return hchk(net::adam(len, theta, m, v, g, (float)lr, (float)beta1, (float)beta2, (float)eps, step,
                          (hipStream_t)stream),
                "adam");
}

}  // extern "C"
