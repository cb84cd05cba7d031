// net.hip -- host side of the learned preconditioner's network: buffers,
// forward, backward, one training step (Adam), and the preconditioner map
// z = s * NN(h^2 r / s) - mean with s = rms(h^2 r).
//
// The scale-free form uses A = (1/h^2)(-Lap_1): A e = r  <=>  (-Lap_1) e =
// h^2 r, so a network trained at one grid spacing applies at any other; the
// normalisation by s makes the map exactly positively homogeneous.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "net.hpp"

namespace pic {
namespace net {

static thread_local std::string n_err;
const char* last_error() { return n_err.c_str(); }

#define NCHK(expr)                                                                       \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) {                                                          \
            n_err = std::string(#expr) + ": " + hipGetErrorString(e_);                   \
            return -2;                                                                   \
        }                                                                                \
    } while (0)

struct LayerSpec {
    const char* name;
    int ci, co, level;
};
static const LayerSpec kSpec[kLayers] = {
    {"e1a", 1, 16, 0},  {"e1b", 16, 16, 0}, {"e2a", 16, 32, 1}, {"e2b", 32, 32, 1},
    {"b3a", 32, 64, 2}, {"b3b", 64, 32, 2}, {"d2a", 32, 32, 1}, {"d2b", 32, 16, 1},
    {"d1a", 16, 16, 0}, {"out", 16, 1, 0}};
enum { E1A, E1B, E2A, E2B, B3A, B3B, D2A, D2B, D1A, OUT };

int64_t param_count() {
    int64_t s = 0;
    for (const auto& l : kSpec) s += 27LL * l.ci * l.co + l.co;
    return s;
}

struct Net {
    int n = 0;
    bool training = false;
    int64_t P = 0;
    int64_t woff[kLayers], boff[kLayers];
    float* params = nullptr;  // FP32 master (device)
    uint16_t* ffrag[kLayers] = {};
    uint16_t* bfrag[kLayers] = {};
    // activations (BF16, channels-last)
    uint16_t *in = nullptr, *e1a = nullptr, *e1b = nullptr, *p1 = nullptr, *e2a = nullptr,
             *e2b = nullptr, *p2 = nullptr, *b3a = nullptr, *b3b = nullptr, *u2 = nullptr,
             *d2a = nullptr, *d2b = nullptr, *u1 = nullptr, *d1a = nullptr;
    float* out = nullptr;
    double* red = nullptr;      // reduction partials (+ tail for scalars)
    double* scal = nullptr;     // device scalars (s)
    double* zbuf = nullptr;
    // training
    float *grads = nullptr, *am = nullptr, *av = nullptr, *wpart = nullptr, *d2 = nullptr;
    float *g1a = nullptr, *g1b = nullptr;          // FP32 16 ch at n
    float *g2a = nullptr, *g2b = nullptr;          // FP32 32 ch at n/2
    float *g2c = nullptr;                          // FP32 16 ch at n/2
    float *g3a = nullptr, *g3b = nullptr;          // FP32 64 / 32 ch at n/4
    uint16_t *gb_out = nullptr, *gb_d1a = nullptr, *gb_d2a = nullptr, *gb1 = nullptr, *gb2 = nullptr,
             *gb3 = nullptr;
    int step = 0;
    std::vector<void*> allocs;
};

static int alloc(Net* net, void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes < 256 ? 256 : bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        n_err = "hipMalloc failed (" + std::to_string(bytes) + " bytes)";
        return -3;
    }
    net->allocs.push_back(*p);
    return 0;
}

#define NALLOC(ptr, bytes)                                      \
    do {                                                        \
        int rc_ = alloc(net, (void**)&(ptr), (size_t)(bytes));  \
        if (rc_) {                                              \
            destroy(net);                                       \
            return rc_;                                         \
        }                                                       \
    } while (0)

int grid(const Net* net) { return net->n; }

int create(Net** out, int n, bool training) {
    *out = nullptr;
    if (n < 16 || n % 16 != 0) {
        n_err = "network grid size must be a multiple of 16";
        return -1;
    }
    Net* net = new Net();
    net->n = n;
    net->training = training;
    net->P = param_count();
    int64_t o = 0;
    for (int l = 0; l < kLayers; ++l) {
        net->woff[l] = o;
        o += 27LL * kSpec[l].ci * kSpec[l].co;
        net->boff[l] = o;
        o += kSpec[l].co;
    }
    const int64_t n1 = (int64_t)n * n * n, n2 = n1 / 8, n3 = n1 / 64;
    const size_t B = 2, F = 4;
    NALLOC(net->params, net->P * F);
    for (int l = 0; l < kLayers; ++l) {
        if (kSpec[l].ci >= 16 && kSpec[l].co >= 16) {
            NALLOC(net->ffrag[l], frag_elems(kSpec[l].ci, kSpec[l].co) * B);
            NALLOC(net->bfrag[l], frag_elems(kSpec[l].co, kSpec[l].ci) * B);
        }
    }
    NALLOC(net->in, n1 * B);
    NALLOC(net->e1a, n1 * 16 * B);
    NALLOC(net->e1b, n1 * 16 * B);
    // inference with the fused up-sampling: d1a reuses e1a (dead after e1b)
    if (training || !conv_up_fused(n, 16, 16)) NALLOC(net->d1a, n1 * 16 * B);
    else net->d1a = net->e1a;
    NALLOC(net->p1, n2 * 16 * B);
    NALLOC(net->e2a, n2 * 32 * B);
    NALLOC(net->e2b, n2 * 32 * B);
    NALLOC(net->d2a, n2 * 32 * B);
    NALLOC(net->d2b, n2 * 16 * B);
    NALLOC(net->p2, n3 * 32 * B);
    NALLOC(net->b3a, n3 * 64 * B);
    NALLOC(net->b3b, n3 * 32 * B);
    if (training) {
        NALLOC(net->u1, n1 * 16 * B);
        NALLOC(net->u2, n2 * 32 * B);
    } else {
        // inference: u1 reuses e1a (dead after e1b; unused when the
        // up-sampling is fused); u2 reuses e2a (dead after e2b)
        net->u1 = net->e1a;
        net->u2 = net->e2a;
    }
    NALLOC(net->out, n1 * F);
    NALLOC(net->red, (size_t)(2 * loss_parts(n) + 2 * pre_parts(n1) + 64) * sizeof(double));
    NALLOC(net->scal, 64 * sizeof(double));
    if (training) {
        NALLOC(net->grads, net->P * F);
        NALLOC(net->am, net->P * F);
        NALLOC(net->av, net->P * F);
        NCHK(hipMemset(net->am, 0, net->P * F));
        NCHK(hipMemset(net->av, 0, net->P * F));
        size_t wp = 0;
        for (int l = 0; l < kLayers; ++l) {
            const int ln = n >> kSpec[l].level;
            const size_t e = dw_part_elems(ln, kSpec[l].ci, kSpec[l].co);
            if (e > wp) wp = e;
        }
        NALLOC(net->wpart, wp * F);
        NALLOC(net->d2, n1 * F);
        NALLOC(net->g1a, n1 * 16 * F);
        NALLOC(net->g1b, n1 * 16 * F);
        NALLOC(net->g2a, n2 * 32 * F);
        NALLOC(net->g2b, n2 * 32 * F);
        NALLOC(net->g2c, n2 * 16 * F);
        NALLOC(net->g3a, n3 * 64 * F);
        NALLOC(net->g3b, n3 * 32 * F);
        NALLOC(net->gb_out, n1 * B);
        NALLOC(net->gb_d1a, n1 * 16 * B);
        NALLOC(net->gb_d2a, n2 * 32 * B);
        NALLOC(net->gb1, n1 * 16 * B);
        NALLOC(net->gb2, n2 * 32 * B);
        NALLOC(net->gb3, n3 * 64 * B);
    }
    *out = net;
    return 0;
}

void destroy(Net* net) {
    if (!net) return;
    (void)hipDeviceSynchronize();
    for (void* p : net->allocs) (void)hipFree(p);
    delete net;
}

static int repack(Net* net, hipStream_t s) {
    for (int l = 0; l < kLayers; ++l) {
        if (!net->ffrag[l]) continue;
        NCHK(pack(net->params + net->woff[l], kSpec[l].ci, kSpec[l].co, 0, net->ffrag[l], s));
        NCHK(pack(net->params + net->woff[l], kSpec[l].ci, kSpec[l].co, 1, net->bfrag[l], s));
    }
    return 0;
}

int set_params(Net* net, const float* params, hipStream_t s) {
    NCHK(hipMemcpyAsync(net->params, params, net->P * sizeof(float), hipMemcpyDeviceToDevice, s));
    net->step = 0;
    if (net->training) {
        NCHK(hipMemsetAsync(net->am, 0, net->P * sizeof(float), s));
        NCHK(hipMemsetAsync(net->av, 0, net->P * sizeof(float), s));
    }
    return repack(net, s);
}

int get_params(const Net* net, float* params, hipStream_t s) {
    NCHK(hipMemcpyAsync(params, net->params, net->P * sizeof(float), hipMemcpyDeviceToDevice, s));
    return 0;
}

// Forward from net->in (BF16).
static int fwd(Net* net, hipStream_t s) {
    const int n = net->n, h = n / 2, q = n / 4;
    const float* P = net->params;
    auto W = [&](int l) { return P + net->woff[l]; };
    auto Bi = [&](int l) { return P + net->boff[l]; };
    NCHK(conv_in_fwd(n, net->in, W(E1A), Bi(E1A), net->e1a, s));
    if (conv_pool_fused(n, 16, 16)) {
        NCHK(conv_fwd_pool(n, 16, 16, net->e1a, net->ffrag[E1B], Bi(E1B), net->e1b, net->p1, s));
    } else {
        NCHK(conv_fwd(n, 16, 16, net->e1a, net->ffrag[E1B], Bi(E1B), nullptr, 1, net->e1b, s));
        NCHK(pool_fwd(h, 16, net->e1b, net->p1, s));
    }
    NCHK(conv_fwd(h, 16, 32, net->p1, net->ffrag[E2A], Bi(E2A), nullptr, 1, net->e2a, s));
    if (conv_pool_fused(h, 32, 32)) {
        NCHK(conv_fwd_pool(h, 32, 32, net->e2a, net->ffrag[E2B], Bi(E2B), net->e2b, net->p2, s));
    } else {
        NCHK(conv_fwd(h, 32, 32, net->e2a, net->ffrag[E2B], Bi(E2B), nullptr, 1, net->e2b, s));
        NCHK(pool_fwd(q, 32, net->e2b, net->p2, s));
    }
    NCHK(conv_fwd(q, 32, 64, net->p2, net->ffrag[B3A], Bi(B3A), nullptr, 1, net->b3a, s));
    NCHK(conv_fwd(q, 64, 32, net->b3a, net->ffrag[B3B], Bi(B3B), nullptr, 1, net->b3b, s));
    // training keeps the up-sampled inputs (the weight gradients read them);
    // inference up-samples inside the convolution's staging where it can
    if (!net->training && conv_up_fused(h, 32, 32)) {
        NCHK(conv_fwd_up(h, 32, 32, net->b3b, net->ffrag[D2A], Bi(D2A), net->e2b, 1, net->d2a, s));
    } else {
        NCHK(up_fwd(h, 32, net->b3b, net->u2, s));
        NCHK(conv_fwd(h, 32, 32, net->u2, net->ffrag[D2A], Bi(D2A), net->e2b, 1, net->d2a, s));
    }
    NCHK(conv_fwd(h, 32, 16, net->d2a, net->ffrag[D2B], Bi(D2B), nullptr, 1, net->d2b, s));
    if (!net->training && conv_up_fused(n, 16, 16)) {
        NCHK(conv_fwd_up(n, 16, 16, net->d2b, net->ffrag[D1A], Bi(D1A), net->e1b, 1, net->d1a, s));
    } else {
        NCHK(up_fwd(n, 16, net->d2b, net->u1, s));
        NCHK(conv_fwd(n, 16, 16, net->u1, net->ffrag[D1A], Bi(D1A), net->e1b, 1, net->d1a, s));
    }
    NCHK(conv_out_fwd(n, net->d1a, W(OUT), Bi(OUT), net->out, s));
    return 0;
}

int forward_f32(Net* net, const float* x, float* out, hipStream_t s) {
    const int64_t n1 = (int64_t)net->n * net->n * net->n;
    NCHK(to_bf16(n1, x, net->in, s));
    int rc = fwd(net, s);
    if (rc) return rc;
    if (out && out != net->out)
        NCHK(hipMemcpyAsync(out, net->out, n1 * sizeof(float), hipMemcpyDeviceToDevice, s));
    return 0;
}

// Backward from the BF16 output gradient in net->gb_out; gradients into g.
static int bwd(Net* net, float* g, hipStream_t s) {
    const int n = net->n, h = n / 2, q = n / 4;
    const int64_t n1 = (int64_t)n * n * n, n2 = n1 / 8, n3 = n1 / 64;
    const float* P = net->params;
    auto W = [&](int l) { return P + net->woff[l]; };
    auto G = [&](int l) { return g + net->woff[l]; };  // weight grads then bias grads follow
    float* part = net->wpart;
    // out
    NCHK(conv_dw_small(n, 16, 1, net->d1a, net->gb_out, part, G(OUT), s));
    NCHK(conv_out_bwd(n, net->gb_out, W(OUT), net->g1a, 0, s));
    NCHK(grad_round(n1 * 16, net->g1a, net->d1a, net->gb_d1a, s));
    // d1a (skip into e1b)
    NCHK(conv_dw(n, 16, 16, net->u1, net->gb_d1a, part, G(D1A), s));
    NCHK(conv_bwd_data(n, 16, 16, net->gb_d1a, net->bfrag[D1A], net->g1a, 0, s));  // g_u1
    NCHK(up_bwd(h, 16, net->g1a, net->g2c, s));                                     // g_d2b
    NCHK(grad_round(n2 * 16, net->g2c, net->d2b, net->gb2, s));
    // d2b
    NCHK(conv_dw(h, 32, 16, net->d2a, net->gb2, part, G(D2B), s));
    NCHK(conv_bwd_data(h, 32, 16, net->gb2, net->bfrag[D2B], net->g2a, 0, s));      // g_d2a
    NCHK(grad_round(n2 * 32, net->g2a, net->d2a, net->gb_d2a, s));
    // d2a (skip into e2b)
    NCHK(conv_dw(h, 32, 32, net->u2, net->gb_d2a, part, G(D2A), s));
    NCHK(conv_bwd_data(h, 32, 32, net->gb_d2a, net->bfrag[D2A], net->g2b, 0, s));   // g_u2
    NCHK(up_bwd(q, 32, net->g2b, net->g3b, s));                                     // g_b3b
    NCHK(grad_round(n3 * 32, net->g3b, net->b3b, net->gb3, s));
    // b3b
    NCHK(conv_dw(q, 64, 32, net->b3a, net->gb3, part, G(B3B), s));
    NCHK(conv_bwd_data(q, 64, 32, net->gb3, net->bfrag[B3B], net->g3a, 0, s));      // g_b3a
    NCHK(grad_round(n3 * 64, net->g3a, net->b3a, net->gb3, s));
    // b3a
    NCHK(conv_dw(q, 32, 64, net->p2, net->gb3, part, G(B3A), s));
    NCHK(conv_bwd_data(q, 32, 64, net->gb3, net->bfrag[B3A], net->g3b, 0, s));      // g_p2
    NCHK(pool_bwd(h, 32, net->g3b, net->g2a, 0, s));                                // g_e2b
    NCHK(add_bf16(n2 * 32, net->gb_d2a, net->g2a, s));
    NCHK(grad_round(n2 * 32, net->g2a, net->e2b, net->gb2, s));
    // e2b
    NCHK(conv_dw(h, 32, 32, net->e2a, net->gb2, part, G(E2B), s));
    NCHK(conv_bwd_data(h, 32, 32, net->gb2, net->bfrag[E2B], net->g2b, 0, s));      // g_e2a
    NCHK(grad_round(n2 * 32, net->g2b, net->e2a, net->gb2, s));
    // e2a
    NCHK(conv_dw(h, 16, 32, net->p1, net->gb2, part, G(E2A), s));
    NCHK(conv_bwd_data(h, 16, 32, net->gb2, net->bfrag[E2A], net->g2c, 0, s));      // g_p1
    NCHK(pool_bwd(n, 16, net->g2c, net->g1b, 0, s));                                // g_e1b
    NCHK(add_bf16(n1 * 16, net->gb_d1a, net->g1b, s));
    NCHK(grad_round(n1 * 16, net->g1b, net->e1b, net->gb1, s));
    // e1b
    NCHK(conv_dw(n, 16, 16, net->e1a, net->gb1, part, G(E1B), s));
    NCHK(conv_bwd_data(n, 16, 16, net->gb1, net->bfrag[E1B], net->g1a, 0, s));      // g_e1a
    NCHK(grad_round(n1 * 16, net->g1a, net->e1a, net->gb1, s));
    // e1a
    NCHK(conv_dw_small(n, 1, 16, net->in, net->gb1, part, G(E1A), s));
    return 0;
}

int backward(Net* net, const float* dout, float* grads, hipStream_t s) {
    if (!net->training) {
        n_err = "network was created without training buffers";
        return -4;
    }
    const int64_t n1 = (int64_t)net->n * net->n * net->n;
    NCHK(to_bf16(n1, dout, net->gb_out, s));
    return bwd(net, grads ? grads : net->grads, s);
}

int train_step(Net* net, const float* rhs, const float* target, double lam, double lr,
               double* loss, hipStream_t s) {
    if (!net->training) {
        n_err = "network was created without training buffers";
        return -4;
    }
    const int n = net->n;
    const int64_t n1 = (int64_t)n * n * n;
    NCHK(to_bf16(n1, rhs, net->in, s));
    int rc = fwd(net, s);
    if (rc) return rc;
    double* normp = net->red;                         // 2 * loss_parts + 4 scalars
    double* lossp = net->red + 2 * loss_parts(n) + 8;  // 2 * loss_parts
    NCHK(loss_norms(n, target, rhs, normp, s));
    NCHK(loss_pass1(n, net->out, target, rhs, net->d2, lossp, s));
    NCHK(loss_pass2(n, net->out, target, net->d2, normp, lam, net->gb_out, s));
    rc = bwd(net, net->grads, s);
    if (rc) return rc;
    net->step += 1;
    NCHK(adam(net->P, net->params, net->am, net->av, net->grads, (float)lr, 0.9f, 0.999f, 1e-8f,
              net->step, s));
    rc = repack(net, s);
    if (rc) return rc;
    if (loss) {
        const int np = loss_parts(n);
        std::vector<double> h(2 * np + 4);
        NCHK(hipMemcpyAsync(h.data(), normp, (2 * np + 4) * sizeof(double), hipMemcpyDeviceToHost, s));
        std::vector<double> hl(2 * np);
        NCHK(hipMemcpyAsync(hl.data(), lossp, 2 * np * sizeof(double), hipMemcpyDeviceToHost, s));
        NCHK(hipStreamSynchronize(s));
        double a = 0, b = 0;
        for (int i = 0; i < np; ++i) {
            a += hl[2 * i];
            b += hl[2 * i + 1];
        }
        const double nt = h[2 * np + 2], nr = h[2 * np + 3];
        *loss = a / nt + lam * b / nr;
    }
    return 0;
}

int eval_loss(Net* net, const float* rhs, const float* target, double lam, double* loss,
              hipStream_t s) {
    if (!net->training) {
        n_err = "network was created without training buffers";
        return -4;
    }
    const int n = net->n;
    const int64_t n1 = (int64_t)n * n * n;
    NCHK(to_bf16(n1, rhs, net->in, s));
    const int rc = fwd(net, s);
    if (rc) return rc;
    const int np = loss_parts(n);
    double* normp = net->red;
    double* lossp = net->red + 2 * np + 8;
    NCHK(loss_norms(n, target, rhs, normp, s));
    NCHK(loss_pass1(n, net->out, target, rhs, net->d2, lossp, s));
    std::vector<double> h(2 * np), hl(2 * np);
    NCHK(hipMemcpyAsync(h.data(), normp, 2 * np * sizeof(double), hipMemcpyDeviceToHost, s));
    NCHK(hipMemcpyAsync(hl.data(), lossp, 2 * np * sizeof(double), hipMemcpyDeviceToHost, s));
    NCHK(hipStreamSynchronize(s));
    double a = 0, b = 0, nt = 0, nr = 0;
    for (int i = 0; i < np; ++i) {
        a += hl[2 * i];
        b += hl[2 * i + 1];
        nt += h[2 * i];
        nr += h[2 * i + 1];
    }
    *loss = a / nt + lam * b / nr;
    return 0;
}

int make_pair(Net* net, const double* b, const double* bp, const double* phi, const double* pp,
              double h2, float* rhs, float* tgt, double* scale, hipStream_t s) {
    const int64_t n1 = (int64_t)net->n * net->n * net->n;
    NCHK(scale_pair(n1, b, bp, phi, pp, h2, net->red, net->scal + 1, rhs, tgt, s));
    if (scale) {
        NCHK(hipMemcpyAsync(scale, net->scal + 1, sizeof(double), hipMemcpyDeviceToHost, s));
        NCHK(hipStreamSynchronize(s));
    }
    return 0;
}

int precondition(Net* net, const double* r, double h2, double* z, hipStream_t s) {
    const int64_t n1 = (int64_t)net->n * net->n * net->n;
    double* part = net->red;
    NCHK(prep_input(n1, r, h2, part, net->scal, net->in, s));
    int rc = fwd(net, s);
    if (rc) return rc;
    NCHK(post_output(n1, net->out, net->scal, z, part, s));
    return 0;
}

}  // namespace net
}  // namespace pic
