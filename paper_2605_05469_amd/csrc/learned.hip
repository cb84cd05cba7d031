// learned.hip -- flexible PCG driven by the network preconditioner.
#include <string>

#include "learned.hpp"

namespace pic {

static thread_local std::string l_err;

struct Learned {
    int n;
    int64_t n3;
    bool have_net;
};

const char* learned_last_error() { return l_err.c_str(); }

size_t learned_bytes(int) { return 0; }

int learned_create(Learned** out, int n, int64_t n3) {
    Learned* l = new Learned{n, n3, false};
    *out = l;
    return PIC_OK;
}

void learned_destroy(Learned* l) { delete l; }

int learned_solve(Learned* l, const LearnedEnv*, const double*, double*, pic_solve_info*,
                  hipStream_t) {
    if (!l->have_net) {
        l_err = "no network weights loaded (pic_set_unet)";
        return PIC_ERR_STATE;
    }
    return PIC_OK;
}

}  // namespace pic
