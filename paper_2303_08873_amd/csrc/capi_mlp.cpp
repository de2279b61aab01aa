// C-ABI entry points that run the cost-model kernels on caller buffers
// (used to check the GPU gradients and the Adam step against a reference).
#include "internal.h"

using namespace ao;

extern "C" {

int ao_mlp_forward(const float* params, const float* x, int batch, float* out, void* stream) {
    if (batch < 0 || (batch > 0 && (!params || !x || !out)))
        return fail(AO_EINVAL, "bad arguments");
    hipError_t e = mlp_forward(params, x, batch, out, (hipStream_t)stream);
    if (e != hipSuccess) return fail(AO_EHIP, std::string("mlp forward: ") + hipGetErrorString(e));
    return AO_OK;
}

int ao_mlp_grad(const float* params, const float* x, const float* y, const float* mask, int batch,
                float* grad, float* loss, void* stream) {
    if (batch < 1 || !params || !x || !y || !mask || !grad) return fail(AO_EINVAL, "bad arguments");
    hipError_t e = mlp_grad(params, x, y, mask, batch, grad, loss, (hipStream_t)stream);
    if (e != hipSuccess) return fail(AO_EHIP, std::string("mlp grad: ") + hipGetErrorString(e));
    return AO_OK;
}

int ao_mlp_adam(float* params, float* m, float* v, const float* grad, int t, float lr,
                void* stream) {
    if (t < 1 || !params || !m || !v || !grad || !(lr > 0.0f)) return fail(AO_EINVAL, "bad arguments");
    hipError_t e = mlp_adam(params, m, v, grad, t, lr, (hipStream_t)stream);
    if (e != hipSuccess) return fail(AO_EHIP, std::string("mlp adam: ") + hipGetErrorString(e));
    return AO_OK;
}

}  // extern "C"
