// C ABI of the learned density's network: parameters, training steps (loss and
// gradient, Adam) and an epoch loop that launches them back to back on one
// stream with no host synchronisation.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "mad_internal.hpp"
#include "mlp.hpp"

using namespace mad;

namespace {

constexpr int kMaxWaves = 2048;

// waves for a batch of `count` samples: about eight samples per wave, a multiple of four
int train_waves(int64_t count) {
    int64_t w = (count + 7) / 8;
    w = std::max<int64_t>(4, std::min<int64_t>(w, kMaxWaves));
    return (int)((w + 3) / 4 * 4);
}

int upload_params(mad_mlp* m, const float* params_host) {
    for (int i = 0; i < kMlpParams; ++i)
        if (!std::isfinite(params_host[i])) return fail(MAD_E_INVALID_ARG, "non-finite network parameter");
    MAD_HIP_TRY(hipMemcpy(m->d_params, params_host, sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
    MAD_HIP_TRY(hipMemset(m->d_m, 0, sizeof(float) * kMlpParams));
    MAD_HIP_TRY(hipMemset(m->d_v, 0, sizeof(float) * kMlpParams));
    MAD_HIP_TRY(hipMemset(m->d_step, 0, sizeof(int64_t)));
    MAD_HIP_TRY(launch_mlp_to_bf16(m->d_params, m->d_wbf, nullptr));
    MAD_HIP_TRY(hipDeviceSynchronize());
    return MAD_OK;
}

void free_mlp(mad_mlp* m) {
    for (void* p : {(void*)m->d_params, (void*)m->d_m, (void*)m->d_v, (void*)m->d_wbf, (void*)m->d_grad,
                    (void*)m->d_loss, (void*)m->d_step, (void*)m->d_partial})
        if (p) (void)hipFree(p);
    delete m;
}

int loss_grad(mad_mlp* m, const float* z, const float* W, const float* dW, const int32_t* idx, int64_t base,
              int64_t count, float c_e, const float* c_g, float lam_g, float* grad, float* loss, hipStream_t s) {
    MlpTrainLaunch L{};
    L.z = z;
    L.W = W;
    L.dW = dW;
    L.idx = idx;
    L.base = base;
    L.count = count;
    L.params = m->d_params;
    for (int i = 0; i < 6; ++i) L.s_in[i] = m->s_in[i];
    L.s_out = m->s_out;
    L.c_e = c_e;
    for (int i = 0; i < 6; ++i) L.c_g[i] = c_g[i];
    L.lam_g = lam_g;
    L.partial = m->d_partial;
    L.n_waves = train_waves(count);
    MAD_HIP_TRY(launch_mlp_train(L, s));
    MAD_HIP_TRY(launch_mlp_reduce(m->d_partial, L.n_waves, grad, loss, s));
    return MAD_OK;
}

int adam(mad_mlp* m, const float* grad, float lr, float b1, float b2, float eps, hipStream_t s) {
    MAD_HIP_TRY(launch_mlp_step_incr(m->d_step, s));
    MAD_HIP_TRY(launch_mlp_adam(m->d_params, m->d_m, m->d_v, grad, m->d_step, lr, b1, b2, eps, m->d_wbf, s));
    return MAD_OK;
}

bool bad_scalars(float c_e, const float* c_g, float lam_g) {
    if (!c_g) return true;
    for (int i = 0; i < 6; ++i)
        if (!(c_g[i] > 0.0f) || !std::isfinite(c_g[i])) return true;
    return !(c_e > 0.0f) || !(lam_g >= 0.0f) || !std::isfinite(c_e) || !std::isfinite(lam_g);
}

bool bad_adam(float lr, float b1, float b2, float eps) {
    return !(lr > 0.0f) || !(b1 >= 0.0f && b1 < 1.0f) || !(b2 >= 0.0f && b2 < 1.0f) || !(eps > 0.0f) ||
           !std::isfinite(lr);
}

}  // namespace

extern "C" {

int32_t mad_mlp_create(int32_t hidden, const float* params_host, const float* s_in_host, float s_out,
                       mad_mlp** out) {
    if (!out) return fail(MAD_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (hidden != kHid) return fail(MAD_E_UNSUPPORTED, "hidden width must be 64");
    if (!params_host || !s_in_host) return fail(MAD_E_INVALID_ARG, "NULL parameters");
    for (int i = 0; i < 6; ++i)
        if (!std::isfinite(s_in_host[i])) return fail(MAD_E_INVALID_ARG, "non-finite input scale");
    if (!std::isfinite(s_out)) return fail(MAD_E_INVALID_ARG, "non-finite output scale");
    mad_mlp* m = new (std::nothrow) mad_mlp();
    if (!m) return fail(MAD_E_OOM, "network");
    for (int i = 0; i < 6; ++i) m->s_in[i] = s_in_host[i];
    m->s_out = s_out;
    int rc = MAD_OK;
    auto alloc = [&](void** p, size_t bytes) {
        if (rc == MAD_OK && hipMalloc(p, bytes) != hipSuccess) rc = fail(MAD_E_OOM, "network device memory");
    };
    if (hipGetDevice(&m->device) != hipSuccess) rc = fail(MAD_E_HIP, "hipGetDevice");
    alloc((void**)&m->d_params, sizeof(float) * kMlpParams);
    alloc((void**)&m->d_m, sizeof(float) * kMlpParams);
    alloc((void**)&m->d_v, sizeof(float) * kMlpParams);
    alloc((void**)&m->d_wbf, sizeof(uint16_t) * kMlpParams);
    alloc((void**)&m->d_grad, sizeof(float) * kMlpParams);
    alloc((void**)&m->d_loss, sizeof(float) * 4);
    alloc((void**)&m->d_step, sizeof(int64_t));
    alloc((void**)&m->d_partial, sizeof(float) * (size_t)kMaxWaves * (kMlpParams + 1));
    m->partial_waves = kMaxWaves;
    if (rc == MAD_OK) rc = upload_params(m, params_host);
    if (rc != MAD_OK) {
        free_mlp(m);
        return rc;
    }
    *out = m;
    return MAD_OK;
}

int32_t mad_mlp_set_params(mad_mlp* m, const float* params_host) {
    if (!m || !params_host) return fail(MAD_E_INVALID_ARG, "NULL argument");
    return upload_params(m, params_host);
}

int32_t mad_mlp_get_params(const mad_mlp* m, int32_t which, float* params_host) {
    if (!m || !params_host) return fail(MAD_E_INVALID_ARG, "NULL argument");
    MAD_HIP_TRY(hipDeviceSynchronize());
    if (which == 0) {
        MAD_HIP_TRY(hipMemcpy(params_host, m->d_params, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost));
    } else if (which == 1) {
        std::vector<uint16_t> b(kMlpParams);
        MAD_HIP_TRY(hipMemcpy(b.data(), m->d_wbf, sizeof(uint16_t) * kMlpParams, hipMemcpyDeviceToHost));
        for (int i = 0; i < kMlpParams; ++i) {
            const uint32_t u = (uint32_t)b[i] << 16;
            std::memcpy(&params_host[i], &u, 4);
        }
    } else {
        return fail(MAD_E_INVALID_ARG, "which must be 0 or 1");
    }
    return MAD_OK;
}

int32_t mad_mlp_loss_grad(mad_mlp* m, const float* z, const float* W, const float* dW, const int32_t* idx,
                          int64_t base, int64_t count, float c_e, const float* c_g, float lam_g, float* grad,
                          float* loss, void* stream) {
    if (!m || !z || !W || !dW || !grad || !loss) return fail(MAD_E_INVALID_ARG, "NULL argument");
    if (count < 1 || base < 0) return fail(MAD_E_INVALID_ARG, "count must be >= 1 and base >= 0");
    if (bad_scalars(c_e, c_g, lam_g)) return fail(MAD_E_INVALID_ARG, "c_e and every c_g[i] must be > 0, lam_g >= 0");
    return loss_grad(m, z, W, dW, idx, base, count, c_e, c_g, lam_g, grad, loss, (hipStream_t)stream);
}

int32_t mad_mlp_adam_step(mad_mlp* m, const float* grad, float lr, float beta1, float beta2, float eps,
                          void* stream) {
    if (!m || !grad) return fail(MAD_E_INVALID_ARG, "NULL argument");
    if (bad_adam(lr, beta1, beta2, eps)) return fail(MAD_E_INVALID_ARG, "bad Adam constants");
    return adam(m, grad, lr, beta1, beta2, eps, (hipStream_t)stream);
}

int32_t mad_mlp_train_epoch(mad_mlp* m, const float* z, const float* W, const float* dW, const int32_t* perm,
                            int64_t n, int32_t batch, float c_e, const float* c_g, float lam_g, float lr,
                            float beta1, float beta2, float eps, float* loss_hist, void* stream) {
    if (!m || !z || !W || !dW || !perm) return fail(MAD_E_INVALID_ARG, "NULL argument");
    if (n < 1 || batch < 1) return fail(MAD_E_INVALID_ARG, "n and batch must be >= 1");
    if (bad_scalars(c_e, c_g, lam_g)) return fail(MAD_E_INVALID_ARG, "c_e and every c_g[i] must be > 0, lam_g >= 0");
    if (bad_adam(lr, beta1, beta2, eps)) return fail(MAD_E_INVALID_ARG, "bad Adam constants");
    hipStream_t s = (hipStream_t)stream;
    int64_t k = 0;
    for (int64_t b = 0; b < n; b += batch, ++k) {
        const int64_t cnt = std::min<int64_t>(batch, n - b);
        int rc = loss_grad(m, z, W, dW, perm, b, cnt, c_e, c_g, lam_g, m->d_grad, loss_hist ? loss_hist + k : m->d_loss,
                           s);
        if (rc != MAD_OK) return rc;
        if ((rc = adam(m, m->d_grad, lr, beta1, beta2, eps, s)) != MAD_OK) return rc;
    }
    return MAD_OK;
}

int32_t mad_mlp_destroy(mad_mlp* m) {
    if (m) free_mlp(m);
    return MAD_OK;
}

}  // extern "C"
