// C-ABI of the learned policy's network (cr_mlp_*, cr_trace_policy).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "devmem.hpp"
#include "mlp.hpp"
#include "plan.hpp"

namespace crf {
int mlp_param_count();
hipError_t launch_mlp_forward(const float *W, const float *X, int R, float *Y, hipStream_t stream);
hipError_t launch_mlp_grad(const float *W, const float *X, const float *T, int R, float *part, float *grad,
                           hipStream_t stream);
hipError_t launch_adam(float *W, float *m, float *v, const float *g, float lr, float b1, float b2, float eps, float c1,
                       float c2, hipStream_t stream);
void set_last_error(const std::string &msg);
bool trace_item(const cr_family *fam, int p, const uint32_t *coeffs, std::vector<CandRow> &rows, std::string &err,
                cr_status &st);
}  // namespace crf

using namespace crf;

struct cr_mlp {
    int device = 0;
    float *W = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;  // device, CR_MLP_PARAMS (+1 for grad)
    float *X = nullptr, *T = nullptr, *Y = nullptr, *part = nullptr;  // device scratch for rows_cap rows
    float *losses = nullptr;
    DevBlock bW, bm, bv, bgrad, bX, bT, bY, bpart, blosses;  // the blocks behind the pointers above
    size_t rows_cap = 0, loss_cap = 0;
    int64_t adam_t = 0;

    static bool take(DevBlock &b, float *&ptr, size_t bytes) {
        dev_free(b);
        ptr = nullptr;
        if (!dev_alloc(b, bytes)) return false;
        ptr = static_cast<float *>(b.ptr);
        return true;
    }
    static void drop(DevBlock &b, float *&ptr) {
        dev_free(b);
        ptr = nullptr;
    }
    bool ensure_rows(size_t rows) {
        if (rows <= rows_cap) return true;
        const size_t cap = std::max(rows, rows_cap + rows_cap / 2);
        drop(bX, X);
        drop(bT, T);
        drop(bY, Y);
        drop(bpart, part);
        rows_cap = 0;
        const size_t nb = (cap + 63) / 64;
        if (!take(bX, X, cap * CR_MLP_INPUTS * sizeof(float))) return false;
        if (!take(bT, T, cap * sizeof(float))) return false;
        if (!take(bY, Y, cap * sizeof(float))) return false;
        if (!take(bpart, part, nb * (CR_MLP_PARAMS + 1) * sizeof(float))) return false;
        rows_cap = cap;
        return true;
    }
    bool ensure_losses(size_t n) {
        if (n <= loss_cap) return true;
        loss_cap = 0;
        if (!take(blosses, losses, n * sizeof(float))) return false;
        loss_cap = n;
        return true;
    }
    void release() {
        drop(bW, W);
        drop(bm, m);
        drop(bv, v);
        drop(bgrad, grad);
        drop(bX, X);
        drop(bT, T);
        drop(bY, Y);
        drop(bpart, part);
        drop(blosses, losses);
    }
};

namespace crf {

// splitmix64: a counter-based generator (Steele, Lea, Flood 2014)
static uint64_t splitmix64(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

bool mlp_score(cr_mlp *m, const float *x, int rows, float *y, hipStream_t stream, std::string &err) {
    if (rows <= 0) return true;
    if (!m->ensure_rows(rows)) {
        err = "device allocation for the network's rows failed";
        return false;
    }
    hipError_t e = hipMemcpyAsync(m->X, x, sizeof(float) * CR_MLP_INPUTS * rows, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = launch_mlp_forward(m->W, m->X, rows, m->Y, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(y, m->Y, sizeof(float) * rows, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        err = std::string("HIP error in the network's forward pass: ") + hipGetErrorString(e);
        return false;
    }
    return true;
}

}  // namespace crf

extern "C" {

cr_status cr_mlp_create(const float *weights, uint64_t seed, cr_mlp **out) {
    if (!out) {
        set_last_error("null output");
        return CR_EINVAL;
    }
    if (mlp_param_count() != CR_MLP_PARAMS) {
        set_last_error("parameter layout mismatch");
        return CR_ESELFCHECK;
    }
    *out = nullptr;
    std::vector<float> w(CR_MLP_PARAMS, 0.f);
    if (weights) {
        std::memcpy(w.data(), weights, sizeof(float) * CR_MLP_PARAMS);
    } else {
        uint64_t s = seed;
        auto uni = [&](float bound) {
            const double u = (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0);
            return (float)((2.0 * u - 1.0) * bound);
        };
        const int I = CR_MLP_INPUTS, H = CR_MLP_HIDDEN;
        for (int k = 0; k < I * H; k++) w[k] = uni(1.f / std::sqrt((float)I));
        for (int k = 0; k < H * H; k++) w[I * H + H + k] = uni(1.f / std::sqrt((float)H));
        for (int k = 0; k < H; k++) w[I * H + H + H * H + H + k] = uni(1.f / std::sqrt((float)H));
    }
    cr_mlp *m = new cr_mlp();
    (void)hipGetDevice(&m->device);
    const size_t bytes = sizeof(float) * (CR_MLP_PARAMS + 1);
    bool ok = cr_mlp::take(m->bW, m->W, bytes) && cr_mlp::take(m->bm, m->m, bytes) &&
              cr_mlp::take(m->bv, m->v, bytes) && cr_mlp::take(m->bgrad, m->grad, bytes);
    std::vector<float> zero(CR_MLP_PARAMS + 1, 0.f);
    ok = ok && hipMemcpy(m->W, w.data(), sizeof(float) * CR_MLP_PARAMS, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->m, zero.data(), bytes, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->v, zero.data(), bytes, hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        cr_mlp_destroy(m);
        set_last_error("device allocation for the network failed");
        return CR_ENOMEM;
    }
    *out = m;
    return CR_OK;
}

cr_status cr_mlp_destroy(cr_mlp *m) {
    if (!m) return CR_OK;
    m->release();
    delete m;
    return CR_OK;
}

cr_status cr_mlp_weights(const cr_mlp *m, float *out) {
    if (!m || !out) {
        set_last_error("null argument");
        return CR_EINVAL;
    }
    if (hipMemcpy(out, m->W, sizeof(float) * CR_MLP_PARAMS, hipMemcpyDeviceToHost) != hipSuccess) {
        set_last_error("HIP copy of the weights failed");
        return CR_EDEVICE;
    }
    return CR_OK;
}

cr_status cr_mlp_forward(cr_mlp *m, int32_t rows, const float *x, float *y, void *hip_stream) {
    if (!m || rows < 0 || (rows > 0 && (!x || !y))) {
        set_last_error("bad arguments");
        return CR_EINVAL;
    }
    std::string err;
    if (!mlp_score(m, x, rows, y, reinterpret_cast<hipStream_t>(hip_stream), err)) {
        set_last_error(err);
        return CR_EDEVICE;
    }
    return CR_OK;
}

cr_status cr_mlp_grad(cr_mlp *m, int32_t rows, const float *x, const float *t, float *grad, float *loss,
                      void *hip_stream) {
    if (!m || rows <= 0 || !x || !t || !grad) {
        set_last_error("bad arguments");
        return CR_EINVAL;
    }
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    if (!m->ensure_rows(rows)) {
        set_last_error("device allocation for the network's rows failed");
        return CR_ENOMEM;
    }
    std::vector<float> g(CR_MLP_PARAMS + 1);
    hipError_t e = hipMemcpyAsync(m->X, x, sizeof(float) * CR_MLP_INPUTS * rows, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(m->T, t, sizeof(float) * rows, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = launch_mlp_grad(m->W, m->X, m->T, rows, m->part, m->grad, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g.data(), m->grad, sizeof(float) * (CR_MLP_PARAMS + 1), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        set_last_error(std::string("HIP error: ") + hipGetErrorString(e));
        return CR_EDEVICE;
    }
    std::memcpy(grad, g.data(), sizeof(float) * CR_MLP_PARAMS);
    if (loss) *loss = g[CR_MLP_PARAMS];
    return CR_OK;
}

cr_status cr_mlp_train(cr_mlp *m, int32_t rows, const float *x, const float *t, const cr_train_opts *opts,
                       float *loss, void *hip_stream) {
    if (!m || rows <= 0 || !x || !t || !opts || opts->epochs < 0 || opts->batch < 1) {
        set_last_error("bad arguments");
        return CR_EINVAL;
    }
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    const float lr = opts->lr > 0 ? opts->lr : 1e-3f, b1 = opts->beta1 > 0 ? opts->beta1 : 0.9f;
    const float b2 = opts->beta2 > 0 ? opts->beta2 : 0.999f, eps = opts->eps > 0 ? opts->eps : 1e-8f;
    const int batch = std::min<int>(opts->batch, rows);
    const int nbatch = (rows + batch - 1) / batch;
    if (!m->ensure_rows(rows) || !m->ensure_losses(nbatch)) {
        set_last_error("device allocation for training failed");
        return CR_ENOMEM;
    }
    std::vector<int> perm(rows);
    for (int i = 0; i < rows; i++) perm[i] = i;
    std::vector<float> xs((size_t)rows * CR_MLP_INPUTS), ts(rows), bl(nbatch);
    uint64_t s = opts->seed;
    for (int ep = 0; ep < opts->epochs; ep++) {
        for (int i = rows - 1; i > 0; i--) {  // Fisher-Yates
            const int j = (int)(splitmix64(s) % (uint64_t)(i + 1));
            std::swap(perm[i], perm[j]);
        }
        for (int i = 0; i < rows; i++) {
            std::memcpy(&xs[(size_t)i * CR_MLP_INPUTS], &x[(size_t)perm[i] * CR_MLP_INPUTS],
                        sizeof(float) * CR_MLP_INPUTS);
            ts[i] = t[perm[i]];
        }
        hipError_t e = hipMemcpyAsync(m->X, xs.data(), sizeof(float) * xs.size(), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(m->T, ts.data(), sizeof(float) * rows, hipMemcpyHostToDevice, stream);
        for (int bi = 0; bi < nbatch && e == hipSuccess; bi++) {
            const int r0 = bi * batch, nr = std::min(batch, rows - r0);
            e = launch_mlp_grad(m->W, m->X + (size_t)r0 * CR_MLP_INPUTS, m->T + r0, nr, m->part, m->grad, stream);
            m->adam_t++;
            const float c1 = 1.f - std::pow(b1, (float)m->adam_t), c2 = 1.f - std::pow(b2, (float)m->adam_t);
            if (e == hipSuccess) e = launch_adam(m->W, m->m, m->v, m->grad, lr, b1, b2, eps, c1, c2, stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(m->losses + bi, m->grad + CR_MLP_PARAMS, sizeof(float), hipMemcpyDeviceToDevice,
                                   stream);
        }
        if (e == hipSuccess) e = hipMemcpyAsync(bl.data(), m->losses, sizeof(float) * nbatch, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            set_last_error(std::string("HIP error in training: ") + hipGetErrorString(e));
            return CR_EDEVICE;
        }
        if (loss) {
            double a = 0;
            for (int bi = 0; bi < nbatch; bi++) a += (double)bl[bi] * std::min(batch, rows - bi * batch);
            loss[ep] = (float)(a / rows);
        }
    }
    return CR_OK;
}

cr_status cr_trace_policy(const cr_family *fam, int32_t p, const uint32_t *coeffs, int32_t cap, float *x, float *t,
                          int32_t *rows) {
    if (!fam || !coeffs || !rows || (x && (!t || cap < 0))) {
        set_last_error("bad arguments");
        return CR_EINVAL;
    }
    std::vector<CandRow> rs;
    std::string err;
    cr_status st = CR_OK;
    if (!trace_item(fam, p, coeffs, rs, err, st)) {
        set_last_error(err);
        return st;
    }
    *rows = (int32_t)rs.size();
    if (!x) return CR_OK;
    if ((int64_t)rs.size() > cap) {
        set_last_error("more rows than cap");
        return CR_EINVAL;
    }
    for (size_t k = 0; k < rs.size(); k++) {
        std::memcpy(x + k * CR_MLP_INPUTS, rs[k].x, sizeof(float) * CR_MLP_INPUTS);
        t[k] = rs[k].label;
    }
    return CR_OK;
}

}  // extern "C"
