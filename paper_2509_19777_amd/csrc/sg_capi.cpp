// C ABI of the learned basis surrogate network (training and inference).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/hplmm_surrogate.h"
#include "handle.h"

namespace hplmm {
namespace {

void sg_check(hipError_t e, const char *what) {
    if (e != hipSuccess) fail(HPLMM_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <class T>
T *sg_alloc(std::vector<void *> &owned, int64_t n) {
    void *p = nullptr;
    if (n > 0 && hipMalloc(&p, sizeof(T) * (size_t)n) != hipSuccess) fail(HPLMM_E_OOM, "hipMalloc failed");
    owned.push_back(p);
    return (T *)p;
}

hipStream_t to_stream(void *s) { return (hipStream_t)s; }

}  // namespace
}  // namespace hplmm

using namespace hplmm;

struct hplmm_sg_net {
    int32_t ch[5] = {0, 0, 0, 0, 0};
    int32_t max_batch = 0;
    int64_t nparam = 0;
    int64_t w_off[4] = {0, 0, 0, 0}, b_off[4] = {0, 0, 0, 0};
    float *params = nullptr, *grads = nullptr, *adam_m = nullptr, *adam_v = nullptr;
    int32_t t = 0;
    int32_t infer_precision = 32;   // forward passes of inference: 32 or 16 (bfloat16 operands)
    float *act[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};   // act[0] unused (caller's x)
    float *gbuf[2] = {nullptr, nullptr};
    float *part = nullptr;
    int32_t chunks = 0;
    double *loss_s = nullptr;
    std::vector<void *> owned;
    ~hplmm_sg_net() {
        for (void *p : owned)
            if (p) (void)hipFree(p);
    }
};

// bf16: bfloat16 operands (inference only; training keeps FP32 throughout)
static void forward_all(hplmm_sg_net &nt, const float *x, int32_t n, float *y, hipStream_t s, bool bf16 = false) {
    const float *in = x;
    for (int l = 0; l < 4; ++l) {
        float *out = (l == 3 && y) ? y : nt.act[l + 1];
        if (bf16)
            sg::launch_conv_fwd_bf16(in, nt.ch[l], nt.params + nt.w_off[l], nt.params + nt.b_off[l], out,
                                     nt.ch[l + 1], n, l < 3 ? 1 : 0, s);
        else
            sg::launch_conv_fwd(in, nt.ch[l], nt.params + nt.w_off[l], nt.params + nt.b_off[l], out, nt.ch[l + 1],
                                n, l < 3 ? 1 : 0, s);
        in = out;
    }
}

extern "C" hplmm_status hplmm_sg_create(const int32_t channels[5], int32_t max_batch, hplmm_sg_net **out) {
    return guarded([&]() -> hplmm_status {
        if (!channels || !out || max_batch < 1) fail(HPLMM_E_ARG, "NULL argument or max_batch < 1");
        for (int i = 0; i < 5; ++i)
            if (channels[i] < 1 || channels[i] > 32) fail(HPLMM_E_ARG, "every channel count must be in [1, 32]");
        auto *nt = new hplmm_sg_net();
        try {
            std::memcpy(nt->ch, channels, sizeof(nt->ch));
            nt->max_batch = max_batch;
            int64_t off = 0;
            int64_t maxc = 0;
            for (int l = 0; l < 4; ++l) {
                nt->w_off[l] = off;
                off += (int64_t)sg::NOFF * channels[l] * channels[l + 1];
                nt->b_off[l] = off;
                off += channels[l + 1];
                maxc = std::max<int64_t>(maxc, std::max(channels[l], channels[l + 1]));
            }
            nt->nparam = off;
            nt->params = sg_alloc<float>(nt->owned, off);
            nt->grads = sg_alloc<float>(nt->owned, off);
            nt->adam_m = sg_alloc<float>(nt->owned, off);
            nt->adam_v = sg_alloc<float>(nt->owned, off);
            for (float *p : {nt->params, nt->grads, nt->adam_m, nt->adam_v})
                sg_check(hipMemset(p, 0, sizeof(float) * (size_t)off), "hipMemset");
            for (int l = 1; l < 5; ++l) nt->act[l] = sg_alloc<float>(nt->owned, (int64_t)max_batch * sg::P * channels[l]);
            for (auto &g : nt->gbuf) g = sg_alloc<float>(nt->owned, (int64_t)max_batch * sg::P * maxc);
            nt->chunks = std::max<int32_t>(1, std::min<int32_t>(64, max_batch));
            int64_t plen = 0;
            for (int l = 0; l < 4; ++l)
                plen = std::max<int64_t>(plen, (int64_t)sg::NOFF * channels[l] * channels[l + 1] + channels[l + 1]);
            nt->part = sg_alloc<float>(nt->owned, plen * nt->chunks);
            nt->loss_s = sg_alloc<double>(nt->owned, max_batch);
        } catch (...) {
            delete nt;
            throw;
        }
        *out = nt;
        return HPLMM_OK;
    });
}

extern "C" hplmm_status hplmm_sg_param_count(const hplmm_sg_net *net, int64_t *count) {
    return guarded([&]() -> hplmm_status {
        if (!net || !count) fail(HPLMM_E_ARG, "NULL argument");
        *count = net->nparam;
        return HPLMM_OK;
    });
}

extern "C" hplmm_status hplmm_sg_set_params(hplmm_sg_net *net, const float *host, int64_t count) {
    return guarded([&]() -> hplmm_status {
        if (!net || !host) fail(HPLMM_E_ARG, "NULL argument");
        if (count != net->nparam) fail(HPLMM_E_ARG, "count differs from the parameter count");
        sg_check(hipMemcpy(net->params, host, sizeof(float) * (size_t)count, hipMemcpyHostToDevice), "copy");
        for (float *p : {net->adam_m, net->adam_v}) sg_check(hipMemset(p, 0, sizeof(float) * (size_t)count), "hipMemset");
        net->t = 0;
        return HPLMM_OK;
    });
}

extern "C" hplmm_status hplmm_sg_get_params(const hplmm_sg_net *net, float *host, int64_t count) {
    return guarded([&]() -> hplmm_status {
        if (!net || !host) fail(HPLMM_E_ARG, "NULL argument");
        if (count != net->nparam) fail(HPLMM_E_ARG, "count differs from the parameter count");
        sg_check(hipMemcpy(host, net->params, sizeof(float) * (size_t)count, hipMemcpyDeviceToHost), "copy");
        return HPLMM_OK;
    });
}

extern "C" hplmm_status hplmm_sg_forward(hplmm_sg_net *net, const float *x, int32_t n, float *y, void *stream) {
    return guarded([&]() -> hplmm_status {
        if (!net || !x || !y) fail(HPLMM_E_ARG, "NULL argument");
        if (n < 1 || n > net->max_batch) fail(HPLMM_E_ARG, "n must be in [1, max_batch]");
        forward_all(*net, x, n, y, to_stream(stream), net->infer_precision == 16);
        sg_check(hipGetLastError(), "kernel launch");
        return HPLMM_OK;
    });
}

extern "C" hplmm_status hplmm_sg_set_inference_precision(hplmm_sg_net *net, int32_t precision) {
    return guarded([&]() -> hplmm_status {
        if (!net) fail(HPLMM_E_ARG, "NULL argument");
        if (precision != 32 && precision != 16) fail(HPLMM_E_ARG, "precision must be 32 or 16");
        net->infer_precision = precision;
        return HPLMM_OK;
    });
}

extern "C" hplmm_status hplmm_sg_gradient(hplmm_sg_net *net, const float *x, const float *y, int32_t n, double *loss,
                                          void *stream) {
    return guarded([&]() -> hplmm_status {
        if (!net || !x || !y) fail(HPLMM_E_ARG, "NULL argument");
        if (n < 1 || n > net->max_batch) fail(HPLMM_E_ARG, "n must be in [1, max_batch]");
        hplmm_sg_net &nt = *net;
        const hipStream_t s = to_stream(stream);
        forward_all(nt, x, n, nullptr, s);
        // d loss / d output, then back through the layers: layer l's output
        // gradient g (ReLU already applied for l < 3) gives its parameter
        // gradients, and its data gradient masked by act[l] > 0 is layer
        // (l - 1)'s output gradient
        float *g = nt.gbuf[0];
        sg::launch_loss(nt.act[4], y, nt.ch[4], x, nt.ch[0], n, g, nt.loss_s, s);
        int cur = 0;
        for (int l = 3; l >= 0; --l) {
            const float *in = l == 0 ? x : nt.act[l];
            sg::launch_conv_bwd_weight(in, nt.ch[l], nt.gbuf[cur], nt.ch[l + 1], n, nt.part, nt.chunks,
                                       nt.grads + nt.w_off[l], s);
            if (l > 0) {
                sg::launch_conv_bwd_data(nt.gbuf[cur], nt.ch[l + 1], nt.params + nt.w_off[l], nt.gbuf[1 - cur], nt.ch[l],
                                         nt.act[l], n, s);
                cur = 1 - cur;
            }
        }
        sg_check(hipGetLastError(), "kernel launch");
        if (loss) {
            std::vector<double> ls((size_t)n);
            sg_check(hipMemcpyAsync(ls.data(), nt.loss_s, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost, s), "copy");
            sg_check(hipStreamSynchronize(s), "sync");
            double t = 0.0;
            for (double v : ls) t += v;
            *loss = t / n;
        }
        return HPLMM_OK;
    });
}

extern "C" hplmm_status hplmm_sg_get_grads(const hplmm_sg_net *net, float *host, int64_t count, void *stream) {
    return guarded([&]() -> hplmm_status {
        if (!net || !host) fail(HPLMM_E_ARG, "NULL argument");
        if (count != net->nparam) fail(HPLMM_E_ARG, "count differs from the parameter count");
        const hipStream_t s = to_stream(stream);
        sg_check(hipMemcpyAsync(host, net->grads, sizeof(float) * (size_t)count, hipMemcpyDeviceToHost, s), "copy");
        sg_check(hipStreamSynchronize(s), "sync");
        return HPLMM_OK;
    });
}

extern "C" hplmm_status hplmm_sg_adam(hplmm_sg_net *net, float lr, void *stream) {
    return guarded([&]() -> hplmm_status {
        if (!net) fail(HPLMM_E_ARG, "NULL argument");
        if (!(lr > 0.f)) fail(HPLMM_E_ARG, "lr must be > 0");
        net->t += 1;
        sg::launch_adam(net->params, net->grads, net->adam_m, net->adam_v, net->nparam, lr, 0.9f, 0.999f, 1e-8f,
                        net->t, to_stream(stream));
        sg_check(hipGetLastError(), "kernel launch");
        return HPLMM_OK;
    });
}

extern "C" void hplmm_sg_destroy(hplmm_sg_net *net) { delete net; }

// ---- samples of a set-up problem --------------------------------------------------
namespace hplmm {

// Box grains only: every grain node and every node of its adjacent interfaces
// must lie in one 9^3 node lattice whose corner is a multiple of 8.
void sg_build_sample_tables(Handle &h, hipStream_t s) {
    if (h.sg_ready) return;
    if (h.mortar_kind != HPLMM_MORTAR_GAUSSIAN)
        fail(HPLMM_E_ARG, "the learned surrogate's inputs need Gaussian mortars");
    const int64_t nG = (int64_t)h.gm_grain.size();
    std::vector<int32_t> origin((size_t)(3 * nG), 0);
    std::vector<float> logmean((size_t)nG, 0.f);
    for (int64_t m = 0; m < nG; ++m) {
        int32_t lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX};
        double lsum = 0.0;
        const int64_t a0 = h.sg_gnodes_ptr[(size_t)m], a1 = h.sg_gnodes_ptr[(size_t)m + 1];
        for (int64_t i = a0; i < a1; ++i) {
            const int32_t v = h.sg_gnodes[(size_t)i];
            for (int d = 0; d < 3; ++d) lo[d] = std::min(lo[d], h.sg_xyz[3 * (size_t)v + d]);
            lsum += h.sg_logtr[(size_t)v];
        }
        logmean[(size_t)m] = a1 > a0 ? (float)(lsum / (double)(a1 - a0)) : 0.f;
        for (int d = 0; d < 3; ++d) origin[(size_t)(3 * m + d)] = (lo[d] / (sg::G - 1)) * (sg::G - 1);
        auto inside = [&](int32_t v) {
            for (int d = 0; d < 3; ++d) {
                const int32_t r = h.sg_xyz[3 * (size_t)v + d] - origin[(size_t)(3 * m + d)];
                if (r < 0 || r >= sg::G) return false;
            }
            return true;
        };
        for (int64_t i = a0; i < a1; ++i)
            if (!inside(h.sg_gnodes[(size_t)i])) fail(HPLMM_E_PARTITION, "surrogate: grain does not fit an 8^3-voxel box");
        for (int64_t q = h.sg_adj_ptr[(size_t)m]; q < h.sg_adj_ptr[(size_t)m + 1]; ++q) {
            const int32_t c = h.sg_adj[(size_t)q];
            for (int64_t t = h.sg_iface_ptr[(size_t)c]; t < h.sg_iface_ptr[(size_t)c + 1]; ++t)
                if (!inside(h.sg_iface_nodes[(size_t)t]))
                    fail(HPLMM_E_PARTITION, "surrogate: an interface of a grain leaves its 8^3-voxel box");
        }
    }
    std::vector<int32_t> lcol;
    h.sg_s_m.clear();
    h.sg_s_c.clear();
    h.sg_s_a.clear();
    for (int64_t m = 0; m < nG; ++m)
        for (int64_t q = h.sg_adj_ptr[(size_t)m]; q < h.sg_adj_ptr[(size_t)m + 1]; ++q) {
            const int32_t c = h.sg_adj[(size_t)q];
            for (int32_t a = 0; a < h.sg_iface_nu[(size_t)c]; ++a) {
                h.sg_s_m.push_back((int32_t)m);
                h.sg_s_c.push_back(c);
                h.sg_s_a.push_back(a);
                lcol.push_back(h.sg_lcol[(size_t)q]);
            }
        }
    h.sg_total = (int64_t)h.sg_s_m.size();
    std::vector<int64_t> ndof((size_t)nG), nt((size_t)nG);
    for (int64_t m = 0; m < nG; ++m) {
        ndof[(size_t)m] = h.gset.n[(size_t)m];
        nt[(size_t)m] = h.gset.nt[(size_t)m];
    }
    sg::SampleArgs &a = h.sg_args;
    a.s_m = h.upload(h.sg_s_m, s);
    a.s_c = h.upload(h.sg_s_c, s);
    a.s_a = h.upload(h.sg_s_a, s);
    a.s_lcol = h.upload(lcol, s);
    a.g_origin = h.upload(origin, s);
    a.g_voff = h.upload(h.gset.voff, s);
    a.g_ndof = h.upload(ndof, s);
    a.g_roff = h.upload(h.gm_roff, s);
    a.g_nt = h.upload(nt, s);
    a.g_logmean = h.upload(logmean, s);
    a.adj_ptr = h.upload(h.sg_adj_ptr, s);
    a.adj = h.upload(h.sg_adj, s);
    a.iface_ptr = h.cm.iface_ptr;
    a.iface_nodes = h.cm.iface_nodes;
    a.H = h.cm.H;
    a.iface_hoff = h.cm.iface_hoff;
    a.iface_nu = h.cm.iface_nu;
    a.xyz = h.upload(h.sg_xyz, s);
    a.logtr = h.upload(h.sg_logtr, s);
    a.fill = h.upload(h.sg_fill, s);
    a.slot_dof = h.d_g_slot_dof;
    a.X = h.ar64;
    sg_check(hipStreamSynchronize(s), "sync");
    h.sg_ready = true;
}

void sg_net_forward(hplmm_sg_net *net, const float *x, int32_t n, float *y, hipStream_t s) {
    forward_all(*net, x, n, y, s, net->infer_precision == 16);
}
int32_t sg_net_max_batch(const hplmm_sg_net *net) { return net->max_batch; }
bool sg_net_is_basis_net(const hplmm_sg_net *net) { return net->ch[0] == 4 && net->ch[4] == 9; }

}  // namespace hplmm

extern "C" hplmm_status hplmm_sg_samples(hplmm_handle *hh, int64_t first, int64_t count, float *x_dev, float *y_dev,
                                         int32_t *meta, int64_t *total, void *stream) {
    return guarded([&]() -> hplmm_status {
        if (!hh) fail(HPLMM_E_ARG, "NULL handle");
        Handle &h = hh->h;
        const hipStream_t s = to_stream(stream);
        sg_build_sample_tables(h, s);
        if (total) *total = h.sg_total;
        if (count == 0) return HPLMM_OK;
        if (first < 0 || count < 0 || first + count > h.sg_total) fail(HPLMM_E_ARG, "sample range outside [0, total)");
        if (!x_dev) fail(HPLMM_E_ARG, "x_dev is NULL");
        if (y_dev && !h.ready) fail(HPLMM_E_STATE, "targets need a completed hplmm_setup");
        sg::launch_fill_samples(h.sg_args, first, count, x_dev, y_dev, s);
        sg_check(hipGetLastError(), "kernel launch");
        if (meta)
            for (int64_t i = 0; i < count; ++i) {
                meta[3 * i] = h.sg_s_m[(size_t)(first + i)];
                meta[3 * i + 1] = h.sg_s_c[(size_t)(first + i)];
                meta[3 * i + 2] = h.sg_s_a[(size_t)(first + i)];
            }
        return HPLMM_OK;
    });
}
