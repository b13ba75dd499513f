// C ABI of the learned warm start (include/sbmds_mlp.h): network handle,
// weights files, features, forward pass, loss/gradient and Adam.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sbmds.h"
#include "../../include/sbmds_mlp.h"
#include "sbmds_mlp_internal.h"

using namespace sbmds;
using namespace sbmds::mlp;

struct sbmds_mlp {
    int k = 0;
    hipStream_t stream = nullptr;
    int64_t np = 0;
    float *theta = nullptr, *grad = nullptr, *adam_m = nullptr, *adam_v = nullptr;
    float *mean = nullptr, *inv_std = nullptr;  // device [19]
    float hmean[kIn], hstd[kIn];
    int64_t adam_t = 0;
    // work buffers, grown on demand
    int64_t cap_rows = 0;
    float *X = nullptr, *Z1 = nullptr, *H1 = nullptr, *Z2 = nullptr, *H2 = nullptr, *Y = nullptr, *dY = nullptr;
    float *dZ1 = nullptr, *dZ2 = nullptr, *feat = nullptr, *T = nullptr, *part = nullptr;
    int cap_seg = 0;
    int64_t *seg = nullptr;
    double *stats = nullptr, *A = nullptr, *loss_seg = nullptr, *gscale = nullptr, *loss = nullptr;
};

namespace {

constexpr int64_t kMaxRows = 4000000;

#define HIPCHK(expr)                                                                                        \
    do {                                                                                                    \
        hipError_t _e = (expr);                                                                             \
        if (_e != hipSuccess) return api_fail(SBMDS_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)
#define OKCHK(expr)            \
    do {                       \
        int _r = (expr);       \
        if (_r < 0) return _r; \
    } while (0)

// offsets of the parameter blocks in the flat vector
struct Layout {
    int64_t W1, b1, W2, b2, W3, b3, total;
    explicit Layout(int k) {
        W1 = 0;
        b1 = W1 + (int64_t)kIn * kHid;
        W2 = b1 + kHid;
        b2 = W2 + (int64_t)kHid * kHid;
        W3 = b2 + kHid;
        b3 = W3 + (int64_t)kHid * k;
        total = b3 + k;
    }
};

int dmalloc(void **p, size_t bytes) {
    *p = nullptr;
    hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 16));
    if (e != hipSuccess) {
        *p = nullptr;
        return api_fail(SBMDS_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    return SBMDS_OK;
}

void dfree(void *p) {
    if (p) (void)hipFree(p);
}

int ensure_rows(sbmds_mlp *net, int64_t rows) {
    if (rows <= net->cap_rows) return SBMDS_OK;
    HIPCHK(hipStreamSynchronize(net->stream));
    for (float *p : {net->X, net->Z1, net->H1, net->Z2, net->H2, net->Y, net->dY, net->dZ1, net->dZ2, net->feat,
                     net->T, net->part})
        dfree(p);
    net->cap_rows = 0;
    const int64_t r = std::max<int64_t>(rows, 1024);
    const int k = net->k;
    OKCHK(dmalloc((void **)&net->X, r * kIn * 4));
    OKCHK(dmalloc((void **)&net->feat, r * kIn * 4));
    OKCHK(dmalloc((void **)&net->Z1, r * kHid * 4));
    OKCHK(dmalloc((void **)&net->H1, r * kHid * 4));
    OKCHK(dmalloc((void **)&net->Z2, r * kHid * 4));
    OKCHK(dmalloc((void **)&net->H2, r * kHid * 4));
    OKCHK(dmalloc((void **)&net->dZ1, r * kHid * 4));
    OKCHK(dmalloc((void **)&net->dZ2, r * kHid * 4));
    OKCHK(dmalloc((void **)&net->Y, r * k * 4));
    OKCHK(dmalloc((void **)&net->dY, r * k * 4));
    OKCHK(dmalloc((void **)&net->T, r * k * 4));
    const int64_t part_elems = (int64_t)wgrad_chunks(r) * (kHid + 1) * kHid;
    OKCHK(dmalloc((void **)&net->part, part_elems * 4));
    net->cap_rows = r;
    return SBMDS_OK;
}

int ensure_segs(sbmds_mlp *net, int nseg) {
    if (nseg <= net->cap_seg) return SBMDS_OK;
    HIPCHK(hipStreamSynchronize(net->stream));
    dfree(net->seg);
    dfree(net->stats);
    dfree(net->A);
    dfree(net->loss_seg);
    dfree(net->gscale);
    dfree(net->loss);
    net->cap_seg = 0;
    const int k = net->k;
    OKCHK(dmalloc((void **)&net->seg, (size_t)(nseg + 1) * 8));
    OKCHK(dmalloc((void **)&net->stats, (size_t)nseg * (2 * k * k + 1) * 8));
    OKCHK(dmalloc((void **)&net->A, (size_t)nseg * k * k * 8));
    OKCHK(dmalloc((void **)&net->loss_seg, (size_t)nseg * 8));
    OKCHK(dmalloc((void **)&net->gscale, (size_t)nseg * 8));
    OKCHK(dmalloc((void **)&net->loss, 8));
    net->cap_seg = nseg;
    return SBMDS_OK;
}

int alloc_net(sbmds_mlp *net) {
    const int64_t np = net->np;
    OKCHK(dmalloc((void **)&net->theta, np * 4));
    OKCHK(dmalloc((void **)&net->grad, np * 4));
    OKCHK(dmalloc((void **)&net->adam_m, np * 4));
    OKCHK(dmalloc((void **)&net->adam_v, np * 4));
    OKCHK(dmalloc((void **)&net->mean, kIn * 4));
    OKCHK(dmalloc((void **)&net->inv_std, kIn * 4));
    HIPCHK(hipMemsetAsync(net->grad, 0, np * 4, net->stream));
    HIPCHK(hipMemsetAsync(net->adam_m, 0, np * 4, net->stream));
    HIPCHK(hipMemsetAsync(net->adam_v, 0, np * 4, net->stream));
    return SBMDS_OK;
}

int upload_norm(sbmds_mlp *net) {
    float inv[kIn];
    for (int i = 0; i < kIn; ++i) inv[i] = 1.0f / net->hstd[i];
    HIPCHK(hipMemcpyAsync(net->mean, net->hmean, kIn * 4, hipMemcpyHostToDevice, net->stream));
    HIPCHK(hipMemcpyAsync(net->inv_std, inv, kIn * 4, hipMemcpyHostToDevice, net->stream));
    HIPCHK(hipStreamSynchronize(net->stream));
    return SBMDS_OK;
}

// splitmix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014) and Box-Muller for the initial weights.
struct SplitMix {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
    double gauss() { return std::sqrt(-2.0 * std::log(uniform())) * std::cos(6.283185307179586 * uniform()); }
};

int copy_in(void *dst, const void *src, size_t bytes, int mem, hipStream_t s) {
    if (bytes == 0) return SBMDS_OK;
    HIPCHK(hipMemcpyAsync(dst, src, bytes, mem == SBMDS_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          s));
    return SBMDS_OK;
}

int forward_impl(sbmds_mlp *net, const float *feat_dev, int64_t rows) {
    const Layout L(net->k);
    hipStream_t s = net->stream;
    HIPCHK(launch_standardise(feat_dev, rows, net->mean, net->inv_std, net->X, s));
    HIPCHK(launch_gemm(1, net->X, rows, kIn, kIn, 1, net->theta + L.W1, kHid, kHid, 1, net->theta + L.b1, net->H1,
                       net->Z1, nullptr, s));
    HIPCHK(launch_gemm(1, net->H1, rows, kHid, kHid, 1, net->theta + L.W2, kHid, kHid, 1, net->theta + L.b2, net->H2,
                       net->Z2, nullptr, s));
    HIPCHK(launch_gemm(0, net->H2, rows, kHid, kHid, 1, net->theta + L.W3, net->k, net->k, 1, net->theta + L.b3,
                       net->Y, nullptr, nullptr, s));
    return SBMDS_OK;
}

int check_rows(int64_t rows) {
    if (rows < 1 || rows > kMaxRows) return api_fail(SBMDS_EINVAL, "rows must be in [1, 4000000]");
    return SBMDS_OK;
}

// ---- work buffer of the forward pass without allocation -------------------
// A fixed array per GPU (it lives until the process ends), large enough for
// one chunk of rows of the standardised features and both hidden layers;
// sbmds_mlp_forward_noalloc runs the rows through it chunk by chunk.  Host
// code never uses the array's name as an address: its device address is
// looked up once per device (hipGetSymbolAddress) and kept.
constexpr int64_t kNoAllocChunk = 8192;
constexpr int64_t kNoAllocFloats = kNoAllocChunk * (kIn + 2 * kHid);
static __device__ __align__(256) float scratch[kNoAllocFloats];
constexpr int kMaxDevices = 64;
std::array<float *, kMaxDevices> g_scratch{};
std::mutex g_scratch_mu;

// Device address of the current device's work buffer (looked up on the
// first use on that device, with the device current).
int scratch_of_current_device(float **out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return api_fail(SBMDS_ENODEV, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return api_fail(SBMDS_EHIP, "hipGetSymbolAddress returned NULL");
        g_scratch[dev] = (float *)p;
    }
    *out = g_scratch[dev];
    return SBMDS_OK;
}

}  // namespace

namespace sbmds {
namespace mlp {
int forward_device(sbmds_mlp *net, const float *feat, int64_t rows, float *Y) {
    OKCHK(check_rows(rows));
    OKCHK(ensure_rows(net, rows));
    OKCHK(forward_impl(net, feat, rows));
    HIPCHK(hipMemcpyAsync(Y, net->Y, rows * net->k * 4, hipMemcpyDeviceToDevice, net->stream));
    return SBMDS_OK;
}
int reserve_rows(sbmds_mlp *net, int64_t rows) {
    OKCHK(check_rows(rows));
    return ensure_rows(net, rows);
}
int out_width(const sbmds_mlp *net) { return net->k; }
}  // namespace mlp
}  // namespace sbmds

extern "C" {

int sbmds_mlp_create(int k, uint64_t seed, void *stream, sbmds_mlp **out) {
    api_clear_error();
    if (!out) return api_fail(SBMDS_EINVAL, "out is NULL");
    *out = nullptr;
    if (k < 1 || k > kMaxOut) return api_fail(SBMDS_EINVAL, "k must be in [1, 8]");
    float *sc = nullptr;
    OKCHK(scratch_of_current_device(&sc));  // set-up of the allocation-free forward pass on this device
    sbmds_mlp *net = new sbmds_mlp();
    net->k = k;
    net->stream = (hipStream_t)stream;
    const Layout L(k);
    net->np = L.total;
    for (int i = 0; i < kIn; ++i) {
        net->hmean[i] = 0.0f;
        net->hstd[i] = 1.0f;
    }
    int rc = alloc_net(net);
    if (rc == SBMDS_OK) {
        std::vector<float> th(net->np, 0.0f);
        SplitMix rng{seed};
        auto fill = [&](int64_t off, int64_t count, double sd) {
            for (int64_t i = 0; i < count; ++i) th[off + i] = (float)(sd * rng.gauss());
        };
        fill(L.W1, (int64_t)kIn * kHid, std::sqrt(2.0 / kIn));
        fill(L.W2, (int64_t)kHid * kHid, std::sqrt(2.0 / kHid));
        fill(L.W3, (int64_t)kHid * k, std::sqrt(1.0 / kHid));
        rc = sbmds_mlp_set_params(net, th.data());
        if (rc == SBMDS_OK) rc = upload_norm(net);
    }
    if (rc < 0) {
        sbmds_mlp_destroy(net);
        return rc;
    }
    *out = net;
    return SBMDS_OK;
}

int sbmds_mlp_load(const char *path, void *stream, sbmds_mlp **out) {
    api_clear_error();
    if (!out || !path) return api_fail(SBMDS_EINVAL, "path and out must be non-NULL");
    *out = nullptr;
    float *sc = nullptr;
    OKCHK(scratch_of_current_device(&sc));  // set-up of the allocation-free forward pass on this device
    FILE *f = std::fopen(path, "rb");
    if (!f) return api_fail(SBMDS_EINVAL, std::string("cannot open ") + path);
    char magic[8];
    int32_t hdr[4];
    float mean[kIn], sd[kIn];
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "SBMDSMLP", 8) == 0 &&
              std::fread(hdr, 4, 4, f) == 4 && hdr[0] == 1 && hdr[1] == kIn && hdr[2] == kHid && hdr[3] >= 1 &&
              hdr[3] <= kMaxOut && std::fread(mean, 4, kIn, f) == (size_t)kIn && std::fread(sd, 4, kIn, f) == (size_t)kIn;
    std::vector<float> th;
    if (ok) {
        th.resize(Layout(hdr[3]).total);
        ok = std::fread(th.data(), 4, th.size(), f) == th.size();
    }
    std::fclose(f);
    if (!ok) return api_fail(SBMDS_EINVAL, std::string("not a valid weights file: ") + path);
    for (int i = 0; i < kIn; ++i)
        if (!(sd[i] > 0.0f) || !std::isfinite(mean[i])) return api_fail(SBMDS_EINVAL, "invalid standardisation in weights file");
    for (float v : th)
        if (!std::isfinite(v)) return api_fail(SBMDS_EINVAL, "non-finite weight in weights file");
    sbmds_mlp *net = nullptr;
    OKCHK(sbmds_mlp_create(hdr[3], 0, stream, &net));
    int rc = sbmds_mlp_set_params(net, th.data());
    if (rc == SBMDS_OK) rc = sbmds_mlp_set_norm(net, mean, sd);
    if (rc < 0) {
        sbmds_mlp_destroy(net);
        return rc;
    }
    *out = net;
    return SBMDS_OK;
}

int sbmds_mlp_save(const sbmds_mlp *net, const char *path) {
    api_clear_error();
    if (!net || !path) return api_fail(SBMDS_EINVAL, "net and path must be non-NULL");
    std::vector<float> th(net->np);
    OKCHK(sbmds_mlp_get_params(net, th.data()));
    FILE *f = std::fopen(path, "wb");
    if (!f) return api_fail(SBMDS_EINVAL, std::string("cannot write ") + path);
    const int32_t hdr[4] = {1, kIn, kHid, net->k};
    bool ok = std::fwrite("SBMDSMLP", 1, 8, f) == 8 && std::fwrite(hdr, 4, 4, f) == 4 &&
              std::fwrite(net->hmean, 4, kIn, f) == (size_t)kIn && std::fwrite(net->hstd, 4, kIn, f) == (size_t)kIn &&
              std::fwrite(th.data(), 4, th.size(), f) == th.size();
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return api_fail(SBMDS_EINVAL, std::string("writing failed: ") + path);
    return SBMDS_OK;
}

int64_t sbmds_mlp_num_params(const sbmds_mlp *net) { return net ? net->np : api_fail(SBMDS_EINVAL, "net is NULL"); }

int sbmds_mlp_get_params(const sbmds_mlp *net, float *theta) {
    if (!net || !theta) return api_fail(SBMDS_EINVAL, "net and theta must be non-NULL");
    HIPCHK(hipMemcpyAsync(theta, net->theta, net->np * 4, hipMemcpyDeviceToHost, net->stream));
    HIPCHK(hipStreamSynchronize(net->stream));
    return SBMDS_OK;
}

int sbmds_mlp_set_params(sbmds_mlp *net, const float *theta) {
    if (!net || !theta) return api_fail(SBMDS_EINVAL, "net and theta must be non-NULL");
    HIPCHK(hipMemcpyAsync(net->theta, theta, net->np * 4, hipMemcpyHostToDevice, net->stream));
    HIPCHK(hipStreamSynchronize(net->stream));
    return SBMDS_OK;
}

int sbmds_mlp_set_norm(sbmds_mlp *net, const float *mean, const float *sd) {
    api_clear_error();
    if (!net || !mean || !sd) return api_fail(SBMDS_EINVAL, "net, mean and std must be non-NULL");
    for (int i = 0; i < kIn; ++i)
        if (!(sd[i] > 0.0f) || !std::isfinite(sd[i]) || !std::isfinite(mean[i]))
            return api_fail(SBMDS_EINVAL, "std must be positive and finite");
    std::memcpy(net->hmean, mean, sizeof(net->hmean));
    std::memcpy(net->hstd, sd, sizeof(net->hstd));
    return upload_norm(net);
}

int sbmds_mlp_features(const float *xyz, int64_t n, const int32_t *lmv, const void *W, int64_t l, int w_double,
                       float *feat, int mem, void *stream) {
    api_clear_error();
    if (!xyz || !lmv || !W || !feat) return api_fail(SBMDS_EINVAL, "NULL argument");
    if (mem != SBMDS_MEM_HOST && mem != SBMDS_MEM_DEVICE) return api_fail(SBMDS_EINVAL, "mem must be 0 or 1");
    if (l < 1 || n < 1 || l > n || l > 4000000) return api_fail(SBMDS_EINVAL, "need 1 <= l <= n, l <= 4000000");
    hipStream_t s = (hipStream_t)stream;
    // landmark ids must address xyz: checked on the host copy
    std::vector<int32_t> hl(l);
    HIPCHK(hipMemcpyAsync(hl.data(), lmv, l * 4, mem == SBMDS_MEM_DEVICE ? hipMemcpyDeviceToHost : hipMemcpyHostToHost,
                          s));
    HIPCHK(hipStreamSynchronize(s));
    for (int64_t j = 0; j < l; ++j)
        if (hl[j] < 0 || hl[j] >= n) return api_fail(SBMDS_EINVAL, "landmark_vertex out of range");
    const size_t wsz = w_double ? 8 : 4;
    void *dW = nullptr, *dx = nullptr, *dl = nullptr, *df = nullptr, *rowmax = nullptr;
    int rc = SBMDS_OK;
    auto release = [&]() {
        (void)hipStreamSynchronize(s);
        if (mem == SBMDS_MEM_HOST) {
            dfree(dW);
            dfree(dx);
            dfree(dl);
            dfree(df);
        }
        dfree(rowmax);
    };
    if (mem == SBMDS_MEM_HOST) {
        if ((rc = dmalloc(&dW, (size_t)l * l * wsz)) == 0 && (rc = dmalloc(&dx, (size_t)n * 12)) == 0 &&
            (rc = dmalloc(&dl, (size_t)l * 4)) == 0 && (rc = dmalloc(&df, (size_t)l * kIn * 4)) == 0) {
            if ((rc = copy_in(dW, W, (size_t)l * l * wsz, mem, s)) == 0 && (rc = copy_in(dx, xyz, (size_t)n * 12, mem, s)) == 0)
                rc = copy_in(dl, hl.data(), (size_t)l * 4, SBMDS_MEM_HOST, s);
        }
    } else {
        dW = const_cast<void *>(W);
        dx = const_cast<float *>(xyz);
        dl = const_cast<int32_t *>(lmv);
        df = feat;
    }
    if (rc == SBMDS_OK) rc = dmalloc(&rowmax, (size_t)l * 8);
    if (rc == SBMDS_OK) {
        hipError_t e = launch_features(dW, w_double, l, l, (const float *)dx, (const int32_t *)dl, (float *)df,
                                       (double *)rowmax, s);
        if (e == hipSuccess && mem == SBMDS_MEM_HOST)
            e = hipMemcpyAsync(feat, df, (size_t)l * kIn * 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = api_fail(SBMDS_EHIP, std::string("features: ") + hipGetErrorString(e));
    }
    release();
    return rc;
}

int sbmds_mlp_forward(sbmds_mlp *net, const float *feat, int64_t rows, float *Y, int mem) {
    api_clear_error();
    if (!net || !feat || !Y) return api_fail(SBMDS_EINVAL, "NULL argument");
    if (mem != SBMDS_MEM_HOST && mem != SBMDS_MEM_DEVICE) return api_fail(SBMDS_EINVAL, "mem must be 0 or 1");
    OKCHK(check_rows(rows));
    OKCHK(ensure_rows(net, rows));
    OKCHK(copy_in(net->feat, feat, (size_t)rows * kIn * 4, mem, net->stream));
    OKCHK(forward_impl(net, net->feat, rows));
    HIPCHK(hipMemcpyAsync(Y, net->Y, (size_t)rows * net->k * 4,
                          mem == SBMDS_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, net->stream));
    HIPCHK(hipStreamSynchronize(net->stream));
    return SBMDS_OK;
}

int sbmds_mlp_forward_noalloc(sbmds_mlp *net, const float *feat, int64_t rows, float *Y) {
    api_clear_error();
    if (!net || !feat || !Y) return api_fail(SBMDS_EINVAL, "NULL argument");
    if (rows < 1 || rows > kMaxRows)
        return api_fail(SBMDS_EINVAL, "rows must be in [1, 4000000] (got " + std::to_string(rows) + ")");
    float *sc = nullptr;
    OKCHK(scratch_of_current_device(&sc));
    const Layout L(net->k);
    hipStream_t s = net->stream;
    float *X = sc;
    float *H1 = X + kNoAllocChunk * kIn;
    float *H2 = H1 + kNoAllocChunk * kHid;
    for (int64_t r0 = 0; r0 < rows; r0 += kNoAllocChunk) {
        const int64_t m = std::min(kNoAllocChunk, rows - r0);
        HIPCHK(launch_standardise(feat + r0 * kIn, m, net->mean, net->inv_std, X, s));
        HIPCHK(launch_gemm(1, X, m, kIn, kIn, 1, net->theta + L.W1, kHid, kHid, 1, net->theta + L.b1, H1, nullptr,
                           nullptr, s));
        HIPCHK(launch_gemm(1, H1, m, kHid, kHid, 1, net->theta + L.W2, kHid, kHid, 1, net->theta + L.b2, H2, nullptr,
                           nullptr, s));
        HIPCHK(launch_gemm(0, H2, m, kHid, kHid, 1, net->theta + L.W3, net->k, net->k, 1, net->theta + L.b3,
                           Y + r0 * net->k, nullptr, nullptr, s));
    }
    return SBMDS_OK;
}

int sbmds_mlp_loss_grad(sbmds_mlp *net, const float *feat, const float *T, const int64_t *seg, int nseg,
                        double *loss, float *grad, int mem) {
    api_clear_error();
    if (!net || !feat || !T || !seg) return api_fail(SBMDS_EINVAL, "NULL argument");
    if (mem != SBMDS_MEM_HOST && mem != SBMDS_MEM_DEVICE) return api_fail(SBMDS_EINVAL, "mem must be 0 or 1");
    if (nseg < 1) return api_fail(SBMDS_EINVAL, "nseg must be >= 1");
    std::vector<int64_t> hs(nseg + 1);
    HIPCHK(hipMemcpyAsync(hs.data(), seg, (size_t)(nseg + 1) * 8,
                          mem == SBMDS_MEM_DEVICE ? hipMemcpyDeviceToHost : hipMemcpyHostToHost, net->stream));
    HIPCHK(hipStreamSynchronize(net->stream));
    if (hs[0] != 0) return api_fail(SBMDS_EINVAL, "seg[0] must be 0");
    for (int i = 0; i < nseg; ++i)
        if (hs[i + 1] <= hs[i]) return api_fail(SBMDS_EINVAL, "every mesh needs at least one row");
    const int64_t rows = hs[nseg];
    OKCHK(check_rows(rows));
    OKCHK(ensure_rows(net, rows));
    OKCHK(ensure_segs(net, nseg));
    const int k = net->k;
    hipStream_t s = net->stream;
    OKCHK(copy_in(net->feat, feat, (size_t)rows * kIn * 4, mem, s));
    OKCHK(copy_in(net->T, T, (size_t)rows * k * 4, mem, s));
    OKCHK(copy_in(net->seg, hs.data(), (size_t)(nseg + 1) * 8, SBMDS_MEM_HOST, s));
    OKCHK(forward_impl(net, net->feat, rows));
    HIPCHK(launch_loss(k, net->Y, net->T, net->seg, nseg, rows, kRidge, net->stats, net->A, net->loss_seg,
                       net->gscale, net->dY, net->loss, s));
    const Layout L(k);
    float *g = net->grad;
    // layer 3: dW3, db3 from H2 and dY; dZ2 = (dY W3^T) * g'(Z2)
    HIPCHK(launch_wgrad(net->H2, rows, kHid, net->dY, k, net->part, g + L.W3, g + L.b3, s));
    HIPCHK(launch_gemm(2, net->dY, rows, k, k, 1, net->theta + L.W3, kHid, 1, k, nullptr, net->dZ2, nullptr, net->Z2,
                       s));
    // layer 2
    HIPCHK(launch_wgrad(net->H1, rows, kHid, net->dZ2, kHid, net->part, g + L.W2, g + L.b2, s));
    HIPCHK(launch_gemm(2, net->dZ2, rows, kHid, kHid, 1, net->theta + L.W2, kHid, 1, kHid, nullptr, net->dZ1, nullptr,
                       net->Z1, s));
    // layer 1
    HIPCHK(launch_wgrad(net->X, rows, kIn, net->dZ1, kHid, net->part, g + L.W1, g + L.b1, s));
    if (loss) HIPCHK(hipMemcpyAsync(loss, net->loss, 8, hipMemcpyDeviceToHost, s));
    if (grad) HIPCHK(hipMemcpyAsync(grad, g, net->np * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return SBMDS_OK;
}

int sbmds_mlp_adam_step(sbmds_mlp *net, float lr) {
    api_clear_error();
    if (!net) return api_fail(SBMDS_EINVAL, "net is NULL");
    if (!(lr > 0.0f) || !std::isfinite(lr)) return api_fail(SBMDS_EINVAL, "lr must be positive");
    net->adam_t += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float bc1 = (float)(1.0 - std::pow(b1, (double)net->adam_t));
    const float bc2 = (float)(1.0 - std::pow(b2, (double)net->adam_t));
    HIPCHK(launch_adam(net->theta, net->grad, net->adam_m, net->adam_v, net->np, lr, (float)b1, (float)b2, 1e-8f, bc1,
                       bc2, net->stream));
    return SBMDS_OK;
}

void sbmds_mlp_destroy(sbmds_mlp *net) {
    if (!net) return;
    (void)hipStreamSynchronize(net->stream);
    for (void *p : {(void *)net->theta, (void *)net->grad, (void *)net->adam_m, (void *)net->adam_v, (void *)net->mean,
                    (void *)net->inv_std, (void *)net->X, (void *)net->Z1, (void *)net->H1, (void *)net->Z2,
                    (void *)net->H2, (void *)net->Y, (void *)net->dY, (void *)net->dZ1, (void *)net->dZ2,
                    (void *)net->feat, (void *)net->T, (void *)net->part, (void *)net->seg, (void *)net->stats,
                    (void *)net->A, (void *)net->loss_seg, (void *)net->gscale, (void *)net->loss})
        dfree(p);
    delete net;
}

}  // extern "C"
