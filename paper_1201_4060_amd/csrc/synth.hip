// Synthetic workload generator on the device: the Kolmogorov-spectrum field
// used for benchmarks and serving loads, generated where it is consumed so
// that 1024^3 snapshots need no host memory or transfers.  It is not part of
// the interpolation method.
//
// Definition (identical to the host generator the tests use): Fourier-series
// coefficients on [0, 2pi)^3 in the real-FFT half-spectrum layout
// uhat[c][k0][k1][k2]; amplitude |k|^(-11/6) for 0 < |k| <= n/3, zero
// elsewhere; phase 2 pi u with u the top 53 bits of SplitMix64 output
// `counter` of stream c (counter = flat half-spectrum index of the canonical
// member of a Hermitian pair; the other member of a k2 = 0 pair takes the
// conjugate); three components projected divergence-free per mode,
// (I - k k^T / |k|^2); one global factor makes the mean over components of
// sum_k |uhat_k|^2 (full Hermitian spectrum) equal to 1.
#include "common.hpp"

namespace bsi {
namespace {

constexpr uint64_t GAMMA = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// uniform double of output `counter` of the (seed, stream) sequence
__device__ __forceinline__ double keyed_uniform(uint64_t seed, uint64_t stream, uint64_t counter) {
    const uint64_t base = mix64((seed * GAMMA) ^ stream);
    return double(mix64(base + (counter + 1) * GAMMA) >> 11) * 0x1.0p-53;
}

struct Mode {
    bool on;
    double re[3], im[3];
    double weight;  // 1 for k2 = 0, 2 otherwise (the mirrored half of the spectrum)
};

__device__ __forceinline__ Mode mode_values(int n, int C, uint64_t seed, int divfree, long i0, long i1, long k2) {
    Mode m{};
    const long h = n / 2 + 1;
    const long k0 = i0 <= n / 2 ? i0 : i0 - n;
    const long k1 = i1 <= n / 2 ? i1 : i1 - n;
    const long r2 = k0 * k0 + k1 * k1 + k2 * k2;
    m.on = r2 > 0 && 9 * r2 <= long(n) * n;
    if (!m.on) return m;
    const double amp = pow(double(r2), -11.0 / 12.0);
    const bool noncanon = k2 == 0 && (k0 < 0 || (k0 == 0 && k1 < 0));
    const long c0 = noncanon ? -k0 : k0, c1 = noncanon ? -k1 : k1;
    const uint64_t counter = uint64_t((((c0 % n) + n) % n * n + ((c1 % n) + n) % n) * h + k2);
    const double sgn = noncanon ? -1.0 : 1.0;
    for (int c = 0; c < C; ++c) {
        const double th = 2.0 * 3.141592653589793 * keyed_uniform(seed, uint64_t(c), counter);
        double s, co;
        sincos(th, &s, &co);
        m.re[c] = amp * co;
        m.im[c] = amp * sgn * s;
    }
    if (C == 3 && divfree) {
        const double kv[3] = {double(k0), double(k1), double(k2)};
        double dre = 0, dim = 0;
        for (int c = 0; c < 3; ++c) {
            dre += kv[c] * m.re[c];
            dim += kv[c] * m.im[c];
        }
        for (int c = 0; c < 3; ++c) {
            m.re[c] -= kv[c] * (dre / double(r2));
            m.im[c] -= kv[c] * (dim / double(r2));
        }
    }
    m.weight = k2 == 0 ? 1.0 : 2.0;
    return m;
}

constexpr int GEN_BLOCK = 256;

__global__ __launch_bounds__(GEN_BLOCK) void k_kolmo_energy(int n, int C, uint64_t seed, int divfree, long total,
                                                            double* partial) {
    __shared__ double sh[GEN_BLOCK];
    const long h = n / 2 + 1;
    double e = 0.0;
    const long idx = blockIdx.x * long(GEN_BLOCK) + threadIdx.x;
    if (idx < total) {
        const long k2 = idx % h, i1 = (idx / h) % n, i0 = idx / (h * n);
        const Mode m = mode_values(n, C, seed, divfree, i0, i1, k2);
        if (m.on)
            for (int c = 0; c < C; ++c) e += m.weight * (m.re[c] * m.re[c] + m.im[c] * m.im[c]);
    }
    sh[threadIdx.x] = e;
    __syncthreads();
    for (int s = GEN_BLOCK / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// one workgroup: sum of partial[0..m) in a fixed order, then the scale factor
__global__ __launch_bounds__(GEN_BLOCK) void k_kolmo_scale(const double* partial, long m, int C, double* scale) {
    __shared__ double sh[GEN_BLOCK];
    double e = 0.0;
    for (long i = threadIdx.x; i < m; i += GEN_BLOCK) e += partial[i];
    sh[threadIdx.x] = e;
    __syncthreads();
    for (int s = GEN_BLOCK / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) scale[0] = sh[0] > 0.0 ? sqrt(double(C) / sh[0]) : 0.0;
}

template <typename T>
__global__ __launch_bounds__(GEN_BLOCK) void k_kolmo_write(int n, int C, uint64_t seed, int divfree, long total,
                                                           const double* scale, T* out) {
    const long idx = blockIdx.x * long(GEN_BLOCK) + threadIdx.x;
    if (idx >= total) return;
    const long h = n / 2 + 1;
    const long k2 = idx % h, i1 = (idx / h) % n, i0 = idx / (h * n);
    const Mode m = mode_values(n, C, seed, divfree, i0, i1, k2);
    const double s = scale[0];
    for (int c = 0; c < C; ++c) {
        out[2 * (c * total + idx)] = m.on ? T(m.re[c] * s) : T(0);
        out[2 * (c * total + idx) + 1] = m.on ? T(m.im[c] * s) : T(0);
    }
}

}  // namespace
}  // namespace bsi

using namespace bsi;

extern "C" bsi_status bsi_synth_kolmogorov(bsi_ctx* ctx, int32_t n, int32_t ncomp, uint64_t seed,
                                           int32_t divergence_free, int32_t prec, void* uhat_dev,
                                           void* stream) {
    clear_error();
    BSI_CHECK(ctx && uhat_dev, BSI_E_INVAL, "NULL argument");
    BSI_CHECK(n >= 2 && n <= 4096 && n % 2 == 0, BSI_E_INVAL, "n must be even, 2 <= n <= 4096");
    BSI_CHECK(ncomp == 1 || ncomp == 3, BSI_E_INVAL, "ncomp must be 1 or 3");
    BSI_CHECK(prec == BSI_F64 || prec == BSI_F32, BSI_E_INVAL, "prec must be F64 (complex128) or F32 (complex64)");
    BSI_HIP(hipSetDevice(ctx->device));
    const hipStream_t s = pick_stream(ctx, stream);
    const long total = long(n) * n * (n / 2 + 1);
    const long blocks = (total + GEN_BLOCK - 1) / GEN_BLOCK;
    double* tmp = nullptr;
    BSI_CHECK(hipMalloc(&tmp, size_t(blocks + 1) * sizeof(double)) == hipSuccess, BSI_E_NOMEM,
              "generator scratch allocation failed");
    const int df = divergence_free ? 1 : 0;
    hipLaunchKernelGGL(k_kolmo_energy, dim3(unsigned(blocks)), dim3(GEN_BLOCK), 0, s, n, ncomp, seed, df, total,
                       tmp + 1);
    hipLaunchKernelGGL(k_kolmo_scale, dim3(1), dim3(GEN_BLOCK), 0, s, tmp + 1, blocks, ncomp, tmp);
    if (prec == BSI_F64)
        hipLaunchKernelGGL(k_kolmo_write<double>, dim3(unsigned(blocks)), dim3(GEN_BLOCK), 0, s, n, ncomp, seed, df,
                           total, tmp, static_cast<double*>(uhat_dev));
    else
        hipLaunchKernelGGL(k_kolmo_write<float>, dim3(unsigned(blocks)), dim3(GEN_BLOCK), 0, s, n, ncomp, seed, df,
                           total, tmp, static_cast<float*>(uhat_dev));
    const hipError_t e = hipGetLastError();
    (void)hipStreamSynchronize(s);
    (void)hipFree(tmp);
    BSI_CHECK(e == hipSuccess, BSI_E_DEVICE, std::string("generator launch failed: ") + hipGetErrorString(e));
    return BSI_OK;
}

extern "C" bsi_status bsi_ctx_trim(bsi_ctx* ctx) {
    clear_error();
    BSI_CHECK(ctx != nullptr, BSI_E_INVAL, "ctx is NULL");
    BSI_HIP(hipSetDevice(ctx->device));
    BSI_HIP(hipDeviceSynchronize());
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (auto& kv : ctx->fft_ws) (void)hipFree(kv.second.ptr);
    for (auto& kv : ctx->eval_ws) (void)hipFree(kv.second.ptr);
    ctx->fft_ws.clear();
    ctx->eval_ws.clear();
    return BSI_OK;
}
