// Error metrics of a reconstruction g against a reference f (the five error
// measures of Section 4.2, used by the paper's round-trip stability test):
//
//   max |f - g|, mean |f - g|, median |f - g|, rms = sqrt(mean |f - g|^2),
//   relative rms = sqrt(sum |f - g|^2 / sum |f|^2)
//
// over n complex entries, in FP64 whatever the input precision.
//
// Sums and maxima: one pass, each thread accumulating a grid-stride share,
// then a wavefront reduction by DPP lane moves (quad permutes and row
// rotations combine the 16 lanes of a row; the four row results are read with
// readlane), one LDS exchange per workgroup, and a one-workgroup pass over the
// workgroup partials.
//
// Median: the two middle order statistics (equal for odd n) by radix
// selection on the bit patterns of |f - g| (non-negative doubles order as
// their 64-bit patterns), 8 bits per pass from the top: each pass histograms,
// among the entries whose higher bits match the prefix chosen so far, the
// next byte (LDS histograms merged with global atomics), and one thread per
// statistic picks the bin that holds its rank.  Eight passes fix all 64 bits,
// so the result is the exact element, not an estimate.
#include <cstdint>

#include "sht_internal.h"

namespace sht {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxBlocks = 1024;
constexpr int kBins = 256;

// workspace layout
struct MetricsWs {
    double part[kMaxBlocks][4];                 // sum d, sum d^2, sum |f|^2, max d
    unsigned long long hist[2][kBins];          // per statistic
    unsigned long long prefix[2], rank[2];      // selection state
};

template <typename T> struct Cplx;
template <> struct Cplx<float> { using type = float2; };
template <> struct Cplx<double> { using type = double2; };

// |f - g| and |f|^2 of entry i, in FP64 (the differences of FP32 inputs are
// exact in FP64)
template <typename T>
__device__ inline void entry(const typename Cplx<T>::type *f, const typename Cplx<T>::type *g, size_t i,
                             double &d, double &f2) {
    const typename Cplx<T>::type a = f[i], b = g[i];
    const double ar = (double)a.x, ai = (double)a.y;
    const double dr = ar - (double)b.x, di = ai - (double)b.y;
    d = sqrt(dr * dr + di * di);
    f2 = ar * ar + ai * ai;
}

// one DPP lane move of a double (both 32-bit halves move the same way)
template <int CTRL>
__device__ inline double dpp(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ inline double readlane(double v, int lane) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// DPP controls: quad permutes [1,0,3,2] and [2,3,0,1] (lane xor 1, xor 2),
// row rotations by 4 and 8 lanes
constexpr int kQuadXor1 = 0xb1, kQuadXor2 = 0x4e, kRowRor4 = 0x124, kRowRor8 = 0x128;

// wavefront reduction (every lane of the wave must be active); the result is
// wave-uniform
template <bool MAX>
__device__ inline double wave_reduce(double v) {
    auto op = [](double a, double b) { return MAX ? fmax(a, b) : a + b; };
    v = op(v, dpp<kQuadXor1>(v));
    v = op(v, dpp<kQuadXor2>(v));
    v = op(v, dpp<kRowRor4>(v));
    v = op(v, dpp<kRowRor8>(v));  // every lane holds its row's result
    return op(op(readlane(v, 0), readlane(v, 16)), op(readlane(v, 32), readlane(v, 48)));
}

// block reduction of the four accumulators; thread 0 gets the result
__device__ inline void block_reduce(double (&acc)[4], double (*lds)[4]) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double r[4];
    r[0] = wave_reduce<false>(acc[0]);
    r[1] = wave_reduce<false>(acc[1]);
    r[2] = wave_reduce<false>(acc[2]);
    r[3] = wave_reduce<true>(acc[3]);
    if (lane == 0)
        for (int q = 0; q < 4; ++q) lds[wave][q] = r[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kThreads / 64; ++w) {
            r[0] += lds[w][0];
            r[1] += lds[w][1];
            r[2] += lds[w][2];
            r[3] = fmax(r[3], lds[w][3]);
        }
        for (int q = 0; q < 4; ++q) acc[q] = r[q];
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_err_sums(const typename Cplx<T>::type *f,
                                                       const typename Cplx<T>::type *g, size_t n, MetricsWs *ws) {
    __shared__ double lds[kThreads / 64][4];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const size_t stride = (size_t)gridDim.x * kThreads;
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
        double d, f2;
        entry<T>(f, g, i, d, f2);
        acc[0] += d;
        acc[1] += d * d;
        acc[2] += f2;
        acc[3] = fmax(acc[3], d);
    }
    block_reduce(acc, lds);
    if (threadIdx.x == 0)
        for (int q = 0; q < 4; ++q) ws->part[blockIdx.x][q] = acc[q];
}

// one workgroup: combine the partials into out[0], out[1], out[3], out[4];
// set up the selection (ranks (n-1)/2 and n/2, empty prefixes, zero bins)
__global__ __launch_bounds__(kThreads) void k_err_finish(int nblocks, size_t n, MetricsWs *ws, double *out) {
    __shared__ double lds[kThreads / 64][4];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += kThreads) {
        acc[0] += ws->part[b][0];
        acc[1] += ws->part[b][1];
        acc[2] += ws->part[b][2];
        acc[3] = fmax(acc[3], ws->part[b][3]);
    }
    block_reduce(acc, lds);
    for (int i = threadIdx.x; i < 2 * kBins; i += kThreads) ws->hist[i / kBins][i % kBins] = 0ull;
    if (threadIdx.x == 0) {
        const double dn = (double)n;
        out[0] = n ? acc[3] : 0.0;
        out[1] = n ? acc[0] / dn : 0.0;
        out[2] = 0.0;
        out[3] = n ? sqrt(acc[1] / dn) : 0.0;
        out[4] = acc[2] > 0.0 ? sqrt(acc[1] / acc[2]) : sqrt(acc[1]);
        ws->prefix[0] = ws->prefix[1] = 0ull;
        ws->rank[0] = n ? (unsigned long long)((n - 1) / 2) : 0ull;
        ws->rank[1] = (unsigned long long)(n / 2);
    }
}

// pass p of the selection: histogram of byte 7 - p of the entries that match
// each statistic's prefix in bytes 0 .. 6 - p (counted from the top)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_err_hist(const typename Cplx<T>::type *f,
                                                       const typename Cplx<T>::type *g, size_t n, int pass,
                                                       MetricsWs *ws) {
    __shared__ unsigned int h[2][kBins];
    for (int i = threadIdx.x; i < 2 * kBins; i += kThreads) h[i / kBins][i % kBins] = 0u;
    __syncthreads();
    const int shift = 56 - 8 * pass;
    const uint64_t hi_mask = pass == 0 ? 0ull : ~0ull << (64 - 8 * pass);
    const uint64_t p0 = ws->prefix[0], p1 = ws->prefix[1];
    const size_t stride = (size_t)gridDim.x * kThreads;
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
        double d, f2;
        entry<T>(f, g, i, d, f2);
        const uint64_t u = __builtin_bit_cast(uint64_t, d);
        const unsigned bin = (unsigned)(u >> shift) & (kBins - 1);
        if (((u ^ p0) & hi_mask) == 0) atomicAdd(&h[0][bin], 1u);
        if (((u ^ p1) & hi_mask) == 0) atomicAdd(&h[1][bin], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 2 * kBins; i += kThreads) {
        const unsigned c = h[i / kBins][i % kBins];
        if (c) atomicAdd(&ws->hist[i / kBins][i % kBins], (unsigned long long)c);
    }
}

// after pass p: each statistic takes the bin that holds its rank; the bins
// are cleared for the next pass; after the last pass the median is written
__global__ void k_err_pick(int pass, size_t n, MetricsWs *ws, double *out) {
    const int t = threadIdx.x;
    if (t < 2) {
        const int shift = 56 - 8 * pass;
        unsigned long long k = ws->rank[t], below = 0ull;
        int b = 0;
        for (; b < kBins - 1; ++b) {
            const unsigned long long c = ws->hist[t][b];
            if (k < below + c) break;
            below += c;
        }
        ws->rank[t] = k - below;
        ws->prefix[t] |= (unsigned long long)b << shift;
    }
    __syncthreads();
    for (int i = t; i < 2 * kBins; i += blockDim.x) ws->hist[i / kBins][i % kBins] = 0ull;
    if (t == 0 && pass == 7 && n > 0)
        out[2] = 0.5 * (__builtin_bit_cast(double, ws->prefix[0]) + __builtin_bit_cast(double, ws->prefix[1]));
}

template <typename T>
hipError_t launch(const void *f, const void *g, size_t n, double *out, MetricsWs *ws, hipStream_t st) {
    using C = typename Cplx<T>::type;
    size_t want = (n + kThreads - 1) / kThreads;
    const int nb = (int)(want < 1 ? 1 : (want > (size_t)kMaxBlocks ? kMaxBlocks : want));
    hipLaunchKernelGGL(k_err_sums<T>, dim3(nb), dim3(kThreads), 0, st, (const C *)f, (const C *)g, n, ws);
    hipLaunchKernelGGL(k_err_finish, dim3(1), dim3(kThreads), 0, st, nb, n, ws, out);
    for (int pass = 0; pass < 8; ++pass) {
        hipLaunchKernelGGL(k_err_hist<T>, dim3(nb), dim3(kThreads), 0, st, (const C *)f, (const C *)g, n, pass, ws);
        hipLaunchKernelGGL(k_err_pick, dim3(1), dim3(64), 0, st, pass, n, ws, out);
    }
    return hipGetLastError();
}

}  // namespace

size_t error_workspace_bytes() { return (sizeof(MetricsWs) + 255) & ~(size_t)255; }

hipError_t launch_error_metrics(bool fp64, const void *f, const void *g, size_t n, double *out, void *ws,
                                hipStream_t st) {
    return fp64 ? launch<double>(f, g, n, out, (MetricsWs *)ws, st)
                : launch<float>(f, g, n, out, (MetricsWs *)ws, st);
}

}  // namespace sht
