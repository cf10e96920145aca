// Torus FFT stages: the phi and theta transforms of Eq. (sht_inv_fast) and
// Eq. (fourier_series) on the odd grid N = 2L - 1 of Eq. (nodes_theta) /
// Eq. (nodes_phi), with the half-sample phases of Eq. (dft_phase) written in.
//
// Every stage is a chirp-z (Bluestein) row transform
//     y_k = b_k sum_{n < nin} (a_n x_n) c_{k-n},      k < kout,
// evaluated as a cyclic convolution of power-of-two length M >= nin + kout - 1
// in LDS: a decimation-in-frequency FFT (bit-reversed output), a product with
// the kernel spectrum (stored bit-reversed, 1/M folded in), and an inverse
// decimation-in-time FFT that takes bit-reversed input.  No bit reversal is
// ever performed.  The chirps are e^{i pi k / N} with k reduced mod 2N in
// integer arithmetic.  One workgroup transforms one row.
#include "sht_internal.h"

namespace sht {

namespace {

constexpr int kRowThreads = 256;

__device__ inline long long mod2n(long long x, long long twoN) {
    long long r = x % twoN;
    return r < 0 ? r + twoN : r;
}

template <typename C>
__device__ inline C rot_ipow(C v, int k) {  // v * i^k
    switch (k & 3) {
        case 0: return v;
        case 1: return C{-v.y, v.x};
        case 2: return C{-v.x, -v.y};
        default: return C{v.y, -v.x};
    }
}

template <typename C>
__device__ void fft_dif(C *buf, const C *tw, int M, int logM) {
    for (int lg = logM; lg >= 1; --lg) {
        const int len = 1 << lg, half = len >> 1, stride = M >> lg;
        for (int idx = threadIdx.x; idx < (M >> 1); idx += blockDim.x) {
            const int j = idx & (half - 1);
            const int i0 = ((idx >> (lg - 1)) << lg) + j, i1 = i0 + half;
            const C u = buf[i0], v = buf[i1];
            buf[i0] = cadd(u, v);
            buf[i1] = cmul(csub(u, v), tw[j * stride]);
        }
        __syncthreads();
    }
}

template <typename C>
__device__ void fft_dit_inv(C *buf, const C *tw, int M, int logM) {
    for (int lg = 1; lg <= logM; ++lg) {
        const int len = 1 << lg, half = len >> 1, stride = M >> lg;
        for (int idx = threadIdx.x; idx < (M >> 1); idx += blockDim.x) {
            const int j = idx & (half - 1);
            const int i0 = ((idx >> (lg - 1)) << lg) + j, i1 = i0 + half;
            const C u = buf[i0], v = cmulc(buf[i1], tw[j * stride]);
            buf[i0] = cadd(u, v);
            buf[i1] = csub(u, v);
        }
        __syncthreads();
    }
}

// buf <- IFFT(FFT(buf) * H): the cyclic convolution with the plan kernel.
template <typename C>
__device__ void convolve(C *buf, const C *H, const C *tw, int M, int logM) {
    fft_dif(buf, tw, M, logM);
    for (int i = threadIdx.x; i < M; i += blockDim.x) buf[i] = cmul(buf[i], H[i]);
    __syncthreads();
    fft_dit_inv(buf, tw, M, logM);
}

// ---------------------------------------------------------------- kernels --

// Inverse theta stage.  Row (b, mu): the Fourier coefficients F_{mu m'},
// m' >= 0, from the contraction output R[|mu|][c][m'] (c = q*B + b with
// q = 0,1 the real/imag part for mu >= 0 and q = 2,3 for mu < 0), times
// (-1)^s i^{-(mu+s)} (and (-1)^{m'} for mu < 0); m' < 0 filled with
// F_{mu,-m'} = (-1)^{mu+s} F_{mu m'} (Eq. (Ffourier_sym)); then
//   g_mu(theta_t) = sum_{m'} F_{mu m'} e^{i m' theta_t},  t < L.
// Output G[b][t][mu + L - 1].
template <typename T>
__global__ __launch_bounds__(kRowThreads) void k_theta_inv(FftTables<T> ft, int s, int B,
                                                           const T *__restrict__ R,
                                                           typename CT<T>::type *__restrict__ G) {
    using C = typename CT<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *buf = reinterpret_cast<C *>(smem_raw);
    const int L = ft.L, N = ft.N, M = ft.M, h = L - 1;
    const long long twoN = 2LL * N;
    const int row = blockIdx.x;
    const int mu_idx = row % N, b = row / N;
    const int mu = mu_idx - h, m = mu < 0 ? -mu : mu, neg = mu < 0;
    const int Cn = 4 * B;
    const T *Rre = R + ((size_t)m * Cn + (size_t)(2 * neg) * B + b) * L;
    const T *Rim = Rre + (size_t)B * L;
    const int phase = -(mu + s);                 // i^{-(mu+s)}
    const T sgn_s = (s & 1) ? T(-1) : T(1);
    const int fill_odd = parity((long long)mu + s);
    for (int n = threadIdx.x; n < M; n += blockDim.x) {
        C x{T(0), T(0)};
        if (n < N) {
            const int mp = n - h, amp = mp < 0 ? -mp : mp;
            C F{Rre[amp] * sgn_s, Rim[amp] * sgn_s};
            F = rot_ipow(F, phase);
            int flip = (neg && (amp & 1)) ^ (mp < 0 && fill_odd);
            if (flip) F = C{-F.x, -F.y};
            x = cmul(F, ft.e2n[mod2n((long long)n * n + n, twoN)]);
        }
        buf[n] = x;
    }
    __syncthreads();
    convolve(buf, ft.h_it, ft.tw, M, ft.logM);
    for (int t = threadIdx.x; t < L; t += blockDim.x) {
        const C y = cmul(buf[t], ft.e2n[mod2n((long long)t * t - 2LL * h * t - h, twoN)]);
        G[((size_t)b * L + t) * N + mu_idx] = y;
    }
}

// Inverse phi stage.  Row (b, t): f(theta_t, phi_p) = sum_mu g_mu(theta_t) e^{i mu phi_p}.
template <typename T>
__global__ __launch_bounds__(kRowThreads) void k_phi_inv(FftTables<T> ft,
                                                         const typename CT<T>::type *__restrict__ G,
                                                         typename CT<T>::type *__restrict__ map) {
    using C = typename CT<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *buf = reinterpret_cast<C *>(smem_raw);
    const int L = ft.L, N = ft.N, M = ft.M, h = L - 1;
    const long long twoN = 2LL * N;
    const size_t row = blockIdx.x;
    const C *in = G + row * N;
    for (int n = threadIdx.x; n < M; n += blockDim.x) {
        C x{T(0), T(0)};
        if (n < N) x = cmul(in[n], ft.e2n[mod2n((long long)n * n + n, twoN)]);
        buf[n] = x;
    }
    __syncthreads();
    convolve(buf, ft.h_ip, ft.tw, M, ft.logM);
    C *out = map + row * N;
    for (int p = threadIdx.x; p < N; p += blockDim.x)
        out[p] = cmul(buf[p], ft.e2n[mod2n((long long)p * p - 2LL * h * p - h, twoN)]);
}

// Forward phi stage.  Row (b, t): Q_mu(t) = N^-1 sum_p f(theta_t, phi_p) e^{-i mu phi_p}.
template <typename T>
__global__ __launch_bounds__(kRowThreads) void k_phi_fwd(FftTables<T> ft,
                                                         const typename CT<T>::type *__restrict__ map,
                                                         typename CT<T>::type *__restrict__ Q) {
    using C = typename CT<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *buf = reinterpret_cast<C *>(smem_raw);
    const int L = ft.L, N = ft.N, M = ft.M, h = L - 1;
    const long long twoN = 2LL * N;
    const size_t row = blockIdx.x;
    const C *in = map + row * N;
    for (int n = threadIdx.x; n < M; n += blockDim.x) {
        C x{T(0), T(0)};
        if (n < N) x = cmul(in[n], ft.e2n[mod2n(-((long long)n * n - 2LL * h * n - h), twoN)]);
        buf[n] = x;
    }
    __syncthreads();
    convolve(buf, ft.h_fd, ft.tw, M, ft.logM);
    const T invN = T(1) / T(N);
    C *out = Q + row * N;
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        const C y = cmul(buf[k], ft.e2n[mod2n(-((long long)k * k + k), twoN)]);
        out[k] = C{y.x * invN, y.y * invN};
    }
}

// Forward theta stage.  Row (b, mu): parity extension of Q_mu to the torus
// rings t < N (Section 3.2: even for mu+s even, odd otherwise), the theta DFT
//   F_{mu m''} = N^-1 sum_t Q~_mu(t) e^{-i m'' theta_t},
// then the exact sin(theta) quadrature folded over +-m' with its real
// even-offset kernel K(p) = 2/(1-p^2) (p even), 0 (p odd):
//   G'_{mu m'} = c_{m'} 2 pi sum_{m''} F_{mu m''} K(m'' - m'),  c_0 = 1, c_{m'>0} = 2.
// Written as X[|mu|][c][m'] with c = q*B + b (q = 0,1 for mu >= 0, 2,3 for
// mu < 0), times (-1)^{m'} for mu < 0 (the d^l_{m',-m} = (-1)^{l+m'} d^l_{m'm}
// symmetry; the (-1)^l part is applied on output).
template <typename T>
__global__ __launch_bounds__(kRowThreads) void k_theta_fwd(FftTables<T> ft, int s, int B,
                                                           const typename CT<T>::type *__restrict__ Q,
                                                           T *__restrict__ X) {
    using C = typename CT<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *buf = reinterpret_cast<C *>(smem_raw);
    const int L = ft.L, N = ft.N, M = ft.M, h = L - 1;
    const long long twoN = 2LL * N;
    const int row = blockIdx.x;
    const int mu_idx = row % N, b = row / N;
    const int mu = mu_idx - h, m = mu < 0 ? -mu : mu, neg = mu < 0;
    const int ext_odd = parity((long long)mu + s);
    const C *Qb = Q + (size_t)b * L * N + mu_idx;
    for (int n = threadIdx.x; n < M; n += blockDim.x) {
        C x{T(0), T(0)};
        if (n < N) {
            if (n < L) {
                x = Qb[(size_t)n * N];
            } else {
                x = Qb[(size_t)(2 * L - 2 - n) * N];
                if (ext_odd) x = C{-x.x, -x.y};
            }
            x = cmul(x, ft.e2n[mod2n(-((long long)n * n - 2LL * h * n - h), twoN)]);
        }
        buf[n] = x;
    }
    __syncthreads();
    convolve(buf, ft.h_fd, ft.tw, M, ft.logM);
    const T invN = T(1) / T(N);
    for (int k = threadIdx.x; k < M; k += blockDim.x) {
        C y{T(0), T(0)};
        if (k < N) {
            y = cmul(buf[k], ft.e2n[mod2n(-((long long)k * k + k), twoN)]);
            y = C{y.x * invN, y.y * invN};
        }
        buf[k] = y;
    }
    __syncthreads();
    convolve(buf, ft.h_fk, ft.tw, M, ft.logM);
    const int Cn = 4 * B;
    T *Xre = X + ((size_t)m * Cn + (size_t)(2 * neg) * B + b) * L;
    T *Xim = Xre + (size_t)B * L;
    const T twopi = T(6.283185307179586476925286766559);
    for (int k = threadIdx.x; k < L; k += blockDim.x) {
        T w = (k == 0 ? T(1) : T(2)) * twopi;
        if (neg && (k & 1)) w = -w;
        Xre[k] = buf[k].x * w;
        Xim[k] = buf[k].y * w;
    }
}

// Plan helper: forward DIF of `rows` sequences of length M, in place, scaled.
template <typename T>
__global__ __launch_bounds__(kRowThreads) void k_dif_rows(FftTables<T> ft, typename CT<T>::type *data,
                                                          T scale) {
    using C = typename CT<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *buf = reinterpret_cast<C *>(smem_raw);
    const int M = ft.M;
    C *row = data + (size_t)blockIdx.x * M;
    for (int i = threadIdx.x; i < M; i += blockDim.x) buf[i] = row[i];
    __syncthreads();
    fft_dif(buf, ft.tw, M, ft.logM);
    for (int i = threadIdx.x; i < M; i += blockDim.x) row[i] = C{buf[i].x * scale, buf[i].y * scale};
}

template <typename T> size_t lds_bytes(const FftTables<T> &ft) {
    return (size_t)ft.M * sizeof(typename CT<T>::type);
}

template <typename K> hipError_t set_lds(K kernel, size_t bytes) {
    if (bytes > 64 * 1024)
        return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    return hipSuccess;
}

}  // namespace

template <typename T>
hipError_t launch_theta_inv(const FftTables<T> &ft, int s, int B, const T *R, void *G, hipStream_t st) {
    const size_t lds = lds_bytes(ft);
    hipError_t e = set_lds(k_theta_inv<T>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_theta_inv<T>, dim3(ft.N * B), dim3(kRowThreads), lds, st, ft, s, B, R,
                       (typename CT<T>::type *)G);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_phi_inv(const FftTables<T> &ft, int B, const void *G, void *map, hipStream_t st) {
    const size_t lds = lds_bytes(ft);
    hipError_t e = set_lds(k_phi_inv<T>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_phi_inv<T>, dim3(ft.L * B), dim3(kRowThreads), lds, st, ft,
                       (const typename CT<T>::type *)G, (typename CT<T>::type *)map);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_phi_fwd(const FftTables<T> &ft, int B, const void *map, void *Q, hipStream_t st) {
    const size_t lds = lds_bytes(ft);
    hipError_t e = set_lds(k_phi_fwd<T>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_phi_fwd<T>, dim3(ft.L * B), dim3(kRowThreads), lds, st, ft,
                       (const typename CT<T>::type *)map, (typename CT<T>::type *)Q);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_theta_fwd(const FftTables<T> &ft, int s, int B, const void *Q, T *X, hipStream_t st) {
    const size_t lds = lds_bytes(ft);
    hipError_t e = set_lds(k_theta_fwd<T>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_theta_fwd<T>, dim3(ft.N * B), dim3(kRowThreads), lds, st, ft, s, B,
                       (const typename CT<T>::type *)Q, X);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fft_dif_inplace(const FftTables<T> &ft, typename CT<T>::type *buf, int rows, double scale,
                                  hipStream_t st) {
    const size_t lds = lds_bytes(ft);
    hipError_t e = set_lds(k_dif_rows<T>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dif_rows<T>, dim3(rows), dim3(kRowThreads), lds, st, ft, buf, (T)scale);
    return hipGetLastError();
}

#define SHT_INST(T)                                                                                      \
    template hipError_t launch_theta_inv<T>(const FftTables<T> &, int, int, const T *, void *, hipStream_t); \
    template hipError_t launch_phi_inv<T>(const FftTables<T> &, int, const void *, void *, hipStream_t);     \
    template hipError_t launch_phi_fwd<T>(const FftTables<T> &, int, const void *, void *, hipStream_t);     \
    template hipError_t launch_theta_fwd<T>(const FftTables<T> &, int, int, const void *, T *, hipStream_t); \
    template hipError_t launch_fft_dif_inplace<T>(const FftTables<T> &, typename CT<T>::type *, int, double, \
                                                  hipStream_t);
SHT_INST(double)
SHT_INST(float)
#undef SHT_INST

}  // namespace sht
