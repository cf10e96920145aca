// Layout kernels between the caller's coefficient array flm[b][l*l + l + m]
// and the order-major panels the contraction streams, [m >= 0][c][l] with
// Cn columns per order, of which this launch's maps (one spin) own
// c = coff + q*B + b:
//   q = 0, 1   Re, Im of f_{l, m}
//   q = 2, 3   Re, Im of (-1)^l f_{l, -m}   (m > 0; zero for m = 0)
// The (-1)^l factor realises d^l_{m',-m} = (-1)^{l+m'} d^l_{m'm}
// (Eq. (wignerd_sym6)), so one Wigner chain per |m| serves both signs.
// Coefficients with l < |s| are read as zero (Section 2.3: no such
// harmonics exist) and written as zero.
//
// Both kernels transpose 32 x 32 (l, m) tiles through LDS so that the
// coefficient rows (contiguous in m) and the panels (contiguous in l) are
// both accessed with unit stride.
//
// flip: the launch's maps (spin s) are contracted with the factors of spin
// -s, d^l_{m',s}(pi/2) = (-1)^{l+m'} d^l_{m',-s}(pi/2) (Eq. (wignerd_sym6)):
// their panels carry one more (-1)^l here, the theta stages the (-1)^{m'}.
//
// Spin 0 (FP32 panels): each complete block of 16 degrees of a panel row is
// stored even degrees first (par16_pos), the order the FP32 and BF16x3
// spin-0 contractions read.
//
// HALF (real spin-0 signals, f_{l,-m} = (-1)^m conj(f_lm), Section 3.3):
// only q = 0, 1 are kept (c = q*B + b, 2B columns); the output side writes
// the negative orders from the symmetry.
#include "sht_internal.h"

namespace sht {

namespace {

constexpr int TL = 32;  // tile edge

template <typename T, bool HALF>
__global__ __launch_bounds__(256) void k_layout_in(int L, int s, int B, int Cn, int coff, int flip,
                                                  const typename CT<T>::type *__restrict__ flm, T *__restrict__ P) {
    using C = typename CT<T>::type;
    __shared__ T tile[4][TL][TL + 1];  // [q][l_local][m_local]
    const int l0 = blockIdx.x * TL, m0 = blockIdx.y * TL, b = blockIdx.z;
    if (l0 + TL - 1 < m0) return;  // tile entirely above the diagonal (l < m)
    const int as = s < 0 ? -s : s;
    const C *fb = flm + (size_t)b * L * L;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    // read: x runs over m (contiguous in flm)
    for (int li = ty; li < TL; li += 8) {
        const int l = l0 + li, m = m0 + tx;
        T v0 = 0, v1 = 0, v2 = 0, v3 = 0;
        if (l < L && m <= l && l >= as) {
            const size_t base = (size_t)l * l + l;
            const C p = fb[base + m];
            const T sl = (flip && (l & 1)) ? T(-1) : T(1);
            v0 = p.x * sl;
            v1 = p.y * sl;
            if (!HALF && m > 0) {
                const C q = fb[base - m];
                const T sg = ((l & 1) && !flip) ? T(-1) : T(1);
                v2 = q.x * sg;
                v3 = q.y * sg;
            }
        }
        tile[0][li][tx] = v0;
        tile[1][li][tx] = v1;
        tile[2][li][tx] = v2;
        tile[3][li][tx] = v3;
    }
    __syncthreads();
    // write: x runs over l (contiguous in the panel)
    constexpr int NQ = HALF ? 2 : 4;
    for (int mi = ty; mi < TL; mi += 8) {
        const int m = m0 + mi, l = l0 + tx;
        if (m >= L || l >= L || l < m) continue;
        const int pl = (s == 0 && sizeof(T) == 4) ? par16_pos(l, L) : l;  // FP32 spin 0: parity blocks
        for (int q = 0; q < NQ; ++q) P[((size_t)m * Cn + coff + (size_t)q * B + b) * L + pl] = tile[q][tx][mi];
    }
}

// Inverse of the above for the forward transform's contraction output
// R[m][c][l], applying the remaining factors of the conjugated Eq. (shf_exp):
//   f_{l, m}  = (-1)^s i^{m+s}              (R0 + i R1)
//   f_{l,-m}  = (-1)^s i^{s-m} (-1)^l       (R2 + i R3)      (m > 0)
template <typename T, bool HALF>
__global__ __launch_bounds__(256) void k_layout_out(int L, int s, int B, int Cn, int coff, int flip,
                                                   const T *__restrict__ R, typename CT<T>::type *__restrict__ flm) {
    using C = typename CT<T>::type;
    __shared__ T tile[4][TL][TL + 1];  // [q][m_local][l_local]
    const int l0 = blockIdx.x * TL, m0 = blockIdx.y * TL, b = blockIdx.z;
    if (l0 + TL - 1 < m0) return;
    const int as = s < 0 ? -s : s;
    constexpr int NQ = HALF ? 2 : 4;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    // read: x runs over l
    for (int mi = ty; mi < TL; mi += 8) {
        const int m = m0 + mi, l = l0 + tx;
        T v[4] = {0, 0, 0, 0};
        if (m < L && l < L && l >= m && l >= as) {
            for (int q = 0; q < NQ; ++q) v[q] = R[((size_t)m * Cn + coff + (size_t)q * B + b) * L + l];
        }
        for (int q = 0; q < 4; ++q) tile[q][mi][tx] = v[q];
    }
    __syncthreads();
    C *fb = flm + (size_t)b * L * L;
    const T sgn_s = (s & 1) ? T(-1) : T(1);
    // write: x runs over m
    for (int li = ty; li < TL; li += 8) {
        const int l = l0 + li, m = m0 + tx;
        if (l >= L || m > l) continue;
        const size_t base = (size_t)l * l + l;
        const T sf = (flip && (l & 1)) ? -sgn_s : sgn_s;
        C p{tile[0][tx][li] * sf, tile[1][tx][li] * sf};
        // multiply by i^{m+s}
        switch ((m + s) & 3) {
            case 0: break;
            case 1: p = C{-p.y, p.x}; break;
            case 2: p = C{-p.x, -p.y}; break;
            default: p = C{p.y, -p.x}; break;
        }
        fb[base + m] = p;
        if (HALF && m > 0) {
            // f_{l,-m} = (-1)^m conj(f_lm)
            fb[base - m] = (m & 1) ? C{-p.x, p.y} : C{p.x, -p.y};
        } else if (m > 0) {
            const T sl = ((l & 1) && !flip) ? -sgn_s : sgn_s;
            C q{tile[2][tx][li] * sl, tile[3][tx][li] * sl};
            switch ((s - m) & 3) {
                case 0: break;
                case 1: q = C{-q.y, q.x}; break;
                case 2: q = C{-q.x, -q.y}; break;
                default: q = C{q.y, -q.x}; break;
            }
            fb[base - m] = q;
        }
    }
}

// Spin pairs (Section 3.3): for f_{-s} = conj(f_s),
//   {}_{-s}f_{lm} = (-1)^{s+m} conj({}_s f_{l,-m}).
template <typename T>
__global__ void k_spin_pair(int L, int s, size_t total, const typename CT<T>::type *__restrict__ in,
                            typename CT<T>::type *__restrict__ out) {
    using C = typename CT<T>::type;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const size_t per = (size_t)L * L;
    const size_t b = i / per;
    const int idx = (int)(i % per);
    int l = (int)sqrt((double)idx);
    while (l * l > idx) --l;
    while ((l + 1) * (l + 1) <= idx) ++l;
    const int m = idx - l * l - l;
    const int as = s < 0 ? -s : s;
    C v{T(0), T(0)};
    if (l >= as) {
        const C x = in[b * per + (size_t)(l * l + l - m)];
        const T sg = ((s + m) & 1) ? T(-1) : T(1);
        v = C{sg * x.x, -sg * x.y};
    }
    out[i] = v;
}

}  // namespace

template <typename T>
hipError_t launch_spin_pair(int L, int s, int B, const void *in, void *out, hipStream_t st) {
    const size_t total = (size_t)B * L * L;
    hipLaunchKernelGGL(k_spin_pair<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, L, s, total,
                       (const typename CT<T>::type *)in, (typename CT<T>::type *)out);
    return hipGetLastError();
}

template hipError_t launch_spin_pair<double>(int, int, int, const void *, void *, hipStream_t);
template hipError_t launch_spin_pair<float>(int, int, int, const void *, void *, hipStream_t);

template <typename T>
hipError_t launch_layout_in(int L, int s, int B, int Cn, int coff, int flip, bool half, const void *flm, T *P,
                            hipStream_t st) {
    dim3 grid((L + TL - 1) / TL, (L + TL - 1) / TL, B);
    const typename CT<T>::type *f = (const typename CT<T>::type *)flm;
    if (half) hipLaunchKernelGGL((k_layout_in<T, true>), grid, dim3(256), 0, st, L, s, B, Cn, coff, flip, f, P);
    else hipLaunchKernelGGL((k_layout_in<T, false>), grid, dim3(256), 0, st, L, s, B, Cn, coff, flip, f, P);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_layout_out(int L, int s, int B, int Cn, int coff, int flip, bool half, const T *R, void *flm,
                             hipStream_t st) {
    dim3 grid((L + TL - 1) / TL, (L + TL - 1) / TL, B);
    typename CT<T>::type *f = (typename CT<T>::type *)flm;
    if (half) hipLaunchKernelGGL((k_layout_out<T, true>), grid, dim3(256), 0, st, L, s, B, Cn, coff, flip, R, f);
    else hipLaunchKernelGGL((k_layout_out<T, false>), grid, dim3(256), 0, st, L, s, B, Cn, coff, flip, R, f);
    return hipGetLastError();
}

template hipError_t launch_layout_in<double>(int, int, int, int, int, int, bool, const void *, double *, hipStream_t);
template hipError_t launch_layout_in<float>(int, int, int, int, int, int, bool, const void *, float *, hipStream_t);
template hipError_t launch_layout_out<double>(int, int, int, int, int, int, bool, const double *, void *,
                                              hipStream_t);
template hipError_t launch_layout_out<float>(int, int, int, int, int, int, bool, const float *, void *, hipStream_t);

}  // namespace sht
