// Layout kernels between the caller's coefficient array flm[b][l*l + l + m]
// and the order-major panels the contraction streams, [m >= 0][c][l] with
// Cn columns per order, of which map b of a segment of B maps (one spin,
// columns from coff on) owns c = coff + q*B + b:
//   q = 0, 1   Re, Im of f_{l, m}
//   q = 2, 3   Re, Im of (-1)^l f_{l, -m}   (m > 0; zero for m = 0)
// The (-1)^l factor realises d^l_{m',-m} = (-1)^{l+m'} d^l_{m'm}
// (Eq. (wignerd_sym6)), so one Wigner chain per |m| serves both signs.
// Coefficients with l < |s| are read as zero (Section 2.3: no such
// harmonics exist) and written as zero.
//
// Both kernels transpose 32 x 32 (l, m) tiles through LDS so that the
// coefficient rows (contiguous in m) and the panels (contiguous in l) are
// both accessed with unit stride.  One launch covers every map of a call:
// work item i takes map i / T and tile i mod T of the T tiles that meet the
// triangle m <= l, and each XCD runs a contiguous range of items, so that
// the tiles that share the cache lines of a coefficient row (the rows start
// at l^2 + l, not on a line) meet in one L2.  Each thread issues all its global loads before the first
// use (indices clamped to a valid entry, the values selected afterwards), so
// that a workgroup has its whole tile in flight at once.
//
// flip: the segment's maps (spin s) are contracted with the factors of spin
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

constexpr int TL = 32;       // tile edge
constexpr int NR = TL / 8;   // tile rows per thread (256 threads, 32 per row)

__host__ __device__ constexpr int tri_count(int nt) { return nt * (nt + 1) / 2; }

// Tile t of the lower triangle of 32 x 32 tiles, row by row: (lt, mt), mt <= lt.
__device__ __forceinline__ void tri_tile(int t, int &lt, int &mt) {
    int r = (int)((sqrtf(8.f * (float)t + 1.f) - 1.f) * 0.5f);
    while (tri_count(r + 1) <= t) ++r;
    while (tri_count(r) > t) --r;
    lt = r;
    mt = t - tri_count(r);
}

template <typename T, bool HALF>
__global__ __launch_bounds__(256) void k_layout_in(int L, int ntri, SpinSegs sg, int Cn,
                                                  const typename CT<T>::type *__restrict__ flm, T *__restrict__ P) {
    using C = typename CT<T>::type;
    __shared__ T tile[4][TL][TL + 1];  // [q][l_local][m_local]
    const int item = xcd_item((int)blockIdx.x, (int)gridDim.x), bg = item / ntri;
    int lt, mt;
    tri_tile(item - bg * ntri, lt, mt);
    const int l0 = lt * TL, m0 = mt * TL;
    const SpinSeg g = find_seg(sg, bg);
    const int s = g.s, as = s < 0 ? -s : s, b = bg - g.b0, flip = g.flip;
    const C *fb = flm + (size_t)bg * L * L;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    // read: x runs over m (contiguous in flm)
    C vp[NR], vn[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const int l = l0 + ty + 8 * i, m = m0 + tx;
        const bool ok = l < L && m <= l && l >= as;
        const size_t base = ok ? (size_t)l * l + l : 0;
        const int mm = ok ? m : 0;
        vp[i] = fb[base + mm];
        if (!HALF) vn[i] = fb[base - mm];
    }
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const int li = ty + 8 * i, l = l0 + li, m = m0 + tx;
        const bool ok = l < L && m <= l && l >= as;
        const T sl = (flip && (l & 1)) ? T(-1) : T(1);
        tile[0][li][tx] = ok ? vp[i].x * sl : T(0);
        tile[1][li][tx] = ok ? vp[i].y * sl : T(0);
        if (!HALF) {
            const bool okn = ok && m > 0;
            const T sn = ((l & 1) && !flip) ? T(-1) : T(1);
            tile[2][li][tx] = okn ? vn[i].x * sn : T(0);
            tile[3][li][tx] = okn ? vn[i].y * sn : T(0);
        }
    }
    __syncthreads();
    // write: x runs over l (contiguous in the panel)
    constexpr int NQ = HALF ? 2 : 4;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const int mi = ty + 8 * i, m = m0 + mi, l = l0 + tx;
        if (m >= L || l >= L || l < m) continue;
        const int pl = (s == 0 && sizeof(T) == 4) ? par16_pos(l, L) : l;  // FP32 spin 0: parity blocks
        T *row = P + ((size_t)m * Cn + g.coff + b) * L + pl;
#pragma unroll
        for (int q = 0; q < NQ; ++q) row[(size_t)q * g.B * L] = tile[q][tx][mi];
    }
}

// Inverse of the above for the forward transform's contraction output
// R[m][c][l], applying the remaining factors of the conjugated Eq. (shf_exp):
//   f_{l, m}  = (-1)^s i^{m+s}              (R0 + i R1)
//   f_{l,-m}  = (-1)^s i^{s-m} (-1)^l       (R2 + i R3)      (m > 0)
template <typename T, bool HALF>
__global__ __launch_bounds__(256) void k_layout_out(int L, int ntri, SpinSegs sg, int Cn, const T *__restrict__ R,
                                                   typename CT<T>::type *__restrict__ flm) {
    using C = typename CT<T>::type;
    __shared__ T tile[4][TL][TL + 1];  // [q][m_local][l_local]
    const int item = xcd_item((int)blockIdx.x, (int)gridDim.x), bg = item / ntri;
    int lt, mt;
    tri_tile(item - bg * ntri, lt, mt);
    const int l0 = lt * TL, m0 = mt * TL;
    const SpinSeg g = find_seg(sg, bg);
    const int s = g.s, as = s < 0 ? -s : s, b = bg - g.b0, flip = g.flip;
    constexpr int NQ = HALF ? 2 : 4;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    // read: x runs over l
    T v[NR][NQ];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const int m = m0 + ty + 8 * i, l = l0 + tx;
        const bool ok = m < L && l < L && l >= m && l >= as;
        const size_t at = ok ? ((size_t)m * Cn + g.coff + b) * L + l : 0;
        const size_t qs = ok ? (size_t)g.B * L : 0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) v[i][q] = R[at + q * qs];
    }
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const int mi = ty + 8 * i, m = m0 + mi, l = l0 + tx;
        const bool ok = m < L && l < L && l >= m && l >= as;
#pragma unroll
        for (int q = 0; q < 4; ++q) tile[q][mi][tx] = (ok && q < NQ) ? v[i][q < NQ ? q : 0] : T(0);
    }
    __syncthreads();
    C *fb = flm + (size_t)bg * L * L;
    const T sgn_s = (s & 1) ? T(-1) : T(1);
    // write: x runs over m
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const int li = ty + 8 * i, l = l0 + li, m = m0 + tx;
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

// Workgroups of a layout launch: T tiles per map, every map of the call.
static bool layout_grid(int L, const SpinSegs &sg, int &ntri, unsigned &nblk) {
    const int nt = (L + TL - 1) / TL;
    ntri = tri_count(nt);
    const long long n = (long long)ntri * sg.batch;
    if (sg.n < 1 || sg.n > SHT_MULTI_SEG_MAX || n < 1 || n > 0x7fffffffLL) return false;
    nblk = (unsigned)n;
    return true;
}

template <typename T>
hipError_t launch_layout_in(int L, const SpinSegs &sg, int Cn, bool half, const void *flm, T *P, hipStream_t st) {
    int ntri;
    unsigned nblk;
    if (!layout_grid(L, sg, ntri, nblk)) return hipErrorInvalidValue;
    const typename CT<T>::type *f = (const typename CT<T>::type *)flm;
    if (half) hipLaunchKernelGGL((k_layout_in<T, true>), dim3(nblk), dim3(256), 0, st, L, ntri, sg, Cn, f, P);
    else hipLaunchKernelGGL((k_layout_in<T, false>), dim3(nblk), dim3(256), 0, st, L, ntri, sg, Cn, f, P);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_layout_out(int L, const SpinSegs &sg, int Cn, bool half, const T *R, void *flm, hipStream_t st) {
    int ntri;
    unsigned nblk;
    if (!layout_grid(L, sg, ntri, nblk)) return hipErrorInvalidValue;
    typename CT<T>::type *f = (typename CT<T>::type *)flm;
    if (half) hipLaunchKernelGGL((k_layout_out<T, true>), dim3(nblk), dim3(256), 0, st, L, ntri, sg, Cn, R, f);
    else hipLaunchKernelGGL((k_layout_out<T, false>), dim3(nblk), dim3(256), 0, st, L, ntri, sg, Cn, R, f);
    return hipGetLastError();
}

template hipError_t launch_layout_in<double>(int, const SpinSegs &, int, bool, const void *, double *, hipStream_t);
template hipError_t launch_layout_in<float>(int, const SpinSegs &, int, bool, const void *, float *, hipStream_t);
template hipError_t launch_layout_out<double>(int, const SpinSegs &, int, bool, const double *, void *,
                                              hipStream_t);
template hipError_t launch_layout_out<float>(int, const SpinSegs &, int, bool, const float *, void *, hipStream_t);

}  // namespace sht
