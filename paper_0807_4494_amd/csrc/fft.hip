// Torus FFT stages: the phi and theta transforms of Eq. (sht_inv_fast) and
// Eq. (fourier_series) on the odd grid N = 2L - 1 of Eq. (nodes_theta) /
// Eq. (nodes_phi), with the half-sample phases of Eq. (dft_phase) written in.
//
// Every stage is a chirp-z (Bluestein) row transform
//     y_k = b_k sum_{n < nin} (a_n x_n) c_{k-n},      k < kout,
// evaluated as a cyclic convolution of power-of-two length M >= nin + kout - 1:
// a Stockham FFT (radix 16 passes, one 2/4/8 pass when log2 M is not a
// multiple of 4) whose first pass reads the row straight from HBM with the
// chirp applied and whose last pass multiplies by the plan kernel's spectrum
// (1/M folded in), then the inverse FFT as conj(FFT(conj(.))) whose last pass
// writes the wanted outputs straight to HBM.  Intermediate passes stay in LDS.
// The chirps are e^{i pi k / N} with k reduced mod 2N in integer arithmetic.
// One workgroup of M/16 threads transforms one row; each thread holds 16
// points in registers during every pass.
#include <mutex>
#include <set>
#include <tuple>
#include <type_traits>

#include "sht_internal.h"

namespace sht {

namespace {

constexpr int kMaxRowThreads = 512;

// Threads per row: M / 16 (each thread owns 16 of the M points in every
// pass), at least one wave, at most kMaxRowThreads (M = 16384: two groups of
// 16 points per thread).
__host__ __device__ constexpr int row_threads(int M) {
    return M / 16 < 64 ? 64 : (M / 16 > kMaxRowThreads ? kMaxRowThreads : M / 16);
}

// Rows whose M-point buffer (with its pad slots) exceeds the LDS of a CU
// (FP64 at M = 16384) run as two M/2-point halves (convolve_split below).
//
// Rows held whole also keep the twiddles of their transform's second pass in
// LDS, after the padded buffer: that pass has Ns = 2^(LOGM mod 4) (16 when 4
// divides LOGM) and every thread's k = j mod Ns is one of those few values,
// so the whole table (16 Ns entries) is small; the convolutions copy it in
// and the pass reads all fifteen w^{rk} instead of forming eleven of them.
__host__ __device__ constexpr int ltw_entries(int logM, bool split) {
    return split || logM < 8 ? 0 : 16 << fft_pass_lr(logM, 0);
}
// LDS slots of an M-point buffer with its pad slots (pad(i) = i + i/16)
__host__ __device__ constexpr int padded_points(int logM) { return (1 << logM) + (1 << logM) / 16; }
template <typename T, int LOGM> __host__ __device__ constexpr bool split_rows() {
    return rows_split(1 << LOGM, 2 * (int)sizeof(T));
}

// Waves per SIMD that a row kernel's LDS buffer admits (workgroups per CU of
// 160 KB, row_threads(M) / 64 waves each), between 2 and 4: the kernels are
// compiled to that occupancy (at most 512 / waves registers per lane), so
// the compiler does not trade it for registers.
template <typename T, int LOGM> constexpr int row_waves() {
    constexpr int M = 1 << LOGM;
    constexpr int m = split_rows<T, LOGM>() ? M / 2 : M;
    constexpr int lds = (m + m / 16 + ltw_entries(LOGM, split_rows<T, LOGM>())) * 2 * (int)sizeof(T);
    constexpr int w = (160 * 1024 / lds) * (row_threads(M) / 64) / 4;
    return w < 2 ? 2 : w > 4 ? 4 : w;
}
#define SHT_ROW_KERNEL(T, LOGM) \
    __global__ __launch_bounds__(kMaxRowThreads) __attribute__((amdgpu_waves_per_eu(row_waves<T, LOGM>())))


// LDS slot of point i: one pad slot after every 16 points, so that the
// stride-16 accesses of the Stockham passes spread over the banks.
__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }

// f(std::integral_constant<int, i>) for i = 0 .. n-1, unrolled at compile time.
template <int n, int i = 0, typename F> __device__ __forceinline__ void static_for(F &&f) {
    if constexpr (i < n) {
        f(std::integral_constant<int, i>{});
        static_for<n, i + 1>(f);
    }
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

template <typename C> __device__ inline C conj(C v) { return C{v.x, -v.y}; }
template <typename C> __device__ inline C mul_mi(C v) { return C{v.y, -v.x}; }  // v * (-i)

// ---- in-register forward DFTs (sign e^{-2 pi i n k / R}) ----
template <typename C> __device__ inline void dft2(C &a, C &b) {
    const C t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <typename C> __device__ inline void dft4(C &x0, C &x1, C &x2, C &x3) {
    const C t0 = cadd(x0, x2), t1 = csub(x0, x2), t2 = cadd(x1, x3), t3 = mul_mi(csub(x1, x3));
    x0 = cadd(t0, t2);
    x2 = csub(t0, t2);
    x1 = cadd(t1, t3);
    x3 = csub(t1, t3);
}

// 8 = 4 x 2: n = n1 + 2 n2, k = 4 k1' ... written out as two radix-4 on even/odd
template <typename C, typename T> __device__ inline void dft8(C *v) {
    // x[n1 + 2 n2]: radix-4 over n2 for n1 = 0, 1
    dft4(v[0], v[2], v[4], v[6]);
    dft4(v[1], v[3], v[5], v[7]);
    // twiddle W8^{n1 k1} on the odd branch
    const T h = T(0.70710678118654752440084436210485);
    v[3] = C{(v[3].x + v[3].y) * h, (v[3].y - v[3].x) * h};   // * e^{-i pi/4}
    v[5] = mul_mi(v[5]);                                       // * e^{-i pi/2}
    v[7] = C{(v[7].y - v[7].x) * h, -(v[7].x + v[7].y) * h};  // * e^{-3 i pi/4}
    // radix-2 over n1; outputs X[k1 + 4 k2]
    C o[8];
    o[0] = cadd(v[0], v[1]); o[4] = csub(v[0], v[1]);
    o[1] = cadd(v[2], v[3]); o[5] = csub(v[2], v[3]);
    o[2] = cadd(v[4], v[5]); o[6] = csub(v[4], v[5]);
    o[3] = cadd(v[6], v[7]); o[7] = csub(v[6], v[7]);
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = o[i];
}

// 16 = 4 x 4: x[n1 + 4 n2] -> DFT4 over n2 -> W16^{n1 k1} -> DFT4 over n1 -> X[k1 + 4 k2].
// HIN: the inputs x[8..15] are zero (the first DFT4s see two zero inputs).
// HOUT: only X[0..7] are wanted (the last DFT4s form two outputs each).
template <typename C, typename T, bool HIN = false, bool HOUT = false> __device__ inline void dft16(C *v) {
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) {
        if constexpr (HIN) {
            const C a = v[n1], b = v[n1 + 4], mb = mul_mi(b);
            v[n1] = cadd(a, b);
            v[n1 + 4] = cadd(a, mb);
            v[n1 + 8] = csub(a, b);
            v[n1 + 12] = csub(a, mb);
        } else {
            dft4(v[n1], v[n1 + 4], v[n1 + 8], v[n1 + 12]);
        }
    }
    // v[n1 + 4 k1] now holds Y[n1][k1]
    const T c1 = T(0.92387953251128675612818318939679), s1 = T(0.38268343236508977172845998403040);
    const T h = T(0.70710678118654752440084436210485);
    auto tw = [&](C a, T c, T s) { return C{a.x * c + a.y * s, a.y * c - a.x * s}; };  // a * e^{-i theta}
    v[5] = tw(v[5], c1, s1);     // W16^1
    v[9] = tw(v[9], h, h);       // W16^2
    v[13] = tw(v[13], s1, c1);   // W16^3
    v[6] = tw(v[6], h, h);       // W16^2
    v[10] = mul_mi(v[10]);       // W16^4
    v[14] = tw(v[14], -h, h);    // W16^6
    v[7] = tw(v[7], s1, c1);     // W16^3
    v[11] = tw(v[11], -h, h);    // W16^6
    v[15] = tw(v[15], -c1, -s1); // W16^9
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        C *x = v + 4 * k1;
        if constexpr (HOUT) {
            const C t0 = cadd(x[0], x[2]), t1 = csub(x[0], x[2]);
            const C t2 = cadd(x[1], x[3]), t3 = mul_mi(csub(x[1], x[3]));
            x[0] = cadd(t0, t2);
            x[1] = cadd(t1, t3);
        } else {
            dft4(x[0], x[1], x[2], x[3]);
        }
    }
    // v[4 k1 + k2] holds X[k1 + 4 k2]; transpose to natural order
    constexpr int K2 = HOUT ? 2 : 4;
    C o[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < K2; ++k2) o[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
    for (int i = 0; i < 4 * K2; ++i) v[i] = o[i];
}

// R-point DFT in place; HIN / HOUT as for dft16 (the smaller radices take the
// zero inputs as they are and form every output).
template <int R, typename C, typename T, bool HIN = false, bool HOUT = false> __device__ inline void dft_r(C *v) {
    if constexpr (R == 16) {
        dft16<C, T, HIN, HOUT>(v);
    } else {
        if constexpr (HIN) {
#pragma unroll
            for (int r = R / 2; r < R; ++r) v[r] = C{T(0), T(0)};
        }
        if constexpr (R == 2) dft2(v[0], v[1]);
        else if constexpr (R == 4) dft4(v[0], v[1], v[2], v[3]);
        else dft8<C, T>(v);
    }
}

// One Stockham radix-R pass over M points, in place in LDS or from/to the
// caller's functors.  Butterfly j < M/R reads src[j + r M/R], multiplies by
// w^{r (j mod Ns)} with w = e^{-2 pi i / (Ns R)}, takes the R-point DFT and
// writes dst[(j div Ns) Ns R + (j mod Ns) + r Ns].  Every load of the pass
// (inputs, twiddles, and pre(k) for each output k, a per-output value the
// store needs, such as a chirp factor) is issued before the barrier that
// separates the reads from the writes, so that src and dst may be the same
// LDS buffer and no load waits inside the compute phase.
// HIN (first pass only, Ns = 1): the points from M/2 on are zero, so only
// r < R/2 is read.  HOUT (last pass only, Ns = M/R): only the outputs below
// M/2 are formed and handed on.
struct NoAux {};
struct NoPre {
    __host__ __device__ NoAux operator()(int) const { return NoAux{}; }
};

// Reads / writes of point n at LDS slot pad(n).  For the accesses of a
// Stockham pass, pad(b + c) = pad(b) + c + (c >> 4) for the butterfly's base
// index b and its constant offsets c = r M/R (reads) or r Ns (writes): the
// low four bits of b plus those of c never carry (b mod 16 is below
// 16 - (c mod 16) for power-of-two M, R, Ns).  The pass therefore forms
// pad(b) once and addresses every point with a constant offset.
template <typename C> struct LdsLd {
    C *buf;
    __device__ C operator()(int n) const { return buf[pad(n)]; }
};
template <typename C> struct LdsSt {
    C *buf;
    __device__ void operator()(int k, C x, NoAux) const { buf[pad(k)] = x; }
};
template <typename F> struct IsLds : std::false_type {};
template <typename C> struct IsLds<LdsLd<C>> : std::true_type {};
template <typename C> struct IsLds<LdsSt<C>> : std::true_type {};
template <int c> constexpr int padc = c + (c >> 4);

// The twiddles w^{rk}, r = 1..15, of a radix-16 butterfly from the four
// table values w^k, w^{2k}, w^{4k}, w^{8k} (t[0] is not set).
template <typename C> __device__ __forceinline__ void radix16_twiddles(const C *w4, C *t) {
    t[1] = w4[0];
    t[2] = w4[1];
    t[4] = w4[2];
    t[8] = w4[3];
    t[3] = cmul(t[1], t[2]);
    t[5] = cmul(t[1], t[4]);
    t[6] = cmul(t[2], t[4]);
    t[7] = cmul(t[3], t[4]);
#pragma unroll
    for (int r = 9; r < 16; ++r) t[r] = cmul(t[r - 8], t[8]);
}

template <int R, int LOGM, int LOGNS, typename T, bool HIN, bool HOUT, bool LW, typename Ld, typename Pre,
          typename St>
__device__ __forceinline__ void stockham_pass(const typename CT<T>::type *ptw, Ld ld, Pre pre, St st) {
    using C = typename CT<T>::type;
    using A = decltype(pre(0));
    constexpr int LOGR = R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : 4;
    constexpr int M = 1 << LOGM;
    constexpr int nb = M >> LOGR;
    constexpr int nt = row_threads(M);                  // threads per row
    constexpr int NP = (nb + nt - 1) / nt;               // butterflies per thread
    // every row kernel runs with row_threads(M) threads (M/2-point halves
    // of split rows too: both counts are kMaxRowThreads there), so with one
    // butterfly per thread and nt of them the butterfly exists and its
    // compute phase needs no guard (the load phase keeps it: without it the
    // compiler hoists loads across passes until the kernel spills)
    constexpr bool FULL = nb == nt;
    constexpr int logNs = LOGNS;
    constexpr int RIN = HIN ? R / 2 : R, ROUT = HOUT ? R / 2 : R;
    // w^{r k} sits at ptw[r Ns + k], so a wave's threads (consecutive k)
    // read one contiguous run per r.  For radix 16 from global memory only
    // w^{k}, w^{2k}, w^{4k}, w^{8k} are loaded and the rest formed as products
    // of at most four table values (loading all fifteen was slower, in FP32
    // too); from the LDS copy (LW) all fifteen are read.
    constexpr bool ALLW = R != 16 || LW;
    constexpr int Ns = 1 << LOGNS;
    constexpr int NW = LOGNS == 0 ? 1 : ALLW ? R : 4;
    static_assert(!HIN || LOGNS == 0, "zero upper half only on the first pass");
    static_assert(!HOUT || LOGNS + LOGR == LOGM, "half output only on the last pass");
    C v[NP][R];
    C w[NP][NW];
    A aux[NP][ROUT];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const int j = threadIdx.x + q * nt;
        if (j < nb) {
            const int k = j & ((1 << logNs) - 1);
            const int base = ((j >> logNs) << (logNs + LOGR)) + k;
            if constexpr (IsLds<Ld>::value) {
                const C *p = ld.buf + pad(j);
                static_for<RIN>([&](auto rr) { v[q][rr.value] = p[padc<rr.value * nb>]; });
            } else {
#pragma unroll
                for (int r = 0; r < RIN; ++r) v[q][r] = ld(j + r * nb);
            }
            if constexpr (LOGNS > 0) {
                const C *wk = ptw + k;
                if constexpr (!ALLW) {
                    w[q][0] = wk[1 * Ns];
                    w[q][1] = wk[2 * Ns];
                    w[q][2] = wk[4 * Ns];
                    w[q][3] = wk[8 * Ns];
                } else {
#pragma unroll
                    for (int r = 1; r < R; ++r) w[q][r] = wk[r * Ns];
                }
            }
#pragma unroll
            for (int r = 0; r < ROUT; ++r) aux[q][r] = pre(base + (r << logNs));
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const int j = threadIdx.x + q * nt;
        if (FULL || j < nb) {
            const int k = j & ((1 << logNs) - 1);
            if constexpr (LOGNS > 0) {
                if constexpr (!ALLW) {
                    C t[16];
                    radix16_twiddles(w[q], t);
#pragma unroll
                    for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], t[r]);
                } else {
#pragma unroll
                    for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], w[q][r]);
                }
            }
            dft_r<R, C, T, HIN, HOUT>(v[q]);
            const int base = ((j >> logNs) << (logNs + LOGR)) + k;
            if constexpr (IsLds<St>::value) {
                C *p = st.buf + pad(base);
                static_for<ROUT>([&](auto rr) { p[padc<(rr.value << logNs)>] = v[q][rr.value]; });
            } else {
#pragma unroll
                for (int r = 0; r < ROUT; ++r) st(base + (r << logNs), v[q][r], aux[q][r]);
            }
        }
    }
    __syncthreads();
}

// Forward DFT of M = 2^LOGM points: the first pass reads ld(n), the last pass
// hands output k to st(k, X_k, pre(k)); intermediate passes live in buf
// (LDS).  The first pass has radix 2^(LOGM mod 4) when LOGM is not a
// multiple of 4, all others radix 16.  HIN: ld(n) is zero for n >= M/2 and is
// not called there.  HOUT: st is called for k < M/2 only.  PSTOP: the last
// pass run (earlier than the transform's last, it leaves its output in buf).
template <int LOGM, int P, int LOGNS, typename T, bool HIN, bool HOUT, int PSTOP = fft_npass(LOGM) - 1,
          bool LTW = false, typename Ld, typename Pre, typename St>
__device__ __forceinline__ void fft_passes(typename CT<T>::type *buf, const typename CT<T>::type *ptw, Ld ld,
                                           Pre pre, St st) {
    using C = typename CT<T>::type;
    constexpr int NPASS = fft_npass(LOGM);
    constexpr int LR = fft_pass_lr(LOGM, P);
    constexpr int RR = 1 << LR;
    constexpr bool FIRST = P == 0, LAST = P == NPASS - 1;
    constexpr bool PIN = HIN && FIRST, POUT = HOUT && LAST;
    // LTW: the second pass's twiddles from their copy in LDS (ltw_load)
    constexpr bool LW = LTW && P == 1;
    const C *tp = LW ? buf + padded_points(LOGM) : ptw + fft_pass_offset(LOGM, P);
    const LdsLd<C> lbuf{buf};
    const LdsSt<C> sbuf{buf};
    if constexpr (FIRST && LAST) stockham_pass<RR, LOGM, LOGNS, T, PIN, POUT, LW>(tp, ld, pre, st);
    else if constexpr (FIRST) stockham_pass<RR, LOGM, LOGNS, T, PIN, POUT, LW>(tp, ld, NoPre{}, sbuf);
    else if constexpr (LAST) stockham_pass<RR, LOGM, LOGNS, T, PIN, POUT, LW>(tp, lbuf, pre, st);
    else stockham_pass<RR, LOGM, LOGNS, T, PIN, POUT, LW>(tp, lbuf, NoPre{}, sbuf);
    if constexpr (P < PSTOP) fft_passes<LOGM, P + 1, LOGNS + LR, T, HIN, HOUT, PSTOP, LTW>(buf, ptw, ld, pre, st);
}

// Copies the second pass's twiddles into LDS after the padded M-point
// buffer (rows held whole; ltw_entries).  Ordered before the second pass's
// reads by the barriers of the first pass.
template <int LOGM, typename T>
__device__ __forceinline__ void ltw_load(typename CT<T>::type *buf, const typename CT<T>::type *ptw) {
    typename CT<T>::type *dst = buf + padded_points(LOGM);
    const typename CT<T>::type *src = ptw + fft_pass_offset(LOGM, 1);
    for (int i = threadIdx.x; i < ltw_entries(LOGM, false); i += blockDim.x) dst[i] = src[i];
}

// Whether a convolution at M = 2^LOGM runs its spectrum product in registers
// (spectrum_pass): M a power of 16 with one butterfly per thread and pass.
template <int LOGM> constexpr bool fused_spectrum() {
    return LOGM % 4 == 0 && LOGM >= 8 && (1 << (LOGM - 4)) == row_threads(1 << LOGM);
}

// The forward transform's last radix-16 pass, the product with the spectrum
// H and the inverse transform's first pass, in registers.  With M = 16^n
// points and nb = M/16 threads, thread j ends the forward transform holding
// its outputs k = j + r nb (r < 16) and starts the inverse holding its inputs
// n = j + r nb: the same points, so the product needs no round trip through
// LDS.  The inverse is taken as conj(FFT(conj(.))), as in convolve.
template <int LOGM, typename T>
__device__ __forceinline__ void spectrum_pass(typename CT<T>::type *buf, const typename CT<T>::type *ptw,
                                              const typename CT<T>::type *H) {
    using C = typename CT<T>::type;
    static_assert(fused_spectrum<LOGM>(), "M = 16^n, one butterfly per thread");
    constexpr int nb = 1 << (LOGM - 4);  // = Ns of the forward's last pass
    const int j = threadIdx.x;
    const C *tp = ptw + fft_pass_offset(LOGM, fft_npass(LOGM) - 1) + j;
    C v[16], h[16], w[4];
    {
        const C *p = buf + pad(j);
        static_for<16>([&](auto rr) { v[rr.value] = p[padc<rr.value * nb>]; });
    }
    w[0] = tp[1 * nb];
    w[1] = tp[2 * nb];
    w[2] = tp[4 * nb];
    w[3] = tp[8 * nb];
#pragma unroll
    for (int r = 0; r < 16; ++r) h[r] = H[j + r * nb];
    __syncthreads();
    C t[16];
    radix16_twiddles(w, t);
#pragma unroll
    for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], t[r]);
    dft_r<16, C, T>(v);
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = conj(cmul(v[r], h[r]));
    dft_r<16, C, T>(v);
    C *q = buf + pad(16 * j);
    static_for<16>([&](auto rr) { q[padc<rr.value>] = v[rr.value]; });
    __syncthreads();
}

template <int LOGM, typename T, typename Ld, typename St>
__device__ __forceinline__ void fft_run(typename CT<T>::type *buf, const typename CT<T>::type *ptw, Ld ld, St st) {
    fft_passes<LOGM, 0, 0, T, false, false>(buf, ptw, ld, NoPre{}, st);
}

// Cyclic convolution with a plan kernel of spectrum H (natural order, 1/M
// folded in): y = IFFT(FFT(x) H), the inverse taken as conj(FFT(conj(.))).
// x is read through ld(n) for n < M/2 (the input must vanish from M/2 on);
// y_k is handed to st(k, y_k, pre(k)) for k < M/2, pre(k) being loaded ahead
// of the last pass's compute phase.  Every chirp-z use satisfies both:
// M >= 2N - 1 is even, so the N inputs and the (at most N) wanted outputs lie
// below M/2.
template <int LOGM, typename T, typename Ld, typename Pre, typename St>
__device__ __forceinline__ void convolve(typename CT<T>::type *buf, const typename CT<T>::type *H,
                                         const typename CT<T>::type *tw, Ld ld, Pre pre, St st) {
    using C = typename CT<T>::type;
    using A = decltype(pre(0));
    constexpr int NPASS = fft_npass(LOGM);
    constexpr bool LTW = ltw_entries(LOGM, split_rows<T, LOGM>()) > 0;
    if constexpr (LTW) ltw_load<LOGM, T>(buf, tw);
    if constexpr (fused_spectrum<LOGM>()) {
        fft_passes<LOGM, 0, 0, T, true, false, NPASS - 2, LTW>(buf, tw, ld, NoPre{}, LdsSt<C>{buf});
        spectrum_pass<LOGM, T>(buf, tw, H);
        fft_passes<LOGM, 1, 4, T, false, true, NPASS - 1, LTW>(buf, tw, LdsLd<C>{buf}, pre,
                                                                [&st](int k, C x, A a) { st(k, conj(x), a); });
    } else {
        fft_passes<LOGM, 0, 0, T, true, false, NPASS - 1, LTW>(
            buf, tw, ld, [H](int k) { return H[k]; },
            [buf](int k, C x, C hk) { buf[pad(k)] = conj(cmul(x, hk)); });
        fft_passes<LOGM, 0, 0, T, false, true, NPASS - 1, LTW>(
            buf, tw, LdsLd<C>{buf}, pre,
            [&st](int k, C x, A a) { st(k, conj(x), a); });
    }
}

// The same convolution for rows whose M-point buffer does not fit in LDS,
// as two independent M/2-point cyclic convolutions (decimation in frequency
// of the forward transform, in time of the inverse).  With w = e^{-2 pi i/M}
// and the input vanishing from M/2 on,
//   X[2k]   = FFT_{M/2}(x)[k],          X[2k+1] = FFT_{M/2}(x w^n)[k],
//   y[n]    = a[n] + w^{-n} b[n]  (n < M/2),
//   a = IDFT_{M/2}(X_even H_even),       b = IDFT_{M/2}(X_odd H_odd)
// (unnormalised inverse sums; H carries 1/M).  LDS holds one M/2-point
// buffer; the workgroup's global scratch slot holds the input (xs: ld may
// read the LDS buffer the halves overwrite) and a (as) between the halves.
// Visibility of the slot across the workgroup's threads comes from the
// barriers that close every pass.  Same ld / pre / st contract as convolve.
template <int LOGH, typename T, typename Ld, typename Pre, typename St>
__device__ __forceinline__ void convolve_split(typename CT<T>::type *buf, typename CT<T>::type *xs,
                                               typename CT<T>::type *as, const typename CT<T>::type *H,
                                               const typename CT<T>::type *twM,
                                               const typename CT<T>::type *ptwh, Ld ld, Pre pre, St st) {
    using C = typename CT<T>::type;
    using A = decltype(pre(0));
    constexpr int MH = 1 << LOGH;
    for (int n = threadIdx.x; n < MH; n += blockDim.x) xs[n] = ld(n);
    __syncthreads();
    const C *xin = xs, *asr = as;
    // even half: a = IDFT(FFT(x) H[2k])
    fft_passes<LOGH, 0, 0, T, false, false>(
        buf, ptwh, [xin](int n) { return xin[n]; }, [H](int k) { return H[2 * k]; },
        [buf](int k, C x, C hk) { buf[pad(k)] = conj(cmul(x, hk)); });
    fft_passes<LOGH, 0, 0, T, false, false>(buf, ptwh, LdsLd<C>{buf}, NoPre{},
                                            [as](int k, C x, NoAux) { as[k] = conj(x); });
    // odd half, combined with a on the way out
    fft_passes<LOGH, 0, 0, T, false, false>(
        buf, ptwh, [xin, twM](int n) { return cmul(xin[n], twM[n]); }, [H](int k) { return H[2 * k + 1]; },
        [buf](int k, C x, C hk) { buf[pad(k)] = conj(cmul(x, hk)); });
    // (a[n] and w^n are read in the store phase: held ahead with the
    // caller's per-output values they would not fit in registers)
    fft_passes<LOGH, 0, 0, T, false, false>(
        buf, ptwh, LdsLd<C>{buf}, pre,
        [&st, asr, twM](int n, C x, A u) { st(n, cadd(asr[n], cmulc(conj(x), twM[n])), u); });
}

// One row convolution of a kernel instantiated at LOGM: in LDS, or split
// with the workgroup's scratch slot (M complex values at scr + blockIdx.x M).
template <int LOGM, typename T, typename Ld, typename Pre, typename St>
__device__ __forceinline__ void row_convolve(const FftTables<T> &ft, typename CT<T>::type *buf,
                                             const typename CT<T>::type *H, typename CT<T>::type *scr, Ld ld,
                                             Pre pre, St st) {
    if constexpr (split_rows<T, LOGM>()) {
        constexpr int MH = 1 << (LOGM - 1);
        typename CT<T>::type *slot = scr + (size_t)blockIdx.x * (2 * MH);
        convolve_split<LOGM - 1, T>(buf, slot, slot + MH, H, ft.tw, ft.ptwh, ld, pre, st);
    } else {
        convolve<LOGM, T>(buf, H, ft.ptw, ld, pre, st);
    }
}

// The work items of a row kernel: one per workgroup (taken through
// xcd_item), or for split rows a loop over items, gridDim.x workgroups each
// with its own scratch slot.
template <bool SPLIT, typename F> __device__ __forceinline__ void for_items(int nitems, F body) {
    if constexpr (SPLIT) {
        for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
            body(it);
            __syncthreads();
        }
    } else {
        body(xcd_item((int)blockIdx.x, (int)gridDim.x));
    }
}

// The two adjacent complex values g[0], g[1] as one aligned piece (16 bytes
// for complex float; two 16-byte stores for complex double).
__device__ __forceinline__ void store_pair(cplx32 *g, cplx32 a, cplx32 b) {
    *reinterpret_cast<float4 *>(g) = make_float4(a.x, a.y, b.x, b.y);
}
__device__ __forceinline__ void store_pair(cplx64 *g, cplx64 a, cplx64 b) {
    g[0] = a;
    g[1] = b;
}
__device__ __forceinline__ void load_pair(const cplx32 *g, cplx32 &a, cplx32 &b) {
    const float4 v = *reinterpret_cast<const float4 *>(g);
    a = cplx32{v.x, v.y};
    b = cplx32{v.z, v.w};
}
__device__ __forceinline__ void load_pair(const cplx64 *g, cplx64 &a, cplx64 &b) {
    a = g[0];
    b = g[1];
}

// Clamped load p[min(n, N-1)]: the chirp-z functors read unconditionally and
// select zero afterwards, so that the loads of a pass issue together instead
// of one branch (and one wait) per point.
template <typename V> __device__ __forceinline__ V ldc(const V *p, int n, int N) { return p[n < N ? n : N - 1]; }

// ---------------------------------------------------------------- kernels --

// Inverse theta stage, two rows per block.  Row (b, mu): the Fourier
// coefficients F_{mu m'}, m' >= 0, from the contraction output R[|mu|][c][m']
// (c = coff + q*B + b for map b of its spin segment, q = 0,1 the real/imag
// part for mu >= 0 and q = 2,3 for mu < 0), times (-1)^s i^{-(mu+s)} (and
// (-1)^{m'} for mu < 0); m' < 0 filled
// with F_{mu,-m'} = sigma F_{mu m'}, sigma = (-1)^{mu+s} (Eq. (Ffourier_sym));
// then g_mu(theta_t) = sum_{m'} F_{mu m'} e^{i m' theta_t}, t < L.
// That symmetry makes g_mu even (sigma = 1) or odd (sigma = -1) under
// theta -> 2 pi - theta, i.e. t -> N-1-t.  Rows mu and mu+1 have opposite
// sigma, so one length-N transform of their sum Z gives both:
//   g_mu(theta_t) = (Z(theta_t) + sigma_mu Z(theta_{N-1-t})) / 2.
// Block (b, i) takes mu = 2i - (L-1) and mu + 1 (the last block of a map
// takes mu = L-1 alone).  Output: columns 2i and 2i + 1 (mu + L - 1 and
// mu + L) of every ring t, stored pair-major, G[b][i][t][2]: the block's
// output is one contiguous run of L 16-byte pieces (strided stores cost far
// more here than strided loads; the phi stage gathers the pairs of a ring).
// HALF (real spin-0 signals): only mu >= 0, from the 2-column panels, pairs
// (2i, 2i+1), rings of L orders, ring-major G[b][t][.].
template <typename T, int LOGM, bool HALF>
SHT_ROW_KERNEL(T, LOGM) void k_theta_inv(FftTables<T> ft, SpinSegs sg, int Cn,
                                                           const T *__restrict__ R,
                                                           typename CT<T>::type *__restrict__ G,
                                                           typename CT<T>::type *scr) {
    using C = typename CT<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *buf = reinterpret_cast<C *>(smem_raw);
    const int L = ft.L, N = ft.N, h = L - 1;
    const int npair = HALF ? (L + 1) / 2 : L;
    for_items<split_rows<T, LOGM>()>(npair * sg.batch, [&](int item) {
    const int pair = item % npair, bg = item / npair;
    const SpinSeg sgm = find_seg(sg, bg);
    const int s = sgm.s, B = sgm.B, coff = sgm.coff, flip = sgm.flip, b = bg - sgm.b0;
    struct Row {
        const T *re, *im;
        int neg, odd;
    };
    auto row_of = [&](int mu) {
        const int m = mu < 0 ? -mu : mu, neg = mu < 0;
        Row r;
        r.re = R + ((size_t)m * Cn + coff + (size_t)(2 * neg) * B + b) * L;
        r.im = r.re + (size_t)B * L;
        r.neg = neg;
        r.odd = parity((long long)mu + s);
        return r;
    };
    const int mua = HALF ? 2 * pair : 2 * pair - h;
    const bool two = mua < h;
    const Row ra = row_of(mua), rb = row_of(two ? mua + 1 : mua);
    // The row factors (-1)^s i^{-(mu+s)} are left out of the transformed
    // sum: the factor of mu + 1 is the factor of mu times -i, so the sum
    // carries F_a + (-i) F_b and the factor of mu multiplies the outputs.
    // Both contraction rows (m' = 0..L-1) are staged in LDS as complex
    // values, each read once (16-byte loads where the row length allows),
    // with (-1)^{m'} applied for mu < 0 and for factors of spin -s, and row b
    // times -i; a missing second row is zero.  The fill of m' < 0 reads them
    // back mirrored (the FFT's first pass only overwrites the buffer after
    // its loads).
    C *Fa = buf, *Fb = buf + L;
    const C zero{T(0), T(0)};
    {
        constexpr int V = 16 / (int)sizeof(T);
        typedef T vec __attribute__((ext_vector_type(V)));
        const bool alta = ra.neg ^ flip, altb = rb.neg ^ flip;
        auto put = [&](int m, T are, T aim, T bre, T bim) {
            const T ga = (alta && (m & 1)) ? T(-1) : T(1), gb = (altb && (m & 1)) ? T(-1) : T(1);
            Fa[m] = C{ga * are, ga * aim};
            Fb[m] = two ? C{gb * bim, -gb * bre} : zero;  // (-i) (bre + i bim)
        };
        if (L % V == 0) {
            for (int i = threadIdx.x; i < L / V; i += blockDim.x) {
                const vec are = reinterpret_cast<const vec *>(ra.re)[i], aim = reinterpret_cast<const vec *>(ra.im)[i];
                const vec bre = reinterpret_cast<const vec *>(rb.re)[i], bim = reinterpret_cast<const vec *>(rb.im)[i];
#pragma unroll
                for (int e = 0; e < V; ++e) put(i * V + e, are[e], aim[e], bre[e], bim[e]);
            }
        } else {
            for (int m = threadIdx.x; m < L; m += blockDim.x) put(m, ra.re[m], ra.im[m], rb.re[m], rb.im[m]);
        }
    }
    __syncthreads();
    // sigma of the two rows for m' < 0: they have opposite parity, so the
    // mirrored half carries sigma_a (F_a - (-i) F_b)
    const T siga = ra.odd ? T(-1) : T(1);
    const C *cha = ft.cha, *chb = ft.chb;
    auto ld = [&](int n) -> C {
        const int nc = n < N ? n : N - 1;
        const int mp = nc - h;
        const bool lo = mp >= 0;
        const int amp = lo ? mp : -mp;
        const C u = Fa[amp], v = Fb[amp], c = cha[nc];
        const T sv = lo ? T(1) : T(-1), su = lo ? T(1) : siga;
        const C x = cmul(C{su * (u.x + sv * v.x), su * (u.y + sv * v.y)}, c);
        return n < N ? x : zero;
    };
    // Z(theta_t), t < N, lands in LDS
    auto pre = [&](int t) { return ldc(chb, t, N); };
    auto st = [&](int t, C y, C c) {
        if (t < N) buf[pad(t)] = cmul(y, c);
    };
    row_convolve<LOGM, T>(ft, buf, ft.h_ip, scr, ld, pre, st);
    // columns mu and mu+1 of the rings G[b][t][.] (ring_len: even, and mu
    // starts at an even column, so a pair is one aligned 16-byte piece)
    const int rl = ring_len(L, HALF);
    // ring-major (HALF): piece t at Ga + t rl; pair-major: at Ga + 2t
    C *Ga = G + (size_t)bg * L * rl + (HALF ? mua : (size_t)pair * rl);
    const size_t ts = HALF ? (size_t)rl : 2;
    // halves, with the row factor (-1)^s i^{-(mua+s)} of both rows
    const T hf = (s & 1) ? T(-0.5) : T(0.5);
    const T sa = ra.odd ? -hf : hf;
    const int ph = -(mua + s);
    for (int t = threadIdx.x; t < L; t += blockDim.x) {
        const C z = buf[pad(t)], zr = buf[pad(N - 1 - t)];
        C *g = Ga + (size_t)t * ts;
        const C ga = rot_ipow(C{hf * z.x + sa * zr.x, hf * z.y + sa * zr.y}, ph);
        if (two) store_pair(g, ga, rot_ipow(C{hf * z.x - sa * zr.x, hf * z.y - sa * zr.y}, ph));
        else g[0] = ga;
    }
    });
}

// Inverse phi stage.  Row (b, t): f(theta_t, phi_p) = sum_mu g_mu(theta_t) e^{i mu phi_p},
// g_mu(theta_t) from the theta stage's pair-major rings: column n of ring t of
// map b at G[b][n / 2][t][n % 2] (rs = 2L values per pair, L rings per map).
template <typename T, int LOGM>
SHT_ROW_KERNEL(T, LOGM) void k_phi_inv(FftTables<T> ft, int rows, int rs,
                                                         const typename CT<T>::type *__restrict__ G,
                                                         typename CT<T>::type *__restrict__ map,
                                                         typename CT<T>::type *scr) {
    using C = typename CT<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *buf = reinterpret_cast<C *>(smem_raw);
    const int N = ft.N;
    for_items<split_rows<T, LOGM>()>(rows, [&](int item) {
    // rows in XCD-grouped order: neighbouring rings share the lines of the
    // pair-major layout, and this keeps them in one XCD's L2
    const size_t row = (size_t)item;
    const int L = ft.L;
    const C *in = G + (row / L) * L * rs + 2 * (row % L);
    C *out = map + row * N;
    const C *cha = ft.cha, *chb = ft.chb;
    // the ring's pairs gathered into LDS, one 16-byte piece per load (the
    // FFT's first pass reads them before it overwrites the buffer)
    C *sr = buf;
    for (int q = threadIdx.x; q < L; q += blockDim.x) {
        C a, c;
        load_pair(in + (size_t)q * rs, a, c);
        sr[2 * q] = a;
        sr[2 * q + 1] = c;
    }
    __syncthreads();
    auto ld = [&](int n) -> C {
        const C x = cmul(sr[n < N ? n : N - 1], ldc(cha, n, N));
        return n < N ? x : C{T(0), T(0)};
    };
    auto pre = [&](int p) { return ldc(chb, p, N); };
    auto st = [&](int p, C y, C c) {
        if (p < N) out[p] = cmul(y, c);
    };
    row_convolve<LOGM, T>(ft, buf, ft.h_ip, scr, ld, pre, st);
    });
}

// Forward phi stage.  Row (b, t): Q_mu(t) = N^-1 sum_p f(theta_t, phi_p) e^{-i mu phi_p}.
template <typename T, int LOGM>
SHT_ROW_KERNEL(T, LOGM) void k_phi_fwd(FftTables<T> ft, int rows, int rs,
                                                         const typename CT<T>::type *__restrict__ map,
                                                         typename CT<T>::type *__restrict__ Q,
                                                         typename CT<T>::type *scr) {
    using C = typename CT<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *buf = reinterpret_cast<C *>(smem_raw);
    const int N = ft.N;
    for_items<split_rows<T, LOGM>()>(rows, [&](int item) {
    const size_t row = split_rows<T, LOGM>() ? (size_t)item : (size_t)blockIdx.x;
    const C *in = map + row * N;
    C *out = Q + row * rs;
    const C *cha = ft.cha, *chb = ft.chb;
    const T invN = T(1) / T(N);
    auto ld = [&](int n) -> C {
        const C x = cmulc(ldc(in, n, N), ldc(chb, n, N));
        return n < N ? x : C{T(0), T(0)};
    };
    auto pre = [&](int k) { return ldc(cha, k, N); };
    auto st = [&](int k, C y, C c) {
        if (k < N) {
            const C z = cmulc(y, c);
            out[k] = C{z.x * invN, z.y * invN};
        }
    };
    row_convolve<LOGM, T>(ft, buf, ft.h_fd, scr, ld, pre, st);
    });
}

// Forward theta stage, two orders per block.  Column mu of the phi-stage rings
// Q[b][t][.] (read in place, stride one ring): parity extension of Q_mu to the torus rings
// t < N (Section 3.2: Q~(t) = sigma Q(2L-2-t) for t >= L, sigma = (-1)^{mu+s}),
// the theta DFT
//   F_{mu m''} = N^-1 sum_t Q~_mu(t) e^{-i m'' theta_t},
// then the exact sin(theta) quadrature, folded over +-m' (Eq. (wignerd_sym6)):
//   X_{mu m'} = c_{m'} 2 pi sum_{m''} (F_{mu m''} + sigma F_{mu,-m''}) K(m'' - m'),
// K(p) = 2/(1-p^2) (p even), 0 (p odd), c_0 = 1/2, c_{m'>0} = 1.
// The weights +-i pi/2 of the integral at p = +-1 cancel in the fold except
// at the top order m' = L-1 of an odd row, where they leave
// -i pi^2 (F_{h-1} + F_{1-h}) = -2 i pi^2 (-1)^{h-1} Q_mu(L-1) / N, the part of
// the theta = pi sample that the odd extension cannot mirror.
// Rows mu and mu+1 have opposite sigma.  With the theta = pi sample of the
// odd row set aside, their extensions are exactly even and odd, so one DFT of
// the summed extension Z gives F_mu + F_{mu+1} with F_mu even and F_{mu+1} odd
// in m'' (or the reverse), and one correlation Y = Z * K over m' in
// [-(L-1), L-1] gives both rows: X_{mu m'} = c_{m'} 2 pi (Y(m') + sigma Y(-m')).
// Written as X[|mu|][c][m'] with c = q*B + b (q = 0,1 for mu >= 0, 2,3 for
// mu < 0), times (-1)^{m'} for mu < 0 (the d^l_{m',-m} = (-1)^{l+m'} d^l_{m'm}
// symmetry; the (-1)^l part is applied on output).  Spin 0 in FP32: each
// complete block of 16 orders m' of a row is stored even orders first
// (par16_pos), the order the FP32 and BF16x3 spin-0 contractions read.
// HALF (real spin-0 signals): only mu >= 0, rings of L orders, pairs
// (2i, 2i+1), 2-column panels.
template <typename T, int LOGM, bool HALF>
SHT_ROW_KERNEL(T, LOGM) void k_theta_fwd(FftTables<T> ft, SpinSegs sg, int Cn,
                                                           const typename CT<T>::type *__restrict__ Q,
                                                           T *__restrict__ X, typename CT<T>::type *scr) {
    using C = typename CT<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *buf = reinterpret_cast<C *>(smem_raw);
    const int L = ft.L, N = ft.N, h = L - 1;
    const int npair = HALF ? (L + 1) / 2 : L;
    for_items<split_rows<T, LOGM>()>(npair * sg.batch, [&](int item) {
    const int pair = item % npair, bg = item / npair;
    const SpinSeg sgm = find_seg(sg, bg);
    const int s = sgm.s, B = sgm.B, coff = sgm.coff, flip = sgm.flip, b = bg - sgm.b0;
    const int mua = HALF ? 2 * pair : 2 * pair - h;
    const bool two = mua < h;
    const int oddA = parity((long long)mua + s);
    // columns mu and mu+1 of the rings Q[b][t][.] (ring_len, even; mu at an
    // even column), t < L
    const int rl = ring_len(L, HALF);
    const C *Qa = Q + (size_t)bg * L * rl + (HALF ? mua : mua + h);
    const C *Qb = two ? Qa + 1 : Qa;
    const C *cha = ft.cha, *chb = ft.chb;
    const T invN = T(1) / T(N);
    // the two columns staged in LDS by parity, one aligned 16-byte piece per
    // ring (each ring read once; the extension reads them back mirrored):
    // se the even row, so the odd one, whose theta = pi sample (t = L-1) is
    // left out of the extension and stored as zero; a missing second row
    // (the last block of a map) is zero
    C *se = buf, *so = buf + L;
    const C zero{T(0), T(0)};
    for (int t = threadIdx.x; t < L; t += blockDim.x) {
        C xa, xb = zero;
        if (two) load_pair(Qa + (size_t)t * rl, xa, xb);
        else xa = Qa[(size_t)t * rl];
        const C xo = oddA ? xa : xb;
        se[t] = oddA ? xb : xa;
        so[t] = t == h ? zero : xo;
    }
    __syncthreads();
    // the extended sum at n < N: even + odd below L, even - odd mirrored
    auto ld = [&](int n) -> C {
        const int nc = n < N ? n : N - 1;
        const bool lo = nc < L;
        const int i = lo ? nc : 2 * L - 2 - nc;
        const C xe = se[i], xo = so[i], c = chb[nc];
        const T sg = lo ? T(1) : T(-1);
        const C x = cmulc(C{xe.x + sg * xo.x, xe.y + sg * xo.y}, c);
        return n < N ? x : zero;
    };
    // the theta DFT lands in LDS (zero from N to M/2) as the input of the correlation
    auto pre = [&](int k) { return ldc(cha, k, N); };
    auto st_mid = [&](int k, C y, C c) {
        const C z = cmulc(y, c);
        buf[pad(k)] = k < N ? C{z.x * invN, z.y * invN} : C{T(0), T(0)};
    };
    row_convolve<LOGM, T>(ft, buf, ft.h_fd, scr, ld, pre, st_mid);
    // Y(m') at buf[m' + h], |m'| <= h
    row_convolve<LOGM, T>(ft, buf, ft.h_fk, scr, LdsLd<C>{buf}, NoPre{},
                          [buf, N](int k, C y, NoAux) { if (k < N) buf[pad(k)] = y; });
    const T twopi = T(6.283185307179586476925286766559);
    const T pi2 = T(9.8696044010893586188344909998762);
    auto store = [&](int mu, int odd, const C *Qr) {
        const int m = mu < 0 ? -mu : mu, neg = mu < 0;
        T *Xre = X + ((size_t)m * Cn + coff + (size_t)(2 * neg) * B + b) * L;
        T *Xim = Xre + (size_t)B * L;
        const T sg = odd ? T(-1) : T(1);
        // top-order term of an odd row: -2 i pi^2 (-1)^{h-1} Q(L-1) / N
        C top{T(0), T(0)};
        if (odd && h >= 1) {
            const C q = Qr[(size_t)h * rl];
            const T f = T(2) * pi2 * invN * ((h - 1) & 1 ? T(-1) : T(1));
            top = C{f * q.y, -f * q.x};
        }
        for (int k = threadIdx.x; k < L; k += blockDim.x) {
            const C yp = buf[pad(h + k)], ym = buf[pad(h - k)];
            const T w = (k == 0 ? T(0.5) : T(1)) * twopi;
            C x{(yp.x + sg * ym.x) * w, (yp.y + sg * ym.y) * w};
            if (k == h) x = cadd(x, top);
            const T sgn = ((neg ^ flip) && (k & 1)) ? T(-1) : T(1);
            const int pk = (s == 0 && sizeof(T) == 4) ? par16_pos(k, L) : k;  // FP32 spin 0: parity blocks
            Xre[pk] = x.x * sgn;
            Xim[pk] = x.y * sgn;
        }
    };
    store(mua, oddA, Qa);
    if (two) store(mua + 1, !oddA, Qb);
    });
}

// Real spin-0 maps, two rings per transform (rows r and r+1 of the [B*L]
// rings).  Inverse phi stage from the orders m >= 0 of G'[r][m] (L entries),
// g_{-m} = conj(g_m) (Section 3.3): each ring's samples are real, so the
// spectrum g_r + i g_{r+1} gives ring r in the real part and ring r+1 in the
// imaginary part of one synthesis.
template <typename T, int LOGM>
SHT_ROW_KERNEL(T, LOGM) void k_phi_inv_real(FftTables<T> ft, int rows,
                                                              const typename CT<T>::type *__restrict__ G,
                                                              T *__restrict__ map, typename CT<T>::type *scr) {
    using C = typename CT<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *buf = reinterpret_cast<C *>(smem_raw);
    const int L = ft.L, N = ft.N, h = L - 1;
    for_items<split_rows<T, LOGM>()>((rows + 1) / 2, [&](int item) {
    const size_t r0 = 2 * (split_rows<T, LOGM>() ? (size_t)item : (size_t)blockIdx.x);
    const bool two = r0 + 1 < (size_t)rows;
    const size_t rl = ring_len(L, true);
    const C *ina = G + r0 * rl, *inb = two ? ina + rl : ina;
    T *outa = map + r0 * N, *outb = outa + N;
    const C *cha = ft.cha, *chb = ft.chb;
    auto ld = [&](int n) -> C {
        const int nc = n < N ? n : N - 1;
        const int mu = nc - h, am = mu < 0 ? -mu : mu;
        C a = ina[am], b = inb[am];
        const C c = cha[nc];
        if (!two) b = C{T(0), T(0)};
        if (mu < 0) {
            a = conj(a);
            b = conj(b);
        }
        const C x = cmul(C{a.x - b.y, a.y + b.x}, c);  // a + i b
        return n < N ? x : C{T(0), T(0)};
    };
    auto pre = [&](int p) { return ldc(chb, p, N); };
    auto st = [&](int p, C y, C c) {
        if (p < N) {
            const C z = cmul(y, c);
            outa[p] = z.x;
            if (two) outb[p] = z.y;
        }
    };
    row_convolve<LOGM, T>(ft, buf, ft.h_ip, scr, ld, pre, st);
    });
}

// Forward phi stage of two real rings r, r+1 at once, keeping the orders
// m >= 0: the DFT Z of x_r + i x_{r+1} gives
//   Q_r(m) = (Z_m + conj(Z_{-m})) / 2,  Q_{r+1}(m) = (Z_m - conj(Z_{-m})) / (2i),
// with Q(m) = N^-1 sum_p x(phi_p) e^{-i m phi_p}.  Output Q[r][m], m < L.
template <typename T, int LOGM>
SHT_ROW_KERNEL(T, LOGM) void k_phi_fwd_real(FftTables<T> ft, int rows,
                                                              const T *__restrict__ map,
                                                              typename CT<T>::type *__restrict__ Q,
                                                              typename CT<T>::type *scr) {
    using C = typename CT<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *buf = reinterpret_cast<C *>(smem_raw);
    const int L = ft.L, N = ft.N, h = L - 1;
    for_items<split_rows<T, LOGM>()>((rows + 1) / 2, [&](int item) {
    const size_t r0 = 2 * (split_rows<T, LOGM>() ? (size_t)item : (size_t)blockIdx.x);
    const bool two = r0 + 1 < (size_t)rows;
    const T *ina = map + r0 * N, *inb = two ? ina + N : ina;
    const size_t rl = ring_len(L, true);
    C *outa = Q + r0 * rl, *outb = outa + rl;
    const C *cha = ft.cha, *chb = ft.chb;
    const T invN = T(1) / T(N);
    auto ld = [&](int n) -> C {
        const int nc = n < N ? n : N - 1;
        const T a = ina[nc], b = inb[nc];
        const C x = cmulc(C{a, two ? b : T(0)}, chb[nc]);
        return n < N ? x : C{T(0), T(0)};
    };
    // Z_{k-h}, k < N, lands in LDS
    auto pre = [&](int k) { return ldc(cha, k, N); };
    auto st = [&](int k, C y, C c) {
        if (k < N) {
            const C z = cmulc(y, c);
            buf[pad(k)] = C{z.x * invN, z.y * invN};
        }
    };
    row_convolve<LOGM, T>(ft, buf, ft.h_fd, scr, ld, pre, st);
    for (int m = threadIdx.x; m < L; m += blockDim.x) {
        const C zp = buf[pad(h + m)], zm = buf[pad(h - m)];
        outa[m] = C{T(0.5) * (zp.x + zm.x), T(0.5) * (zp.y - zm.y)};
        if (two) outb[m] = C{T(0.5) * (zp.y + zm.y), T(0.5) * (zm.x - zp.x)};
    }
    });
}

// Theta DFT alone, for the paper's own forward transform (per-order
// triangular systems).  Row (b, mu) of Q'[b][mu][t]: the extension of
// Section 3.2 chosen by the parity of mu+s (the theta = pi sample kept as it
// is) and F_{mu m'} = N^-1 sum_t Q~_mu(t) e^{-i m' theta_t} for m' in [0, L),
// written to F[b][mu + L - 1][m'].
template <typename T, int LOGM>
SHT_ROW_KERNEL(T, LOGM) void k_theta_dft(FftTables<T> ft, int s,
                                                           const typename CT<T>::type *__restrict__ Q,
                                                           typename CT<T>::type *__restrict__ F) {
    using C = typename CT<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *buf = reinterpret_cast<C *>(smem_raw);
    const int L = ft.L, N = ft.N, h = L - 1;
    const size_t row = blockIdx.x;                  // b * N + mu_idx
    const int mu = (int)(row % N) - h;
    const int odd = parity((long long)mu + s);
    const C *Qr = Q + row * L;
    C *Fr = F + row * L;
    const C *cha = ft.cha, *chb = ft.chb;
    const T invN = T(1) / T(N);
    auto ld = [&](int n) -> C {
        const int nc = n < N ? n : N - 1;
        C x = Qr[nc < L ? nc : 2 * L - 2 - nc];
        if (odd && nc >= L) x = C{-x.x, -x.y};
        const C y = cmulc(x, chb[nc]);
        return n < N ? y : C{T(0), T(0)};
    };
    auto pre = [&](int k) { return ldc(cha, k, N); };
    auto st = [&](int k, C y, C c) {
        if (k >= h && k < N) {
            const C z = cmulc(y, c);
            Fr[k - h] = C{z.x * invN, z.y * invN};
        }
    };
    convolve<LOGM, T>(buf, ft.h_fd, ft.ptw, ld, pre, st);
}

// out[b][c][r] = in[b][r][c], 32 x 32 tiles through LDS.
template <typename T>
__global__ __launch_bounds__(256) void k_transpose(int rows, int cols, const typename CT<T>::type *__restrict__ in,
                                                   typename CT<T>::type *__restrict__ out) {
    using C = typename CT<T>::type;
    __shared__ C tile[32][33];
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32, b = blockIdx.z;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const C *ib = in + (size_t)b * rows * cols;
    C *ob = out + (size_t)b * rows * cols;
    for (int i = ty; i < 32; i += 8) {
        const int r = r0 + i, c = c0 + tx;
        if (r < rows && c < cols) tile[i][tx] = ib[(size_t)r * cols + c];
    }
    __syncthreads();
    for (int i = ty; i < 32; i += 8) {
        const int c = c0 + i, r = r0 + tx;
        if (r < rows && c < cols) ob[(size_t)c * rows + r] = tile[tx][i];
    }
}

// Plan helper: forward DFT (natural order) of `rows` sequences of length M, in place, scaled.
template <typename T, int LOGM>
SHT_ROW_KERNEL(T, LOGM) void k_fft_rows(FftTables<T> ft, typename CT<T>::type *data,
                                                          T scale) {
    using C = typename CT<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *buf = reinterpret_cast<C *>(smem_raw);
    C *row = data + (size_t)blockIdx.x * ft.M;
    fft_run<LOGM, T>(buf, ft.ptw, [row](int n) { return row[n]; },
                     [row, scale](int k, C x, NoAux) { row[k] = C{x.x * scale, x.y * scale}; });
}

template <typename T> bool split_host(const FftTables<T> &ft) { return rows_split(ft.M, 2 * (int)sizeof(T)); }

// LDS of a row kernel: the M-point buffer with one pad slot per 16 points
// (half of it for split rows).
template <typename T> size_t lds_bytes(const FftTables<T> &ft) {
    const bool split = split_host(ft);
    const size_t m = split ? (size_t)ft.M / 2 : (size_t)ft.M;
    return (m + m / 16 + (size_t)ltw_entries(ft.logM, split)) * sizeof(typename CT<T>::type);
}

// Launch shape of a row kernel over n items: one workgroup per item, or for
// split rows at most kSplitSlots workgroups looping over the items.
template <typename T> dim3 row_grid(const FftTables<T> &ft, int n) {
    if (split_host(ft)) return dim3((unsigned)(n < kSplitSlots ? n : kSplitSlots));
    return dim3((unsigned)n);
}

// Raises a kernel's dynamic-LDS limit once per (device, kernel, size), so a
// launch sequence after the first one (e.g. under graph capture) is kernel
// launches only.
template <typename K> hipError_t set_lds(K kernel, size_t bytes) {
    if (bytes <= 64 * 1024) return hipSuccess;
    static std::mutex mu;
    static std::set<std::tuple<int, const void *, size_t>> done;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const auto key = std::make_tuple(dev, (const void *)kernel, bytes);
    std::lock_guard<std::mutex> lk(mu);
    if (done.count(key)) return hipSuccess;
    e = hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) done.insert(key);
    return e;
}

}  // namespace

// Calls f(std::integral_constant<int, LOGM>) for the plan's log2 M (3 .. 14).
template <typename F> hipError_t with_logm(int logM, F f) {
    switch (logM) {
        case 3: return f(std::integral_constant<int, 3>{});
        case 4: return f(std::integral_constant<int, 4>{});
        case 5: return f(std::integral_constant<int, 5>{});
        case 6: return f(std::integral_constant<int, 6>{});
        case 7: return f(std::integral_constant<int, 7>{});
        case 8: return f(std::integral_constant<int, 8>{});
        case 9: return f(std::integral_constant<int, 9>{});
        case 10: return f(std::integral_constant<int, 10>{});
        case 11: return f(std::integral_constant<int, 11>{});
        case 12: return f(std::integral_constant<int, 12>{});
        case 13: return f(std::integral_constant<int, 13>{});
        case 14: return f(std::integral_constant<int, 14>{});
        default: return hipErrorInvalidValue;
    }
}

// Rows of a theta launch over every map of a call (order pairs per map
// times maps), or 0 when the table is malformed or the count overflows.
static long long theta_rows(int L, bool half, const SpinSegs &sg) {
    if (sg.n < 1 || sg.n > SHT_MULTI_SEG_MAX || sg.batch < 1) return 0;
    const long long n = (long long)(half ? (L + 1) / 2 : L) * sg.batch;
    return n <= 0x7fffffffLL ? n : 0;
}

template <typename T>
hipError_t launch_theta_inv(const FftTables<T> &ft, const SpinSegs &sg, int Cn, bool half, const T *R, void *G,
                            void *scr, hipStream_t st) {
    const long long rows = theta_rows(ft.L, half, sg);
    if (rows == 0) return hipErrorInvalidValue;
    return with_logm(ft.logM, [&](auto lm) {
        constexpr int LM = decltype(lm)::value;
        const size_t lds = lds_bytes(ft);
        typename CT<T>::type *g = (typename CT<T>::type *)G, *w = (typename CT<T>::type *)scr;
        if (half) {
            hipError_t e = set_lds(k_theta_inv<T, LM, true>, lds);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL((k_theta_inv<T, LM, true>), row_grid(ft, (int)rows), dim3(row_threads(ft.M)), lds, st,
                               ft, sg, Cn, R, g, w);
        } else {
            hipError_t e = set_lds(k_theta_inv<T, LM, false>, lds);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL((k_theta_inv<T, LM, false>), row_grid(ft, (int)rows), dim3(row_threads(ft.M)), lds, st,
                               ft, sg, Cn, R, g, w);
        }
        return hipGetLastError();
    });
}

template <typename T>
hipError_t launch_phi_inv(const FftTables<T> &ft, int B, int rs, const void *G, void *map, void *scr,
                          hipStream_t st) {
    return with_logm(ft.logM, [&](auto lm) {
        constexpr int LM = decltype(lm)::value;
        const size_t lds = lds_bytes(ft);
        hipError_t e = set_lds(k_phi_inv<T, LM>, lds);
        if (e != hipSuccess) return e;
        const int rows = ft.L * B;
        hipLaunchKernelGGL((k_phi_inv<T, LM>), row_grid(ft, rows), dim3(row_threads(ft.M)), lds, st, ft, rows, rs,
                           (const typename CT<T>::type *)G, (typename CT<T>::type *)map, (typename CT<T>::type *)scr);
        return hipGetLastError();
    });
}

template <typename T>
hipError_t launch_phi_fwd(const FftTables<T> &ft, int B, int rs, const void *map, void *Q, void *scr,
                          hipStream_t st) {
    return with_logm(ft.logM, [&](auto lm) {
        constexpr int LM = decltype(lm)::value;
        const size_t lds = lds_bytes(ft);
        hipError_t e = set_lds(k_phi_fwd<T, LM>, lds);
        if (e != hipSuccess) return e;
        const int rows = ft.L * B;
        hipLaunchKernelGGL((k_phi_fwd<T, LM>), row_grid(ft, rows), dim3(row_threads(ft.M)), lds, st, ft, rows, rs,
                           (const typename CT<T>::type *)map, (typename CT<T>::type *)Q, (typename CT<T>::type *)scr);
        return hipGetLastError();
    });
}

template <typename T>
hipError_t launch_theta_fwd(const FftTables<T> &ft, const SpinSegs &sg, int Cn, bool half, const void *Q, T *X,
                            void *scr, hipStream_t st) {
    const long long rows = theta_rows(ft.L, half, sg);
    if (rows == 0) return hipErrorInvalidValue;
    return with_logm(ft.logM, [&](auto lm) {
        constexpr int LM = decltype(lm)::value;
        const size_t lds = lds_bytes(ft);
        const typename CT<T>::type *q = (const typename CT<T>::type *)Q;
        typename CT<T>::type *w = (typename CT<T>::type *)scr;
        if (half) {
            hipError_t e = set_lds(k_theta_fwd<T, LM, true>, lds);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL((k_theta_fwd<T, LM, true>), row_grid(ft, (int)rows), dim3(row_threads(ft.M)), lds, st,
                               ft, sg, Cn, q, X, w);
        } else {
            hipError_t e = set_lds(k_theta_fwd<T, LM, false>, lds);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL((k_theta_fwd<T, LM, false>), row_grid(ft, (int)rows), dim3(row_threads(ft.M)), lds, st,
                               ft, sg, Cn, q, X, w);
        }
        return hipGetLastError();
    });
}

template <typename T>
hipError_t launch_phi_inv_real(const FftTables<T> &ft, int B, const void *G, T *map, void *scr, hipStream_t st) {
    return with_logm(ft.logM, [&](auto lm) {
        constexpr int LM = decltype(lm)::value;
        const size_t lds = lds_bytes(ft);
        hipError_t e = set_lds(k_phi_inv_real<T, LM>, lds);
        if (e != hipSuccess) return e;
        const int rows = ft.L * B;
        hipLaunchKernelGGL((k_phi_inv_real<T, LM>), row_grid(ft, (rows + 1) / 2), dim3(row_threads(ft.M)), lds, st,
                           ft, rows, (const typename CT<T>::type *)G, map, (typename CT<T>::type *)scr);
        return hipGetLastError();
    });
}

template <typename T>
hipError_t launch_phi_fwd_real(const FftTables<T> &ft, int B, const T *map, void *Q, void *scr, hipStream_t st) {
    return with_logm(ft.logM, [&](auto lm) {
        constexpr int LM = decltype(lm)::value;
        const size_t lds = lds_bytes(ft);
        hipError_t e = set_lds(k_phi_fwd_real<T, LM>, lds);
        if (e != hipSuccess) return e;
        const int rows = ft.L * B;
        hipLaunchKernelGGL((k_phi_fwd_real<T, LM>), row_grid(ft, (rows + 1) / 2), dim3(row_threads(ft.M)), lds, st,
                           ft, rows, map, (typename CT<T>::type *)Q, (typename CT<T>::type *)scr);
        return hipGetLastError();
    });
}

// (the triangular forward's theta DFT and the plan's in-place FFT run only
// at sizes whose rows fit in LDS)
template <typename T>
hipError_t launch_theta_dft(const FftTables<T> &ft, int s, int B, const void *Q, void *F, hipStream_t st) {
    if (split_host(ft)) return hipErrorInvalidValue;
    return with_logm(ft.logM, [&](auto lm) {
        constexpr int LM = decltype(lm)::value;
        const size_t lds = lds_bytes(ft);
        hipError_t e = set_lds(k_theta_dft<T, LM>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_theta_dft<T, LM>), dim3(ft.N * B), dim3(row_threads(ft.M)), lds, st, ft, s,
                           (const typename CT<T>::type *)Q, (typename CT<T>::type *)F);
        return hipGetLastError();
    });
}

template <typename T>
hipError_t launch_fft_inplace(const FftTables<T> &ft, typename CT<T>::type *buf, int rows, double scale,
                              hipStream_t st) {
    if (split_host(ft)) return hipErrorInvalidValue;
    return with_logm(ft.logM, [&](auto lm) {
        constexpr int LM = decltype(lm)::value;
        const size_t lds = lds_bytes(ft);
        hipError_t e = set_lds(k_fft_rows<T, LM>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_fft_rows<T, LM>), dim3(rows), dim3(row_threads(ft.M)), lds, st, ft, buf, (T)scale);
        return hipGetLastError();
    });
}

template <typename T>
hipError_t launch_transpose(int B, int rows, int cols, const void *in, void *out, hipStream_t st) {
    const dim3 grid((cols + 31) / 32, (rows + 31) / 32, B);
    hipLaunchKernelGGL(k_transpose<T>, grid, dim3(256), 0, st, rows, cols, (const typename CT<T>::type *)in,
                       (typename CT<T>::type *)out);
    return hipGetLastError();
}

template <typename T> hipError_t prepare_row_kernels(const FftTables<T> &ft) {
    return with_logm(ft.logM, [&](auto lm) {
        constexpr int LM = decltype(lm)::value;
        const size_t lds = lds_bytes(ft);
        hipError_t e = set_lds(k_theta_inv<T, LM, true>, lds);
        if (e == hipSuccess) e = set_lds(k_theta_inv<T, LM, false>, lds);
        if (e == hipSuccess) e = set_lds(k_phi_inv<T, LM>, lds);
        if (e == hipSuccess) e = set_lds(k_phi_fwd<T, LM>, lds);
        if (e == hipSuccess) e = set_lds(k_theta_fwd<T, LM, true>, lds);
        if (e == hipSuccess) e = set_lds(k_theta_fwd<T, LM, false>, lds);
        if (e == hipSuccess) e = set_lds(k_phi_inv_real<T, LM>, lds);
        if (e == hipSuccess) e = set_lds(k_phi_fwd_real<T, LM>, lds);
        if (e == hipSuccess && !split_host(ft)) e = set_lds(k_theta_dft<T, LM>, lds);
        return e;
    });
}

template <typename T> size_t split_scratch_bytes(const FftTables<T> &ft) {
    return split_host(ft) ? (size_t)kSplitSlots * ft.M * sizeof(typename CT<T>::type) : 0;
}

#define SHT_INST(T)                                                                                      \
    template hipError_t launch_theta_inv<T>(const FftTables<T> &, const SpinSegs &, int, bool, const T *,     \
                                            void *, void *, hipStream_t);                                \
    template hipError_t launch_phi_inv_real<T>(const FftTables<T> &, int, const void *, T *, void *, hipStream_t); \
    template hipError_t launch_phi_fwd_real<T>(const FftTables<T> &, int, const T *, void *, void *, hipStream_t); \
    template hipError_t launch_phi_inv<T>(const FftTables<T> &, int, int, const void *, void *, void *,    \
                                          hipStream_t);                                                  \
    template hipError_t launch_phi_fwd<T>(const FftTables<T> &, int, int, const void *, void *, void *,    \
                                          hipStream_t);                                                  \
    template hipError_t launch_theta_dft<T>(const FftTables<T> &, int, int, const void *, void *, hipStream_t); \
    template hipError_t launch_theta_fwd<T>(const FftTables<T> &, const SpinSegs &, int, bool, const void *,  \
                                            T *, void *, hipStream_t);                                   \
    template size_t split_scratch_bytes<T>(const FftTables<T> &);                                        \
    template hipError_t launch_transpose<T>(int, int, int, const void *, void *, hipStream_t);                \
    template hipError_t launch_fft_inplace<T>(const FftTables<T> &, typename CT<T>::type *, int, double, \
                                                  hipStream_t);                                          \
    template hipError_t prepare_row_kernels<T>(const FftTables<T> &);
SHT_INST(double)
SHT_INST(float)
#undef SHT_INST

}  // namespace sht
