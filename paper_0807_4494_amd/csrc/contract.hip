// The O(L^3) core: the contraction of Eq. (fourier_coeff) between torus
// Fourier coefficients and harmonic coefficients, for every order m >= 0,
//
//   inverse  R[m][c][m'] = sum_{l >= max(m, m')} M_m(m', l) P[m][c][l]
//   forward  R[m][c][l]  = sum_{m' = 0}^{l}      M_m(m', l) X[m][c][m']
//
// with M_m(m', l) = sqrt((2l+1)/4pi) d^l_{m'm}(pi/2) d^l_{m',-s}(pi/2), and the
// columns c running over {Re, Im} x {+m, -m} x maps (the phases and signs
// that distinguish the columns are applied by the neighbouring stages).
//
// M is never stored.  Each workgroup owns GM consecutive orders, a tile of TJ
// output indices j (m' for the inverse, l for the forward) and up to CTILE
// columns; every thread owns the Wigner chains of one j:
//   inverse: chains in l (the GEMM's K axis) for (m', m) and (m', -s);
//   forward: chains in m' (the K axis) for (l, m) and (l, -s).
// The chains run in FP64 (chain.h), emit one K-slab of M into LDS per step
// of TK, and the slab is multiplied on the matrix cores:
//   out[c][j] += sum_k X^T[c][k] M[k][j]   (v_mfma 16x16x4, f32 or f64).
#include "chain.h"

namespace sht {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
// Output layout of the 16x16x4 MFMAs (measured on gfx950): element r of lane
// holds D[row][lane % 16] with row = 4*(lane/16) + r for f32 and
// row = 4*r + lane/16 for f64.
template <> struct Mfma<float> {
    using acc = f32x4;
    static __device__ inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
    static __device__ inline acc op(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma<double> {
    using acc = f64x4;
    static __device__ inline int row(int lane, int r) { return 4 * r + (lane >> 4); }
    static __device__ inline acc op(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

template <typename T> struct Tile;
template <> struct Tile<float> { static constexpr int TJ = 256, WJ = 64; };
template <> struct Tile<double> { static constexpr int TJ = 128, WJ = 32; };

constexpr int GM = 2;   // orders per workgroup
constexpr int TK = 16;  // K slab
constexpr int NT = 256; // threads

template <typename T> struct Args {
    int L, s, B, C;       // C = 4B columns
    int njt, ncb;         // j tiles, column blocks
    const T *X;           // [L][C][L]
    T *Y;                 // [L][C][L]
    EdgeTable E;
    const SpinState *ss;  // [L][L], inverse only
};

template <typename T, int MODE, int CTILE>
__global__ __launch_bounds__(NT) void k_contract(Args<T> a) {
    constexpr int TJ = Tile<T>::TJ, WJ = Tile<T>::WJ;
    constexpr int NSUB = NT / TJ;   // threads sharing one j
    constexpr int NCH = GM / NSUB;  // main chains per thread
    constexpr int NCI = CTILE / 16, NJI = WJ / 16;
    using acc_t = typename Mfma<T>::acc;

    __shared__ T Mt[GM][TK][TJ];
    __shared__ T Xt[GM][TK][CTILE];
    __shared__ double fam[GM + 1][TK], fbm[GM + 1][TK], fcl[TK];

    const int L = a.L, s = a.s, Cn = a.C;
    const int sigma = -s, asg = s < 0 ? -s : s;
    int bid = blockIdx.x;
    const int cb = bid % a.ncb;
    bid /= a.ncb;
    const int jt = bid % a.njt;
    const int mg = bid / a.njt;
    const int m0 = mg * GM, j0 = jt * TJ, c0 = cb * CTILE;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int jl = tid % TJ, sub = tid / TJ;
    const int j = j0 + jl;
    const bool jvalid = j < L;

    if (MODE == kForward) {
        // outputs l < max(m0, |s|) are never read
        const int need = m0 > asg ? m0 : asg;
        if (j0 + TJ - 1 < need) return;
    }

    acc_t acc[GM][NCI][NJI];
#pragma unroll
    for (int g = 0; g < GM; ++g)
#pragma unroll
        for (int ci = 0; ci < NCI; ++ci)
#pragma unroll
            for (int ji = 0; ji < NJI; ++ji) acc[g][ci][ji] = acc_t{0, 0, 0, 0};

    Chain ch[NCH], sc;
    int mch[NCH];
    bool vch[NCH];
#pragma unroll
    for (int g = 0; g < NCH; ++g) {
        mch[g] = m0 + sub * NCH + g;
        ch[g].zero();
    }
    sc.zero();

    // K range and per-thread chain bookkeeping
    int kfirst, klast;  // inclusive, in iteration order
    double q = 0.0;     // inverse: sqrt(l^2 - m'^2) at the current l
    double gprev = 0.0; // forward: sqrt((l+m'+1)(l-m')) for the previous m'
    double clj = 0.0;   // forward: sqrt((2l+1)/4pi)
    int l0s = 0;
    if (MODE == kInverse) {
        const int l_lo = m0 > j0 ? m0 : j0;
        kfirst = (l_lo / TK) * TK;
        klast = L - 1;
#pragma unroll
        for (int g = 0; g < NCH; ++g) vch[g] = jvalid && mch[g] < L;
        l0s = j > asg ? j : asg;
        if (jvalid && l0s < kfirst) {
            const SpinState st = a.ss[(size_t)kfirst * L + j];
            sc.d = st.d;
            sc.dp = st.dp;
            sc.k = st.k;
            sc.es = emit_scale(st.k);
        }
        const double Y = (double)kfirst * kfirst - (double)j * j;
        q = Y > 0.0 ? sqrt(Y) : 0.0;
    } else {
        int top = j0 + TJ - 1;
        if (top > L - 1) top = L - 1;
        kfirst = ((top + TK) / TK) * TK - 1;  // chunk-aligned top, >= top
        klast = 0;
#pragma unroll
        for (int g = 0; g < NCH; ++g) vch[g] = jvalid && mch[g] < L && j >= mch[g];
        clj = sqrt((2.0 * j + 1.0) / (4.0 * 3.14159265358979323846));
    }

    const int nchunks = MODE == kInverse ? (L - kfirst + TK - 1) / TK : (kfirst + 1) / TK;
    for (int chunk = 0; chunk < nchunks; ++chunk) {
        // K rows kk = 0..TK-1 of this slab correspond to k = kbase + kk
        const int kbase = MODE == kInverse ? kfirst + chunk * TK : kfirst - (chunk + 1) * TK + 1;

        if (MODE == kInverse && tid < (GM + 1) * TK) {
            const int gi = tid / TK, kk = tid % TK;
            const int l = kbase + kk;
            const int idx = gi < GM ? m0 + gi : sigma;
            double am, bm;
            lrec_factor_full(l, idx, am, bm);
            fam[gi][kk] = am;
            fbm[gi][kk] = bm;
            if (gi == 0) fcl[kk] = sqrt((2.0 * l + 1.0) / (4.0 * 3.14159265358979323846));
        }
        // X slab: Xt[g][kk][c] = X[m0+g][c0+c][kbase+kk]
#pragma unroll
        for (int g = 0; g < GM; ++g) {
            const int m = m0 + g;
            for (int e = tid; e < CTILE * TK; e += NT) {
                const int c = e / TK, kk = e % TK;
                const int k = kbase + kk;
                bool ok = m < L && (c0 + c) < Cn && k >= 0 && k < L;
                if (MODE == kInverse) ok = ok && k >= m;
                Xt[g][kk][c] = ok ? a.X[((size_t)m * Cn + c0 + c) * L + k] : T(0);
            }
        }
        __syncthreads();

        // ---- generate the M slab ----
        if (MODE == kInverse) {
            for (int kk = 0; kk < TK; ++kk) {
                const int l = kbase + kk;
                if (l == l0s && jvalid) sc.inject(edge_seed(a.E, j, sigma));
#pragma unroll
                for (int g = 0; g < NCH; ++g) {
                    const int l0 = j > mch[g] ? j : mch[g];
                    if (vch[g] && l == l0) ch[g].inject(edge_seed(a.E, j, mch[g]));
                }
                const double W = (l < L) ? fcl[kk] * sc.value() : 0.0;
#pragma unroll
                for (int g = 0; g < NCH; ++g)
                    Mt[sub * NCH + g][kk][jl] = (T)(vch[g] ? ch[g].value() * W : 0.0);
                // step l -> l+1
                const double Xl = (double)(l + 1) * (l + 1) - (double)j * j;
                const double r = rsqrt(Xl > 1.0 ? Xl : 1.0);
                const double ap = (double)j * r, bp = q * r;
                q = Xl > 0.0 ? Xl * r : 0.0;
                {
                    const double dn = -(ap * fam[GM][kk] * sc.d + bp * fbm[GM][kk] * sc.dp);
                    if (l >= l0s) sc.push(dn);
                }
#pragma unroll
                for (int g = 0; g < NCH; ++g) {
                    const int gi = sub * NCH + g;
                    const double dn = -(ap * fam[gi][kk] * ch[g].d + bp * fbm[gi][kk] * ch[g].dp);
                    const int l0 = j > mch[g] ? j : mch[g];
                    if (l >= l0) ch[g].push(dn);
                }
            }
        } else {
            for (int kk = TK - 1; kk >= 0; --kk) {
                const int k = kbase + kk;  // m'
                if (k == j && jvalid) {
                    if (j >= asg) sc.inject(edge_seed(a.E, j, sigma));
#pragma unroll
                    for (int g = 0; g < NCH; ++g)
                        if (vch[g]) ch[g].inject(edge_seed(a.E, j, mch[g]));
                    gprev = 0.0;
                }
                const bool live = k >= 0 && k <= j && jvalid;
                const double W = live ? clj * sc.value() : 0.0;
#pragma unroll
                for (int g = 0; g < NCH; ++g)
                    Mt[sub * NCH + g][kk][jl] = (T)(vch[g] ? ch[g].value() * W : 0.0);
                // step m' -> m'-1
                const double Xk = (double)(j + k) * (double)(j - k + 1);
                const double y = rsqrt(Xk > 1.0 ? Xk : 1.0);
                const double gcur = Xk > 0.0 ? Xk * y : 0.0;
                if (live) {
                    sc.push((2.0 * sigma * sc.d - gprev * sc.dp) * y);
#pragma unroll
                    for (int g = 0; g < NCH; ++g)
                        ch[g].push((2.0 * mch[g] * ch[g].d - gprev * ch[g].dp) * y);
                }
                gprev = gcur;
            }
        }
        __syncthreads();

        // ---- matrix cores ----
        const int wj0 = j0 + wave * WJ;  // first j of this wave
        bool active;
        if (MODE == kInverse) {
            const int start = m0 > wj0 ? m0 : wj0;
            active = kbase + TK - 1 >= start && wj0 < L;
        } else {
            active = kbase <= wj0 + WJ - 1 && wj0 < L;
        }
        if (active) {
#pragma unroll
            for (int g = 0; g < GM; ++g) {
#pragma unroll
                for (int ks = 0; ks < TK / 4; ++ks) {
                    const int kr = ks * 4 + (lane >> 4);
                    T av[NCI], bv[NJI];
#pragma unroll
                    for (int ci = 0; ci < NCI; ++ci) av[ci] = Xt[g][kr][ci * 16 + (lane & 15)];
#pragma unroll
                    for (int ji = 0; ji < NJI; ++ji) bv[ji] = Mt[g][kr][wave * WJ + ji * 16 + (lane & 15)];
#pragma unroll
                    for (int ci = 0; ci < NCI; ++ci)
#pragma unroll
                        for (int ji = 0; ji < NJI; ++ji)
                            acc[g][ci][ji] = Mfma<T>::op(av[ci], bv[ji], acc[g][ci][ji]);
                }
            }
        }
        __syncthreads();
    }

    // ---- write out[c][j] ----
#pragma unroll
    for (int g = 0; g < GM; ++g) {
        const int m = m0 + g;
        if (m >= L) continue;
#pragma unroll
        for (int ci = 0; ci < NCI; ++ci)
#pragma unroll
            for (int ji = 0; ji < NJI; ++ji)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int c = c0 + ci * 16 + Mfma<T>::row(lane, r);
                    const int jj = j0 + wave * WJ + ji * 16 + (lane & 15);
                    if (c < Cn && jj < L) a.Y[((size_t)m * Cn + c) * L + jj] = acc[g][ci][ji][r];
                }
    }
}

template <typename T, int MODE, int CTILE>
hipError_t launch_one(const Args<T> &a, hipStream_t st) {
    const int nmg = (a.L + GM - 1) / GM;
    const dim3 grid(nmg * a.njt * a.ncb);
    hipLaunchKernelGGL((k_contract<T, MODE, CTILE>), grid, dim3(NT), 0, st, a);
    return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_contract(int mode, int L, int s, int B, const T *X, T *Y, const EdgeTable &E,
                           const SpinState *ss, hipStream_t st) {
    Args<T> a;
    a.L = L;
    a.s = s;
    a.B = B;
    a.C = 4 * B;
    a.njt = (L + Tile<T>::TJ - 1) / Tile<T>::TJ;
    a.X = X;
    a.Y = Y;
    a.E = E;
    a.ss = ss;
    if (a.C <= 16) {
        a.ncb = 1;
        return mode == kInverse ? launch_one<T, kInverse, 16>(a, st) : launch_one<T, kForward, 16>(a, st);
    }
    a.ncb = (a.C + 63) / 64;
    return mode == kInverse ? launch_one<T, kInverse, 64>(a, st) : launch_one<T, kForward, 64>(a, st);
}

template hipError_t launch_contract<double>(int, int, int, int, const double *, double *, const EdgeTable &,
                                            const SpinState *, hipStream_t);
template hipError_t launch_contract<float>(int, int, int, int, const float *, float *, const EdgeTable &,
                                           const SpinState *, hipStream_t);

hipError_t launch_contract_bf16x3(int, int, int, int, const float *, float *, const EdgeTable &,
                                  const SpinState *, hipStream_t) {
    return hipErrorNotSupported;
}

}  // namespace sht
