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
// columns.  Its producer waves own the Wigner chains of the tile's j:
//   inverse: chains in l (the GEMM's K axis) for (m', m);
//   forward: chains in m' (the K axis) for (l, m),
// run them in FP64 (chain.h), multiply by the spin factor
// sqrt((2l+1)/4pi) d^l_{m',-s}(pi/2) (the same for every order, so it is
// tabulated once per (L, s) in the plan) and emit one K-slab of M at a time;
// its consumer waves multiply the previous slab on the matrix cores
//   out[c][j] += sum_k X^T[c][k] M[k][j]
// while the producers fill the next one (double-buffered LDS).  Three
// precisions share the kernel:
//   FP64    M and X in FP64, v_mfma_f64_16x16x4;
//   FP32    M rounded to FP32, v_mfma_f32_16x16x4;
//   BF16x3  M and X split into BF16 pairs hi + lo, three v_mfma_f32_16x16x16
//           BF16 products hi*hi + hi*lo + lo*hi accumulated in FP32 (the
//           lo*lo term, ~2^-16 relative, is dropped).
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <utility>
#include <vector>

#include "chain.h"

namespace sht {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));

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

// Raw buffer loads (gfx9 resource word 3; offsets past the resource's size
// read zero).
constexpr int kBufWord3 = 0x00020000;
template <typename T>
__device__ __forceinline__ T buffer_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}

__device__ __forceinline__ double2 buffer_load_d2(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    typedef double d2v __attribute__((ext_vector_type(2)));
    const d2v v = __builtin_bit_cast(d2v, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
    return make_double2(v.x, v.y);
}

__device__ __forceinline__ float4 buffer_load_f4(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
}

// BF16 pair of an FP32 value: hi = v rounded to BF16 (nearest, ties to
// even), lo = the remainder v - hi rounded the same way; hi + lo carries
// about 16 significant bits.  Finite inputs only.
__device__ inline unsigned short bf16_rne(float v) {
    const unsigned u = __float_as_uint(v);
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float bf16_value(unsigned short h) { return __uint_as_float((unsigned)h << 16); }
__device__ inline void bf16_split(float v, unsigned short &hi, unsigned short &lo) {
    hi = bf16_rne(v);
    lo = bf16_rne(v - bf16_value(hi));
}

constexpr int GM = 4;    // orders per workgroup
constexpr int TK = 16;   // K slab

// Precision policies.  The first NCONS threads of a workgroup consume (MFMA),
// the NPROD after them produce (FP64 Wigner chains).  TJ output
// indices j per workgroup, WJ per consumer wave; GM orders m; TK rows of K per
// slab.  kP32W is the FP32 tile of 128 columns: two consumer waves per SIMD,
// each with the j block and accumulators of a 64-column tile, over one
// column half, beside one producer wave, so each Wigner entry generated
// serves 128 columns for the producer time a 64-column tile spends.
enum { kP64 = 0, kP32 = 1, kPBF = 2, kP32W = 3 };
template <int P> struct Prec;
template <> struct Prec<kP64> { using T = double; static constexpr int TJ = 64, WJ = 16, NCONS = 256, NPROD = 256; };
template <> struct Prec<kP32> { using T = float; static constexpr int TJ = 128, WJ = 32, NCONS = 256, NPROD = 256; };
template <> struct Prec<kPBF> { using T = float; static constexpr int TJ = 128, WJ = 32, NCONS = 256, NPROD = 256; };
template <> struct Prec<kP32W> { using T = float; static constexpr int TJ = 128, WJ = 32, NCONS = 512, NPROD = 256; };
template <int P> constexpr int kThreads = Prec<P>::NCONS + Prec<P>::NPROD;
template <int P> constexpr bool kIsF32 = P == kP32 || P == kP32W;

// LDS slabs.  FP32 / FP64: M slab [k][j] with rows padded by 16 so the four K
// rows an MFMA fragment spans hit disjoint banks; X slab [c][k] with rows of
// TK + 1 (FP64) or TK + 4 (FP32: four consecutive k are one aligned 16-byte
// store, and the fragment reads, 16 columns x 4 k, still hit 64 distinct
// banks).  BF16x3: the 16x16x16 BF16 fragments hold four consecutive k
// per lane, so M is stored [k/4][j][k%4] and X [c][k] (row of TK + 4, so a
// lane's four k are one aligned 8-byte read), each as hi and lo planes.
// KP (FP32 forward): M stored [k/2][j][k%2] for K-paired fragments (see the
// consumers).
// kP32W: X rows of TK unpadded, filled by LDS-direct loads (each lane's 16
// bytes land at the next 16-byte slot), with slot q of row c holding k quad
// q ^ ((c >> 2) & 3): the 16 columns of a fragment read then spread over 64
// banks.
template <int P> constexpr int kXRow = P == kP32W ? TK : (kIsF32<P> ? TK + 4 : TK + 1);
template <int P, int CTILE, bool KP = false> struct Slabs {
    using T = typename Prec<P>::T;
    static constexpr int XROW = kXRow<P>;
    T M[2][GM][TK][Prec<P>::TJ + 16];
    alignas(16) T X[2][GM][CTILE][XROW];
};
template <int P, int CTILE> struct Slabs<P, CTILE, true> {
    static constexpr int TJ = Prec<P>::TJ, XROW = kXRow<P>;
    alignas(16) float M[2][GM][TK / 2][TJ + 16][2];
    alignas(16) float X[2][GM][CTILE][XROW];
};
template <int CTILE> struct Slabs<kPBF, CTILE, false> {
    static constexpr int TJ = Prec<kPBF>::TJ;
    static constexpr int XROW = TK + 4;
    alignas(16) unsigned short Mh[2][GM][TK / 4][TJ + 16][4];
    alignas(16) unsigned short Ml[2][GM][TK / 4][TJ + 16][4];
    alignas(16) unsigned short Xh[2][GM][CTILE][TK + 4];
    alignas(16) unsigned short Xl[2][GM][CTILE][TK + 4];
};

// Column blocks of one launch: block y takes columns [c0[y], c0[y] + CTILE)
// clipped to cend[y] (the end of its spin's columns), with that spin's
// factor table, |s| and (table mode) cached table.  One launch can so serve
// the maps of several spins at one L.
constexpr int kMaxColBlocks = 32;

template <typename T> struct Args {
    int L, C;             // C columns in all (4 per map; 2 per map for real signals)
    int njt, ncb;         // j tiles, column blocks
    const T *X;           // [L][C][L]
    T *Y;                 // [L][C][L]
    EdgeTable E;
    const double2 *jtab;  // [L][L] j-side step factors at [k][j] (jti or jtf)
    const double2 *fab;   // [L][L] order-side l-recursion factors
    const double *cl;     // [L] sqrt((2l+1)/4pi)
    const int *sched;     // workgroup order: (group << 8) | j tile, longest K loop first
    const T *wtab[kMaxColBlocks];  // [L][L] spin factor at [k][j] (wi or wf) of block y's spin
    const T *mtab[kMaxColBlocks];  // table mode: M_m(m', l) at [m][l][m'] (plan's cached table)
    int c0[kMaxColBlocks], cend[kMaxColBlocks], asg[kMaxColBlocks];
};

// TAB: the producers copy the slab of M from the plan's cached table instead
// of running the Wigner chains (the measured comparison of a precomputed-Delta
// design with on-the-fly generation).
template <int P, int MODE, int CTILE, bool TAB, bool PAR>
__global__ __launch_bounds__(kThreads<P>) void k_contract(Args<typename Prec<P>::T> a) {
    using T = typename Prec<P>::T;
    constexpr bool BF = P == kPBF;
    constexpr int TJ = Prec<P>::TJ, WJ = Prec<P>::WJ;
    constexpr int NC = Prec<P>::NCONS;        // consumer threads
    constexpr int NPJ = Prec<P>::NPROD / TJ;  // producer threads sharing one j
    constexpr int NCH = GM / NPJ;   // main chains per producer thread
    constexpr int NJW = TJ / WJ;    // consumer waves across the j tile
    constexpr int CW = CTILE * NJW * 64 / NC;  // columns per consumer wave
    constexpr int NCI = CW / 16, NJI = WJ / 16;
    constexpr int XPT = GM * CTILE * TK / NC;  // X slab elements per consumer thread
    static_assert(NCH * NPJ == GM && CW * (NC / 64 / NJW) == CTILE, "tile shape");
    static_assert(XPT % 4 == 0, "X slab quadruples");
    using acc_t = typename Mfma<T>::acc;

    // FP32 forward: K-paired MFMA fragments (measured faster there; the
    // inverse keeps the plain layout, where pairing measured slower)
    constexpr bool KP = kIsF32<P> && MODE == kForward;
    constexpr bool DX = P == kP32W;  // X slab by LDS-direct loads, swizzled rows
    __shared__ Slabs<P, CTILE, KP> sm;
    __shared__ double fam[2][GM][TK], fbm[2][GM][TK];

    const int L = a.L, Cn = a.C;
    // Workgroup x takes the x-th (order group, j tile) pair of the plan's
    // schedule, longest K loop first, so the short ones fill the tail; the
    // column block is blockIdx.y.
    const int code = a.sched[blockIdx.x];
    if (code < 0) return;  // padding of the schedule
    const int mg = code >> 8, jt = code & 255, cb = (int)blockIdx.y;
    const int m0 = mg * GM, j0 = jt * TJ, c0 = a.c0[cb], cend = a.cend[cb], asg = a.asg[cb];
    const T *wtab = a.wtab[cb], *mtab = a.mtab[cb];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // PAR: the parity kernel, launched on spin-0 blocks of FP32 data only.
    // Delta^l_{m',0}(pi/2) = 0 for odd l + m' (K index and j of opposite
    // parity).  The tile places its even j in the first TJ / 2 positions and
    // its odd j after them (pj), so the j of a consumer wave share one parity;
    // the K slabs of complete 16-blocks arrive with even K in positions 0-7
    // and odd K in 8-15 (par16_pos; the producers emit in the same order), and
    // the consumers skip the products of the other parity.  BF16x3 (one MFMA
    // spans the slab's 16 K) keeps the K order of the FP32 panels but skips
    // nothing.  FP64 data keeps the natural order, and the 128-column tile
    // takes no spin-0 blocks.
    static_assert(!PAR || P == kP32 || P == kPBF, "parity kernels");
    constexpr bool par = PAR, pj = PAR && P == kP32;
    // j of tile position p, and (producers, which keep consecutive j for
    // contiguous table loads) the position of j0 + jl
    auto jpos = [&](int p) { return pj ? 2 * (p % (TJ / 2)) + p / (TJ / 2) : p; };
    auto jcol = [&](int jl) { return pj ? (jl & 1) * (TJ / 2) + (jl >> 1) : jl; };
    // slab in parity blocks: a spin-0 block's slab inside [0, L)
    auto pk_of = [&](int kbase) { return par && kbase + TK <= L; };
    const bool producer = tid >= NC;

    if (MODE == kForward) {
        // outputs l < max(m0, |s|) are never read
        const int need = m0 > asg ? m0 : asg;
        if (j0 + TJ - 1 < need) return;
    }

    // ---- K schedule (shared by both roles) ----
    int kfirst, nchunks;
    if (MODE == kInverse) {
        const int l_lo = m0 > j0 ? m0 : j0;
        kfirst = (l_lo / TK) * TK;
        nchunks = (L - kfirst + TK - 1) / TK;
    } else {
        int top = j0 + TJ - 1;
        if (top > L - 1) top = L - 1;
        kfirst = ((top + TK) / TK) * TK - 1;  // chunk-aligned top, >= top
        nchunks = (kfirst + 1) / TK;
    }
    auto kbase_of = [&](int chunk) {
        return MODE == kInverse ? kfirst + chunk * TK : kfirst - (chunk + 1) * TK + 1;
    };

    if (TAB && producer) {
        // ================= producers, table mode: copy M slabs =================
        const int ptid = tid - NC;
        const int jl = ptid % TJ, sub = ptid / TJ;
        const int j = j0 + jl, jc = jcol(jl);
        T vc[NCH][TK], vn[NCH][TK];
        auto load_slab = [&](int chunk, T (&dst)[NCH][TK]) {
            const int kbase = kbase_of(chunk);
#pragma unroll
            for (int g = 0; g < NCH; ++g) {
                const int m = m0 + sub * NCH + g;
#pragma unroll
                for (int kk = 0; kk < TK; ++kk) {
                    const int k = kbase + kk;
                    const bool ok = chunk < nchunks && j < L && m < L && k >= 0 && k < L;
                    size_t idx = 0;
                    if (ok) idx = MODE == kInverse ? ((size_t)m * L + k) * L + j : ((size_t)m * L + j) * L + k;
                    dst[g][kk] = ok ? mtab[idx] : T(0);
                }
            }
        };
        auto emit_t = [&](int buf, int gi, int kk, T v) {
            if constexpr (BF) {
                unsigned short hi, lo;
                bf16_split(v, hi, lo);
                sm.Mh[buf][gi][kk >> 2][jc][kk & 3] = hi;
                sm.Ml[buf][gi][kk >> 2][jc][kk & 3] = lo;
            } else if constexpr (KP) {
                sm.M[buf][gi][kk >> 1][jc][kk & 1] = v;
            } else {
                sm.M[buf][gi][kk][jc] = v;
            }
        };
        auto store_slab = [&](int chunk, int buf) {
            auto store = [&](auto pk_tag) {
                constexpr bool PK = decltype(pk_tag)::value;
#pragma unroll
                for (int g = 0; g < NCH; ++g)
#pragma unroll
                    for (int kk = 0; kk < TK; ++kk) emit_t(buf, sub * NCH + g, PK ? par16_pos(kk, TK) : kk, vc[g][kk]);
            };
            if (pk_of(kbase_of(chunk))) store(std::true_type{});
            else store(std::false_type{});
        };
        auto advance = [&]() {
#pragma unroll
            for (int g = 0; g < NCH; ++g)
#pragma unroll
                for (int kk = 0; kk < TK; ++kk) vc[g][kk] = vn[g][kk];
        };
        // same barrier sequence as the chain producers below
        load_slab(0, vc);
        __syncthreads();
        load_slab(1, vn);
        store_slab(0, 0);
        __syncthreads();
        for (int chunk = 1; chunk <= nchunks; ++chunk) {
            if (chunk < nchunks) {
                advance();
                load_slab(chunk + 1, vn);
                store_slab(chunk, chunk & 1);
            }
            __syncthreads();
        }
        return;
    }

    if (producer) {
        // ================= producers: FP64 Wigner chains =================
        // (FP32 / BF16x3: the producers issue ahead of the matrix-core waves)
        if constexpr (P != kP64) __builtin_amdgcn_s_setprio(2);
        const int ptid = tid - NC;
        // sub (the order rows of this thread) is uniform across a wave
        const int jl = ptid % TJ, sub = __builtin_amdgcn_readfirstlane(ptid / TJ);
        const int j = j0 + jl, jc = jcol(jl);
        const bool jvalid = j < L;
        Chain ch[NCH];
        int l0[NCH];
        double sv[NCH], twom[NCH];
        bool vch[NCH];
        // chains start at zero with the scale of their seed; the seed is added
        // by the step that reaches the chain's edge (degree for the inverse,
        // order for the forward)
#pragma unroll
        for (int g = 0; g < NCH; ++g) {
            const int m = m0 + sub * NCH + g;
            vch[g] = jvalid && m < L && (MODE == kInverse || j >= m);
            const Seed sd = vch[g] ? edge_seed(a.E, j, m) : Seed{0.0, 0};
            ch[g].d = 0.0;
            ch[g].dp = 0.0;
            ch[g].k = sd.k;
            ch[g].es = emit_scale(sd.k);
            sv[g] = sd.v;
            l0[g] = !vch[g] ? -2 : (MODE == kInverse ? (j > m ? j : m) : j);
            twom[g] = 2.0 * m;
        }
        double gprev = 0.0;  // forward: sqrt((l+m'+1)(l-m')) of the previous m'
#pragma unroll
        for (int g = 0; g < NCH; ++g)
            if (l0[g] == kfirst) ch[g].d = sv[g];

        // j-side step factors (plan table: (ap, bp) of the l-recursion for the
        // inverse, (y, g) of the m'-recursion for the forward) and the spin
        // factor sqrt((2l+1)/4pi) d^l_{.,-s}, PD steps ahead: set kk % PD
        // holds step kk of the slab until it is consumed and is then refilled
        // with step kk + PD (in this slab or the next), so no register copies.
        // The steps visit table rows one after another (up in l for the
        // inverse, down in m' for the forward), so each load takes a running
        // uniform row offset and a fixed lane offset into the table viewed as
        // a buffer: no address arithmetic per step.  The rows a tile visits
        // outside [0, L) lie in the tables' zero padding (kTabPad rows each
        // side); they only reach steps whose chains are zero or whose
        // emissions meet zero rows of X.  (The spin factor is held in the
        // output precision: it multiplies a value rounded to T on emission
        // anyway.)
        constexpr int PD = P == kP32W ? TK / 4 : TK / 2;  // fewer in flight where 3 waves share a SIMD
        const unsigned jo = (unsigned)(jvalid ? j : 0);
        double2 tj[PD];
        T wj[PD];
        const unsigned rowj = (unsigned)L * (unsigned)sizeof(double2), roww = (unsigned)L * (unsigned)sizeof(T);
        const int prow = L + 2 * kTabPad;
        const __amdgpu_buffer_rsrc_t jrs = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(a.jtab - (size_t)kTabPad * L), (short)0, prow * L * (int)sizeof(double2), kBufWord3);
        const __amdgpu_buffer_rsrc_t wrs = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(wtab - (size_t)kTabPad * L), (short)0, prow * L * (int)sizeof(T), kBufWord3);
        const unsigned jvo = jo * (unsigned)sizeof(double2), wvo = jo * (unsigned)sizeof(T);
        // padded row of the next step to load, in processing order
        const int krow0 = kbase_of(0) + (MODE == kInverse ? 0 : TK - 1) + kTabPad;
        unsigned soj = (unsigned)krow0 * rowj, sow = (unsigned)krow0 * roww;
        auto load_next = [&](double2 &t, T &w) {
            t = buffer_load_d2(jrs, jvo, soj);
            w = buffer_load<T>(wrs, wvo, sow);
            if (MODE == kInverse) {
                soj += rowj;
                sow += roww;
            } else {
                soj -= rowj;
                sow -= roww;
            }
        };
        // order-side factors of the l-recursion (inverse), staged through LDS
        // one slab ahead: loaded at the start of a slab, stored at its end
        double2 fnext = make_double2(0.0, 0.0);
        const int fgi = ptid / TK, fkk = ptid % TK;
        auto fetch_factors = [&](int chunk) {
            if (MODE == kInverse && ptid < GM * TK) {
                const int l = kbase_of(chunk) + fkk, idx = m0 + fgi;
                const bool ok = chunk < nchunks && l < L && idx < L;
                fnext = a.fab[ok ? (size_t)idx * L + l : 0];
                if (!ok) fnext = make_double2(0.0, 0.0);
            }
        };
        auto store_factors = [&](int buf) {
            if (MODE == kInverse && ptid < GM * TK) {
                fam[buf][fgi][fkk] = fnext.x;
                fbm[buf][fgi][fkk] = fnext.y;
            }
        };
        // one entry of M, rounded to the MFMA precision, into LDS at slab
        // position pos (the step kk, or par16_pos(kk) in parity blocks).
        // KP: the two entries of a position pair are written together as one
        // 8-byte store when the one in the even position is emitted (in
        // processing order, m' descending, it comes last: one step after its
        // partner, or two in parity blocks); the first waits in `held`, slot
        // (pos >> 3) & 1 (a pair of odd steps and one of even steps may wait
        // at once in parity blocks)
        T held[NCH][2];
        auto emit = [&](int buf, int g, int pos, double dv, T W) {
            const int gi = sub * NCH + g;
            if constexpr (BF) {
                unsigned short hi, lo;
                bf16_split((float)dv * W, hi, lo);
                sm.Mh[buf][gi][pos >> 2][jc][pos & 3] = hi;
                sm.Ml[buf][gi][pos >> 2][jc][pos & 3] = lo;
            } else if constexpr (KP) {
                const T v = (T)dv * W;
                if (pos & 1) {
                    held[g][(pos >> 3) & 1] = v;
                } else {
                    typedef float f32x2 __attribute__((ext_vector_type(2)));
                    *(f32x2 *)&sm.M[buf][gi][pos >> 1][jc][0] = f32x2{v, held[g][(pos >> 3) & 1]};
                }
            } else {
                sm.M[buf][gi][pos][jc] = (T)dv * W;
            }
        };
        // keep |d| < 2^512 for chains still below the double range (checked once
        // per slab: one slab grows a chain by far less than 2^400)
        auto renorm = [&](Chain &c) {
            if (c.k > 1 && fabs(c.d) > kBig) {
                c.d *= kSmall;
                c.dp *= kSmall;
                --c.k;
                c.es = emit_scale(c.k);
            }
        };
        // one slab.  INJ: some lane of the wave reaches a chain edge in it.
        // ES1: every chain of the wave is at scale level 0 (emission needs no
        // unscaling).
        // PK: the slab is stored in parity blocks.  (Always inlined: a call
        // would move the chain state it works on to scratch memory.)
        auto steps = [&](int chunk, int buf, auto inj_tag, auto es_tag, auto pk_tag) __attribute__((always_inline)) {
            constexpr bool INJ = decltype(inj_tag)::value, ES1 = decltype(es_tag)::value;
            constexpr bool PK = decltype(pk_tag)::value;
            const int kbase = kbase_of(chunk);
            // the step kk at which chain g reaches its edge (compared with the
            // unrolled kk, so no per-step constants are kept in registers)
            int edge[NCH];
#pragma unroll
            for (int g = 0; g < NCH; ++g) edge[g] = MODE == kInverse ? l0[g] - 1 - kbase : l0[g] + 1 - kbase;
            if (MODE == kInverse) {
                // order-side factors of step kk are read from LDS during step
                // kk-1; a scheduling barrier closes every step, so the reads
                // neither wait inside their own step nor all move to the slab
                // start (which needs more registers than the wave has)
                double fa[NCH], fb[NCH];
#pragma unroll
                for (int g = 0; g < NCH; ++g) {
                    fa[g] = fam[buf][sub * NCH + g][0];
                    fb[g] = fbm[buf][sub * NCH + g][0];
                }
#pragma unroll
                for (int kk = 0; kk < TK; ++kk) {  // degree l = kbase + kk
                    const double2 t = tj[kk % PD];
                    const T W = wj[kk % PD];
                    double am[NCH], bm[NCH];
#pragma unroll
                    for (int g = 0; g < NCH; ++g) {
                        am[g] = fa[g];
                        bm[g] = fb[g];
                        if (kk + 1 < TK) {
                            fa[g] = fam[buf][sub * NCH + g][kk + 1];
                            fb[g] = fbm[buf][sub * NCH + g][kk + 1];
                        }
                    }
                    load_next(tj[kk % PD], wj[kk % PD]);
#pragma unroll
                    for (int g = 0; g < NCH; ++g)
                        emit(buf, g, PK ? par16_pos(kk, TK) : kk, ES1 ? ch[g].d : ch[g].d * ch[g].es, W);
                    // step l -> l+1
#pragma unroll
                    for (int g = 0; g < NCH; ++g) {
                        double dn = -(t.x * am[g] * ch[g].d + t.y * bm[g] * ch[g].dp);
                        if constexpr (INJ) dn += (kk == edge[g]) ? sv[g] : 0.0;
                        ch[g].dp = ch[g].d;
                        ch[g].d = dn;
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            } else {
#pragma unroll
                for (int kk = TK - 1; kk >= 0; --kk) {  // m' = kbase + kk
                    const double2 t = tj[kk % PD];
                    const T W = wj[kk % PD];
                    load_next(tj[kk % PD], wj[kk % PD]);
#pragma unroll
                    for (int g = 0; g < NCH; ++g)
                        emit(buf, g, PK ? par16_pos(kk, TK) : kk, ES1 ? ch[g].d : ch[g].d * ch[g].es, W);
                    // step m' -> m'-1
#pragma unroll
                    for (int g = 0; g < NCH; ++g) {
                        double dn = (twom[g] * ch[g].d - gprev * ch[g].dp) * t.x;
                        if constexpr (INJ) dn += (kk == edge[g]) ? sv[g] : 0.0;
                        ch[g].dp = ch[g].d;
                        ch[g].d = dn;
                    }
                    gprev = t.y;
                }
            }
        };
        auto generate = [&](int chunk, int buf) __attribute__((always_inline)) {
            const int kbase = kbase_of(chunk);
            fetch_factors(chunk + 1);
            // edges reached in this slab: inverse l+1 in (kbase, kbase+TK],
            // forward m'-1 in [kbase-1, kbase+TK-2]
            bool mine = false, lvl0 = true;
#pragma unroll
            for (int g = 0; g < NCH; ++g) {
                const int e = l0[g];
                mine |= MODE == kInverse ? (e > kbase && e <= kbase + TK) : (e >= kbase - 1 && e <= kbase + TK - 2);
                lvl0 = lvl0 && ch[g].k == 0;
            }
            const bool inj = __any(mine), es1 = __all(lvl0);
            auto run = [&](auto pk_tag) __attribute__((always_inline)) {
                if (inj) {
                    if (es1) steps(chunk, buf, std::true_type{}, std::true_type{}, pk_tag);
                    else steps(chunk, buf, std::true_type{}, std::false_type{}, pk_tag);
                } else {
                    if (es1) steps(chunk, buf, std::false_type{}, std::true_type{}, pk_tag);
                    else steps(chunk, buf, std::false_type{}, std::false_type{}, pk_tag);
                }
            };
            if (pk_of(kbase)) run(std::true_type{});
            else run(std::false_type{});
#pragma unroll
            for (int g = 0; g < NCH; ++g) renorm(ch[g]);
            store_factors(buf ^ 1);
        };

        // ---- pipeline: producers run one slab ahead of the consumers.  Each
        // role has its own loop (disjoint register live ranges); both execute
        // the same number of workgroup barriers, and every wave takes one role.
        // the first PD steps of slab 0 in processing order
#pragma unroll
        for (int i = 0; i < PD; ++i) {
            const int kk = MODE == kInverse ? i : TK - 1 - i;
            load_next(tj[kk % PD], wj[kk % PD]);
        }
        fetch_factors(0);
        store_factors(0);
        __syncthreads();
        generate(0, 0);
        __syncthreads();
        for (int chunk = 1; chunk <= nchunks; ++chunk) {
            if (chunk < nchunks) generate(chunk, chunk & 1);
            __syncthreads();
        }
        return;
    }

    // ================= consumers: MFMA =================
    // this wave's j block and column range within the tile
    const int jw = wave % NJW, cwo = (wave / NJW) * CW;
    acc_t acc[GM][NCI][NJI];
#pragma unroll
    for (int g = 0; g < GM; ++g)
#pragma unroll
        for (int ci = 0; ci < NCI; ++ci)
#pragma unroll
            for (int ji = 0; ji < NJI; ++ji) acc[g][ci][ji] = acc_t{0, 0, 0, 0};

    auto mfma_slab = [&](int chunk, int buf) {
        const int kbase = kbase_of(chunk);
        // this wave's j: positions jw WJ .. jw WJ + WJ - 1 of the tile, i.e.
        // WJ consecutive j, or (parity placement) every other j from wj0
        const int wj0 = j0 + jpos(jw * WJ), wj1 = wj0 + (pj ? 2 : 1) * (WJ - 1);
        bool active = c0 + cwo < cend;  // some column of this wave exists
        if (MODE == kInverse) {
            const int start = m0 > wj0 ? m0 : wj0;
            active = active && kbase + TK - 1 >= start && wj0 < L;
        } else {
            active = active && kbase <= wj1 && wj0 < L;
        }
        if (!active) return;
        if constexpr (BF) {
            // one 16x16x16 BF16 MFMA spans the whole slab: per order, fragments
            // of group g+1 are read while the 3 NCI NJI MFMAs of group g run
            s16x4 ah[2][NCI], al[2][NCI], bh[2][NJI], bl[2][NJI];
            const int kg = lane >> 4;
            auto ldfrag = [&](int g, int slot) {
#pragma unroll
                for (int ci = 0; ci < NCI; ++ci) {
                    const int c = cwo + ci * 16 + (lane & 15);
                    ah[slot][ci] = *(const s16x4 *)&sm.Xh[buf][g][c][4 * kg];
                    al[slot][ci] = *(const s16x4 *)&sm.Xl[buf][g][c][4 * kg];
                }
#pragma unroll
                for (int ji = 0; ji < NJI; ++ji) {
                    const int jj = jw * WJ + ji * 16 + (lane & 15);
                    bh[slot][ji] = *(const s16x4 *)&sm.Mh[buf][g][kg][jj][0];
                    bl[slot][ji] = *(const s16x4 *)&sm.Ml[buf][g][kg][jj][0];
                }
            };
            ldfrag(0, 0);
#pragma unroll
            for (int g = 0; g < GM; ++g) {
                if (g + 1 < GM) ldfrag(g + 1, (g + 1) & 1);
                const int sl = g & 1;
#pragma unroll
                for (int ci = 0; ci < NCI; ++ci)
#pragma unroll
                    for (int ji = 0; ji < NJI; ++ji) {
                        acc_t c = acc[g][ci][ji];
                        c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al[sl][ci], bh[sl][ji], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[sl][ci], bl[sl][ji], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[sl][ci], bh[sl][ji], c, 0, 0, 0);
                        acc[g][ci][ji] = c;
                    }
            }
        } else if constexpr (KP) {
            // K slots in pairs: pair group (g, h) covers steps 2h and 2h + 1
            // of order g; slot q of step 2h + e takes k = 8h + 2q + e, so a
            // lane's two operands of a pair group are one 8-byte read from each
            // slab.  Fragments double-buffered as below.  This lane's X base
            // for pair group h is k = 8h + 2 (lane >> 4); in the swizzled rows
            // its quad 2h + (lane >> 5) sits at slot (2h + (lane >> 5)) ^
            // ((lane >> 2) & 3).
            typedef float f32x2 __attribute__((ext_vector_type(2)));
            f32x2 av[2][NCI], bv[2][NJI];
            constexpr int XR = Slabs<P, CTILE, KP>::XROW, MR = (TJ + 16) * 2;
            // halves of the slab (parity kernel): pair group h of every order,
            // in a loop that is not unrolled (one copy of the body)
            auto halves = [&](int h0, int nhalf) __attribute__((always_inline)) {
#pragma clang loop unroll(disable)
                for (int hf = 0; hf < nhalf; ++hf) {
                    const int h = h0 + hf;
                    const int q = DX ? (2 * h + (lane >> 5)) ^ ((lane >> 2) & 3) : 2 * h + (lane >> 5);
                    const float *xl = &sm.X[buf][0][cwo + (lane & 15)][4 * q + 2 * ((lane >> 4) & 1)];
                    const float *ml = &sm.M[buf][0][lane >> 4][jw * WJ + (lane & 15)][0] + 4 * h * MR;
                    auto ldfrag = [&](int g, int slot) {
#pragma unroll
                        for (int ci = 0; ci < NCI; ++ci) av[slot][ci] = *(const f32x2 *)&xl[(g * CTILE + ci * 16) * XR];
#pragma unroll
                        for (int ji = 0; ji < NJI; ++ji) bv[slot][ji] = *(const f32x2 *)&ml[g * (TK / 2) * MR + ji * 32];
                    };
                    ldfrag(0, 0);
#pragma unroll
                    for (int g = 0; g < GM; ++g) {
                        if (g + 1 < GM) ldfrag(g + 1, (g + 1) & 1);
#pragma unroll
                        for (int e = 0; e < 2; ++e)
#pragma unroll
                            for (int ci = 0; ci < NCI; ++ci)
#pragma unroll
                                for (int ji = 0; ji < NJI; ++ji)
                                    acc[g][ci][ji] = Mfma<T>::op(av[g & 1][ci][e], bv[g & 1][ji][e], acc[g][ci][ji]);
                    }
                }
            };
            // the whole slab in one pass
            auto whole = [&]() __attribute__((always_inline)) {
                constexpr int NPG = GM * 2;
                const float *xlh[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int q = DX ? (2 * h + (lane >> 5)) ^ ((lane >> 2) & 3) : 2 * h + (lane >> 5);
                    xlh[h] = &sm.X[buf][0][cwo + (lane & 15)][4 * q + 2 * ((lane >> 4) & 1)];
                }
                const float *ml = &sm.M[buf][0][lane >> 4][jw * WJ + (lane & 15)][0];
                auto ldfrag = [&](int idx, int slot) {
                    const int g = idx / 2, h = idx % 2;
#pragma unroll
                    for (int ci = 0; ci < NCI; ++ci) av[slot][ci] = *(const f32x2 *)&xlh[h][(g * CTILE + ci * 16) * XR];
#pragma unroll
                    for (int ji = 0; ji < NJI; ++ji) bv[slot][ji] = *(const f32x2 *)&ml[(g * (TK / 2) + 4 * h) * MR + ji * 32];
                };
                ldfrag(0, 0);
#pragma unroll
                for (int idx = 0; idx < NPG; ++idx) {
                    if (idx + 1 < NPG) ldfrag(idx + 1, (idx + 1) & 1);
                    const int g = idx / 2;
#pragma unroll
                    for (int e = 0; e < 2; ++e)
#pragma unroll
                        for (int ci = 0; ci < NCI; ++ci)
#pragma unroll
                            for (int ji = 0; ji < NJI; ++ji)
                                acc[g][ci][ji] = Mfma<T>::op(av[idx & 1][ci][e], bv[idx & 1][ji][e], acc[g][ci][ji]);
                }
            };
            // parity kernel: in a parity-block slab only the half of the
            // wave's parity, else both halves
            if constexpr (P == kP32 && PAR) {
                const bool pk = pk_of(kbase);  // one call: one copy of the body
                halves(pk ? (jw * WJ) / (TJ / 2) : 0, pk ? 1 : 2);
            } else {
                whole();
            }
        } else {
            // operand fragments double-buffered: group idx+1 is read from LDS
            // while the MFMAs of group idx run.  This lane's fragment bases in
            // the slab (X: k quad q, at slot q ^ ((lane >> 2) & 3) in swizzled
            // rows); every fragment is a constant offset from them.
            T av[2][NCI], bv[2][NJI];
            constexpr int XR = Slabs<P, CTILE, KP>::XROW, MR = TJ + 16;
            // halves of the slab (parity kernel): k quads 2h and 2h + 1 of
            // every order, in a loop that is not unrolled (one copy of the body)
            auto halves = [&](int h0, int nhalf) __attribute__((always_inline)) {
#pragma clang loop unroll(disable)
                for (int hf = 0; hf < nhalf; ++hf) {
                    const int kq0 = 2 * (h0 + hf);
                    const T *xl[2];
#pragma unroll
                    for (int e = 0; e < 2; ++e) {
                        const int q = DX ? (kq0 + e) ^ ((lane >> 2) & 3) : kq0 + e;
                        xl[e] = &sm.X[buf][0][cwo + (lane & 15)][4 * q + (lane >> 4)];
                    }
                    const T *ml = &sm.M[buf][0][lane >> 4][jw * WJ + (lane & 15)] + 4 * kq0 * MR;
                    constexpr int NG = GM * 2;
                    auto ldfrag = [&](int idx, int slot) {
                        const int g = idx / 2, e = idx % 2;
#pragma unroll
                        for (int ci = 0; ci < NCI; ++ci) av[slot][ci] = xl[e][(g * CTILE + ci * 16) * XR];
#pragma unroll
                        for (int ji = 0; ji < NJI; ++ji) bv[slot][ji] = ml[(g * TK + e * 4) * MR + ji * 16];
                    };
                    ldfrag(0, 0);
#pragma unroll
                    for (int idx = 0; idx < NG; ++idx) {
                        if (idx + 1 < NG) ldfrag(idx + 1, (idx + 1) & 1);
                        const int g = idx / 2;
#pragma unroll
                        for (int ci = 0; ci < NCI; ++ci)
#pragma unroll
                            for (int ji = 0; ji < NJI; ++ji)
                                acc[g][ci][ji] = Mfma<T>::op(av[idx & 1][ci], bv[idx & 1][ji], acc[g][ci][ji]);
                    }
                }
            };
            // the whole slab in one pass
            auto whole = [&]() __attribute__((always_inline)) {
                constexpr int NKS = TK / 4, NGRP = GM * NKS;
                const T *xlk[NKS];
#pragma unroll
                for (int ks = 0; ks < NKS; ++ks) {
                    const int q = DX ? ks ^ ((lane >> 2) & 3) : ks;
                    xlk[ks] = &sm.X[buf][0][cwo + (lane & 15)][4 * q + (lane >> 4)];
                }
                const T *ml = &sm.M[buf][0][lane >> 4][jw * WJ + (lane & 15)];
                auto ldfrag = [&](int idx, int slot) {
                    const int g = idx / NKS, ks = idx % NKS;
#pragma unroll
                    for (int ci = 0; ci < NCI; ++ci) av[slot][ci] = xlk[ks][(g * CTILE + ci * 16) * XR];
#pragma unroll
                    for (int ji = 0; ji < NJI; ++ji) bv[slot][ji] = ml[(g * TK + ks * 4) * MR + ji * 16];
                };
                ldfrag(0, 0);
#pragma unroll
                for (int idx = 0; idx < NGRP; ++idx) {
                    if (idx + 1 < NGRP) ldfrag(idx + 1, (idx + 1) & 1);
                    const int g = idx / NKS;
#pragma unroll
                    for (int ci = 0; ci < NCI; ++ci)
#pragma unroll
                        for (int ji = 0; ji < NJI; ++ji)
                            acc[g][ci][ji] = Mfma<T>::op(av[idx & 1][ci], bv[idx & 1][ji], acc[g][ci][ji]);
                }
            };
            // parity kernel: as in the paired path above
            if constexpr (P == kP32 && PAR) {
                const bool pk = pk_of(kbase);  // one call: one copy of the body
                halves(pk ? (jw * WJ) / (TJ / 2) : 0, pk ? 1 : 2);
            } else {
                whole();
            }
        }
    };

    if constexpr (DX) {
        // X slab by LDS-direct loads: instruction i of consumer wave w moves
        // the 64 16-byte slots s = (NSL w + i) 64 + lane of the slab
        // [g][c][TK] (4 slots a row), i.e. rows (g_i, cb_i + lane / 4) with
        // cb_i a multiple of 16; slot q' of row c holds the k quad
        // q' ^ ((c >> 2) & 3) = q' ^ ((lane >> 4) & 3).  A lane's global
        // offset is then one per-lane part, fixed for the whole K loop, plus
        // a uniform part per instruction and the uniform slab offset.
        constexpr int NSL = GM * CTILE * TK / 4 / NC;  // slots per consumer thread
        static_assert(NSL * NC * 4 == GM * CTILE * TK && TK == 16 && CTILE % 16 == 0, "slot map");
        const int wv = __builtin_amdgcn_readfirstlane(wave);
        const int lrow = lane >> 2, lq = (lane & 3) ^ ((lane >> 4) & 3);
        const unsigned vlane = (unsigned)((lrow * L + 4 * lq) * (int)sizeof(T));
        auto slot_g = [&](int i) { return (wv * NSL + i) * 64 / (CTILE * 4); };
        auto slot_cb = [&](int i) { return ((wv * NSL + i) * 16) % CTILE; };
        bool rok = true;
#pragma unroll
        for (int i = 0; i < NSL; ++i) rok = rok && (m0 + slot_g(i)) < L && (c0 + slot_cb(i) + lrow) < cend;
        const T *xbase = a.X + (size_t)m0 * Cn * L;
        // every row this wave moves exists, and the rows are 16-byte aligned
        const bool wall = __all(rok) && (L & 3) == 0;
        const __amdgpu_buffer_rsrc_t xrsrc = __builtin_amdgcn_make_buffer_rsrc(
            (void *)xbase, (short)0, wall ? GM * Cn * L * (int)sizeof(T) : 0, kBufWord3);
        auto full_slab = [&](int chunk) {
            const int kbase = kbase_of(chunk);
            return wall && kbase >= 0 && kbase + TK <= L && (MODE != kInverse || kbase >= m0 + GM - 1);
        };
        // whole slab inside rows that exist: straight into LDS
        auto load_direct = [&](int chunk, int buf) {
            const unsigned so = (unsigned)kbase_of(chunk) * (unsigned)sizeof(T);
#pragma unroll
            for (int i = 0; i < NSL; ++i) {
                T *dst = &sm.X[buf][0][0][0] + (wv * NSL + i) * 64 * 4;
                const unsigned si = (unsigned)((slot_g(i) * Cn + c0 + slot_cb(i)) * L * (int)sizeof(T)) + so;
                __builtin_amdgcn_raw_ptr_buffer_load_lds(xrsrc, (__attribute__((address_space(3))) void *)dst, 16,
                                                         vlane, si, 0, 0);
            }
        };
        // otherwise element by element with the bounds of the panel rows
        // (inverse: l >= m, with l the degree a position holds), through
        // registers
        auto load_masked = [&](int chunk, int buf) {
            const int kbase = kbase_of(chunk);
            const bool pk = pk_of(kbase);
#pragma unroll
            for (int i = 0; i < NSL; ++i) {
                const int sl = (wv * NSL + i) * 64 + lane;
                const int g = slot_g(i), c = slot_cb(i) + lrow;
                const bool row = (m0 + g) < L && (c0 + c) < cend;
                const T *src = xbase + (size_t)(g * Cn + c0 + c) * L;
                T v[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int k = kbase + 4 * lq + e, kt = kbase + (pk ? par16_idx(4 * lq + e) : 4 * lq + e);
                    const bool ok = row && k >= 0 && k < L && (MODE != kInverse || kt >= m0 + g);
                    v[e] = ok ? src[k] : T(0);
                }
                *(float4 *)(&sm.X[buf][0][0][0] + sl * 4) = make_float4(v[0], v[1], v[2], v[3]);
            }
        };
        // the direct loads must have landed before the barrier publishes them
        auto wait_direct = [&]() { __builtin_amdgcn_s_waitcnt(0x0F70); };  // vmcnt(0)

        __syncthreads();
        if (full_slab(0)) {
            load_direct(0, 0);
            wait_direct();
        } else {
            load_masked(0, 0);
        }
        __syncthreads();
        for (int chunk = 1; chunk <= nchunks; ++chunk) {
            const int cur = chunk & 1, prev = cur ^ 1;
            const bool more = chunk < nchunks, direct = more && full_slab(chunk);
            if (direct) load_direct(chunk, cur);
            mfma_slab(chunk - 1, prev);
            if (more && !direct) load_masked(chunk, cur);
            if (direct) wait_direct();
            __syncthreads();
        }
    } else {
        // X slab: element i of this thread is (g, c, kk); 32-bit offsets from the
        // group's panel base, fixed for the whole K loop.  FP32 / BF16x3: element
        // 4 q + r is k = 4 kq + r of the q-th (g, c, kq) quadruple, so a thread's
        // four consecutive elements are four consecutive k of one row (one
        // 16-byte load when the rows are 16-byte aligned)
        constexpr bool V4 = P != kP64;
        constexpr int XROW = Slabs<P, CTILE, KP>::XROW;
        int xoff[XPT], xsl[XPT], xkk[XPT], xg[XPT];
        bool xok[XPT];
    #pragma unroll
        for (int i = 0; i < XPT; ++i) {
            int g, c, kk;
            if constexpr (V4) {
                const int e4 = tid + (i / 4) * NC;  // over [GM][CTILE][TK / 4]
                g = e4 / (CTILE * TK / 4);
                const int rem = e4 % (CTILE * TK / 4);
                c = rem / (TK / 4);
                kk = 4 * (rem % (TK / 4)) + i % 4;
            } else {
                const int e = tid + i * NC;  // over [GM][CTILE][TK]
                g = e / (CTILE * TK);
                const int rem = e % (CTILE * TK);
                c = rem / TK;
                kk = rem % TK;
            }
            xg[i] = g;
            xkk[i] = kk;
            xok[i] = (m0 + g) < L && (c0 + c) < cend;
            xoff[i] = (g * Cn + c0 + c) * L + kk;
            xsl[i] = (g * CTILE + c) * XROW + kk;
        }
        const T *xbase = a.X + (size_t)m0 * Cn * L;
        bool xall = true;
    #pragma unroll
        for (int i = 0; i < XPT; ++i) xall = xall && xok[i];
        xall = __all(xall);  // every (order, column) of the tile exists
        // the group's panel rows as a buffer resource (used only when xall: then
        // the GM rows of Cn x L entries all exist)
        const __amdgpu_buffer_rsrc_t xrsrc =
            __builtin_amdgcn_make_buffer_rsrc((void *)xbase, (short)0, xall ? GM * Cn * L * (int)sizeof(T) : 0, kBufWord3);
        unsigned xvo[P != kP64 ? XPT : 1];
        if constexpr (P != kP64) {
    #pragma unroll
            for (int i = 0; i < XPT; ++i) xvo[i] = (unsigned)xoff[i] * (unsigned)sizeof(T);
        }
        T xr[XPT];
        auto load_x = [&](int chunk) {
            const int kbase = kbase_of(chunk);
            // whole slab inside the panel rows that exist (inverse: l >= m for
            // every order of the group): plain loads from a uniform base
            // (FP64 tiles keep the masked loads: their accumulators leave no
            // room for the buffer offsets)
            const bool full = P != kP64 && xall && kbase >= 0 && kbase + TK <= L && (MODE != kInverse || kbase >= m0 + GM - 1);
            if (full) {
                // buffer loads: the tile's panel as a resource, the lane offset
                // (fixed for the whole K loop) and the slab offset (uniform) both
                // added by the memory unit
                const unsigned so = (unsigned)kbase * (unsigned)sizeof(T);
                if constexpr (P != kP64) {
                    if ((L & 3) == 0) {
                        // rows and slab start 16-byte aligned (kbase is a multiple of TK)
    #pragma unroll
                        for (int i = 0; i < XPT; i += 4) {
                            const float4 v = buffer_load_f4(xrsrc, xvo[i], so);
                            xr[i] = v.x;
                            xr[i + 1] = v.y;
                            xr[i + 2] = v.z;
                            xr[i + 3] = v.w;
                        }
                    } else {
    #pragma unroll
                        for (int i = 0; i < XPT; ++i) xr[i] = buffer_load<T>(xrsrc, xvo[i], so);
                    }
                }
            } else {
    #pragma unroll
                for (int i = 0; i < XPT; ++i) {
                    const int k = kbase + xkk[i];
                    bool ok = xok[i] && k >= 0 && k < L;
                    // the degree this position holds (parity blocks: par16_idx)
                    const int kt = kbase + (pk_of(kbase) ? par16_idx(xkk[i]) : xkk[i]);
                    if (MODE == kInverse) ok = ok && kt >= m0 + xg[i];
                    xr[i] = ok ? xbase[xoff[i] + kbase] : T(0);
                }
            }
        };
        auto store_x = [&](int buf) {
            if constexpr (BF) {
                unsigned short *xh = &sm.Xh[buf][0][0][0], *xl = &sm.Xl[buf][0][0][0];
    #pragma unroll
                for (int i = 0; i < XPT; ++i) {
                    unsigned short hi, lo;
                    bf16_split(xr[i], hi, lo);
                    xh[xsl[i]] = hi;
                    xl[xsl[i]] = lo;
                }
            } else if constexpr (kIsF32<P>) {
                float *xt = &sm.X[buf][0][0][0];
    #pragma unroll
                for (int i = 0; i < XPT; i += 4) *(float4 *)&xt[xsl[i]] = make_float4(xr[i], xr[i + 1], xr[i + 2], xr[i + 3]);
            } else {
                T *xt = &sm.X[buf][0][0][0];
    #pragma unroll
                for (int i = 0; i < XPT; ++i) xt[xsl[i]] = xr[i];
            }
        };

        __syncthreads();
        load_x(0);
        store_x(0);
        __syncthreads();
        for (int chunk = 1; chunk <= nchunks; ++chunk) {
            const int cur = chunk & 1, prev = cur ^ 1;
            if (chunk < nchunks) load_x(chunk);
            mfma_slab(chunk - 1, prev);
            if (chunk < nchunks) store_x(cur);
            __syncthreads();
        }

    }

    // ---- write out[c][j] ----
#pragma unroll
    for (int g = 0; g < GM; ++g) {
        const int m = m0 + g;
        if (m >= L) continue;
        T *yrow = a.Y + (size_t)m * Cn * L;
#pragma unroll
        for (int ci = 0; ci < NCI; ++ci)
#pragma unroll
            for (int ji = 0; ji < NJI; ++ji)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int c = c0 + cwo + ci * 16 + Mfma<T>::row(lane, r);
                    const int jj = j0 + jpos(jw * WJ + ji * 16 + (lane & 15));
                    if (c < cend && jj < L) yrow[c * L + jj] = acc[g][ci][ji][r];
                }
    }
}

// par: the parity kernel (spin-0 blocks of FP32 data; 64-column-or-narrower
// FP32 and BF16x3 tiles)
template <int P, int MODE, int CTILE>
hipError_t launch_one(Args<typename Prec<P>::T> a, int nsched, bool tab, bool par, hipStream_t st) {
    if (nsched == 0 || a.ncb == 0) return hipSuccess;
    const dim3 grid(nsched, a.ncb);
    if constexpr (P == kP32 || P == kPBF) {
        if (par) {
            if (tab) hipLaunchKernelGGL((k_contract<P, MODE, CTILE, true, true>), grid, dim3(kThreads<P>), 0, st, a);
            else hipLaunchKernelGGL((k_contract<P, MODE, CTILE, false, true>), grid, dim3(kThreads<P>), 0, st, a);
            return hipGetLastError();
        }
    }
    if (par) return hipErrorInvalidValue;
    if (tab) hipLaunchKernelGGL((k_contract<P, MODE, CTILE, true, false>), grid, dim3(kThreads<P>), 0, st, a);
    else hipLaunchKernelGGL((k_contract<P, MODE, CTILE, false, false>), grid, dim3(kThreads<P>), 0, st, a);
    return hipGetLastError();
}

// Table of M_m(m', l) = sqrt((2l+1)/4pi) d^l_{m'm}(pi/2) d^l_{m',-s}(pi/2),
// rounded to T as the chain producers round it, at [m][l][m'] (zero for
// l < max(m, m')).  One thread per (m, m'): the l-chain of the inverse
// producers run over the whole degree range.
template <typename T>
__global__ void k_mtable(int L, EdgeTable E, const double *ri, const double2 *fab, const T *w, T *tab) {
    const int mp = blockIdx.x * blockDim.x + threadIdx.x, m = blockIdx.y;
    if (mp >= L) return;
    const int l0 = mp > m ? mp : m;
    const Seed sd = edge_seed(E, mp, m);
    Chain c;
    c.d = 0.0;
    c.dp = 0.0;
    c.k = sd.k;
    c.es = emit_scale(sd.k);
    double q = 0.0;
    for (int l = 0; l < L; ++l) {
        const size_t o = ((size_t)m * L + l) * L + mp;
        if (l < l0) {
            tab[o] = T(0);
            continue;
        }
        if (l == l0) c.d = sd.v;
        tab[o] = (T)(c.d * c.es) * w[(size_t)l * L + mp];
        const double r = ri[(size_t)l * L + mp];
        const double ap = (double)mp * r, bp = q * r;
        q = ((double)(l + 1) * (l + 1) - (double)mp * mp) * r;
        const double2 f = fab[(size_t)m * L + l];
        const double dn = -(ap * f.x * c.d + bp * f.y * c.dp);
        c.dp = c.d;
        c.d = dn;
        if (((l - l0) & 15) == 15 && c.k > 1 && fabs(c.d) > kBig) {
            c.d *= kSmall;
            c.dp *= kSmall;
            --c.k;
            c.es = emit_scale(c.k);
        }
    }
}

// Column tile of the contraction for (device, L, columns, precision): the
// choice recorded by set_contract_tile (pinned, or picked by the timing
// autotuner), else the tile t in {16, 32, 64} (FP32 also 128) that minimises
// the sum over column blocks of (its columns rounded up to t, or to 64 in the
// 128-column tile, whose consumer waves each take 64 columns and skip
// theirs when absent) + 24: every block pays its columns on the matrix cores
// plus the Wigner generation, which costs about as much as 24 columns.
std::mutex g_tile_mu;
std::map<std::tuple<int, int, int, int>, int> g_tiles;

// (several spins: the cost is summed over their column ranges; a pinned tile
// is looked up under the total column count)
// Segments a launch takes: all, only those of spin 0, or only the others.
enum { kAllSpins = 0, kSpinZero = 1, kSpinNonzero = 2 };
bool seg_in(const ContractSeg &sg, int which) {
    return which == kAllSpins || ((sg.sp->spin == 0) == (which == kSpinZero));
}

// the cost model's best tile up to tmax over the segments `which` selects
int best_tile(int nseg, const ContractSeg *seg, int tmax, int which) {
    int best = 16;
    long best_cost = -1;
    for (int t = 16; t <= tmax; t *= 2) {
        const int gran = t > 64 ? 64 : t;
        long cost = 0;
        for (int k = 0; k < nseg; ++k) {
            if (!seg_in(seg[k], which)) continue;
            for (int c = 0; c < seg[k].ncol; c += t) {
                const int n = seg[k].ncol - c < t ? seg[k].ncol - c : t;
                cost += (n + gran - 1) / gran * gran + 24;
            }
        }
        if (best_cost < 0 || cost < best_cost) {
            best = t;
            best_cost = cost;
        }
    }
    return best;
}

int contract_tile(int L, int nseg, const ContractSeg *seg, int P) {
    int C = 0;
    for (int k = 0; k < nseg; ++k) C += seg[k].ncol;
    int dev = 0;
    (void)hipGetDevice(&dev);
    {
        std::lock_guard<std::mutex> lk(g_tile_mu);
        auto it = g_tiles.find(std::make_tuple(dev, L, C, P));
        if (it != g_tiles.end()) return it->second;
    }
    return best_tile(nseg, seg, P == kP32 ? 128 : 64, kAllSpins);
}

template <int P>
hipError_t launch_tiled(int mode, int L, int nseg, const ContractSeg *seg, int ct, const typename Prec<P>::T *X,
                        typename Prec<P>::T *Y, const EdgeTable &E, const RecTables &rt, hipStream_t st, int which,
                        bool par) {
    using T = typename Prec<P>::T;
    Args<T> a;
    a.L = L;
    a.C = 0;
    for (int k = 0; k < nseg; ++k) a.C += seg[k].ncol;
    a.njt = (L + Prec<P>::TJ - 1) / Prec<P>::TJ;
    a.X = X;
    a.Y = Y;
    a.E = E;
    a.jtab = mode == kInverse ? rt.jti : rt.jtf;
    a.fab = rt.fab;
    a.cl = rt.cl;
    const int cls = Prec<P>::TJ == 64 ? 0 : 1;
    a.sched = rt.sched[mode][cls];
    const int ns = rt.nsched[mode][cls];
    // column blocks, spin by spin; table mode only when every spin has its table
    bool tab = true;
    int nb = 0, c = 0;
    for (int k = 0; k < nseg; ++k) {
        if (!seg_in(seg[k], which)) {  // another launch's columns
            c += seg[k].ncol;
            continue;
        }
        const SpinPlan &sp = *seg[k].sp;
        const T *w, *mt;
        if constexpr (P == kP64) {
            w = mode == kInverse ? sp.wi : sp.wf;
            mt = sp.mtab64;
        } else {
            w = mode == kInverse ? sp.wi32 : sp.wf32;
            mt = sp.mtab32;
        }
        tab = tab && mt != nullptr;
        for (int c0 = 0; c0 < seg[k].ncol; c0 += ct) {
            if (nb == kMaxColBlocks) return hipErrorInvalidValue;
            a.c0[nb] = c + c0;
            a.cend[nb] = c + seg[k].ncol;
            a.asg[nb] = sp.spin < 0 ? -sp.spin : sp.spin;
            a.wtab[nb] = w;
            a.mtab[nb] = mt;
            ++nb;
        }
        c += seg[k].ncol;
    }
    a.ncb = nb;
    if constexpr (P == kP32W) {
        return mode == kInverse ? launch_one<P, kInverse, 128>(a, ns, tab, par, st)
                                : launch_one<P, kForward, 128>(a, ns, tab, par, st);
    } else {
        if (ct == 16)
            return mode == kInverse ? launch_one<P, kInverse, 16>(a, ns, tab, par, st)
                                    : launch_one<P, kForward, 16>(a, ns, tab, par, st);
        if (ct == 32)
            return mode == kInverse ? launch_one<P, kInverse, 32>(a, ns, tab, par, st)
                                    : launch_one<P, kForward, 32>(a, ns, tab, par, st);
        return mode == kInverse ? launch_one<P, kInverse, 64>(a, ns, tab, par, st)
                                : launch_one<P, kForward, 64>(a, ns, tab, par, st);
    }
}

template <int P>
hipError_t launch_prec(int mode, int L, int nseg, const ContractSeg *seg, const typename Prec<P>::T *X,
                       typename Prec<P>::T *Y, const EdgeTable &E, const RecTables &rt, hipStream_t st) {
    const int ct = contract_tile(L, nseg, seg, P);
    if constexpr (P == kP64) {
        return launch_tiled<P>(mode, L, nseg, seg, ct, X, Y, E, rt, st, kAllSpins, false);
    } else {
        // FP32 data: the spin-0 segments (their panels in parity blocks) go to
        // the parity kernel, on a tile of at most 64 columns; the others to
        // the plain one, the 128-column tile when chosen (two launches on the
        // stream when there are both)
        bool zero = false, other = false;
        for (int k = 0; k < nseg; ++k) (seg[k].sp->spin == 0 ? zero : other) = true;
        hipError_t e = hipSuccess;
        if (other) {
            const int which = zero ? kSpinNonzero : kAllSpins;
            if (P == kP32 && ct == 128) e = launch_tiled<kP32W>(mode, L, nseg, seg, ct, X, Y, E, rt, st, which, false);
            else e = launch_tiled<P>(mode, L, nseg, seg, ct, X, Y, E, rt, st, which, false);
        }
        if (e == hipSuccess && zero) {
            const int ct0 = ct > 64 ? best_tile(nseg, seg, 64, kSpinZero) : ct;
            e = launch_tiled<P>(mode, L, nseg, seg, ct0, X, Y, E, rt, st, other ? kSpinZero : kAllSpins, true);
        }
        return e;
    }
}

}  // namespace

template <typename T>
hipError_t launch_contract(int mode, int L, int nseg, const ContractSeg *seg, const T *X, T *Y, const EdgeTable &E,
                           const RecTables &rt, hipStream_t st) {
    constexpr int P = sizeof(T) == 8 ? kP64 : kP32;
    return launch_prec<P>(mode, L, nseg, seg, X, Y, E, rt, st);
}

template hipError_t launch_contract<double>(int, int, int, const ContractSeg *, const double *, double *,
                                            const EdgeTable &, const RecTables &, hipStream_t);
template hipError_t launch_contract<float>(int, int, int, const ContractSeg *, const float *, float *,
                                           const EdgeTable &, const RecTables &, hipStream_t);

int build_contract_schedules(int L, RecTables &rt) {
    static_assert(Prec<kP64>::TJ == 64 && Prec<kP32>::TJ == 128 && Prec<kPBF>::TJ == 128, "tile classes");
    const int tjs[2] = {64, 128};
    for (int mode = 0; mode < 2; ++mode)
        for (int cls = 0; cls < 2; ++cls) {
            const int TJ = tjs[cls];
            const int nmg = (L + GM - 1) / GM, njt = (L + TJ - 1) / TJ;
            std::vector<std::pair<int, int>> items;  // (K slabs, code)
            for (int mg = 0; mg < nmg; ++mg)
                for (int jt = 0; jt < njt; ++jt) {
                    const int m0 = mg * GM, j0 = jt * TJ;
                    int cost;
                    if (mode == kInverse) {
                        const int lo = m0 > j0 ? m0 : j0;
                        cost = (L - (lo / TK) * TK + TK - 1) / TK;
                    } else {
                        if (j0 + TJ - 1 < m0) continue;  // outputs l < m are never read
                        const int top = j0 + TJ - 1 < L - 1 ? j0 + TJ - 1 : L - 1;
                        cost = (top + TK) / TK;
                    }
                    items.push_back({cost, (mg << 8) | jt});
                }
            std::stable_sort(items.begin(), items.end(),
                             [](const std::pair<int, int> &x, const std::pair<int, int> &y) { return x.first > y.first; });
            // Workgroups go to the 8 XCDs round-robin (x mod 8).  Order group
            // mg goes to XCD mg mod 8 with all its j tiles, which read the
            // same panel rows, so those rows are fetched into one L2; each
            // XCD's list stays longest first.  Interleaved entry 8i + k is
            // the i-th of XCD k's list, padded with -1 (no work) to a
            // multiple of 8, which keeps x mod 8 the XCD in every column block.
            std::vector<int> per[8];
            for (const auto &it : items) per[(it.second >> 8) & 7].push_back(it.second);
            size_t n = 0;
            for (int k = 0; k < 8; ++k) n = per[k].size() > n ? per[k].size() : n;
            std::vector<int> codes(8 * n, -1);
            for (size_t i = 0; i < n; ++i)
                for (int k = 0; k < 8; ++k)
                    if (i < per[k].size()) codes[8 * i + k] = per[k][i];
            if (hipMalloc(&rt.sched[mode][cls], codes.size() * sizeof(int)) != hipSuccess) return -1;
            if (hipMemcpy(rt.sched[mode][cls], codes.data(), codes.size() * sizeof(int), hipMemcpyHostToDevice) !=
                hipSuccess)
                return -1;
            rt.nsched[mode][cls] = (int)codes.size();
        }
    return 0;
}

hipError_t launch_mtable(int L, int precision_fp64, const EdgeTable &E, const RecTables &rt, SpinPlan &sp,
                         hipStream_t st) {
    const dim3 grid((L + 63) / 64, L);
    if (precision_fp64)
        hipLaunchKernelGGL(k_mtable<double>, grid, dim3(64), 0, st, L, E, rt.ri, rt.fab, sp.wi, sp.mtab64);
    else
        hipLaunchKernelGGL(k_mtable<float>, grid, dim3(64), 0, st, L, E, rt.ri, rt.fab, sp.wi32, sp.mtab32);
    return hipGetLastError();
}

hipError_t launch_contract_bf16x3(int mode, int L, int nseg, const ContractSeg *seg, const float *X, float *Y,
                                  const EdgeTable &E, const RecTables &rt, hipStream_t st) {
    return launch_prec<kPBF>(mode, L, nseg, seg, X, Y, E, rt, st);
}

int contract_precision_class(bool fp64, bool bf16x3) { return fp64 ? kP64 : (bf16x3 ? kPBF : kP32); }

void set_contract_tile(int L, int C, int pclass, int ctile) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_tile_mu);
    const auto key = std::make_tuple(dev, L, C, pclass);
    if (ctile == 0) g_tiles.erase(key);
    else g_tiles[key] = ctile;
}

int get_contract_tile(int L, int C, int pclass) {
    const ContractSeg one{C, nullptr};
    return contract_tile(L, 1, &one, pclass);
}

}  // namespace sht
