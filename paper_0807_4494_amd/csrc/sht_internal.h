// Internal declarations shared by the HIP translation units of libsht.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "sht.h"

namespace sht {

// ---------------------------------------------------------------- numbers ---
struct cplx64 { double x, y; };
struct cplx32 { float x, y; };

template <typename T> struct CT;
template <> struct CT<double> { using type = cplx64; };
template <> struct CT<float> { using type = cplx32; };

template <typename C> __host__ __device__ inline C cmul(C a, C b) {
    return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename C> __host__ __device__ inline C cmulc(C a, C b) {  // a * conj(b)
    return C{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename C> __host__ __device__ inline C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __host__ __device__ inline C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }

// Extended-range scale for Wigner chains: a chain value is stored as
// d * 2^(-512 k); k = 0 means plain.  Seeds as small as 2^-2048 occur.
constexpr double kBig = 0x1p512;
constexpr double kSmall = 0x1p-512;

__host__ __device__ inline int parity(long long x) { return (int)(x & 1); }
__host__ __device__ inline double sgn_pow(long long x) { return parity(x) ? -1.0 : 1.0; }

// ---------------------------------------------------------------- plans -----
// Edge table: E[l][k] = 2^-l sqrt(C(2l, l+k)), 0 <= k <= l < SHT_L_MAX, as a
// mantissa in [1, 2) and a binary exponent, at index l(l+1)/2 + k.
struct EdgeTable {
    double *mant = nullptr;
    int *expo = nullptr;
    int lmax = 0;
};

// Per-(L, precision) tables for the torus FFT stages.
template <typename T> struct FftTables {
    using C = typename CT<T>::type;
    int L = 0, N = 0, M = 0, logM = 0;
    C *tw = nullptr;      // e^{-2 pi i k / M}, k < M
    C *e2n = nullptr;     // e^{i pi k / N}, k < 2N
    C *cha = nullptr;     // e^{i pi (n^2 + n) / N}, n < N          (chirps of the stages)
    C *chb = nullptr;     // e^{i pi (n^2 - 2 h n - h) / N}, n < N, h = L - 1
    C *ptw = nullptr;     // per-pass Stockham twiddles (fft_pass_offset)
    C *h_ip = nullptr;    // spectra (natural order, 1/M folded in) of the chirp-z kernels:
    C *h_fd = nullptr;    //   inverse DFT, forward DFT,
    C *h_fk = nullptr;    //   and the forward quadrature's real kernel K
    C *ptwh = nullptr;    // pass twiddles of an M/2-point FFT (rows split in two halves;
                          //   allocated when M > 8192)
};

// Row length of the rings between the theta and phi stages: 2L complex
// values per ring for complex maps (the N = 2L - 1 orders and one unused
// slot, so that every ring starts 16-byte aligned and a pair of orders is one
// aligned 16-byte piece), L + (L & 1) for real maps (orders m >= 0).
__host__ __device__ constexpr int ring_len(int L, bool half) { return half ? L + (L & 1) : 2 * L; }

// Spin-0 panel order (FP32 data).  Delta^l_{m',0}(pi/2) vanishes for odd
// l + m', so spin-0 contractions pair even degrees with even m' and odd with
// odd.  The FP32 contraction inputs of spin 0 (degrees l of the inverse's
// coefficient panels, orders m' of the forward's theta-stage output)
// therefore hold each complete aligned block of 16 indices as its 8 even
// entries followed by its 8 odd ones; an incomplete last block keeps the
// natural order.
__host__ __device__ constexpr int par16_pos(int k, int L) {
    return (k | 15) < L ? (k & ~15) | ((k & 1) << 3) | ((k & 15) >> 1) : k;
}
// offset within a complete block: position p holds index 2 (p & 7) + (p >> 3)
__host__ __device__ constexpr int par16_idx(int p) { return ((p & 7) << 1) | ((p >> 3) & 1); }

// Rows whose M-point buffer exceeds the LDS (FP64 at M = 16384) run as two
// halves with a global scratch slot of M complex values per workgroup; a
// launch uses at most kSplitSlots workgroups.
constexpr int kSplitSlots = 256;
constexpr size_t kLdsBytes = 160 * 1024;   // LDS of one CU
__host__ __device__ constexpr bool rows_split(int M, int cbytes) {
    return (size_t)(M + M / 16) * (size_t)cbytes > kLdsBytes;
}

// Per-L reciprocal square roots of the two Wigner recursions (FP64):
//   ri[l*L + j] = 1/sqrt((l+1)^2 - j^2)        (l-recursion, j <= l; else 0)
//   rf[k*L + l] = 1/sqrt((l+k)(l-k+1))          (m'-recursion at m' = k; 0 if k > l)
// and the order-side factors of the l-recursion, for a >= 0 and l < L:
//   fab[a*L + l] = { a (2l+1) / (l sqrt((l+1)^2 - a^2)),
//                    sqrt(l^2 - a^2) (l+1) / (l sqrt((l+1)^2 - a^2)) }  (0 at l = 0 or a > l)
//   cl[l] = sqrt((2l+1)/(4 pi))
//
// and the contraction's workgroup order: for each mode (inverse, forward) and
// tile width class (TJ = 64: FP64, TJ = 128: FP32 / BF16x3), the
// (order group, j tile) pairs that have work, as (group << 8) | tile, sorted
// by the length of their K loop, longest first (nsched entries each).
// The tables the contraction streams row by row (jti, jtf and the spin
// factors wi, wf, wi32, wf32) are stored with kTabPad zero rows before row 0
// and after row L - 1: a tile's K loop may run up to two slabs past either end
// of [0, L), and the padding lets it load those rows unguarded.  The pointers
// point at row 0; the allocation starts kTabPad rows earlier.
constexpr int kTabPad = 32;

struct RecTables {
    double *ri = nullptr;
    double *rf = nullptr;
    double2 *fab = nullptr;
    double2 *jti = nullptr;  // [l][j]: (j r, sqrt(l^2 - j^2) r), r = ri[l][j] (l-recursion, j side)
    double2 *jtf = nullptr;  // [k][j]: (y, (j+k)(j-k+1) y), y = rf[k][j] (m'-recursion)
    double *cl = nullptr;
    int *sched[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    int nsched[2][2] = {{0, 0}, {0, 0}};
};

struct Plan {
    int device = 0, L = 0, prec = 0;
    FftTables<double> f64;
    FftTables<float> f32;
    RecTables rec;
};

// Per-(L, spin) spin factors of the contraction, sqrt((2l+1)/4pi) d^l_{m',-s}(pi/2),
// in the two layouts the K loops stream (FP64, and rounded to FP32 for the
// FP32 path):
//   wi[l*L + m'] (inverse, K = l),   wf[m'*L + l] (forward, K = m')
struct SpinPlan {
    int device = 0, L = 0, spin = 0;
    double *wi = nullptr, *wf = nullptr;
    float *wi32 = nullptr, *wf32 = nullptr;
    // optional cached tables of the full contraction factor M_m(m', l) at
    // [m][l][m'] (L^3 entries), FP64 and FP32 (the latter also feeds BF16x3)
    double *mtab64 = nullptr;
    float *mtab32 = nullptr;
    // captured graphs whose transforms stream a table ([0] FP32, [1] FP64):
    // the table is not freed while any of them exists
    int mtab_users[2] = {0, 0};
};

// -------------------------------------------------------- kernel launches ---
// plan.hip
hipError_t launch_edge_table(EdgeTable &E, hipStream_t st);
hipError_t launch_spin_tables(const EdgeTable &E, const RecTables &rt, SpinPlan &sp, hipStream_t st);
hipError_t launch_rec_tables(int L, RecTables &rt, hipStream_t st);
template <typename T> hipError_t launch_fft_tables(FftTables<T> &ft, FftTables<double> *src, hipStream_t st);

// Workgroups are dealt to the 8 XCDs round-robin; this maps workgroup i to
// the work item it takes so that each XCD runs one contiguous range of items
// in order (the tail n mod 8 keeps its own index).  Neighbouring items share
// cache lines (the strided rows the theta stages read or write, the rows of
// unaligned coefficient blocks in the layout stages), and then meet in one
// L2.
__device__ __forceinline__ int xcd_item(int i, int n) {
    const int per = n >> 3;
    return i < (per << 3) ? (i & 7) * per + (i >> 3) : i;
}

// The spin segments of one call, as the layout and theta kernels see them:
// segment k holds the caller's maps [b0, b0 + B) of spin s (their rings and
// coefficient arrays follow those of the segments before), and those maps
// own the panel columns coff + q*B + (b - b0) of Cn.  flip: the segment's
// maps are contracted with the factors of spin -s (the layout stages then
// apply (-1)^l, the theta stages (-1)^{m'}; Eq. (wignerd_sym6)).
struct SpinSeg {
    int s, B, b0, coff, flip;
};
struct SpinSegs {
    int n, batch;
    SpinSeg seg[SHT_MULTI_SEG_MAX];
};
// The segment holding map bg (uniform over a workgroup).
__device__ __forceinline__ SpinSeg find_seg(const SpinSegs &sg, int bg) {
    int k = 0;
    while (k + 1 < sg.n && bg >= sg.seg[k + 1].b0) ++k;
    return sg.seg[k];
}

// layout.hip: one launch over every map of a call.  half: real spin-0
// signals, orders m >= 0 only (2 columns per map)
template <typename T>
hipError_t launch_layout_in(int L, const SpinSegs &sg, int Cn, bool half, const void *flm, T *P, hipStream_t st);
template <typename T>
hipError_t launch_layout_out(int L, const SpinSegs &sg, int Cn, bool half, const T *R, void *flm, hipStream_t st);

// {}_{-s}f_{lm} = (-1)^{s+m} conj({}_s f_{l,-m}) for spin pairs f_{-s} = conj(f_s)
template <typename T>
hipError_t launch_spin_pair(int L, int s, int B, const void *in, void *out, hipStream_t st);

// fft.hip: row transforms.  scr: split-row scratch of split_scratch_bytes(ft)
// bytes (unused, may be NULL, when that is 0)
template <typename T> size_t split_scratch_bytes(const FftTables<T> &ft);
// The theta stages of every map of a call (one launch); G / Q point at the
// first map's rings.
template <typename T>
hipError_t launch_theta_inv(const FftTables<T> &ft, const SpinSegs &sg, int Cn, bool half, const T *R, void *G,
                            void *scr, hipStream_t st);
// rs: row stride of the rings G / Q (ring_len(L, false), or N for the
// triangular forward's rows)
template <typename T>
hipError_t launch_phi_inv(const FftTables<T> &ft, int B, int rs, const void *G, void *map, void *scr,
                          hipStream_t st);
template <typename T>
hipError_t launch_phi_fwd(const FftTables<T> &ft, int B, int rs, const void *map, void *Q, void *scr,
                          hipStream_t st);
template <typename T>
hipError_t launch_theta_fwd(const FftTables<T> &ft, const SpinSegs &sg, int Cn, bool half, const void *Q, T *X,
                            void *scr, hipStream_t st);
// real maps (spin 0): phi synthesis from orders m >= 0, phi analysis keeping m >= 0
template <typename T>
hipError_t launch_phi_inv_real(const FftTables<T> &ft, int B, const void *G, T *map, void *scr, hipStream_t st);
template <typename T>
hipError_t launch_phi_fwd_real(const FftTables<T> &ft, int B, const T *map, void *Q, void *scr, hipStream_t st);
// theta DFT of the extended rows alone, F[b][mu][m'] for m' in [0, L)
template <typename T>
hipError_t launch_theta_dft(const FftTables<T> &ft, int s, int B, const void *Q, void *F, hipStream_t st);
// out[b][c][r] = in[b][r][c] for complex T
template <typename T>
hipError_t launch_transpose(int B, int rows, int cols, const void *in, void *out, hipStream_t st);
// raises the dynamic-LDS limit of every row kernel at the plan's FFT size
// once (plan building), so that later launches set no attributes
template <typename T> hipError_t prepare_row_kernels(const FftTables<T> &ft);
// forward FFT (natural order) of one sequence per block, in place (plan building)
template <typename T>
hipError_t launch_fft_inplace(const FftTables<T> &ft, typename CT<T>::type *buf, int rows,
                                  double scale, hipStream_t st);

// contract.hip
enum ContractMode { kInverse = 0, kForward = 1 };
// One launch contracts the columns of several spins at one L: segment k owns
// the next ncol columns and contracts them with its spin's factors.  Columns:
// 4 per map for complex signals (Re, Im of f_{l,m} and of (-1)^l f_{l,-m}),
// 2 per map for real spin-0 signals (m >= 0 only).
struct ContractSeg {
    int ncol;
    const SpinPlan *sp;
};
template <typename T>
hipError_t launch_contract(int mode, int L, int nseg, const ContractSeg *seg, const T *X, T *Y, const EdgeTable &E,
                           const RecTables &rt, hipStream_t st);
hipError_t launch_mtable(int L, int precision_fp64, const EdgeTable &E, const RecTables &rt, SpinPlan &sp,
                         hipStream_t st);
// fills rt.sched / rt.nsched for L (host sort, synchronous copy); 0 on success
int build_contract_schedules(int L, RecTables &rt);

// metrics.hip: error metrics of g against f (n complex entries, complex double
// if fp64 else complex float) into out[0..4] (device), asynchronous on st
size_t error_workspace_bytes();
hipError_t launch_error_metrics(bool fp64, const void *f, const void *g, size_t n, double *out, void *ws,
                                hipStream_t st);
// Column tile of the contraction (16, 32 or 64 columns per workgroup) for
// (current device, L, columns C, precision class): set_contract_tile pins it
// (0 restores the default cost model).
int contract_precision_class(bool fp64, bool bf16x3);
void set_contract_tile(int L, int C, int pclass, int ctile);
int get_contract_tile(int L, int C, int pclass);

hipError_t launch_contract_bf16x3(int mode, int L, int nseg, const ContractSeg *seg, const float *X, float *Y,
                                  const EdgeTable &E, const RecTables &rt, hipStream_t st);

// tri.hip: the paper's per-order triangular systems (FP64, L <= SHT_TRI_L_MAX)
hipError_t launch_tri_solve(int L, int s, int B, const void *F, void *flm, const EdgeTable &E,
                            const SpinPlan &sp, const RecTables &rt, hipStream_t st);
// ... and the least-squares solution of all their rows (the stable comparison)
hipError_t launch_tri_lstsq(int L, int s, int B, const void *F, void *flm, const EdgeTable &E,
                            const SpinPlan &sp, const RecTables &rt, hipStream_t st);

// ------------------------------------------------------------- helpers -----
inline int next_pow2(int x) { int p = 1; while (p < x) p <<= 1; return p; }
inline int ilog2(int x) { int r = 0; while ((1 << r) < x) ++r; return r; }

// Stockham pass structure of an M = 2^logM point FFT: pass 0 has radix
// 2^(logM mod 4) when that is non-zero, every other pass radix 16.  Pass p
// (p >= 1) keeps its twiddles w^{r k}, k < Ns_p, r < R_p, at
// ptw[fft_pass_offset(logM, p) + r Ns_p + k] (consecutive k adjacent: the
// threads of a wave, which hold consecutive k, read one contiguous run).
__host__ __device__ constexpr int fft_pass_lr(int logM, int p) { return (p == 0 && (logM & 3)) ? (logM & 3) : 4; }
__host__ __device__ constexpr int fft_npass(int logM) { return (logM + 3) / 4; }
__host__ __device__ constexpr int fft_pass_logns(int logM, int p) {
    int s = 0;
    for (int q = 0; q < p; ++q) s += fft_pass_lr(logM, q);
    return s;
}
__host__ __device__ constexpr int fft_pass_offset(int logM, int p) {
    int o = 0;
    for (int q = 1; q < p; ++q) o += 1 << (fft_pass_logns(logM, q) + fft_pass_lr(logM, q));
    return o;
}

}  // namespace sht
