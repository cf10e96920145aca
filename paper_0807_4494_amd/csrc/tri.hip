// The paper's own forward transform: per-order triangular systems
// (Section 3.4.2, Eq. (matrix_fwd)), FP64.
//
// For one order m0 (spin s fixed) the lower half of Eq. (fourier_coeff) is
//
//   F_{m0 m'} = sum_{l >= m'} D[m', l] f_{l m0},   m' = 0 .. L-1,
//   D[m', l]  = (-1)^s i^{-(m0+s)} sqrt((2l+1)/4pi) Delta^l_{m' m0} Delta^l_{m',-s},
//
// upper triangular in (m', l).  Coefficients with l < l0 = max(|m0|, |s|) do
// not exist; the system is solved on the square block of rows and columns
// l0 .. L-1 by back substitution, from l = L-1 downwards.  The method is the
// paper's, including its instability beyond small L (Section 4.2); it is
// offered for L <= SHT_TRI_L_MAX.
//
// One workgroup per order (beyond L = kTriLdsMaxL a persistent workgroup
// takes orders in turn and keeps D in its own slot of global scratch: the
// L x L factor no longer fits in LDS).  Thread j (= m') runs the l-chain of
// Delta^l_{j |m0|} (chain.h, the same recursion and edge seeds as the
// contraction) and writes its row of the real factor of D into LDS, stored
// transposed, Dt[l][j], so that the column a back-substitution step needs is
// contiguous across threads.  The phase (-1)^s i^{-(m0+s)} is taken out of D
// and applied to the solution.  Maps are solved MB at a time with one
// accumulator per thread and map: at step l thread l forms
// x_l = acc_l / D[l][l], publishes it through LDS, and every thread j < l
// subtracts D[j][l] x_l from its own accumulator.  For spin 0 the system
// splits into the independent rows and columns of even and of odd l + m'
// (D vanishes elsewhere, Eq. (wignerd_sym6); Section 3.4.2): a step only
// updates the rows of its own parity class, so the two classes are solved
// as separate systems.
#include "chain.h"

namespace sht {

namespace {

constexpr int MB = 8;              // maps per pass
constexpr int kTriThreads = 512;   // one thread per row: L <= SHT_TRI_L_MAX
constexpr int kTriLdsMaxL = 128;   // D in LDS up to this L, in a global slot beyond
constexpr int kTriSlots = 256;     // persistent workgroups (global slots) beyond it

// Orders o = blockIdx.x, blockIdx.x + gridDim.x, ... (one per workgroup when
// the grid has one workgroup per order).
template <typename F> __device__ __forceinline__ void for_orders(int norders, F body) {
    for (int o = blockIdx.x; o < norders; o += gridDim.x) {
        body(o);
        __syncthreads();
    }
}

template <bool GLB>
__global__ __launch_bounds__(kTriThreads) void k_tri_solve(int L, int s, int B, const cplx64 *__restrict__ F,
                                                          cplx64 *__restrict__ flm, EdgeTable E,
                                                          const double *__restrict__ wi,
                                                          const double *__restrict__ ri,
                                                          const double2 *__restrict__ fab, double *gscr) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    // Dt [L][L]: LDS, or this workgroup's global slot
    double *Dt = GLB ? gscr + (size_t)blockIdx.x * L * L : reinterpret_cast<double *>(smem_raw);
    cplx64 *xs = GLB ? reinterpret_cast<cplx64 *>(smem_raw)
                     : reinterpret_cast<cplx64 *>(Dt + (size_t)L * L);  // [MB][L]
    const int N = 2 * L - 1, h = L - 1;
    for_orders(N, [&](int o) {
    const int m0 = o - h;
    const int am = m0 < 0 ? -m0 : m0;
    const int as = s < 0 ? -s : s;
    const int l0 = am > as ? am : as;
    const int j = threadIdx.x;

    // ---- rows of the real factor: Dt[l][j] = wi[l][j] Delta^l_{j m0}, l >= j ----
    if (j < L && j >= l0) {
        Chain c;
        c.inject(edge_seed(E, j, am));  // edge of the (j, |m0|) chain at l = max(j, |m0|) = j
        double q = 0.0;                 // sqrt(l^2 - j^2) at the current l (0 at l = j)
        for (int l = j; l < L; ++l) {
            double d = c.value();
            if (m0 < 0 && ((l + j) & 1)) d = -d;  // Delta^l_{j,-m} = (-1)^{l+j} Delta^l_{jm}
            Dt[(size_t)l * L + j] = wi[(size_t)l * L + j] * d;
            if (l + 1 < L) {
                const double r = ri[(size_t)l * L + j];
                const double ap = (double)j * r, bp = q * r;
                q = ((double)(l + 1) * (l + 1) - (double)j * j) * r;
                const double2 f = fab[(size_t)am * L + l];
                c.push(-(ap * f.x * c.d + bp * f.y * c.dp));
            }
        }
    }
    __syncthreads();

    // phase of D taken out: f = x (-1)^s i^{m0+s} with D_real x = F
    const int ph = ((m0 + s) % 4 + 4) % 4;
    const double sgn = (s & 1) ? -1.0 : 1.0;
    for (int b0 = 0; b0 < B; b0 += MB) {
        const int nb = B - b0 < MB ? B - b0 : MB;
        cplx64 acc[MB];
#pragma unroll
        for (int q = 0; q < MB; ++q) {
            acc[q] = cplx64{0.0, 0.0};
            if (q < nb && j < L) acc[q] = F[((size_t)(b0 + q) * N + (m0 + h)) * L + j];
        }
        for (int l = L - 1; l >= l0; --l) {
            if (j == l) {
                const double inv = 1.0 / Dt[(size_t)l * L + l];
#pragma unroll
                for (int q = 0; q < MB; ++q) xs[q * L + l] = cplx64{acc[q].x * inv, acc[q].y * inv};
            }
            __syncthreads();
            if (j >= l0 && j < l && (s != 0 || ((l - j) & 1) == 0)) {
                const double dj = Dt[(size_t)l * L + j];
#pragma unroll
                for (int q = 0; q < MB; ++q) {
                    const cplx64 x = xs[q * L + l];
                    acc[q].x -= dj * x.x;
                    acc[q].y -= dj * x.y;
                }
            }
        }
        __syncthreads();
        if (j < L) {
            for (int q = 0; q < nb; ++q) {
                cplx64 v{0.0, 0.0};
                if (j >= l0) {
                    const cplx64 x = xs[q * L + j];
                    switch (ph) {  // times i^{m0+s}
                        case 0: v = x; break;
                        case 1: v = cplx64{-x.y, x.x}; break;
                        case 2: v = cplx64{-x.x, -x.y}; break;
                        default: v = cplx64{x.y, -x.x}; break;
                    }
                    v = cplx64{v.x * sgn, v.y * sgn};
                }
                if (am <= j) flm[(size_t)(b0 + q) * L * L + (size_t)j * j + j + m0] = v;
            }
        }
        __syncthreads();
    }
    });
}

// The stable comparison: for one order, all rows m' = 0 .. L-1 of the same
// system (columns l0 .. L-1), solved in the least-squares sense.  The rows
// m' < l0 that the square block drops make these systems well conditioned.
// Solved by conjugate gradients on the normal equations (CGNR: x, the
// residual r = F - D x and z = D^T r), MBL maps (2 MBL real right-hand sides,
// since the real factor of D is real) at a time, until every z has fallen by
// kLsqTol relative to its start or after 2 L + 32 iterations.  D is stored
// transposed with rows padded to L + 1, Dt[l][j], so both products read it
// with at most 2-way bank conflicts:
//   w = D p:    thread j sums Dt[l][j] p_l over l >= max(j, l0)
//   z = D^T r:  thread l sums Dt[l][j] r_j over j <= l
// With D in global memory (beyond kTriLdsMaxL) the second product reads a
// row-major copy Dr[j][l] instead, so that both read consecutive addresses
// across the threads.
constexpr int MBL = 4;
constexpr int NV = 2 * MBL;
constexpr double kLsqTol = 1e-28;  // on |z|^2, i.e. 1e-14 on |z|

__device__ inline double wave_sum64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <bool GLB>
__global__ __launch_bounds__(kTriThreads) void k_tri_lstsq(int L, int s, int B, const cplx64 *__restrict__ F,
                                                          cplx64 *__restrict__ flm, EdgeTable E,
                                                          const double *__restrict__ wi,
                                                          const double *__restrict__ ri,
                                                          const double2 *__restrict__ fab, double *gscr) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int LP = L + 1;
    // Dt [L][L + 1] (and, in global memory, Dr [L][L]): LDS, or this workgroup's slot
    double *Dt = GLB ? gscr + (size_t)blockIdx.x * L * (LP + L) : reinterpret_cast<double *>(smem_raw);
    double *Dr = GLB ? Dt + (size_t)L * LP : nullptr;
    double *vs = GLB ? reinterpret_cast<double *>(smem_raw) : Dt + (size_t)L * LP;  // [NV][L]: p, then r
    double *red = vs + (size_t)NV * L;                  // [NV][waves] partial sums
    const int N = 2 * L - 1, h = L - 1;
    for_orders(N, [&](int o) {
    const int m0 = o - h;
    const int am = m0 < 0 ? -m0 : m0;
    const int as = s < 0 ? -s : s;
    const int l0 = am > as ? am : as;
    const int t = threadIdx.x, nw = (int)blockDim.x / 64, wave = t >> 6, lane = t & 63;

    // ---- the real factor of D at columns l >= l0, every row j ----
    for (int i = t; i < L * LP; i += blockDim.x) Dt[i] = 0.0;
    if constexpr (GLB) {
        for (int i = t; i < L * L; i += blockDim.x) Dr[i] = 0.0;
    }
    __syncthreads();
    if (t < L) {
        const int j = t;
        const int lc = j > am ? j : am;  // edge of the (j, |m0|) chain
        Chain c;
        c.inject(edge_seed(E, j, am));
        double q = 0.0;  // multiplies d^{l-1}, which is zero at the edge
        for (int l = lc; l < L; ++l) {
            if (l >= l0) {
                double d = c.value();
                if (m0 < 0 && ((l + j) & 1)) d = -d;  // Delta^l_{j,-m} = (-1)^{l+j} Delta^l_{jm}
                const double v = wi[(size_t)l * L + j] * d;
                Dt[(size_t)l * LP + j] = v;
                if constexpr (GLB) Dr[(size_t)j * L + l] = v;
            }
            if (l + 1 < L) {
                const double r = ri[(size_t)l * L + j];
                const double ap = (double)j * r, bp = q * r;
                q = ((double)(l + 1) * (l + 1) - (double)j * j) * r;
                const double2 f = fab[(size_t)am * L + l];
                c.push(-(ap * f.x * c.d + bp * f.y * c.dp));
            }
        }
    }
    __syncthreads();

    const bool row = t < L;                 // owns row j = t of the m-side vectors
    const bool col = t >= l0 && t < L;      // owns column l = t of the n-side vectors
    auto block_sums = [&](double (&v)[NV], double (&out)[NV]) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const double w = wave_sum64(v[k]);
            if (lane == 0) red[k * nw + wave] = w;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double a = 0.0;
            for (int i = 0; i < nw; ++i) a += red[k * nw + i];
            out[k] = a;
        }
        __syncthreads();
    };
    // z = D^T r for the r held by the row owners
    auto at_times = [&](const double (&r)[NV], double (&z)[NV]) {
        if (row) {
#pragma unroll
            for (int k = 0; k < NV; ++k) vs[k * L + t] = r[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NV; ++k) z[k] = 0.0;
        if (col) {
            for (int j = 0; j <= t; ++j) {
                const double d = GLB ? Dr[(size_t)j * L + t] : Dt[(size_t)t * LP + j];
#pragma unroll
                for (int k = 0; k < NV; ++k) z[k] += d * vs[k * L + j];
            }
        }
        __syncthreads();
    };
    // w = D p for the p held by the column owners
    auto a_times = [&](const double (&p)[NV], double (&w)[NV]) {
        if (t < L) {
#pragma unroll
            for (int k = 0; k < NV; ++k) vs[k * L + t] = col ? p[k] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NV; ++k) w[k] = 0.0;
        if (row) {
            for (int l = t > l0 ? t : l0; l < L; ++l) {
                const double d = Dt[(size_t)l * LP + t];
#pragma unroll
                for (int k = 0; k < NV; ++k) w[k] += d * vs[k * L + l];
            }
        }
        __syncthreads();
    };

    const int ph = ((m0 + s) % 4 + 4) % 4;
    const double sgn = (s & 1) ? -1.0 : 1.0;
    const int max_iter = 2 * L + 32;
    for (int b0 = 0; b0 < B; b0 += MBL) {
        double r[NV], x[NV], z[NV], p[NV], w[NV], zz[NV], zz0[NV], ww[NV], sq[NV];
#pragma unroll
        for (int q = 0; q < MBL; ++q) {
            cplx64 f{0.0, 0.0};
            if (row && b0 + q < B) f = F[((size_t)(b0 + q) * N + (m0 + h)) * L + t];
            r[2 * q] = f.x;
            r[2 * q + 1] = f.y;
        }
#pragma unroll
        for (int k = 0; k < NV; ++k) x[k] = 0.0;
        at_times(r, z);
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            p[k] = z[k];
            sq[k] = z[k] * z[k];
        }
        block_sums(sq, zz);
#pragma unroll
        for (int k = 0; k < NV; ++k) zz0[k] = zz[k];
        for (int it = 0; it < max_iter; ++it) {
            bool done = true;  // uniform: zz is a block sum
#pragma unroll
            for (int k = 0; k < NV; ++k) done = done && zz[k] <= kLsqTol * zz0[k];
            if (done) break;
            a_times(p, w);
#pragma unroll
            for (int k = 0; k < NV; ++k) sq[k] = w[k] * w[k];
            block_sums(sq, ww);
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                const double alpha = (zz[k] > 0.0 && ww[k] > 0.0) ? zz[k] / ww[k] : 0.0;
                x[k] += alpha * p[k];
                r[k] -= alpha * w[k];
            }
            at_times(r, z);
#pragma unroll
            for (int k = 0; k < NV; ++k) sq[k] = z[k] * z[k];
            double zn[NV];
            block_sums(sq, zn);
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                const double beta = zz[k] > 0.0 ? zn[k] / zz[k] : 0.0;
                p[k] = z[k] + beta * p[k];
                zz[k] = zn[k];
            }
        }
        // f_{l m0} = x (-1)^s i^{m0+s}
        if (t < L && am <= t) {
#pragma unroll
            for (int q = 0; q < MBL; ++q) {
                if (b0 + q >= B) continue;
                cplx64 v{0.0, 0.0};
                if (col) {
                    const cplx64 xv{x[2 * q], x[2 * q + 1]};
                    switch (ph) {
                        case 0: v = xv; break;
                        case 1: v = cplx64{-xv.y, xv.x}; break;
                        case 2: v = cplx64{-xv.x, -xv.y}; break;
                        default: v = cplx64{xv.y, -xv.x}; break;
                    }
                    v = cplx64{v.x * sgn, v.y * sgn};
                }
                flm[(size_t)(b0 + q) * L * L + (size_t)t * t + t + m0] = v;
            }
        }
    }
    });
}

}  // namespace

// Launch of one of the kernels above: one workgroup per order with D in LDS
// up to kTriLdsMaxL, else kTriSlots persistent workgroups with D in global
// slots allocated on the stream (stream-ordered, freed after the launch).
template <typename K>
hipError_t tri_launch(K klds, K kglb, int L, size_t lds_small, size_t lds_glb, size_t slot_doubles, int s, int B,
                      const void *F, void *flm, const EdgeTable &E, const SpinPlan &sp, const RecTables &rt,
                      hipStream_t st) {
    if (L > SHT_TRI_L_MAX) return hipErrorInvalidValue;
    const int threads = ((L + 63) / 64) * 64;
    const int norders = 2 * L - 1;
    if (L <= kTriLdsMaxL) {
        if (lds_small > 64 * 1024) {
            hipError_t e = hipFuncSetAttribute((const void *)klds, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)lds_small);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(klds, dim3(norders), dim3(threads), lds_small, st, L, s, B, (const cplx64 *)F,
                           (cplx64 *)flm, E, sp.wi, rt.ri, rt.fab, (double *)nullptr);
        return hipGetLastError();
    }
    const int grid = norders < kTriSlots ? norders : kTriSlots;
    double *scr = nullptr;
    hipError_t e = hipMallocAsync((void **)&scr, (size_t)grid * slot_doubles * sizeof(double), st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kglb, dim3(grid), dim3(threads), lds_glb, st, L, s, B, (const cplx64 *)F, (cplx64 *)flm, E,
                       sp.wi, rt.ri, rt.fab, scr);
    e = hipGetLastError();
    const hipError_t ef = hipFreeAsync(scr, st);
    return e != hipSuccess ? e : ef;
}

hipError_t launch_tri_lstsq(int L, int s, int B, const void *F, void *flm, const EdgeTable &E, const SpinPlan &sp,
                            const RecTables &rt, hipStream_t st) {
    const int nw = (L + 63) / 64;
    const size_t vecs = ((size_t)NV * L + (size_t)NV * nw) * sizeof(double);
    const size_t lds_small = (size_t)L * (L + 1) * sizeof(double) + vecs;
    return tri_launch(k_tri_lstsq<false>, k_tri_lstsq<true>, L, lds_small, vecs, (size_t)L * (2 * L + 1), s, B, F,
                      flm, E, sp, rt, st);
}

hipError_t launch_tri_solve(int L, int s, int B, const void *F, void *flm, const EdgeTable &E, const SpinPlan &sp,
                            const RecTables &rt, hipStream_t st) {
    const size_t xs = (size_t)MB * L * sizeof(cplx64);
    const size_t lds_small = (size_t)L * L * sizeof(double) + xs;
    return tri_launch(k_tri_solve<false>, k_tri_solve<true>, L, lds_small, xs, (size_t)L * L, s, B, F, flm, E, sp,
                      rt, st);
}

}  // namespace sht
