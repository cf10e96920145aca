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
// One workgroup per order.  Thread j (= m') runs the l-chain of
// Delta^l_{j |m0|} (chain.h, the same recursion and edge seeds as the
// contraction) and writes its row of the real factor of D into LDS, stored
// transposed, Dt[l][j], so that the column a back-substitution step needs is
// contiguous across threads.  The phase (-1)^s i^{-(m0+s)} is taken out of D
// and applied to the solution.  Maps are solved MB at a time with one
// accumulator per thread and map: at step l thread l forms
// x_l = acc_l / D[l][l], publishes it through LDS, and every thread j < l
// subtracts D[j][l] x_l from its own accumulator.
#include "chain.h"

namespace sht {

namespace {

constexpr int MB = 8;  // maps per pass

__global__ __launch_bounds__(SHT_TRI_L_MAX) void k_tri_solve(int L, int s, int B, const cplx64 *__restrict__ F,
                                                            cplx64 *__restrict__ flm, EdgeTable E,
                                                            const double *__restrict__ wi,
                                                            const double *__restrict__ ri,
                                                            const double2 *__restrict__ fab) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *Dt = reinterpret_cast<double *>(smem_raw);            // [L][L]
    cplx64 *xs = reinterpret_cast<cplx64 *>(Dt + (size_t)L * L);  // [MB][L]
    const int N = 2 * L - 1, h = L - 1;
    const int m0 = (int)blockIdx.x - h;
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
            if (j >= l0 && j < l) {
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
}

}  // namespace

hipError_t launch_tri_solve(int L, int s, int B, const void *F, void *flm, const EdgeTable &E, const SpinPlan &sp,
                            const RecTables &rt, hipStream_t st) {
    if (L > SHT_TRI_L_MAX) return hipErrorInvalidValue;
    const size_t lds = (size_t)L * L * sizeof(double) + (size_t)MB * L * sizeof(cplx64);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)k_tri_solve, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
    }
    const int threads = ((L + 63) / 64) * 64;
    hipLaunchKernelGGL(k_tri_solve, dim3(2 * L - 1), dim3(threads), lds, st, L, s, B, (const cplx64 *)F,
                       (cplx64 *)flm, E, sp.wi, rt.ri, rt.fab);
    return hipGetLastError();
}

}  // namespace sht
