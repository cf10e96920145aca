// Plan kernels: Wigner edge seeds, spin-chain states, torus FFT tables.
//
// Everything here runs once per (device), (device, L, precision) or
// (device, L, spin) and is cached by the host library.
#include "chain.h"

namespace sht {

// ----------------------------------------------------------- edge table ---
// E(l, k) = 2^-l sqrt(C(2l, l+k)) for 0 <= k <= l.  Its square is built as a
// product of factors below one,
//   4^-l C(2l, l)       = prod_{j=1..l} (2j-1)/(2j),
//   C(2l,l+k+1)/C(2l,l+k) = (l-k)/(l+k+1),
// with the binary exponent carried separately (E(l,l) = 2^-l underflows
// double precision for l > 1074).  One thread per degree l.
__global__ void k_edge_table(double *mant, int *expo, int lmax) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= lmax) return;
    double m = 1.0;
    int e = 0;
    for (int j = 1; j <= l; ++j) {
        m *= (double)(2 * j - 1) / (double)(2 * j);
        if (m < 0x1p-500) { m *= 0x1p500; e -= 500; }
    }
    const long long base = (long long)l * (l + 1) / 2;
    for (int k = 0; k <= l; ++k) {
        // sqrt(m 2^e) as mantissa in [1, 2) and exponent
        double mm = m;
        int ee = e;
        if (ee & 1) { mm *= 2.0; ee -= 1; }
        double r = sqrt(mm);
        int e2;
        double fr = frexp(r, &e2);  // r = fr 2^e2, fr in [0.5, 1)
        mant[base + k] = fr * 2.0;
        expo[base + k] = ee / 2 + e2 - 1;
        if (k < l) {
            m *= (double)(l - k) / (double)(l + k + 1);
            if (m < 0x1p-500) { m *= 0x1p500; e -= 500; }
        }
    }
}

hipError_t launch_edge_table(EdgeTable &E, hipStream_t st) {
    const int threads = 64;
    hipLaunchKernelGGL(k_edge_table, dim3((E.lmax + threads - 1) / threads), dim3(threads), 0, st,
                       E.mant, E.expo, E.lmax);
    return hipGetLastError();
}

// ------------------------------------------------------- spin tables -----
// For each m' in [0, L): the chain d^l_{m', sigma}(pi/2), sigma = -s, run in l
// from its edge l0 = max(m', |sigma|) with the l-recursion, written as
// wi[l][m'] = cl[l] d^l_{m',sigma}.  Values below the double
// range (scale level >= 1) are stored as their unscaled product, i.e. 0 or a
// subnormal: they multiply Wigner values <= 1 and vanish in the sums.
__global__ void k_spin_inverse(EdgeTable E, const double *ri, const double *cl, double *wi, int L, int sigma) {
    const int mp = blockIdx.x * blockDim.x + threadIdx.x;
    if (mp >= L) return;
    const int asg = sigma < 0 ? -sigma : sigma;
    const int l0 = mp > asg ? mp : asg;
    Chain c;
    c.zero();
    double q = 0.0;  // sqrt(l^2 - m'^2) at the current l
    for (int l = 0; l < L; ++l) {
        if (l == l0) c.inject(edge_seed(E, mp, sigma));
        const size_t idx = (size_t)l * L + mp;
        wi[idx] = cl[l] * c.value();
        // transition l -> l+1
        const double X = (double)(l + 1) * (l + 1) - (double)mp * mp;
        const double r = ri[idx];
        const double ap = (double)mp * r, bp = q * r;
        q = X > 0.0 ? X * r : 0.0;
        double am, bm;
        lrec_factor_full(l, sigma, am, bm);
        const double dn = -(ap * am * c.d + bp * bm * c.dp);
        if (l >= l0) c.push(dn);
    }
}

// wf[m'][l] = wi[l][m'], and both rounded to FP32
__global__ void k_spin_forward(const double *wi, double *wf, float *wi32, float *wf32, int L) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)L * L) return;
    const int k = (int)(idx / L), l = (int)(idx % L);
    const double w = wi[(size_t)l * L + k];
    wf[idx] = w;
    wf32[idx] = (float)w;
    wi32[idx] = (float)wi[idx];
}

hipError_t launch_spin_tables(const EdgeTable &E, const RecTables &rt, SpinPlan &sp, hipStream_t st) {
    const int threads = 64;
    hipLaunchKernelGGL(k_spin_inverse, dim3((sp.L + threads - 1) / threads), dim3(threads), 0, st, E, rt.ri,
                       rt.cl, sp.wi, sp.L, -sp.spin);
    const size_t n = (size_t)sp.L * sp.L;
    hipLaunchKernelGGL(k_spin_forward, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, sp.wi, sp.wf, sp.wi32,
                       sp.wf32, sp.L);
    return hipGetLastError();
}

// ------------------------------------------------ recursion factors ------
// The arguments are exact integers in double precision; the reciprocal square
// roots are taken once per L here instead of once per chain step.
__global__ void k_rec_tables(int L, double *ri, double *rf, double2 *fab, double *cl, double2 *jti, double2 *jtf) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)L * L) return;
    const int a = (int)(idx / L), b = (int)(idx % L);
    {   // fab[a][l], l = b
        double am = 0.0, bm = 0.0;
        if (b >= 1 && a <= b) lrec_factor_full(b, a, am, bm);
        fab[idx] = make_double2(am, bm);
        if (a == 0) cl[b] = sqrt((2.0 * b + 1.0) / (4.0 * 3.14159265358979323846));
    }
    {   // ri[l][j], l = a, j = b, and the j-side factors of the l-recursion
        // step l -> l+1: ap = j r, bp = sqrt(l^2 - j^2) r
        const double X = (double)(a + 1) * (a + 1) - (double)b * b;
        const double r = (b <= a) ? 1.0 / sqrt(X) : 0.0;
        ri[idx] = r;
        const double Y = (double)a * a - (double)b * b;
        const double q = (b < a) ? Y * (1.0 / sqrt(Y)) : 0.0;
        jti[idx] = make_double2((double)b * r, q * r);
    }
    {   // rf[k][l], k = a, l = b, and the factors of the m'-recursion step
        // m' = k -> k-1: y = rf[k][l], g = (l+k)(l-k+1) y
        const double X = (double)(b + a) * (double)(b - a + 1);
        const double y = (a <= b && X > 0.0) ? 1.0 / sqrt(X) : 0.0;
        rf[idx] = y;
        jtf[idx] = make_double2(y, X * y);
    }
}

hipError_t launch_rec_tables(int L, RecTables &rt, hipStream_t st) {
    const size_t n = (size_t)L * L;
    const int th = 256;
    hipLaunchKernelGGL(k_rec_tables, dim3((unsigned)((n + th - 1) / th)), dim3(th), 0, st, L, rt.ri, rt.rf,
                       rt.fab, rt.cl, rt.jti, rt.jtf);
    return hipGetLastError();
}

// ------------------------------------------------------- FFT tables ------
// Angles are pi * (integer) / N or 2 pi * (integer) / M with the integer
// reduced exactly first, then evaluated with sincospi in double precision.
__global__ void k_fill_tw(cplx64 *tw, int M) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    double s, c;
    sincospi(-2.0 * (double)k / (double)M, &s, &c);
    tw[k] = cplx64{c, s};
}

__global__ void k_fill_e2n(cplx64 *e, int N) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 2 * N) return;
    double s, c;
    sincospi((double)k / (double)N, &s, &c);
    e[k] = cplx64{c, s};
}

// Chirp-z kernel sequence c_j for j in [-(nin-1), kout-1], stored at j mod M.
//   type 0: e^{-i pi j^2 / N}      (inverse stages)
//   type 1: e^{+i pi j^2 / N}      (forward DFT stages)
//   type 2: K(j)                   (forward sin-theta quadrature, real)
//           K(p) = 2/(1-p^2) for even p, 0 for odd p
__global__ void k_fill_kernel_seq(cplx64 *c, int M, int N, int L, int nin, int kout, int type) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    // j such that j mod M == i, within the range
    long long j;
    if (i < kout) j = i;
    else if (i >= M - (nin - 1)) j = (long long)i - M;
    else { c[i] = cplx64{0.0, 0.0}; return; }
    if (type == 2) {
        const long long p = j;
        const double v = (p & 1) ? 0.0 : 2.0 / (1.0 - (double)p * (double)p);
        c[i] = cplx64{v, 0.0};
        return;
    }
    const long long twoN = 2LL * N;
    long long r = (j * j) % twoN;
    double s, cc;
    sincospi((double)r / (double)N, &s, &cc);
    c[i] = cplx64{cc, type == 0 ? -s : s};
}

// Stage chirps: cha[n] = e^{i pi (n^2+n)/N}, chb[n] = e^{i pi (n^2 - 2hn - h)/N}.
__global__ void k_fill_chirps(cplx64 *cha, cplx64 *chb, int N, int L) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const long long twoN = 2LL * N, h = L - 1;
    long long ra = ((long long)n * n + n) % twoN;
    long long rb = ((long long)n * n - 2 * h * n - h) % twoN;
    if (rb < 0) rb += twoN;
    double s, c;
    sincospi((double)ra / (double)N, &s, &c);
    cha[n] = cplx64{c, s};
    sincospi((double)rb / (double)N, &s, &c);
    chb[n] = cplx64{c, s};
}

// Twiddles of Stockham pass p: ptw[off + r Ns + k] = e^{-2 pi i r k / (Ns R)}.
__global__ void k_fill_pass_tw(cplx64 *ptw, int off, int logNs, int logR) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = 1 << (logNs + logR);
    if (i >= n) return;
    const int r = i >> logNs, k = i & ((1 << logNs) - 1);
    const long long num = ((long long)r * k) % n;
    double s, c;
    sincospi(-2.0 * (double)num / (double)n, &s, &c);
    ptw[off + i] = cplx64{c, s};
}

// Plain DFT of one length-M row per block row, out[k] = scale sum_n in[n]
// w^{nk} with w = e^{-2 pi i/M} taken from the plan's table at nk mod M: the
// spectra of plans whose M-point FFT does not fit in LDS (built once).
__global__ void k_dft_rows(const cplx64 *in, cplx64 *out, const cplx64 *tw, int M, double scale) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    const cplx64 *x = in + (size_t)blockIdx.y * M;
    double re = 0.0, im = 0.0;
    int idx = 0;  // n k mod M
    for (int n = 0; n < M; ++n) {
        const cplx64 a = x[n], w = tw[idx];
        re += a.x * w.x - a.y * w.y;
        im += a.x * w.y + a.y * w.x;
        idx += k;
        if (idx >= M) idx -= M;
    }
    out[(size_t)blockIdx.y * M + k] = cplx64{re * scale, im * scale};
}

template <typename T> __global__ void k_convert_table(typename CT<T>::type *dst, const cplx64 *src, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    dst[i].x = (T)src[i].x;
    dst[i].y = (T)src[i].y;
}

template <>
hipError_t launch_fft_tables<double>(FftTables<double> &ft, FftTables<double> *, hipStream_t st) {
    const int M = ft.M, N = ft.N, L = ft.L;
    const int th = 256;
    hipLaunchKernelGGL(k_fill_tw, dim3((M + th - 1) / th), dim3(th), 0, st, ft.tw, M);
    hipLaunchKernelGGL(k_fill_e2n, dim3((2 * N + th - 1) / th), dim3(th), 0, st, ft.e2n, N);
    hipLaunchKernelGGL(k_fill_chirps, dim3((N + th - 1) / th), dim3(th), 0, st, ft.cha, ft.chb, N, L);
    for (int p = 1; p < fft_npass(ft.logM); ++p) {
        const int lns = fft_pass_logns(ft.logM, p), lr = fft_pass_lr(ft.logM, p);
        const int n = 1 << (lns + lr);
        hipLaunchKernelGGL(k_fill_pass_tw, dim3((n + th - 1) / th), dim3(th), 0, st, ft.ptw,
                           fft_pass_offset(ft.logM, p), lns, lr);
    }
    hipLaunchKernelGGL(k_fill_kernel_seq, dim3((M + th - 1) / th), dim3(th), 0, st, ft.h_ip, M, N, L, N, N, 0);
    hipLaunchKernelGGL(k_fill_kernel_seq, dim3((M + th - 1) / th), dim3(th), 0, st, ft.h_fd, M, N, L, N, N, 1);
    hipLaunchKernelGGL(k_fill_kernel_seq, dim3((M + th - 1) / th), dim3(th), 0, st, ft.h_fk, M, N, L, N, N, 2);
    if (ft.ptwh) {
        // pass twiddles of the M/2-point halves of split rows
        const int lh = ft.logM - 1;
        for (int p = 1; p < fft_npass(lh); ++p) {
            const int lns = fft_pass_logns(lh, p), lr = fft_pass_lr(lh, p);
            const int n = 1 << (lns + lr);
            hipLaunchKernelGGL(k_fill_pass_tw, dim3((n + th - 1) / th), dim3(th), 0, st, ft.ptwh,
                               fft_pass_offset(lh, p), lns, lr);
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // spectra: forward DFT (natural order), scaled by 1/M (the inverse transform's normalisation)
    const double inv = 1.0 / (double)M;
    if (rows_split(M, (int)sizeof(cplx64))) {
        // the three kernel rows are contiguous (h_ip, h_fd, h_fk): transform
        // them out of a temporary copy
        cplx64 *tmp = nullptr;
        if ((e = hipMalloc((void **)&tmp, 3 * (size_t)M * sizeof(cplx64))) != hipSuccess) return e;
        e = hipMemcpyAsync(tmp, ft.h_ip, 3 * (size_t)M * sizeof(cplx64), hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_dft_rows, dim3((M + th - 1) / th, 3), dim3(th), 0, st, tmp, ft.h_ip, ft.tw, M,
                               inv);
            e = hipGetLastError();
        }
        const hipError_t es = hipStreamSynchronize(st);
        const hipError_t ef = hipFree(tmp);
        return e != hipSuccess ? e : (es != hipSuccess ? es : ef);
    }
    if ((e = launch_fft_inplace<double>(ft, ft.h_ip, 1, inv, st)) != hipSuccess) return e;
    if ((e = launch_fft_inplace<double>(ft, ft.h_fd, 1, inv, st)) != hipSuccess) return e;
    if ((e = launch_fft_inplace<double>(ft, ft.h_fk, 1, inv, st)) != hipSuccess) return e;
    return hipSuccess;
}

template <>
hipError_t launch_fft_tables<float>(FftTables<float> &ft, FftTables<double> *src, hipStream_t st) {
    const int th = 256;
    auto conv = [&](cplx32 *d, const cplx64 *s, int n) {
        if (n > 0) hipLaunchKernelGGL(k_convert_table<float>, dim3((n + th - 1) / th), dim3(th), 0, st, d, s, n);
    };
    conv(ft.tw, src->tw, ft.M);
    conv(ft.e2n, src->e2n, 2 * ft.N);
    conv(ft.cha, src->cha, ft.N);
    conv(ft.chb, src->chb, ft.N);
    conv(ft.ptw, src->ptw, fft_pass_offset(ft.logM, fft_npass(ft.logM)));
    conv(ft.h_ip, src->h_ip, ft.M);
    conv(ft.h_fd, src->h_fd, ft.M);
    conv(ft.h_fk, src->h_fk, ft.M);
    return hipGetLastError();
}

}  // namespace sht
