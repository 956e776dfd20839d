// gfx950 FP64 particle loader: drifting Maxwell-Juttner momenta by the method
// of Melzani et al., "Apar-T" (arXiv:1308.5892), Sect. 4.3 and App. D, with
// co-located pairs (Sect. 2.1) and the relativistic Harris sheet (App. C).
//
// The p_y marginal (App. D, eq. distr_y) is tabulated as an inverse CDF in
// FP64 on the device: Gauss-Legendre integrals over a fine grid, a block scan,
// and a safeguarded Newton solve for each quantile.  Each pair then draws its
// position and two momenta from a counter-based Philox4x64-10 stream.
#include <hip/hip_runtime.h>

#include "pic_internal.h"

namespace pic {

// ------------------------------------------------------------ Philox4x64-10

// Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3"
// (SC'11): ten rounds; each multiplies counter words 0 and 2 by fixed odd
// constants, swaps halves and xors in words 1 and 3 and the round key; the key
// advances by two Weyl increments between rounds.
__device__ inline void philox4x64_10(uint64_t ctr[4], uint64_t k0, uint64_t k1)
{
    constexpr uint64_t kMulA = 0xD2E7470EE14C6C93ull, kMulB = 0xCA5A826395121157ull;
    constexpr uint64_t kWeylA = 0x9E3779B97F4A7C15ull, kWeylB = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t hA = __umul64hi(kMulA, ctr[0]), lA = kMulA * ctr[0];
        const uint64_t hB = __umul64hi(kMulB, ctr[2]), lB = kMulB * ctr[2];
        const uint64_t w0 = hB ^ ctr[1] ^ k0, w2 = hA ^ ctr[3] ^ k1;
        ctr[0] = w0; ctr[1] = lB; ctr[2] = w2; ctr[3] = lA;
        k0 += kWeylA;
        k1 += kWeylB;
    }
}

__device__ inline double unit53(uint64_t w) { return (double)(w >> 11) * (1.0 / 9007199254740992.0); }

// ------------------------------------------------- p_y marginal and its table

struct MJShape {
    double mu, G, beta0;   // 1/theta, Gamma0, beta0
};

// App. D, eq. distr_y without its constant factor, scaled by exp(mu) so that it
// is O(1) at the drift momentum y = Gamma0 beta0.
__device__ inline double py_density(double y, const MJShape &m)
{
    const double gy = sqrt(1.0 + y * y);
    return (1.0 + m.mu * m.G * gy) * exp(m.mu - m.mu * m.G * (gy - m.beta0 * y));
}

// five-point Gauss-Legendre integral of the density over [a, b]
__device__ inline double py_integral(double a, double b, const MJShape &m)
{
    const double x1 = 0.5384693101056831, x2 = 0.9061798459386640;
    const double w0 = 0.5688888888888889, w1 = 0.4786286704993665, w2 = 0.2369268850561891;
    const double c = 0.5 * (a + b), h = 0.5 * (b - a);
    return h * (w0 * py_density(c, m) + w1 * (py_density(c - h * x1, m) + py_density(c + h * x1, m)) +
                w2 * (py_density(c - h * x2, m) + py_density(c + h * x2, m)));
}

__global__ void mj_intervals_kernel(MJShape m, double ylo, double h, int M, double *cum)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < M) cum[i + 1] = py_integral(ylo + i * h, ylo + (i + 1) * h, m);
}

// In-place inclusive prefix sum of cum[1..M] (cum[0] = 0), one block of 1024
// threads: per-thread compensated serial sums over contiguous chunks, then a
// scan of the chunk totals.
__global__ void __launch_bounds__(1024) mj_scan_kernel(double *cum, int M)
{
    __shared__ double tot[1024];
    const int t = threadIdx.x;
    const int per = (M + 1023) / 1024;
    const int i0 = 1 + t * per, i1 = min(M + 1, i0 + per);
    double s = 0.0, comp = 0.0;
    for (int i = i0; i < i1; ++i) {
        const double y = cum[i] - comp;
        const double z = s + y;
        comp = (z - s) - y;
        s = z;
        cum[i] = s;          // local running sum
    }
    tot[t] = s;
    __syncthreads();
    if (t == 0) {
        double run = 0.0, c2 = 0.0;
        for (int q = 0; q < 1024; ++q) {   // exclusive offsets, compensated
            const double v = tot[q];
            tot[q] = run;
            const double y = v - c2;
            const double z = run + y;
            c2 = (z - run) - y;
            run = z;
        }
    }
    __syncthreads();
    const double base = tot[t];
    for (int i = i0; i < i1; ++i) cum[i] += base;
    if (t == 0) cum[0] = 0.0;
}

// tab[i] = J^{-1}(i/N) for 0 < i < N (App. D), tab[0] = ylo, tab[N] = yhi.
__global__ void mj_invert_kernel(MJShape m, double ylo, double yhi, double h, int M, const double *cum, int N,
                                 double *tab)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > N) return;
    if (i == 0) { tab[0] = ylo; return; }
    if (i == N) { tab[N] = yhi; return; }
    const double target = cum[M] * ((double)i / (double)N);
    int lo = 0, hi = M;                     // cum[lo] <= target < cum[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (cum[mid] <= target) lo = mid; else hi = mid;
    }
    const double a = ylo + lo * h;
    double left = a, right = a + h;
    const double rem = target - cum[lo];
    const double piece = cum[lo + 1] - cum[lo];
    double y = a + h * (piece > 0.0 ? rem / piece : 0.5);
    for (int it = 0; it < 80; ++it) {
        const double F = py_integral(a, y, m) - rem;
        if (F > 0.0) right = y; else left = y;
        const double f = py_density(y, m);
        double yn = f > 0.0 ? y - F / f : 0.5 * (left + right);
        if (!(yn > left && yn < right)) yn = 0.5 * (left + right);
        const bool done = fabs(yn - y) <= 1e-15 * (fabs(y) + 1e-3);
        y = yn;
        if (done) break;
    }
    tab[i] = y;
}

// ------------------------------------------------------------- pair loading

// u from (quantile t, radial w in (0,1], azimuth v): p_y from the table by
// linear interpolation; r from l(x) = w l(a) (App. D, eq. finding_u), solved
// by Newton on the logarithm in d = x - a >= 0 from d = 0; azimuth uniform;
// then the drift axis y is carried onto `axis` by a cyclic relabelling.
__device__ inline void mj_momentum(const MJPop &P, int N, double t, double w, double v, double out[3])
{
    const double f = t * N;
    int i = (int)f;
    if (i > N - 1) i = N - 1;
    const double py = P.tab[i] + (f - i) * (P.tab[i + 1] - P.tab[i]);
    const double gy = sqrt(1.0 + py * py);
    const double a = P.mu * P.G * gy;
    const double lw = log(w);
    double dx = 0.0;
    for (int it = 0; it < 60; ++it) {
        const double gval = log1p(dx / (1.0 + a)) - dx - lw;        // decreasing in dx
        const double slope = (a + dx) / (1.0 + a + dx);              // -d(gval)/d(dx)
        const double step = gval / slope;
        dx = fmax(dx + step, 0.0);
        if (it >= 3 && fabs(step) <= 1e-15 * (dx + 1e-300)) break;
    }
    const double um1 = dx / a;
    const double r = sqrt(um1 * (2.0 + um1));
    double sn, cs;
    sincos(6.283185307179586 * v, &sn, &cs);
    const double q[3] = {gy * r * cs, py, gy * r * sn};
    const int sh = (P.axis + 2) % 3;          // component 1 -> axis
    for (int c = 0; c < 3; ++c) out[(c + sh) % 3] = q[c];
}

template <typename R>
__device__ inline void to_storage(const BoxDev<R> &B, const double x[3], int32_t &cell, R d[3])
{
    int c[3];
    for (int a = 0; a < 3; ++a) {
        double s = fmod(x[a], (double)B.n[a]);
        if (s < 0.0) s += B.n[a];
        if (s >= B.n[a]) s -= B.n[a];
        double f = floor(s);
        R off = (R)(s - f);
        int ci = (int)f;
        if (off >= R(1)) {           // rounding reached the next cell
            off = R(0);
            ci += 1;
        }
        if (ci >= B.n[a]) ci -= B.n[a];
        c[a] = ci;
        d[a] = off;
    }
    cell = pack_cell(c[0], c[1], c[2]);
}

template <typename R>
__global__ void __launch_bounds__(256) load_pairs_kernel(const BoxDev<R> *__restrict__ boxes, LoadArgs L)
{
    const BoxDev<R> &B = boxes[L.box];
    const SpeciesDev<R> &SA = B.sp[L.sa];
    const SpeciesDev<R> &SB = B.sp[L.sb];
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < L.npairs;
         p += (int64_t)gridDim.x * blockDim.x) {
        uint64_t w[3][4];
        for (int j = 0; j < 3; ++j) {
            w[j][0] = (uint64_t)p; w[j][1] = (uint64_t)j; w[j][2] = 0; w[j][3] = 0;
            philox4x64_10(w[j], L.seed, L.stream);
        }
        // word map: (0,0..2) position, (0,3) A quantile, (1,0) A radial,
        // (1,1) A azimuth, (1,2) B quantile, (1,3) B radial, (2,0) B azimuth
        double x[3];
        for (int a = 0; a < 3; ++a) {
            const double U = unit53(w[0][a]);
            if (L.profile == PIC_PROFILE_HARRIS && a == L.paxis)
                x[a] = L.centre + L.thick * atanh((2.0 * U - 1.0) * tanh(L.halfw / L.thick));
            else
                x[a] = U * B.n[a];
        }
        double ua[3], ub[3];
        mj_momentum(L.A, L.N, unit53(w[0][3]), 1.0 - unit53(w[1][0]), unit53(w[1][1]), ua);
        mj_momentum(L.B, L.N, unit53(w[1][2]), 1.0 - unit53(w[1][3]), unit53(w[2][0]), ub);
        int32_t cell;
        R d[3];
        to_storage(B, x, cell, d);
        const int ia = L.offa + (int)p, ib = L.offb + (int)p;
        SA.stage.cell[ia] = cell;
        SB.stage.cell[ib] = cell;
        for (int a = 0; a < 3; ++a) {
            SA.stage.d[a][ia] = d[a];
            SB.stage.d[a][ib] = d[a];
            SA.stage.u[a][ia] = (R)ua[a];
            SB.stage.u[a][ib] = (R)ub[a];
        }
        if (SA.stage.id) SA.stage.id[ia] = L.ida + (int32_t)p;
        if (SB.stage.id) SB.stage.id[ib] = L.idb + (int32_t)p;
    }
}

// Harris-sheet b component at its staggered position (App. C,
// eq. B_field_Harris), one or two sheets.
template <typename R>
__global__ void __launch_bounds__(256) harris_field_kernel(const BoxDev<R> *__restrict__ boxes,
                                                           pic_harris_field H)
{
    const BoxDev<R> &B = boxes[H.box];
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= B.nc) return;
    const int n0 = B.n[0], n1 = B.n[1];
    const int idx[3] = {(int)(p % n0), (int)((p / n0) % n1), (int)(p / ((int64_t)n0 * n1))};
    // b_c sits half a cell off the node along the two axes other than c
    const double s = idx[H.grad_axis] + (H.grad_axis != H.field_axis ? 0.5 : 0.0);
    double v = tanh((s - H.centre[0]) / H.thickness);
    if (H.n_sheets == 2) v = v - tanh((s - H.centre[1]) / H.thickness) - 1.0;
    B.b[H.field_axis * B.nc + p] = (R)(H.b0 * v);
}

// ----------------------------------------------------------- host launchers

hipError_t launch_mj_table(double theta, double gamma_beta, double *cum, int M, int N, double *tab,
                           hipStream_t st)
{
    MJShape m;
    m.mu = 1.0 / theta;
    m.G = sqrt(1.0 + gamma_beta * gamma_beta);
    m.beta0 = gamma_beta / m.G;
    // support: where the exponent is 70 below its peak, gy - beta0 y = H
    const double H = 1.0 / m.G + 70.0 / (m.mu * m.G);
    const double rt = sqrt(H * H - 1.0 / (m.G * m.G));
    const double ylo = m.G * m.G * (H * m.beta0 - rt), yhi = m.G * m.G * (H * m.beta0 + rt);
    const double h = (yhi - ylo) / M;
    hipLaunchKernelGGL(mj_intervals_kernel, dim3((M + 255) / 256), dim3(256), 0, st, m, ylo, h, M, cum);
    hipLaunchKernelGGL(mj_scan_kernel, dim3(1), dim3(1024), 0, st, cum, M);
    hipLaunchKernelGGL(mj_invert_kernel, dim3((N + 1 + 255) / 256), dim3(256), 0, st, m, ylo, yhi, h, M, cum, N, tab);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_load_pairs(const BoxDev<R> *boxes, const LoadArgs &L, hipStream_t st)
{
    int64_t blocks = (L.npairs + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(load_pairs_kernel<R>, dim3((unsigned)blocks), dim3(256), 0, st, boxes, L);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_harris_field(const BoxDev<R> *boxes, int64_t nc, const pic_harris_field &H, hipStream_t st)
{
    hipLaunchKernelGGL(harris_field_kernel<R>, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, boxes, H);
    return hipGetLastError();
}

template hipError_t launch_load_pairs<float>(const BoxDev<float> *, const LoadArgs &, hipStream_t);
template hipError_t launch_load_pairs<double>(const BoxDev<double> *, const LoadArgs &, hipStream_t);
template hipError_t launch_harris_field<float>(const BoxDev<float> *, int64_t, const pic_harris_field &, hipStream_t);
template hipError_t launch_harris_field<double>(const BoxDev<double> *, int64_t, const pic_harris_field &, hipStream_t);

} // namespace pic
