// gfx950 kernels of the PIC hot path: fused gather + Boris push + deposit per
// spatial tile, Yee field updates, counting-sort repack and FP64 diagnostics.
//
// Paper: Melzani et al., "Apar-T" (arXiv:1308.5892), App. A.  The readings of
// the paper used here (cyclic node averaging, standard Boris rotation,
// splitting of cell-crossing moves at node planes) are stated where they are
// used.  Every kernel is templated on the storage/arithmetic type R: float is
// the production form (int64 fixed-point current), double the FP64 form.
#include <hip/hip_runtime.h>

#include "pic_internal.h"

namespace pic {

// ------------------------------------------------------------ arithmetic

__device__ inline float fast_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline double fast_rsqrt(double x) { return 1.0 / sqrt(x); }
__device__ inline float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double fast_rcp(double x) { return 1.0 / x; }

template <typename R> __device__ inline R qscale_bits();
template <> __device__ inline float qscale_bits<float>() { return 2147483648.0f; }  // 2^31
template <> __device__ inline double qscale_bits<double>() { return 1.0; }

__device__ inline long long quantize(float v) { return (long long)__float2int_rn(v); }
__device__ inline double quantize(double v) { return v; }

__device__ inline void atomic_add_lds(long long *p, long long v)
{
    atomicAdd(reinterpret_cast<unsigned long long *>(p), (unsigned long long)v);
}
__device__ inline void atomic_add_lds(double *p, double v) { atomicAdd(p, v); }
__device__ inline void atomic_add_global(long long *p, long long v)
{
    atomicAdd(reinterpret_cast<unsigned long long *>(p), (unsigned long long)v);
}
__device__ inline void atomic_add_global(double *p, double v) { atomicAdd(p, v); }

// Relativistic Boris step (App. A.3.3, eq. mover) with hk = k h / 2:
// half electric kick, rotation about b with t = hk B / gamma^t and
// s = 2 t / (1 + t^2) (READING: the printed rotation is garbled; this is the
// rotation that solves the implicit mover equation), half electric kick.
template <typename R>
__device__ inline void boris(R hk, const R E[3], const R Bf[3], R u[3])
{
    R um0 = u[0] + hk * E[0], um1 = u[1] + hk * E[1], um2 = u[2] + hk * E[2];
    R ig = fast_rsqrt(R(1) + um0 * um0 + um1 * um1 + um2 * um2);
    R f = hk * ig;
    R t0 = f * Bf[0], t1 = f * Bf[1], t2 = f * Bf[2];
    R sf = R(2) * fast_rcp(R(1) + t0 * t0 + t1 * t1 + t2 * t2);
    R s0 = sf * t0, s1 = sf * t1, s2 = sf * t2;
    R v0 = um0 + (um1 * t2 - um2 * t1);
    R v1 = um1 + (um2 * t0 - um0 * t2);
    R v2 = um2 + (um0 * t1 - um1 * t0);
    u[0] = um0 + (v1 * s2 - v2 * s1) + hk * E[0];
    u[1] = um1 + (v2 * s0 - v0 * s2) + hk * E[1];
    u[2] = um2 + (v0 * s1 - v1 * s0) + hk * E[2];
}

// Charge-conserving deposit of the straight move d -> d + D, in the frame of
// the start cell (d in [0,1)^3, |D| < 1).  The volume change of the particle
// cube in the eight grid-B cells is attributed per component as in App. A.3.4
// (eq. current_dep): dV_a = -D_a (W_b W_c + sigma D_b D_c / 12).  READING (the
// paper defers cell-crossing moves to references not given): the move is cut
// at each node plane it crosses, in order of the crossing parameter, and each
// piece is deposited in its own cell; breakpoints sit exactly on their plane.
// add(a, ox, oy, oz, v): value v for component a at node (start cell + o).
template <typename R, typename Add>
__device__ inline void deposit_move(const R d[3], const R D[3], R scale, Add &&add)
{
    R x1[3];
    int dir[3];
    R lam[3];
    for (int a = 0; a < 3; ++a) {
        x1[a] = d[a] + D[a];
        dir[a] = x1[a] < R(0) ? -1 : (x1[a] >= R(1) ? 1 : 0);
        lam[a] = dir[a] != 0 ? (R(dir[a] > 0) - d[a]) * fast_rcp(D[a]) : R(2);
    }
    // order the axes by crossing parameter (non-crossing axes last)
    int o0 = 0, o1 = 1, o2 = 2;
    if (lam[o1] < lam[o0]) { int t = o0; o0 = o1; o1 = t; }
    if (lam[o2] < lam[o1]) { int t = o1; o1 = o2; o2 = t; }
    if (lam[o1] < lam[o0]) { int t = o0; o0 = o1; o1 = t; }
    const int ord[3] = {o0, o1, o2};
    const int nb = (dir[0] != 0) + (dir[1] != 0) + (dir[2] != 0);
    R p[3] = {d[0], d[1], d[2]};
    int off[3] = {0, 0, 0};
    int crossed[3] = {0, 0, 0};
    for (int k = 0; k <= nb; ++k) {
        R q[3];
        if (k < nb) {
            const int ax = ord[k];
            const R l = lam[ax];
            for (int a = 0; a < 3; ++a) {
                if (a == ax) {
                    q[a] = R(dir[a] > 0);
                } else {
                    R v = d[a] + l * D[a];
                    if (dir[a] > 0) v = crossed[a] ? fmax(v, R(1)) : fmin(v, R(1));
                    else if (dir[a] < 0) v = crossed[a] ? fmin(v, R(0)) : fmax(v, R(0));
                    q[a] = v;
                }
            }
        } else {
            q[0] = x1[0]; q[1] = x1[1]; q[2] = x1[2];
        }
        R s[3], dd[3];
        for (int a = 0; a < 3; ++a) {
            s[a] = p[a] - R(off[a]);
            dd[a] = q[a] - p[a];
        }
        if (dd[0] != R(0) || dd[1] != R(0) || dd[2] != R(0)) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int b1 = a == 2 ? 0 : a + 1, b2 = a == 0 ? 2 : a - 1;
                const R m1 = s[b1] + R(0.5) * dd[b1], m2 = s[b2] + R(0.5) * dd[b2];
                const R w1[2] = {R(1) - m1, m1}, w2[2] = {R(1) - m2, m2};
                const R K = dd[b1] * dd[b2] * R(1.0 / 12.0);
                const R sa = scale * dd[a];
#pragma unroll
                for (int pp = 0; pp < 2; ++pp)
#pragma unroll
                    for (int qq = 0; qq < 2; ++qq) {
                        const R v = sa * (w1[pp] * w2[qq] + (pp == qq ? K : -K));
                        int o[3] = {off[0], off[1], off[2]};
                        o[b1] += pp;
                        o[b2] += qq;
                        add(a, o[0], o[1], o[2], v);
                    }
            }
        }
        if (k < nb) {
            off[ord[k]] = dir[ord[k]];
            crossed[ord[k]] = 1;
        }
        p[0] = q[0]; p[1] = q[1]; p[2] = q[2];
    }
}

// ------------------------------------------------------ global-memory reads

template <typename R>
__device__ inline R fld(const R *F, const BoxDev<R> &B, int c, int i, int j, int k)
{
    i = wrap_idx(i, B.n[0]);
    j = wrap_idx(j, B.n[1]);
    k = wrap_idx(k, B.n[2]);
    return F[c * B.nc + i + (int64_t)B.n[0] * (j + (int64_t)B.n[1] * k)];
}

// b^t = b^{t-dt/2} - (dt/2) curl e^t at the b_c position of cell (i,j,k)
template <typename R>
__device__ inline R bt_global(const BoxDev<R> &B, int c, int i, int j, int k, R hdt)
{
    const R *e = B.e;
    R curl;
    if (c == 0)
        curl = (fld(e, B, 2, i, j + 1, k) - fld(e, B, 2, i, j, k)) - (fld(e, B, 1, i, j, k + 1) - fld(e, B, 1, i, j, k));
    else if (c == 1)
        curl = (fld(e, B, 0, i, j, k + 1) - fld(e, B, 0, i, j, k)) - (fld(e, B, 2, i + 1, j, k) - fld(e, B, 2, i, j, k));
    else
        curl = (fld(e, B, 1, i + 1, j, k) - fld(e, B, 1, i, j, k)) - (fld(e, B, 0, i, j + 1, k) - fld(e, B, 0, i, j, k));
    return fld(B.b, B, c, i, j, k) - hdt * curl;
}

// Node-averaged fields (App. A.3.3; READING: e_c averaged over the two edges
// along c meeting at the node, b_c over the four faces normal to c) weighted
// trilinearly at (cell, d).  Slow path: everything read from HBM.
template <typename R>
__device__ inline void gather_global(const BoxDev<R> &B, int ix, int iy, int iz, const R d[3], R hdt,
                                     R E[3], R Bf[3])
{
    for (int a = 0; a < 3; ++a) { E[a] = R(0); Bf[a] = R(0); }
    for (int kk = 0; kk < 2; ++kk)
        for (int jj = 0; jj < 2; ++jj)
            for (int ii = 0; ii < 2; ++ii) {
                const int i = ix + ii, j = iy + jj, k = iz + kk;
                const R w = (ii ? d[0] : R(1) - d[0]) * (jj ? d[1] : R(1) - d[1]) * (kk ? d[2] : R(1) - d[2]);
                E[0] += w * R(0.5) * (fld(B.e, B, 0, i - 1, j, k) + fld(B.e, B, 0, i, j, k));
                E[1] += w * R(0.5) * (fld(B.e, B, 1, i, j - 1, k) + fld(B.e, B, 1, i, j, k));
                E[2] += w * R(0.5) * (fld(B.e, B, 2, i, j, k - 1) + fld(B.e, B, 2, i, j, k));
                Bf[0] += w * R(0.25) * (bt_global(B, 0, i, j, k, hdt) + bt_global(B, 0, i, j - 1, k, hdt) +
                                        bt_global(B, 0, i, j - 1, k - 1, hdt) + bt_global(B, 0, i, j, k - 1, hdt));
                Bf[1] += w * R(0.25) * (bt_global(B, 1, i, j, k, hdt) + bt_global(B, 1, i, j, k - 1, hdt) +
                                        bt_global(B, 1, i - 1, j, k - 1, hdt) + bt_global(B, 1, i - 1, j, k, hdt));
                Bf[2] += w * R(0.25) * (bt_global(B, 2, i, j, k, hdt) + bt_global(B, 2, i - 1, j, k, hdt) +
                                        bt_global(B, 2, i - 1, j - 1, k, hdt) + bt_global(B, 2, i, j - 1, k, hdt));
            }
}

// ------------------------------------------------------------ slot claims

__device__ inline uint64_t lanemask_lt() { return (1ull << __lane_id()) - 1ull; }

// Wave-aggregated claim of one slot per pending lane in the counter of its
// target segment: one atomic per distinct target in the wave.
__device__ inline int claim_slot(int32_t *cnt, int target, bool pending)
{
    int slot = -1;
    uint64_t m;
    while ((m = __ballot(pending)) != 0ull) {
        const int leader = __ffsll((unsigned long long)m) - 1;
        const int tgt = __shfl(target, leader);
        const bool mine = pending && target == tgt;
        const uint64_t mm = __ballot(mine);
        int base = 0;
        if (__lane_id() == leader) base = atomicAdd(&cnt[tgt], (int)__popcll(mm));
        base = __shfl(base, leader);
        if (mine) {
            slot = base + (int)__popcll(mm & lanemask_lt());
            pending = false;
        }
    }
    return slot;
}

// Store a particle into copy `dst` at the segment of tile `tgt` (or overflow).
template <typename R>
__device__ inline void store_particle(const BoxDev<R> &B, const SpeciesDev<R> &S, int dst, int tgt, bool valid,
                                      int32_t cell, const R d[3], const R u[3], int32_t id, uint32_t *flags)
{
    int32_t *cnt = S.cnt[dst];
    int slot = claim_slot(cnt, tgt, valid);
    if (!valid) return;
    int idx;
    if (slot < S.seg_cap[dst][tgt]) {
        idx = S.seg_start[dst][tgt] + slot;
    } else {
        const int o = atomicAdd(&cnt[B.ntiles], 1);
        if (o >= S.ovf_cap) {
            atomicOr(flags, PIC_FLAG_LOST);
            return;
        }
        idx = S.seg_start[dst][B.ntiles] + o;
    }
    const PBuf<R> &P = S.buf[dst];
    P.cell[idx] = cell;
    P.d[0][idx] = d[0]; P.d[1][idx] = d[1]; P.d[2][idx] = d[2];
    P.u[0][idx] = u[0]; P.u[1][idx] = u[1]; P.u[2][idx] = u[2];
    if (P.id) P.id[idx] = id;
}

// New cell and offset after the move x1 = d + D (home-cell frame), wrapped.
template <typename R>
__device__ inline int32_t advance_cell(const BoxDev<R> &B, int ix, int iy, int iz, const R x1[3], R dn[3])
{
    int c[3] = {ix, iy, iz};
    for (int a = 0; a < 3; ++a) {
        int f = x1[a] < R(0) ? -1 : (x1[a] >= R(1) ? 1 : 0);
        R v = x1[a] - R(f);
        if (v >= R(1)) {        // x1 a hair below 0: rounds to the cell boundary
            v = R(0);
            f += 1;
        }
        dn[a] = v;
        int ci = c[a] + f;
        if (ci < 0) ci += B.n[a];
        else if (ci >= B.n[a]) ci -= B.n[a];
        c[a] = ci;
    }
    return pack_cell(c[0], c[1], c[2]);
}

// ------------------------------------------------- fused per-tile push kernel

template <typename R>
struct TileGeom {
    int o[3], ext[3];
    int NX, NY, NN;      // node region (ext+1)^3, origin o
    int JX, JY, JN;      // J / raw-e region (ext+3)^3, origin o-1
    int BX, BY, BN;      // raw-b region (ext+2)^3, origin o-1
};

template <typename R>
__device__ inline TileGeom<R> tile_geom(const BoxDev<R> &B, int T)
{
    TileGeom<R> g;
    const int tx = T % B.ntile[0];
    const int r = T / B.ntile[0];
    const int ty = r % B.ntile[1], tz = r / B.ntile[1];
    g.o[0] = tx << B.tshift[0];
    g.o[1] = ty << B.tshift[1];
    g.o[2] = tz << B.tshift[2];
    for (int a = 0; a < 3; ++a) g.ext[a] = min(1 << B.tshift[a], B.n[a] - g.o[a]);
    g.NX = g.ext[0] + 1; g.NY = g.ext[1] + 1; g.NN = g.NX * g.NY * (g.ext[2] + 1);
    g.JX = g.ext[0] + 3; g.JY = g.ext[1] + 3; g.JN = g.JX * g.JY * (g.ext[2] + 3);
    g.BX = g.ext[0] + 2; g.BY = g.ext[1] + 2; g.BN = g.BX * g.BY * (g.ext[2] + 2);
    return g;
}

// Bytes of dynamic LDS for a tile with edges (t0, t1, t2).
template <typename R>
__host__ __device__ inline size_t tile_lds_bytes(int t0, int t1, int t2)
{
    const size_t nn = (size_t)(t0 + 1) * (t1 + 1) * (t2 + 1);
    const size_t jn = (size_t)(t0 + 3) * (t1 + 3) * (t2 + 3);
    const size_t bn = (size_t)(t0 + 2) * (t1 + 2) * (t2 + 2);
    const size_t raw = 3 * (jn + bn) * sizeof(R);
    const size_t jb = 3 * jn * sizeof(typename JType<R>::T);
    const size_t u = raw > jb ? raw : jb;
    return nn * 8 * sizeof(R) + ((u + 15) & ~size_t(15));
}

template <typename R>
__global__ void __launch_bounds__(kBlock) push_kernel(const BoxDev<R> *__restrict__ boxes,
                                                      const Item *__restrict__ items, StepConst<R> C);

// Overflow sweep: same physics, fields from HBM, current by global atomics.
template <typename R>
__device__ void push_overflow(const BoxDev<R> &B, int kblk, const StepConst<R> &C)
{
    using JT = typename JType<R>::T;
    const R hdt = R(0.5) * C.dt;
    for (int s = 0; s < C.nsp; ++s) {
        const SpeciesDev<R> &S = B.sp[s];
        const int n = min(S.cnt[C.cur][B.ntiles], S.ovf_cap);
        const int start = S.seg_start[C.cur][B.ntiles];
        const PBuf<R> &P = S.buf[C.cur];
        const R hk = R(0.5) * C.kq[s] * C.dt;
        const R scale = -C.qs[s] * qscale_bits<R>();
        for (int pb = kblk * kBlock; pb < n; pb += kBlock * kOvfBlocks) {
            const int p = pb + (int)threadIdx.x;
            const bool valid = p < n;
            const int idx = start + (valid ? p : 0);
            int32_t cell = 0, id = 0;
            R d[3] = {R(0.5), R(0.5), R(0.5)}, u[3] = {R(0), R(0), R(0)};
            if (valid) {
                cell = P.cell[idx];
                for (int a = 0; a < 3; ++a) { d[a] = P.d[a][idx]; u[a] = P.u[a][idx]; }
                if (P.id) id = P.id[idx];
            }
            const int ix = cell_x(cell), iy = cell_y(cell), iz = cell_z(cell);
            R E[3], Bf[3];
            if (valid) gather_global(B, ix, iy, iz, d, hdt, E, Bf);
            else for (int a = 0; a < 3; ++a) { E[a] = R(0); Bf[a] = R(0); }
            boris(hk, E, Bf, u);
            if (!(isfinite(u[0]) && isfinite(u[1]) && isfinite(u[2]))) {
                if (valid) atomicOr(C.flags, PIC_FLAG_NONFINITE);
                u[0] = u[1] = u[2] = R(0);
            }
            const R ig = C.dt * fast_rsqrt(R(1) + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            R D[3] = {ig * u[0], ig * u[1], ig * u[2]};
            if (valid) {
                JT *J = B.J;
                deposit_move(d, D, scale, [&](int a, int ox, int oy, int oz, R v) {
                    const int i = wrap_idx(ix + ox, B.n[0]), j = wrap_idx(iy + oy, B.n[1]),
                              k = wrap_idx(iz + oz, B.n[2]);
                    atomic_add_global(&J[a * B.nc + i + (int64_t)B.n[0] * (j + (int64_t)B.n[1] * k)],
                                      quantize(v));
                });
            }
            R x1[3] = {d[0] + D[0], d[1] + D[1], d[2] + D[2]}, dn[3];
            const int32_t nc = advance_cell(B, ix, iy, iz, x1, dn);
            store_particle(B, S, C.cur ^ 1, tile_of(B, nc), valid, nc, dn, u, id, C.flags);
        }
    }
}

template <typename R>
__global__ void __launch_bounds__(kBlock) push_kernel(const BoxDev<R> *__restrict__ boxes,
                                                      const Item *__restrict__ items, StepConst<R> C)
{
    using JT = typename JType<R>::T;
    extern __shared__ __align__(16) unsigned char smem[];
    const Item it = items[blockIdx.x];
    const BoxDev<R> &B = boxes[it.box];
    if (it.tile < 0) {
        push_overflow(B, -1 - it.tile, C);
        return;
    }
    const int T = it.tile;
    const int tid = threadIdx.x;
    const TileGeom<R> g = tile_geom(B, T);
    R *node = reinterpret_cast<R *>(smem);
    unsigned char *uni = smem + (((size_t)g.NN * 8 * sizeof(R) + 15) & ~size_t(15));
    R *re = reinterpret_cast<R *>(uni);          // raw e, 3 x JN, origin o-1
    R *rb = re + 3 * g.JN;                        // raw b, 3 x BN, origin o-1
    JT *jl = reinterpret_cast<JT *>(uni);         // J, 3 x JN, origin o-1 (after staging)

    int nsp_n[kMaxSpecies];
    for (int s = 0; s < C.nsp; ++s)
        nsp_n[s] = min(B.sp[s].cnt[C.cur][T], B.sp[s].seg_cap[C.cur][T]);

    // 1. stage e^t and b^{t-dt/2} of the tile and its halo
    const int64_t n0 = B.n[0], n01 = (int64_t)B.n[0] * B.n[1];
    for (int q = tid; q < 3 * g.JN; q += kBlock) {
        const int c = q / g.JN, r = q - c * g.JN;
        const int i = r % g.JX, j = (r / g.JX) % g.JY, k = r / (g.JX * g.JY);
        const int gi = wrap_idx(g.o[0] - 1 + i, B.n[0]), gj = wrap_idx(g.o[1] - 1 + j, B.n[1]),
                  gk = wrap_idx(g.o[2] - 1 + k, B.n[2]);
        re[q] = B.e[c * B.nc + gi + n0 * gj + n01 * gk];
    }
    for (int q = tid; q < 3 * g.BN; q += kBlock) {
        const int c = q / g.BN, r = q - c * g.BN;
        const int i = r % g.BX, j = (r / g.BX) % g.BY, k = r / (g.BX * g.BY);
        const int gi = wrap_idx(g.o[0] - 1 + i, B.n[0]), gj = wrap_idx(g.o[1] - 1 + j, B.n[1]),
                  gk = wrap_idx(g.o[2] - 1 + k, B.n[2]);
        rb[q] = B.b[c * B.nc + gi + n0 * gj + n01 * gk];
    }
    __syncthreads();
    if (tid == 0)
        for (int s = 0; s < C.nsp; ++s) B.sp[s].cnt[C.cur][T] = 0;   // read above; reused as output next step

    // 2. b^t = b^{t-dt/2} - (dt/2) curl e^t (App. A.3.1 item 1), in place
    const R hdt = R(0.5) * C.dt;
    {
        const int JX = g.JX, JXY = g.JX * g.JY;
        for (int q = tid; q < 3 * g.BN; q += kBlock) {
            const int c = q / g.BN, r = q - c * g.BN;
            const int i = r % g.BX, j = (r / g.BX) % g.BY, k = r / (g.BX * g.BY);
            const int p = i + JX * j + JXY * k;
            const R *ex = re, *ey = re + g.JN, *ez = re + 2 * g.JN;
            R curl;
            if (c == 0) curl = (ez[p + JX] - ez[p]) - (ey[p + JXY] - ey[p]);
            else if (c == 1) curl = (ex[p + JXY] - ex[p]) - (ez[p + 1] - ez[p]);
            else curl = (ey[p + 1] - ey[p]) - (ex[p + JX] - ex[p]);
            rb[q] -= hdt * curl;
        }
    }
    __syncthreads();

    // 3. node fields on the (ext+1)^3 nodes of the tile (App. A.3.3)
    {
        const int JX = g.JX, JXY = g.JX * g.JY, BX = g.BX, BXY = g.BX * g.BY;
        const R *ex = re, *ey = re + g.JN, *ez = re + 2 * g.JN;
        const R *bx = rb, *by = rb + g.BN, *bz = rb + 2 * g.BN;
        for (int q = tid; q < g.NN; q += kBlock) {
            const int i = q % g.NX, j = (q / g.NX) % g.NY, k = q / (g.NX * g.NY);
            // raw coordinates of node (i,j,k) are (i+1, j+1, k+1)
            const int pe = (i + 1) + JX * (j + 1) + JXY * (k + 1);
            const int pb = (i + 1) + BX * (j + 1) + BXY * (k + 1);
            R *nf = node + 8 * q;
            nf[0] = R(0.5) * (ex[pe - 1] + ex[pe]);
            nf[1] = R(0.5) * (ey[pe - JX] + ey[pe]);
            nf[2] = R(0.5) * (ez[pe - JXY] + ez[pe]);
            nf[3] = R(0.25) * (bx[pb] + bx[pb - BX] + bx[pb - BX - BXY] + bx[pb - BXY]);
            nf[4] = R(0.25) * (by[pb] + by[pb - BXY] + by[pb - 1 - BXY] + by[pb - 1]);
            nf[5] = R(0.25) * (bz[pb] + bz[pb - 1] + bz[pb - 1 - BX] + bz[pb - BX]);
            nf[6] = R(0);
            nf[7] = R(0);
        }
    }
    __syncthreads();
    for (int q = tid; q < 3 * g.JN; q += kBlock) jl[q] = JT(0);
    __syncthreads();

    // 4. particles of every species: gather, push, move, deposit, re-bin
    const int NX = g.NX, NXY = g.NX * g.NY;
    const int JX = g.JX, JXY = g.JX * g.JY;
    for (int s = 0; s < C.nsp; ++s) {
        const SpeciesDev<R> &S = B.sp[s];
        const PBuf<R> &P = S.buf[C.cur];
        const int n = nsp_n[s];
        const int start = S.seg_start[C.cur][T];
        const R hk = R(0.5) * C.kq[s] * C.dt;
        const R scale = -C.qs[s] * qscale_bits<R>();
        for (int pb = 0; pb < n; pb += kBlock) {
            const int p = pb + tid;
            const bool valid = p < n;
            const int idx = start + (valid ? p : 0);
            int32_t cell = pack_cell(g.o[0], g.o[1], g.o[2]), id = 0;
            R d[3] = {R(0.5), R(0.5), R(0.5)}, u[3] = {R(0), R(0), R(0)};
            if (valid) {
                cell = P.cell[idx];
                d[0] = P.d[0][idx]; d[1] = P.d[1][idx]; d[2] = P.d[2][idx];
                u[0] = P.u[0][idx]; u[1] = P.u[1][idx]; u[2] = P.u[2][idx];
                if (P.id) id = P.id[idx];
            }
            const int ix = cell_x(cell), iy = cell_y(cell), iz = cell_z(cell);
            const int lx = ix - g.o[0], ly = iy - g.o[1], lz = iz - g.o[2];
            // every particle of the segment has its cell in the tile; anything
            // else would index the tile's LDS out of range, so it takes the
            // HBM path instead
            const bool inside = (unsigned)lx < (unsigned)g.ext[0] && (unsigned)ly < (unsigned)g.ext[1] &&
                                (unsigned)lz < (unsigned)g.ext[2];
            // gather: trilinear weights on the eight nodes of the cell
            R E[3] = {R(0), R(0), R(0)}, Bf[3] = {R(0), R(0), R(0)};
            if (!inside) {
                gather_global(B, ix, iy, iz, d, hdt, E, Bf);
            } else {
                const R wx[2] = {R(1) - d[0], d[0]}, wy[2] = {R(1) - d[1], d[1]}, wz[2] = {R(1) - d[2], d[2]};
                const int q0 = lx + NX * ly + NXY * lz;
#pragma unroll
                for (int kk = 0; kk < 2; ++kk)
#pragma unroll
                    for (int jj = 0; jj < 2; ++jj) {
                        const R wyz = wy[jj] * wz[kk];
#pragma unroll
                        for (int ii = 0; ii < 2; ++ii) {
                            const R w = wx[ii] * wyz;
                            const R *nf = node + 8 * (q0 + ii + NX * jj + NXY * kk);
                            E[0] += w * nf[0]; E[1] += w * nf[1]; E[2] += w * nf[2];
                            Bf[0] += w * nf[3]; Bf[1] += w * nf[4]; Bf[2] += w * nf[5];
                        }
                    }
            }
            boris(hk, E, Bf, u);
            if (!(isfinite(u[0]) && isfinite(u[1]) && isfinite(u[2]))) {
                if (valid) atomicOr(C.flags, PIC_FLAG_NONFINITE);
                u[0] = u[1] = u[2] = R(0);
            }
            const R ig = C.dt * fast_rsqrt(R(1) + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            R D[3] = {ig * u[0], ig * u[1], ig * u[2]};
            if (valid && inside) {
                const int jb = (lx + 1) + JX * (ly + 1) + JXY * (lz + 1);
                const int JN = g.JN;
                deposit_move(d, D, scale, [&](int a, int ox, int oy, int oz, R v) {
                    atomic_add_lds(&jl[a * JN + jb + ox + JX * oy + JXY * oz], quantize(v));
                });
            } else if (valid) {
                JT *J = B.J;
                deposit_move(d, D, scale, [&](int a, int ox, int oy, int oz, R v) {
                    const int i = wrap_idx(ix + ox, B.n[0]), j = wrap_idx(iy + oy, B.n[1]),
                              k = wrap_idx(iz + oz, B.n[2]);
                    atomic_add_global(&J[a * B.nc + i + (int64_t)B.n[0] * (j + (int64_t)B.n[1] * k)],
                                      quantize(v));
                });
            }
            R x1[3] = {d[0] + D[0], d[1] + D[1], d[2] + D[2]}, dn[3];
            const int32_t nc = advance_cell(B, ix, iy, iz, x1, dn);
            const int tn = tile_of(B, nc);
            store_particle(B, S, C.cur ^ 1, tn, valid, nc, dn, u, id, C.flags);
        }
    }
    __syncthreads();

    // 5. flush the tile current to HBM (integer sums: order-independent)
    for (int q = tid; q < 3 * g.JN; q += kBlock) {
        const JT v = jl[q];
        if (v != JT(0)) {
            const int c = q / g.JN, r = q - c * g.JN;
            const int i = r % g.JX, j = (r / g.JX) % g.JY, k = r / (g.JX * g.JY);
            const int gi = wrap_idx(g.o[0] - 1 + i, B.n[0]), gj = wrap_idx(g.o[1] - 1 + j, B.n[1]),
                      gk = wrap_idx(g.o[2] - 1 + k, B.n[2]);
            atomic_add_global(&B.J[c * B.nc + gi + n0 * gj + n01 * gk], v);
        }
    }
}

// ------------------------------------------------------------- Yee updates

// b <- b - h curl e (App. A.3.2)
template <typename R>
__global__ void __launch_bounds__(kBlock) advance_b_kernel(const BoxDev<R> *__restrict__ boxes,
                                                           const CellBlock *__restrict__ blocks, R h)
{
    const CellBlock cb = blocks[blockIdx.x];
    const BoxDev<R> &B = boxes[cb.box];
    const int64_t p = (int64_t)cb.first + threadIdx.x;
    if (p >= B.nc) return;
    const int n0 = B.n[0], n1 = B.n[1], n2 = B.n[2];
    const int i = (int)(p % n0), j = (int)((p / n0) % n1), k = (int)(p / ((int64_t)n0 * n1));
    const int64_t sx = (i + 1 < n0) ? 1 : 1 - n0;
    const int64_t sy = (j + 1 < n1) ? n0 : (int64_t)n0 * (1 - n1);
    const int64_t sz = (k + 1 < n2) ? (int64_t)n0 * n1 : (int64_t)n0 * n1 * (1 - n2);
    const R *ex = B.e, *ey = B.e + B.nc, *ez = B.e + 2 * B.nc;
    const R cx = (ez[p + sy] - ez[p]) - (ey[p + sz] - ey[p]);
    const R cy = (ex[p + sz] - ex[p]) - (ez[p + sx] - ez[p]);
    const R cz = (ey[p + sx] - ey[p]) - (ex[p + sy] - ex[p]);
    B.b[p] -= h * cx;
    B.b[B.nc + p] -= h * cy;
    B.b[2 * B.nc + p] -= h * cz;
}

// e <- e + dt curl b + alpha0 J (App. A.3.2 and A.2, eq. max2bis); J <- 0.
// Also clears the overflow counters of the copy the push just read.
template <typename R>
__global__ void __launch_bounds__(kBlock) advance_e_kernel(const BoxDev<R> *__restrict__ boxes,
                                                           const CellBlock *__restrict__ blocks, R dt,
                                                           int nsp, int clear_copy)
{
    using JT = typename JType<R>::T;
    const CellBlock cb = blocks[blockIdx.x];
    const BoxDev<R> &B = boxes[cb.box];
    if (cb.first == 0 && threadIdx.x < (unsigned)nsp && clear_copy >= 0)
        B.sp[threadIdx.x].cnt[clear_copy][B.ntiles] = 0;
    const int64_t p = (int64_t)cb.first + threadIdx.x;
    if (p >= B.nc) return;
    const int n0 = B.n[0], n1 = B.n[1], n2 = B.n[2];
    const int i = (int)(p % n0), j = (int)((p / n0) % n1), k = (int)(p / ((int64_t)n0 * n1));
    const int64_t sx = (i > 0) ? 1 : 1 - n0;
    const int64_t sy = (j > 0) ? n0 : (int64_t)n0 * (1 - n1);
    const int64_t sz = (k > 0) ? (int64_t)n0 * n1 : (int64_t)n0 * n1 * (1 - n2);
    const R *bx = B.b, *by = B.b + B.nc, *bz = B.b + 2 * B.nc;
    const R cx = (bz[p] - bz[p - sy]) - (by[p] - by[p - sz]);
    const R cy = (bx[p] - bx[p - sz]) - (bz[p] - bz[p - sx]);
    const R cz = (by[p] - by[p - sx]) - (bx[p] - bx[p - sy]);
    JT *J = B.J;
    const double a = B.alpha0 / (double)qscale_bits<R>();
    const R jx = (R)(a * (double)J[p]), jy = (R)(a * (double)J[B.nc + p]), jz = (R)(a * (double)J[2 * B.nc + p]);
    B.e[p] += dt * cx + jx;
    B.e[B.nc + p] += dt * cy + jy;
    B.e[2 * B.nc + p] += dt * cz + jz;
    J[p] = JT(0);
    J[B.nc + p] = JT(0);
    J[2 * B.nc + p] = JT(0);
}

// ------------------------------------------------------ counting-sort repack

template <typename R>
__device__ inline void seg_range(const BoxDev<R> &B, const SpeciesDev<R> &S, int copy, int tile, int &start,
                                 int &n, int &first, int &stride)
{
    if (tile >= 0) {
        start = S.seg_start[copy][tile];
        n = min(S.cnt[copy][tile], S.seg_cap[copy][tile]);
        first = threadIdx.x;
        stride = kBlock;
    } else {
        start = S.seg_start[copy][B.ntiles];
        n = min(S.cnt[copy][B.ntiles], S.ovf_cap);
        first = (-1 - tile) * kBlock + threadIdx.x;
        stride = kBlock * kOvfBlocks;
    }
}

template <typename R>
__global__ void __launch_bounds__(kBlock) repack_count_kernel(const BoxDev<R> *__restrict__ boxes,
                                                              const Item *__restrict__ items, int nsp, int cur)
{
    const Item it = items[blockIdx.x];
    const BoxDev<R> &B = boxes[it.box];
    for (int s = 0; s < nsp; ++s) {
        const SpeciesDev<R> &S = B.sp[s];
        int start, n, first, stride;
        seg_range(B, S, cur, it.tile, start, n, first, stride);
        for (int p = first; p < n; p += stride)
            atomicAdd(&S.tcount[tile_of(B, S.buf[cur].cell[start + p])], 1);
    }
}

template <typename R>
__global__ void __launch_bounds__(kBlock) repack_count_stage_kernel(const BoxDev<R> *__restrict__ boxes,
                                                                    const StageItem *__restrict__ items)
{
    const StageItem it = items[blockIdx.x];
    const BoxDev<R> &B = boxes[it.box];
    const SpeciesDev<R> &S = B.sp[it.species];
    const int p = it.first + threadIdx.x;
    if (p < it.last) atomicAdd(&S.tcount[tile_of(B, S.stage.cell[p])], 1);
}

// One block per (box, species): new segment layout from the tile counts.
// Free slots are shared in proportion to (count + 1); the overflow region is
// the fixed tail of the arrays.
template <typename R>
__global__ void __launch_bounds__(kBlock) repack_layout_kernel(const BoxDev<R> *__restrict__ boxes, int nsp,
                                                               int dst, uint32_t *flags)
{
    __shared__ long long part[kBlock];
    const int box = blockIdx.x / nsp, s = blockIdx.x % nsp;
    const BoxDev<R> &B = boxes[box];
    const SpeciesDev<R> &S = B.sp[s];
    const int nt = B.ntiles;
    const int tid = threadIdx.x;
    const int per = (nt + kBlock - 1) / kBlock;
    const int t0 = min(nt, tid * per), t1 = min(nt, t0 + per);
    long long mine = 0;
    for (int t = t0; t < t1; ++t) mine += S.tcount[t];
    part[tid] = mine;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {   // total
        if (tid < off) part[tid] += part[tid + off];
        __syncthreads();
    }
    const long long total = part[0];
    __syncthreads();
    const long long region = (long long)S.slots - S.ovf_cap;
    if (total > region) {                              // uniform: the whole block leaves
        if (tid == 0) atomicOr(flags, PIC_FLAG_LOST);
        return;
    }
    const long long freeslots = region - total;
    const long long den = total + nt;
    long long mycap = 0;
    for (int t = t0; t < t1; ++t) mycap += S.tcount[t] + (freeslots * (S.tcount[t] + 1)) / den;
    part[tid] = mycap;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {       // inclusive scan of the caps
        const long long v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    long long run = part[tid] - mycap;
    for (int t = t0; t < t1; ++t) {
        const long long cap = S.tcount[t] + (freeslots * (S.tcount[t] + 1)) / den;
        S.seg_start[dst][t] = (int32_t)run;
        S.seg_cap[dst][t] = (int32_t)cap;
        S.cnt[dst][t] = 0;
        S.tcount[t] = 0;
        run += cap;
    }
    if (tid == 0) {
        S.seg_start[dst][nt] = S.slots - S.ovf_cap;
        S.seg_cap[dst][nt] = S.ovf_cap;
        S.cnt[dst][nt] = 0;
    }
}

template <typename R>
__global__ void __launch_bounds__(kBlock) repack_scatter_kernel(const BoxDev<R> *__restrict__ boxes,
                                                                const Item *__restrict__ items, int nsp, int cur,
                                                                uint32_t *flags)
{
    const Item it = items[blockIdx.x];
    const BoxDev<R> &B = boxes[it.box];
    for (int s = 0; s < nsp; ++s) {
        const SpeciesDev<R> &S = B.sp[s];
        int start, n, first, stride;
        seg_range(B, S, cur, it.tile, start, n, first, stride);
        const PBuf<R> &P = S.buf[cur];
        // wave-uniform trip count so that the ballots in store_particle see every lane
        const int trips = n > first - (int)threadIdx.x ? (n - (first - (int)threadIdx.x) + stride - 1) / stride : 0;
        for (int tr = 0; tr < trips; ++tr) {
            const int p = first + tr * stride;
            const bool valid = p < n;
            int32_t cell = 0, id = 0;
            R d[3] = {R(0), R(0), R(0)}, u[3] = {R(0), R(0), R(0)};
            if (valid) {
                const int idx = start + p;
                cell = P.cell[idx];
                for (int a = 0; a < 3; ++a) { d[a] = P.d[a][idx]; u[a] = P.u[a][idx]; }
                if (P.id) id = P.id[idx];
            }
            store_particle(B, S, cur ^ 1, tile_of(B, cell), valid, cell, d, u, id, flags);
        }
    }
}

template <typename R>
__global__ void __launch_bounds__(kBlock) repack_scatter_stage_kernel(const BoxDev<R> *__restrict__ boxes,
                                                                      const StageItem *__restrict__ items,
                                                                      StepConst<R> C)
{
    const StageItem it = items[blockIdx.x];
    const BoxDev<R> &B = boxes[it.box];
    const SpeciesDev<R> &S = B.sp[it.species];
    const int p = it.first + threadIdx.x;
    const bool valid = p < it.last;
    int32_t cell = 0, id = 0;
    R d[3] = {R(0), R(0), R(0)}, u[3] = {R(0), R(0), R(0)};
    if (valid) {
        cell = S.stage.cell[p];
        for (int a = 0; a < 3; ++a) { d[a] = S.stage.d[a][p]; u[a] = S.stage.u[a][p]; }
        if (S.stage.id) id = S.stage.id[p];
        if (it.half) {
            // backward half step (App. A.3.1): u^t -> u^{t-dt/2} in e^t, b^t
            R E[3], Bf[3];
            gather_global(B, cell_x(cell), cell_y(cell), cell_z(cell), d, R(0.5) * C.dt, E, Bf);
            boris(R(-0.25) * C.kq[it.species] * C.dt, E, Bf, u);
        }
    }
    store_particle(B, S, C.cur ^ 1, tile_of(B, cell), valid, cell, d, u, id, C.flags);
}

// After a repack into copy 1-old: clear the counters of copy `old` (all tiles
// and the overflow entry) and give it the new segment layout too.
template <typename R>
__global__ void __launch_bounds__(kBlock) clear_counts_kernel(const BoxDev<R> *__restrict__ boxes, int nboxes,
                                                              int nsp, int old)
{
    const int box = blockIdx.y;
    if (box >= nboxes) return;
    const BoxDev<R> &B = boxes[box];
    for (int t = blockIdx.x * kBlock + threadIdx.x; t <= B.ntiles; t += gridDim.x * kBlock)
        for (int s = 0; s < nsp; ++s) {
            const SpeciesDev<R> &S = B.sp[s];
            S.cnt[old][t] = 0;
            S.seg_start[old][t] = S.seg_start[old ^ 1][t];
            S.seg_cap[old][t] = S.seg_cap[old ^ 1][t];
        }
}

// -------------------------------------------------------------- diagnostics

template <typename R>
__device__ inline void block_sum_to(double *dst, double v)
{
    __shared__ double red[kBlock / 64];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if (__lane_id() == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < kBlock / 64; ++q) t += red[q];
        atomicAdd(dst, t);
    }
}

// Per-particle diagnostics of one box (items of that box only): gamma^t from
// u^- = u^{t-dt/2} + (k dt/2) E(x^t) (READING: the mover's own gamma^t), the
// k = 0 momentum, the gamma-1 histogram and the CIC charge density.
template <typename R>
__global__ void __launch_bounds__(kBlock) diag_particles_kernel(const BoxDev<R> *__restrict__ boxes,
                                                                const Item *__restrict__ items, StepConst<R> C)
{
    const Item it = items[blockIdx.x];
    const BoxDev<R> &B = boxes[it.box];
    const R hdt = R(0.5) * C.dt;
    for (int s = 0; s < C.nsp; ++s) {
        const SpeciesDev<R> &S = B.sp[s];
        int start, n, first, stride;
        seg_range(B, S, C.cur, it.tile, start, n, first, stride);
        const PBuf<R> &P = S.buf[C.cur];
        double acc[6] = {0, 0, 0, 0, 0, 0};
        for (int p = first; p < n; p += stride) {
            const int idx = start + p;
            const int32_t cell = P.cell[idx];
            const int ix = cell_x(cell), iy = cell_y(cell), iz = cell_z(cell);
            R d[3] = {P.d[0][idx], P.d[1][idx], P.d[2][idx]};
            R E[3], Bf[3];
            gather_global(B, ix, iy, iz, d, hdt, E, Bf);
            double um[3];
            for (int a = 0; a < 3; ++a)
                um[a] = (double)P.u[a][idx] + 0.5 * (double)C.kq[s] * (double)C.dt * (double)E[a];
            const double gm1 = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]) - 1.0;
            acc[0] += (double)C.mass[s] * gm1;
            acc[1] += um[0]; acc[2] += um[1]; acc[3] += um[2];
            acc[4] += 1.0;
            acc[5] += gm1;
            if (C.hist_bins > 0) {
                const double v = log10(gm1 > 1e-300 ? gm1 : 1e-300);
                int bin = (int)floor((v - C.hist_lo) / (C.hist_hi - C.hist_lo) * C.hist_bins);
                bin = bin < 0 ? 0 : (bin >= C.hist_bins ? C.hist_bins - 1 : bin);
                atomicAdd(reinterpret_cast<unsigned long long *>(&B.hist[s * C.hist_bins + bin]), 1ull);
            }
            const double q = (double)C.qs[s] * B.alpha0;
            for (int kk = 0; kk < 2; ++kk)
                for (int jj = 0; jj < 2; ++jj)
                    for (int ii = 0; ii < 2; ++ii) {
                        const double w = (ii ? (double)d[0] : 1.0 - (double)d[0]) *
                                         (jj ? (double)d[1] : 1.0 - (double)d[1]) *
                                         (kk ? (double)d[2] : 1.0 - (double)d[2]);
                        const int i = wrap_idx(ix + ii, B.n[0]), j = wrap_idx(iy + jj, B.n[1]),
                                  k = wrap_idx(iz + kk, B.n[2]);
                        atomicAdd(&B.rho[i + (int64_t)B.n[0] * (j + (int64_t)B.n[1] * k)], q * w);
                    }
        }
        for (int q = 0; q < 6; ++q) block_sum_to<R>(&B.acc[kAccSp + 6 * s + q], acc[q]);
    }
}

__device__ inline void atomic_max_pos(double *p, double v)
{
    atomicMax(reinterpret_cast<unsigned long long *>(p), (unsigned long long)__double_as_longlong(v));
}

// Field energies (e^t, b^t) and the Gauss-law residual div e - rho at the nodes.
template <typename R>
__global__ void __launch_bounds__(kBlock) diag_fields_kernel(const BoxDev<R> *__restrict__ boxes, int box,
                                                             R dt)
{
    const BoxDev<R> &B = boxes[box];
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    double gmax = 0.0;
    if (p < B.nc) {
        const int n0 = B.n[0], n1 = B.n[1];
        const int i = (int)(p % n0), j = (int)((p / n0) % n1), k = (int)(p / ((int64_t)n0 * n1));
        for (int c = 0; c < 3; ++c) {
            const double ec = (double)B.e[c * B.nc + p];
            const double bc = (double)bt_global(B, c, i, j, k, R(0.5) * dt);
            v[c] = 0.5 * ec * ec;
            v[3 + c] = 0.5 * bc * bc;
        }
        const double div = (double)fld(B.e, B, 0, i, j, k) - (double)fld(B.e, B, 0, i - 1, j, k) +
                           (double)fld(B.e, B, 1, i, j, k) - (double)fld(B.e, B, 1, i, j - 1, k) +
                           (double)fld(B.e, B, 2, i, j, k) - (double)fld(B.e, B, 2, i, j, k - 1);
        const double r = div - B.rho[p];
        v[6] = r * r;
        gmax = fabs(r);
    }
    for (int q = 0; q < 6; ++q) block_sum_to<R>(&B.acc[kAccField + q], v[q]);
    block_sum_to<R>(&B.acc[kAccField + 7], v[6]);
    for (int off = 32; off > 0; off >>= 1) gmax = fmax(gmax, __shfl_down(gmax, off));
    if (__lane_id() == 0) atomic_max_pos(&B.acc[kAccField + 6], gmax);
}

// ----------------------------------------------------------- host launchers

template <typename R>
size_t push_lds_bytes(int t0, int t1, int t2) { return tile_lds_bytes<R>(t0, t1, t2); }

template <typename R>
hipError_t launch_push(const BoxDev<R> *boxes, const Item *items, int nitems, size_t lds, const StepConst<R> &C,
                       hipStream_t st)
{
    if (lds > 65536) {
        static bool raised = false;
        if (!raised) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&push_kernel<R>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            raised = true;
        }
    }
    hipLaunchKernelGGL(push_kernel<R>, dim3(nitems), dim3(kBlock), lds, st, boxes, items, C);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_fields(const BoxDev<R> *boxes, const CellBlock *blocks, int nblocks, R dt, int nsp,
                         int clear_copy, hipStream_t st)
{
    hipLaunchKernelGGL(advance_b_kernel<R>, dim3(nblocks), dim3(kBlock), 0, st, boxes, blocks, dt);
    hipLaunchKernelGGL(advance_e_kernel<R>, dim3(nblocks), dim3(kBlock), 0, st, boxes, blocks, dt, nsp,
                       clear_copy);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_advance_b(const BoxDev<R> *boxes, const CellBlock *blocks, int nblocks, R h, hipStream_t st)
{
    hipLaunchKernelGGL(advance_b_kernel<R>, dim3(nblocks), dim3(kBlock), 0, st, boxes, blocks, h);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_repack(const BoxDev<R> *boxes, int nboxes, const Item *items, int nitems,
                         const StageItem *sitems, int nsitems, const StepConst<R> &C, hipStream_t st)
{
    if (nitems) hipLaunchKernelGGL(repack_count_kernel<R>, dim3(nitems), dim3(kBlock), 0, st, boxes, items, C.nsp, C.cur);
    if (nsitems) hipLaunchKernelGGL(repack_count_stage_kernel<R>, dim3(nsitems), dim3(kBlock), 0, st, boxes, sitems);
    hipLaunchKernelGGL(repack_layout_kernel<R>, dim3(nboxes * C.nsp), dim3(kBlock), 0, st, boxes, C.nsp, C.cur ^ 1,
                       C.flags);
    if (nitems) hipLaunchKernelGGL(repack_scatter_kernel<R>, dim3(nitems), dim3(kBlock), 0, st, boxes, items, C.nsp, C.cur,
                                   C.flags);
    if (nsitems) hipLaunchKernelGGL(repack_scatter_stage_kernel<R>, dim3(nsitems), dim3(kBlock), 0, st, boxes, sitems, C);
    hipLaunchKernelGGL(clear_counts_kernel<R>, dim3(64, nboxes), dim3(kBlock), 0, st, boxes, nboxes, C.nsp, C.cur);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_diag(const BoxDev<R> *boxes, int box, int64_t nc, const Item *items, int nitems,
                       const StepConst<R> &C, hipStream_t st)
{
    if (nitems) hipLaunchKernelGGL(diag_particles_kernel<R>, dim3(nitems), dim3(kBlock), 0, st, boxes, items, C);
    const int nb = (int)((nc + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(diag_fields_kernel<R>, dim3(nb), dim3(kBlock), 0, st, boxes, box, C.dt);
    return hipGetLastError();
}

#define PIC_INSTANTIATE(R)                                                                                     \
    template size_t push_lds_bytes<R>(int, int, int);                                                         \
    template hipError_t launch_push<R>(const BoxDev<R> *, const Item *, int, size_t, const StepConst<R> &,   \
                                       hipStream_t);                                                          \
    template hipError_t launch_fields<R>(const BoxDev<R> *, const CellBlock *, int, R, int, int, hipStream_t); \
    template hipError_t launch_advance_b<R>(const BoxDev<R> *, const CellBlock *, int, R, hipStream_t);       \
    template hipError_t launch_repack<R>(const BoxDev<R> *, int, const Item *, int, const StageItem *, int,    \
                                         const StepConst<R> &, hipStream_t);                                  \
    template hipError_t launch_diag<R>(const BoxDev<R> *, int, int64_t, const Item *, int,                    \
                                       const StepConst<R> &, hipStream_t);

PIC_INSTANTIATE(float)
PIC_INSTANTIATE(double)

} // namespace pic
