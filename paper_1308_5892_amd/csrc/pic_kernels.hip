// gfx950 kernels of the PIC hot path: fused gather + Boris push + deposit per
// spatial tile, Yee field updates, counting-sort repack and FP64 diagnostics.
//
// Paper: Melzani et al., "Apar-T" (arXiv:1308.5892), App. A.  The readings of
// the paper used here (cyclic node averaging, standard Boris rotation,
// splitting of cell-crossing moves at node planes) are stated where they are
// used.  Every kernel is templated on the storage/arithmetic type R: float is
// the production form (int64 fixed-point current), double the FP64 form.
#include <hip/hip_runtime.h>

#include <limits>

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

// FP32 form: a value already scaled by 2^31 rounded to the nearest integer,
// ties upward, in one conversion (|value| < 2^31 since every face value of one
// move is below one cell volume)
__device__ inline int quantize(float v)
{
    int r;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(v));
    return r;
}
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

// ------------------------------------------------------ global-memory reads

template <typename R>
__device__ inline R fld(const PIC_GLOBAL R *F, const BoxDev<R> &B, int c, int i, int j, int k)
{
    i = wrap_idx(i, B.n[0]);
    j = wrap_idx(j, B.n[1]);
    k = wrap_idx(k, B.n[2]);
    return F[c * B.nc + i + (int64_t)B.n[0] * (j + (int64_t)B.n[1] * k)];
}

// Fourth-order field solver (App. A.3.2, last paragraph; App. B, third item;
// READING: the paper prints no stencil): Faraday's law takes the staggered
// fourth-order difference along each axis, (9/8)(f[+1/2] - f[-1/2]) -
// (1/24)(f[+3/2] - f[-3/2]); Ampere's law keeps the second-order curl, so the
// second-order divergence of e still changes only by the charge-conserving
// current (Gauss's law as with Yee).  d4_e: that difference along axis a of
// component f of e at the point half a cell above (i,j,k) along a.
template <typename R>
__device__ inline R d4_e(const BoxDev<R> &B, int f, int i, int j, int k, int a)
{
    const int o0 = a == 0, o1 = a == 1, o2 = a == 2;
    const R near = fld(B.e, B, f, i + o0, j + o1, k + o2) - fld(B.e, B, f, i, j, k);
    const R far = fld(B.e, B, f, i + 2 * o0, j + 2 * o1, k + 2 * o2) - fld(B.e, B, f, i - o0, j - o1, k - o2);
    return R(9.0 / 8.0) * near - R(1.0 / 24.0) * far;
}

// (curl e)_c of the fourth-order solver at the b_c position of cell (i,j,k)
template <typename R>
__device__ inline R curl4_e(const BoxDev<R> &B, int c, int i, int j, int k)
{
    if (c == 0) return d4_e(B, 2, i, j, k, 1) - d4_e(B, 1, i, j, k, 2);
    if (c == 1) return d4_e(B, 0, i, j, k, 2) - d4_e(B, 2, i, j, k, 0);
    return d4_e(B, 1, i, j, k, 0) - d4_e(B, 0, i, j, k, 1);
}

// b^t = b^{t-dt/2} - (dt/2) curl e^t at the b_c position of cell (i,j,k).
// F4: 1 the fourth-order curl, 0 Yee's, -1 as the box says (the push kernel
// is compiled for one solver, so its loop carries only that one's code).
template <typename R, int F4 = -1>
__device__ inline R bt_global(const BoxDev<R> &B, int c, int i, int j, int k, R hdt)
{
    if (F4 == 1 || (F4 < 0 && B.faraday4)) return fld(B.b, B, c, i, j, k) - hdt * curl4_e(B, c, i, j, k);
    const PIC_GLOBAL R *e = B.e;
    R curl;
    if (c == 0)
        curl = (fld(e, B, 2, i, j + 1, k) - fld(e, B, 2, i, j, k)) - (fld(e, B, 1, i, j, k + 1) - fld(e, B, 1, i, j, k));
    else if (c == 1)
        curl = (fld(e, B, 0, i, j, k + 1) - fld(e, B, 0, i, j, k)) - (fld(e, B, 2, i + 1, j, k) - fld(e, B, 2, i, j, k));
    else
        curl = (fld(e, B, 1, i + 1, j, k) - fld(e, B, 1, i, j, k)) - (fld(e, B, 0, i, j + 1, k) - fld(e, B, 0, i, j, k));
    return fld(B.b, B, c, i, j, k) - hdt * curl;
}

// Node-averaged field values (App. A.3.3; READING: e_c averaged over the two
// edges along c that meet at the node, b_c over the four faces normal to c).
// The tile set-up forms the same sums in the same order from its LDS copy.
template <typename R>
__device__ inline R node_avg2(R a, R b) { return R(0.5) * (a + b); }
template <typename R>
__device__ inline R node_avg4(R a, R b, R c, R d) { return R(0.25) * (a + b + c + d); }

// Component c (0-2: e, 3-5: b^t) at node (i,j,k), read from HBM.
template <typename R, int F4 = -1>
__device__ inline R node_value_global(const BoxDev<R> &B, int c, int i, int j, int k, R hdt)
{
    switch (c) {
    case 0: return node_avg2(fld(B.e, B, 0, i - 1, j, k), fld(B.e, B, 0, i, j, k));
    case 1: return node_avg2(fld(B.e, B, 1, i, j - 1, k), fld(B.e, B, 1, i, j, k));
    case 2: return node_avg2(fld(B.e, B, 2, i, j, k - 1), fld(B.e, B, 2, i, j, k));
    case 3: return node_avg4(bt_global<R, F4>(B, 0, i, j, k, hdt), bt_global<R, F4>(B, 0, i, j - 1, k, hdt),
                             bt_global<R, F4>(B, 0, i, j - 1, k - 1, hdt), bt_global<R, F4>(B, 0, i, j, k - 1, hdt));
    case 4: return node_avg4(bt_global<R, F4>(B, 1, i, j, k, hdt), bt_global<R, F4>(B, 1, i, j, k - 1, hdt),
                             bt_global<R, F4>(B, 1, i - 1, j, k - 1, hdt), bt_global<R, F4>(B, 1, i - 1, j, k, hdt));
    default: return node_avg4(bt_global<R, F4>(B, 2, i, j, k, hdt), bt_global<R, F4>(B, 2, i - 1, j, k, hdt),
                              bt_global<R, F4>(B, 2, i - 1, j - 1, k, hdt), bt_global<R, F4>(B, 2, i, j - 1, k, hdt));
    }
}

// The trilinear interpolant of the eight node values of a cell, f[q] at node
// (q & 1, (q >> 1) & 1, q >> 2), written as c0 + c1 x + c2 y + c3 z + c4 xy +
// c5 yz + c6 zx + c7 xyz in the in-cell offsets: its coefficients, and its
// value at d, nested as c0 + x (c1 + y (c4 + z c7) + z c6) + y (c2 + z c5) +
// z c3 (seven multiply-adds, no products of the offsets).  The tile path and
// the HBM path both use these two, so the fields a particle sees do not
// depend on the path it takes.
template <typename R, typename P>
__device__ inline void trilinear_coef(const R f[8], P cf)
{
    const R ax = f[1] - f[0], ay = f[2] - f[0], az = f[4] - f[0];
    const R axy = (f[3] - f[2]) - ax, ayz = (f[6] - f[4]) - ay, azx = (f[5] - f[1]) - az;
    cf[0] = f[0];
    cf[1] = ax;
    cf[2] = ay;
    cf[3] = az;
    cf[4] = axy;
    cf[5] = ayz;
    cf[6] = azx;
    cf[7] = ((f[7] - f[6]) - (f[5] - f[4])) - axy;
}
template <typename R, typename P>
__device__ inline R trilinear_eval(P k8, const R d[3])
{
    const R t = fma(d[2], k8[7], k8[4]);
    const R u = fma(d[2], k8[6], fma(d[1], t, k8[1]));
    const R v = fma(d[2], k8[5], k8[2]);
    return fma(d[2], k8[3], fma(d[1], v, fma(d[0], u, k8[0])));
}

// e^t and b^t at (cell, d) from HBM: the node values, the interpolant's
// coefficients and its value, as the tile path computes them.
template <typename R, int F4 = -1>
__device__ inline void gather_global(const BoxDev<R> &B, int ix, int iy, int iz, const R d[3], R hdt,
                                     R E[3], R Bf[3])
{
    if constexpr (sizeof(R) == 8) {
        // the component loop stays rolled (each pass inlines eight node
        // values); in the FP64 form, at three waves per SIMD, its results are
        // selected into registers, since an array indexed by the loop counter
        // would live in scratch there
        R o[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
        for (int c = 0; c < 6; ++c) {
            R f[8], cf[8];
            for (int q = 0; q < 8; ++q)
                f[q] = node_value_global<R, F4>(B, c, ix + (q & 1), iy + ((q >> 1) & 1), iz + (q >> 2), hdt);
            trilinear_coef(f, cf);
            const R v = trilinear_eval(cf, d);
#pragma unroll
            for (int k = 0; k < 6; ++k) o[k] = c == k ? v : o[k];
        }
        E[0] = o[0]; E[1] = o[1]; E[2] = o[2];
        Bf[0] = o[3]; Bf[1] = o[4]; Bf[2] = o[5];
    } else {
        for (int c = 0; c < 6; ++c) {
            R f[8], cf[8];
            for (int q = 0; q < 8; ++q)
                f[q] = node_value_global<R, F4>(B, c, ix + (q & 1), iy + ((q >> 1) & 1), iz + (q >> 2), hdt);
            trilinear_coef(f, cf);
            const R v = trilinear_eval(cf, d);
            if (c < 3) E[c] = v;
            else Bf[c - 3] = v;
        }
    }
}

// ------------------------------------------------------------ slot claims

// Number of lanes below this one whose bit is set in the wave mask m.
__device__ inline int lane_rank(uint64_t m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Wave-aggregated claim of one slot per pending lane in the counter of its
// target segment: one atomic per distinct target in the wave.
__device__ inline int claim_slot(PIC_GLOBAL int32_t *cnt, int target, bool pending)
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
            slot = base + lane_rank(mm);
            pending = false;
        }
    }
    return slot;
}

// Element i of a particle array as a 32-bit byte offset from the array's
// (wave-uniform) base: slot counts stay below 2^29, so the offset fits and the
// access is one scalar base plus one vector offset.
template <typename T>
__device__ inline PIC_GLOBAL T &slot_ref(PIC_GLOBAL T *base, int i)
{
    return *reinterpret_cast<PIC_GLOBAL T *>(reinterpret_cast<PIC_GLOBAL char *>(base) +
                                             (uint32_t)i * (uint32_t)sizeof(T));
}

// Store a particle at slot `at` of copy P.  wide: the slot is in the overflow
// region or stages a leaver, and takes the packed cell; otherwise it is in
// the ranges of the cell's tile and takes the tile-local code.
template <typename R>
__device__ inline void write_particle(const PBuf<R> &P, int at, bool wide, int32_t cell, int code, const R d[3],
                                      const R u[3], int32_t id)
{
    if (wide) slot_ref(P.cell, at) = cell;
    else slot_ref(P.lc, at) = (uint8_t)code;
    slot_ref(P.d[0], at) = d[0]; slot_ref(P.d[1], at) = d[1]; slot_ref(P.d[2], at) = d[2];
    slot_ref(P.u[0], at) = u[0]; slot_ref(P.u[1], at) = u[1]; slot_ref(P.u[2], at) = u[2];
    if (P.id) slot_ref(P.id, at) = id;
}

// Slot of copy `dst` for position `pos` of the B range of tile `tgt`, or of the
// overflow region when the segment is full; -1 (and the LOST flag) when both are.
template <typename R>
__device__ inline int b_range_slot(const BoxDev<R> &B, const SpeciesDev<R> &S, int dst, int tgt, int pos,
                                   PIC_GLOBAL uint32_t *flags)
{
    if (pos < S.seg_cap[dst][tgt]) return S.seg_start[dst][tgt] + pos;
    const int o = atomicAdd(&S.nb[dst][B.ntiles], 1);
    if (o >= S.ovf_cap) {
        atomicOr(flags, PIC_FLAG_LOST);
        return -1;
    }
    return S.seg_start[dst][B.ntiles] + o;
}

// Store a particle into the B range of tile `tgt` of copy `dst` (or the
// overflow region); slots are claimed with one atomic per distinct target in
// the wave.  Every lane of the wave must call it.
template <typename R>
__device__ inline void store_particle(const BoxDev<R> &B, const SpeciesDev<R> &S, int dst, int tgt, bool valid,
                                      int32_t cell, const R d[3], const R u[3], int32_t id,
                                      PIC_GLOBAL uint32_t *flags)
{
    const int slot = claim_slot(S.nb[dst], tgt, valid);
    if (!valid) return;
    const int at = b_range_slot(B, S, dst, tgt, S.bs[dst][tgt] + slot, flags);
    if (at >= 0) write_particle(S.buf[dst], at, at >= S.slots - S.ovf_cap, cell, local_code(B, cell), d, u, id);
}

// The particles of tile T in copy c: the A range then the clamped B range.
struct TileRanges {
    int start, na, bs, n;
    __device__ int slot(int q) const { return start + (q < na ? q : bs + (q - na)); }
};

template <typename R>
__device__ inline TileRanges tile_ranges(const SpeciesDev<R> &S, int c, int T)
{
    TileRanges r;
    r.start = S.seg_start[c][T];
    r.na = S.na[c][T];
    r.bs = S.bs[c][T];
    r.n = r.na + max(0, min(S.nb[c][T], S.seg_cap[c][T] - r.bs));
    return r;
}

// The overflow region of copy c as a range.
template <typename R>
__device__ inline TileRanges overflow_range(const BoxDev<R> &B, const SpeciesDev<R> &S, int c)
{
    TileRanges r;
    r.start = S.seg_start[c][B.ntiles];
    r.na = min(S.nb[c][B.ntiles], S.ovf_cap);
    r.bs = 0;
    r.n = r.na;
    return r;
}

// Offset of x in its cell, x - floor(x), kept below 1: an x a hair below a
// node plane, whose difference would round up to 1, stays in the lower cell
// at the largest offset below 1 (one v_fract_f32, which clamps so).
__device__ inline float offset_in_cell(float x) { return __builtin_amdgcn_fractf(x); }
__device__ inline double offset_in_cell(double x) { return fmin(x - floor(x), 1.0 - 0x1p-53); }

// New cell and offset after the move x1 = d + D (home-cell frame), wrapped.
template <typename R>
__device__ inline int32_t advance_cell(const BoxDev<R> &B, int ix, int iy, int iz, const R x1[3], R dn[3])
{
    int c[3] = {ix, iy, iz};
    for (int a = 0; a < 3; ++a) {
        const int f = (int)floor(x1[a]);      // -1, 0 or 1: x1 lies in (-1, 2)
        dn[a] = offset_in_cell(x1[a]);
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

// Geometry of tile T.  The LDS regions are laid out for the full tile shape
// (1 << tshift per axis; ext only limits which cells hold particles), so with
// FIX = 1 (every tile 4x4x4) all their strides are compile-time constants.
template <typename R, int FIX = 0>
__device__ inline TileGeom<R> tile_geom(const BoxDev<R> &B, int T)
{
    TileGeom<R> g;
    const int sx = FIX ? 2 : B.tshift[0], sy = FIX ? 2 : B.tshift[1], sz = FIX ? 2 : B.tshift[2];
    const int tx = T % B.ntile[0];
    const int r = T / B.ntile[0];
    const int ty = r % B.ntile[1], tz = r / B.ntile[1];
    g.o[0] = tx << sx;
    g.o[1] = ty << sy;
    g.o[2] = tz << sz;
    const int t0 = 1 << sx, t1 = 1 << sy, t2 = 1 << sz;
    g.ext[0] = min(t0, B.n[0] - g.o[0]);
    g.ext[1] = min(t1, B.n[1] - g.o[1]);
    g.ext[2] = min(t2, B.n[2] - g.o[2]);
    g.NX = t0 + 1; g.NY = t1 + 1; g.NN = g.NX * g.NY * (t2 + 1);
    g.JX = t0 + 3; g.JY = t1 + 3; g.JN = g.JX * g.JY * (t2 + 3);
    g.BX = t0 + 2; g.BY = t1 + 2; g.BN = g.BX * g.BY * (t2 + 2);
    return g;
}

// Per-wave queue of unfinished moves (LDS ring buffer): a move that crosses
// node planes deposits its first piece at once and waits here for the rest;
// the wave deposits the next piece of 64 queued moves at a time and puts back
// those that still have pieces left.  An entry holds the start of the next
// piece and the end of the move (home-cell frame), the LDS index of the home
// cell with the species sign, and the meta word of the move (move_meta).
// FP32 form: two waves' worth of entries, so that a put after a drain always
// fits.  FP64 form: one wave's worth (a wave drains before a put that would
// not fit), which keeps a 4x4x4 block within the LDS of three blocks per CU.
template <typename R> struct QCap { static constexpr int value = 128; };
template <> struct QCap<double> { static constexpr int value = 64; };
constexpr int kWaves = kBlock / 64;

template <typename R>
__host__ __device__ inline size_t queue_bytes()
{
    return (size_t)kWaves * QCap<R>::value * (2 * sizeof(int32_t) + 6 * sizeof(R));
}

// Bytes of dynamic LDS for a tile with edges (t0, t1, t2): the trilinear
// coefficients of every cell (48 values), the piece queues, then a region that
// first holds the staged raw fields and node fields and then the tile current.
// Values per cell in the gather's coefficient table: 8 per field component,
// padded from 48 to 52 so that the 16-byte reads of lanes in different cells
// start on different LDS banks.  (A coefficient-major table, one dword per
// lane per read, ran the push 43 % slower.)
constexpr int kCoef = 52;

// LDS of one push block for tiles of t0 x t1 x t2 cells, three regions:
//   [coef]   the gather's coefficient table (kCoef values per cell);
//   [stage]  the piece queues during the particle loop, the staged raw e and
//            b (tile plus halo) during set-up;
//   [union]  the node fields during set-up, the tile current afterwards.
struct TileLds {
    size_t coef, stage, uni;
    __host__ __device__ size_t total() const { return coef + stage + uni; }
};

template <typename R>
__host__ __device__ inline TileLds tile_lds(int t0, int t1, int t2)
{
    const size_t nc = (size_t)t0 * t1 * t2;
    const size_t nn = (size_t)(t0 + 1) * (t1 + 1) * (t2 + 1);
    const size_t jn = (size_t)(t0 + 3) * (t1 + 3) * (t2 + 3);
    const size_t bn = (size_t)(t0 + 2) * (t1 + 2) * (t2 + 2);
    const size_t raw = 3 * (jn + bn) * sizeof(R), q = queue_bytes<R>();
    const size_t nodes = 6 * nn * sizeof(R), jb = 3 * jn * sizeof(typename JType<R>::T);
    TileLds L;
    L.coef = (nc * kCoef * sizeof(R) + 15) & ~size_t(15);
    L.stage = ((raw > q ? raw : q) + 15) & ~size_t(15);
    L.uni = ((nodes > jb ? nodes : jb) + 15) & ~size_t(15);
    return L;
}

template <typename R>
__host__ __device__ inline size_t tile_lds_bytes(int t0, int t1, int t2)
{
    return tile_lds<R>(t0, t1, t2).total();
}

// q / m for 0 <= q < 4096 and 1 <= m <= 16, with mul = 65536 / m + 1: the
// rounding error q (mul - 65536/m) / 65536 < 1/16 never reaches the next
// integer because q/m is at least 1/m below it.
__device__ inline int div_small(int q, int mul) { return (int)(__umul24((unsigned)q, (unsigned)mul) >> 16); }

// v wrapped into [0, n) for v in [-n, 2n) (one correction step)
__device__ inline int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// The twelve fluxes of one piece (start offset s in its cell, displacement
// dd), eq. current_dep (App. A.3.4) with the sign and scale of the species,
// rounded to the fixed-point current: per component a, the four faces around
// the cell's a-edge, f = 0 at the cell, 1 one step along b2, 2 one step along
// b1, 3 both (b1, b2 the two other axes in cyclic order).  With
// m = s + dd/2 and K = dd_b1 dd_b2 / 12 the weights are (1-m1)(1-m2)+K,
// (1-m1)m2-K, m1(1-m2)-K and m1 m2+K; they sum to one, so the f = 0 value is
// the rounded total minus the other three rounded values, and a piece moves
// exactly its charge.  add(a, f, q) receives each rounded value.
template <typename R, typename Add>
__device__ inline void piece_fluxes(const R s[3], const R dd[3], R scale, Add &&add)
{
    const R m[3] = {s[0] + R(0.5) * dd[0], s[1] + R(0.5) * dd[1], s[2] + R(0.5) * dd[2]};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int b1 = a == 2 ? 0 : a + 1, b2 = a == 0 ? 2 : a - 1;
        const R PK = m[b1] * m[b2] + dd[b1] * dd[b2] * R(1.0 / 12.0);
        const R F = scale * dd[a];
        const R t11 = F * PK, t01 = fma(F, m[b2], -t11), t10 = fma(F, m[b1], -t11);
        const auto q11 = quantize(t11), q01 = quantize(t01), q10 = quantize(t10);
        const auto q00 = quantize(F) - q01 - q10 - q11;
        add(a, 0, q00);
        add(a, 1, q01);
        add(a, 2, q10);
        add(a, 3, q11);
    }
}

// The fluxes of one piece added to the LDS tile current at jl[cb + off[a][f]].
template <typename R>
__device__ inline void deposit_piece(typename JType<R>::T *jl, int cb, const int (&off)[3][4], const R s[3],
                                     const R dd[3], R scale)
{
    piece_fluxes(s, dd, scale, [&](int a, int f, auto q) { atomic_add_lds(&jl[cb + off[a][f]], q); });
}

template <typename R>
__device__ inline R sel3(int i, R a0, R a1, R a2) { return i == 0 ? a0 : (i == 1 ? a1 : a2); }

// Node planes crossed by the move d -> x1 = d + D in the home-cell frame
// (|D| < 1: at most one per axis): direction per axis and the crossing
// parameter lambda in (0, 1] (2 where no plane is crossed).
template <typename R>
__device__ inline void move_crossings(const R d[3], const R D[3], R x1[3], int dir[3], R lam[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        x1[a] = d[a] + D[a];
        dir[a] = (int)floor(x1[a]);       // -1, 0 or 1, since x1 lies in (-1, 2)
        lam[a] = dir[a] != 0 ? ((dir[a] > 0 ? R(1) : R(0)) - d[a]) * fast_rcp(D[a]) : R(2);
    }
}

// Conducting wall on axis w (App. A.4): when the move d -> d + D (home-cell
// frame; cw = home cell index along w, nw = cells along w) leaves the box
// through a wall, the move is cut where it meets the wall: D1 takes it there,
// P = d + D1 is that point as the deposit computes it, D2 takes the rest
// mirrored back into the box along w, and u_w changes sign.  Returns whether
// the move hit the wall.
template <typename R>
__device__ inline bool wall_hit(int w, int cw, int nw, const R d[3], const R D[3], R D1[3], R P[3], R D2[3],
                                R u[3])
{
    const R xw = d[w] + D[w];
    const bool lo = cw == 0 && xw < R(0), hi = cw == nw - 1 && xw >= R(1);
    if (!lo && !hi) return false;
    const R plane = hi ? R(1) : R(0);
    const R l = (plane - d[w]) / D[w];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        D1[a] = a == w ? plane - d[w] : l * D[a];
        asm volatile("" : "+v"(D1[a]));
        P[a] = d[a] + D1[a];
    }
    R xr = R(2) * plane - xw;                    // the mirrored end along w
    if (xr >= R(1)) xr = R(1) - R(1) / R(1 << 23);  // a move ending exactly on the upper wall
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        D2[a] = (a == w ? xr : d[a] + D[a]) - P[a];
        asm volatile("" : "+v"(D2[a]));
    }
    u[w] = -u[w];
    return true;
}

// The mirrored rest of a wall move starts at P (home-cell frame), which lies
// in a neighbouring cell along each other axis that the first piece crossed.
// Rebase it onto that cell: s = the cell's offset from the home cell (0 along
// the wall axis, where P is on a face of the home cell), P in [0, 1) of it.
template <typename R>
__device__ inline void wall_rest_start(int w, R P[3], int s[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        s[a] = a == w ? 0 : (P[a] < R(0) ? -1 : (P[a] >= R(1) ? 1 : 0));
        R v = P[a] - R(s[a]);
        if (v >= R(1)) v = R(1) - R(0.5) * std::numeric_limits<R>::epsilon();   // -tiny + 1 rounded up
        if (a != w) P[a] = v;
    }
}

__device__ inline float clamp01(float v) { return __builtin_amdgcn_fmed3f(v, 0.0f, 1.0f); }
__device__ inline double clamp01(double v) { return fmin(fmax(v, 0.0), 1.0); }

// First breakpoint of a move d -> d + D: where its first crossing axis ax
// meets its plane (parameter l).  That coordinate is the plane itself; no
// other plane is crossed before it, so every other coordinate lies in the
// closed home cell [0, 1] (clamped there against rounding).  A plane crossed
// at the same parameter is left at the plane: its own piece then has length
// zero.
template <typename R>
__device__ inline void first_breakpoint(const R d[3], const R D[3], const int dir[3], int ax, R l, R q[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const R c = clamp01(fma(l, D[a], d[a]));
        q[a] = a == ax ? (dir[a] > 0 ? R(1) : R(0)) : c;
    }
}

// Meta word of a queued move: next piece k (bits 0-1), crossings nb (2-3),
// the crossing axes in order o0, o1, o2 (4-9), and per axis the crossing
// direction + 1 (10-15).
__device__ inline int move_meta(int k, int nb, int o0, int o1, int o2, const int dir[3])
{
    return k | (nb << 2) | (o0 << 4) | (o1 << 6) | (o2 << 8) | ((dir[0] + 1) << 10) | ((dir[1] + 1) << 12) |
           ((dir[2] + 1) << 14);
}

// Piece k of a queued move (0 <= k <= nb crossings), from its start ps (the
// previous breakpoint; home-cell frame) towards the move's end x1.  The piece
// lies in the cell offset `offc` from the home cell: the directions of the
// crossings before it (axes o_0 .. o_{k-1} of the meta word).  Its end pe is
// x1 for the last piece; otherwise the point where axis o_k meets its plane,
// reached along the rest of the move, with every other coordinate clamped
// into the piece's cell (against rounding).  Every later breakpoint of a
// move is computed this way from the one before, on the tile path and on
// the HBM path alike, so consecutive pieces share their breakpoints exactly
// and the last piece ends exactly at the particle's new position.  Returns
// the piece's start in its cell (sv) and displacement (dd).
template <typename R>
__device__ inline void chain_piece(const R ps[3], const R x1[3], int meta, int k, R pe[3], int offc[3], R sv[3],
                                   R dd[3])
{
    const int nb = (meta >> 2) & 3;
    int crossed = 0;
    if (k > 0) crossed |= 1 << ((meta >> 4) & 3);
    if (k > 1) crossed |= 1 << ((meta >> 6) & 3);
    if (k > 2) crossed |= 1 << ((meta >> 8) & 3);
#pragma unroll
    for (int a = 0; a < 3; ++a) offc[a] = (crossed >> a) & 1 ? ((meta >> (10 + 2 * a)) & 3) - 1 : 0;
    if (k < nb) {
        const int ax = (meta >> (4 + 2 * k)) & 3;
        const R Dp[3] = {x1[0] - ps[0], x1[1] - ps[1], x1[2] - ps[2]};
        const R plane = ((meta >> (10 + 2 * ax)) & 3) == 2 ? R(1) : R(0);
        // the parameter of the crossing along the rest of the move; a rest
        // that no longer moves along the axis (0 * inf) gives 0
        R l = (plane - sel3(ax, ps[0], ps[1], ps[2])) * fast_rcp(sel3(ax, Dp[0], Dp[1], Dp[2]));
        l = fmin(fmax(l, R(0)), R(1));
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const R lo = R(offc[a]);
            const R v = fmin(fmax(fma(l, Dp[a], ps[a]), lo), lo + R(1));
            pe[a] = a == ax ? plane : v;
        }
    } else {
        pe[0] = x1[0]; pe[1] = x1[1]; pe[2] = x1[2];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        sv[a] = ps[a] - R(offc[a]);
        dd[a] = pe[a] - ps[a];
    }
}

// The pieces k, k+1, ..., nb of a queued move, from breakpoint ps to the
// move's end x1 (see chain_piece), as the queue deposits them.
// add(a, ox, oy, oz, q): rounded flux q of component a at node (cell + o).
template <typename R, typename Add>
__device__ inline void deposit_chain(const R ps0[3], const R x1[3], int meta, int k, R scale, Add &&add)
{
    const int nb = (meta >> 2) & 3;
    R ps[3] = {ps0[0], ps0[1], ps0[2]};
    for (; k <= nb; ++k) {
        R pe[3], sv[3], dd[3];
        int offc[3];
        chain_piece(ps, x1, meta, k, pe, offc, sv, dd);
        piece_fluxes(sv, dd, scale, [&](int a, int f, auto q) {
            const int b1 = a == 2 ? 0 : a + 1, b2 = a == 0 ? 2 : a - 1;
            int o[3] = {offc[0], offc[1], offc[2]};
            if (f & 1) o[b2] += 1;
            if (f & 2) o[b1] += 1;
            add(a, o[0], o[1], o[2], q);
        });
        ps[0] = pe[0]; ps[1] = pe[1]; ps[2] = pe[2];
    }
}

// Crossings of the move d -> d + D, their order and the meta word (next piece
// k), as the push computes them.
template <typename R>
__device__ inline int move_order(const R d[3], const R D[3], int k, R x1[3], int dir[3], R lam[3], int &o0,
                                 R &l0)
{
    move_crossings(d, D, x1, dir, lam);
    const int nb = (dir[0] != 0) + (dir[1] != 0) + (dir[2] != 0);
    int q0 = 0, q1 = 1, q2 = 2;
    R m0 = lam[0], m1 = lam[1], m2 = lam[2];
    if (m1 < m0) { R t = m0; m0 = m1; m1 = t; int q = q0; q0 = q1; q1 = q; }
    if (m2 < m1) { R t = m1; m1 = m2; m2 = t; int q = q1; q1 = q2; q2 = q; }
    if (m1 < m0) { R t = m0; m0 = m1; m1 = t; int q = q0; q0 = q1; q1 = q; }
    o0 = q0;
    l0 = m0;
    return move_meta(k, nb, q0, q1, q2, dir);
}

// Charge-conserving deposit of the straight move d -> d + D from the start
// cell (d in [0,1)^3, |D| < 1), for the particles that take the HBM path.
// READING (the paper defers cell-crossing moves to references not given): the
// move is cut at each node plane it crosses, in order of the crossing
// parameter, and each piece deposits its fluxes (eq. current_dep, App. A.3.4)
// in its own cell.  The first breakpoint comes from d and the crossing
// parameter, the later ones from chain_piece, the fluxes from piece_fluxes:
// exactly as the tile path computes them (its first piece at once, the
// others from the queue), so a move deposits the same integers whichever
// path it takes.  add(a, ox, oy, oz, q): rounded flux q of component a at
// node (start cell + o).
template <typename R, typename Add>
__device__ inline void deposit_move(const R d[3], const R D[3], R scale, Add &&add)
{
    R x1[3], lam[3], l0;
    int dir[3], o0;
    const int meta = move_order(d, D, 1, x1, dir, lam, o0, l0);
    const int nb = (meta >> 2) & 3;
    R p1[3];
    if (nb == 0) {
        p1[0] = x1[0]; p1[1] = x1[1]; p1[2] = x1[2];
    } else {
        first_breakpoint(d, D, dir, o0, l0, p1);
    }
    const R dd[3] = {p1[0] - d[0], p1[1] - d[1], p1[2] - d[2]};
    piece_fluxes(d, dd, scale, [&](int a, int f, auto q) {
        const int b1 = a == 2 ? 0 : a + 1, b2 = a == 0 ? 2 : a - 1;
        int o[3] = {0, 0, 0};
        if (f & 1) o[b2] += 1;
        if (f & 2) o[b1] += 1;
        add(a, o[0], o[1], o[2], q);
    });
    if (nb > 0) deposit_chain(p1, x1, meta, 1, scale, add);
}

// The whole move d -> d + D as one chain from its start (the mirrored rest of
// a move through a conducting wall, queued from its first piece).
template <typename R, typename Add>
__device__ inline void deposit_rest(const R d[3], const R D[3], R scale, Add &&add)
{
    R x1[3], lam[3], l0;
    int dir[3], o0;
    const int meta = move_order(d, D, 0, x1, dir, lam, o0, l0);
    deposit_chain(d, x1, meta, 0, scale, add);
}

// The Boris step, the non-finite check and the displacement D = dt u / gamma
// of the move, shared by the tile and HBM paths.  D stays the rounded product
// (opaque to the compiler, so that no multiply-add fuses it into d + D): the
// move's end x1 = d + D and its crossings must come out identical wherever
// they are computed.
template <typename R>
__device__ inline void boris_move(R hk, const R E[3], const R Bf[3], R u[3], R dt, bool valid,
                                  PIC_GLOBAL uint32_t *flags, R D[3])
{
    boris(hk, E, Bf, u);
    // one test catches NaN and infinity (and |u| beyond 1e15)
    R u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const bool bad = !(u2 < R(1e30));
    if (__builtin_expect(__ballot(bad) != 0, 0)) {     // wave-uniform: the fix-up costs nothing otherwise
        if (bad) {
            if (valid) atomicOr(flags, PIC_FLAG_NONFINITE);
            u[0] = u[1] = u[2] = R(0);
            u2 = R(0);
        }
    }
    const R ig = dt * fast_rsqrt(R(1) + u2);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        D[a] = ig * u[a];
        asm volatile("" : "+v"(D[a]));
    }
}

// Tile one step away from tile T in direction code = (dx+1) + 3(dy+1) + 9(dz+1).
template <typename R>
__device__ inline int neighbor_tile(const BoxDev<R> &B, const TileGeom<R> &g, int code)
{
    int t = 0, mul = 1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int dl = code % 3 - 1;
        code /= 3;
        int ta = (g.o[a] >> B.tshift[a]) + dl;
        ta = ta < 0 ? ta + B.ntile[a] : (ta >= B.ntile[a] ? ta - B.ntile[a] : ta);
        t += ta * mul;
        mul *= B.ntile[a];
    }
    return t;
}

// Cells just outside tile g along each axis (wrapped into the box).
struct TileRim {
    int lo[3], hi[3];
};

template <typename R>
__device__ inline TileRim tile_rim(const BoxDev<R> &B, const TileGeom<R> &g)
{
    TileRim r;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r.lo[a] = g.o[a] == 0 ? B.n[a] - 1 : g.o[a] - 1;
        r.hi[a] = g.o[a] + g.ext[a] == B.n[a] ? 0 : g.o[a] + g.ext[a];
    }
    return r;
}

// Direction code of a particle in cell c relative to tile g: 13 if it is
// inside g, (dx+1) + 3(dy+1) + 9(dz+1) for a cell in the layer around g (the
// adjacent tile in that direction is then the particle's tile, since a cell
// one step outside a tile lies in the next tile along that axis), or -1
// otherwise.  A pure function of the stored cell, so that the push and the
// hand-over of the leavers classify a particle the same way.
template <typename R>
__device__ inline int move_bin(const TileGeom<R> &g, const TileRim &rim, const int c[3])
{
    int code = 0, mul = 1;
    bool bad = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int dl = (unsigned)(c[a] - g.o[a]) < (unsigned)g.ext[a] ? 0
                       : (c[a] == rim.lo[a] ? -1 : (c[a] == rim.hi[a] ? 1 : 2));
        bad |= dl == 2;
        code += (dl + 1) * mul;
        mul *= 3;
    }
    return bad ? -1 : code;
}

template <typename R> struct PushWaves { static constexpr int value = 4; };
template <> struct PushWaves<double> { static constexpr int value = 3; };

template <typename R, int FIX, int WALLS, int F4>
__global__ void __launch_bounds__(kBlock, PushWaves<R>::value) push_kernel(const BoxDev<R> *__restrict__ boxes,
                                                      const Item *__restrict__ items, StepConst<R> C);

// Overflow sweep: same physics, fields from HBM, current by global atomics.
template <typename R, int WALLS, int F4>
__device__ void push_overflow(const BoxDev<R> &B, int kblk, const StepConst<R> &C)
{
    using JT = typename JType<R>::T;
    const R hdt = R(0.5) * C.dt;
    for (int s = 0; s < C.nsp; ++s) {
        const SpeciesDev<R> &S = B.sp[s];
        const TileRanges rg = overflow_range(B, S, C.cur);
        const int n = rg.n;
        const int start = rg.start;
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
            if (valid) gather_global<R, F4>(B, ix, iy, iz, d, hdt, E, Bf);
            else for (int a = 0; a < 3; ++a) { E[a] = R(0); Bf[a] = R(0); }
            R D[3];
            boris_move(hk, E, Bf, u, C.dt, valid, C.flags, D);
            // a move through a conducting wall (App. A.4): deposit up to the
            // wall, then the mirrored rest; the particle ends at P2 + D2
            R D1[3], P2[3], D2[3];
            const bool hitw = WALLS && B.wall >= 0 && valid &&
                              wall_hit(B.wall, B.wall == 0 ? ix : (B.wall == 1 ? iy : iz), B.n[B.wall], d, D, D1, P2,
                                       D2, u);
            if (valid) {
                JT *J = B.J;
                auto put_j = [&](int a, int ox, int oy, int oz, JT q) {
                    if (q == JT(0)) return;
                    const int i = wrap_idx(ix + ox, B.n[0]), j = wrap_idx(iy + oy, B.n[1]),
                              k = wrap_idx(iz + oz, B.n[2]);
                    atomic_add_global(&J[a * B.nc + i + (int64_t)B.n[0] * (j + (int64_t)B.n[1] * k)], q);
                };
                if (hitw) {
                    deposit_move(d, D1, scale, put_j);
                    R Q2[3] = {P2[0], P2[1], P2[2]};
                    int s2[3];
                    wall_rest_start(B.wall, Q2, s2);
                    deposit_rest(Q2, D2, scale, [&](int a, int ox, int oy, int oz, JT q) {
                        put_j(a, s2[0] + ox, s2[1] + oy, s2[2] + oz, q);
                    });
                } else {
                    deposit_move(d, D, scale, put_j);
                }
            }
            R x1[3] = {d[0] + D[0], d[1] + D[1], d[2] + D[2]}, dn[3];
            if (hitw)
                for (int a = 0; a < 3; ++a) x1[a] = P2[a] + D2[a];
            const int32_t nc = advance_cell(B, ix, iy, iz, x1, dn);
            store_particle(B, S, C.cur ^ 1, tile_of(B, nc), valid, nc, dn, u, id, C.flags);
        }
    }
}

// FP32 form: four waves per SIMD (at most 128 VGPRs), the occupancy that
// hides the latency of the LDS gather and of the particle loads best on
// gfx950.  FP64 form: three (at most 168 VGPRs; with its 64-entry queues a
// 4x4x4 block's LDS allows three blocks per CU as well).
template <typename R, int FIX, int WALLS, int F4>
__global__ void __launch_bounds__(kBlock, PushWaves<R>::value) push_kernel(const BoxDev<R> *__restrict__ boxes,
                                                      const Item *__restrict__ items, StepConst<R> C)
{
    using JT = typename JType<R>::T;
    extern __shared__ __align__(16) unsigned char smem[];
    const Item it = items[blockIdx.x];
    if (it.box < 0) return;                       // padding of the push order
    const BoxDev<R> &B = boxes[it.box];
    if (it.tile < 0) {
        push_overflow<R, WALLS, F4>(B, -1 - it.tile, C);
        return;
    }
    const int T = it.tile;
    const int tid = threadIdx.x;
    const TileGeom<R> g = tile_geom<R, FIX>(B, T);
    const TileRim rim = tile_rim(B, g);
    // per axis: box edge length, whether the tile touches the box edge (only
    // then can a move wrap), and whether one tile spans the box
    int bn[3];
    bool edge[3], span[3];
    bool fastbin = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        bn[a] = B.n[a];
        edge[a] = g.o[a] == 0 || g.o[a] + g.ext[a] >= bn[a];
        span[a] = B.ntile[a] == 1;
        // with two tiles along an axis the cells on both sides of a tile are
        // the same cells, and a partial tile at the box's far end has its
        // own extent: move_bin's rule decides there
        fastbin &= B.ntile[a] != 2 && g.ext[a] == 4;
    }
    // LDS: per-cell trilinear coefficients | piece queues | union of {raw e,
    // raw b, node fields} (set-up) and the tile current (particle loop)
    const int tsx = FIX ? 2 : B.tshift[0], tsxy = FIX ? 4 : B.tshift[0] + B.tshift[1];
    const int tsz = FIX ? 2 : B.tshift[2];
    const TileLds lds = FIX ? tile_lds<R>(4, 4, 4) : tile_lds<R>(1 << B.tshift[0], 1 << B.tshift[1], 1 << B.tshift[2]);
    R *coef = reinterpret_cast<R *>(smem);
    unsigned char *qmem = smem + lds.coef;
    unsigned char *uni = qmem + lds.stage;
    R *re = reinterpret_cast<R *>(qmem);          // raw e, 3 x JN, origin o-1 (set-up)
    R *rb = re + 3 * g.JN;                        // raw b, 3 x BN, origin o-1 (set-up)
    R *node = reinterpret_cast<R *>(uni);         // node fields, 6 x NN, origin o (set-up)
    JT *jl = reinterpret_cast<JT *>(uni);         // J, 3 x JN, origin o-1 (particle loop)

    // re-binning counters: per species the stayers (from the front of the
    // tile's new A range), the leavers (staged from the back) and the leavers
    // per neighbour direction
    __shared__ int sh_front[kMaxSpecies], sh_back[kMaxSpecies];
    __shared__ int sh_bin[kMaxSpecies][27], sh_base[kMaxSpecies][27];
    // hand-over targets per (species, direction): first slot of the claimed
    // part of the target tile's segment, and the segment's end
    __shared__ int sh_tseg[kMaxSpecies][27], sh_tend[kMaxSpecies][27];
    // hand-over sources per species: the arrays of copy cur^1, and the slot
    // of leaver q of the block's combined leaver range is q + sh_loff[s]
    __shared__ PBuf<R> sh_q[kMaxSpecies];
    __shared__ int sh_loff[kMaxSpecies], sh_lend[kMaxSpecies];
    // per species the tile's ranges in copy cur (start, na, bs, n) and its
    // segment start in copy cur^1, read here, while the fields are staged,
    // instead of at the start of each species' loop and in the hand-over
    __shared__ int sh_rng[kMaxSpecies][5];
    if (tid < kMaxSpecies) {
        sh_front[tid] = 0;
        sh_back[tid] = 0;
    }
    if (tid < kMaxSpecies * 27) (&sh_bin[0][0])[tid] = 0;
    if (tid < C.nsp) {
        const TileRanges r = tile_ranges(B.sp[tid], C.cur, T);
        sh_rng[tid][0] = r.start;
        sh_rng[tid][1] = r.na;
        sh_rng[tid][2] = r.bs;
        sh_rng[tid][3] = r.n;
        sh_rng[tid][4] = B.sp[tid].seg_start[C.cur ^ 1][T];
    }

    // region indices are decoded by multiply-shift (edges of at most 11 and
    // fewer than 2^11 points: exact)
    const int mJX = 65536 / g.JX + 1, mJY = 65536 / g.JY + 1;
    const int mBX = 65536 / g.BX + 1, mBY = 65536 / g.BY + 1;
    const int mNX = 65536 / g.NX + 1, mNY = 65536 / g.NY + 1;
    const int JX = g.JX, JXY = g.JX * g.JY, BX = g.BX, BXY = g.BX * g.BY;
    const int NX = g.NX, NXY = g.NX * g.NY;
    const int64_t n0 = B.n[0], n01 = (int64_t)B.n[0] * B.n[1];
    // grid index of the point (o-1) + (i,j,k), wrapped periodically
    auto gidx = [&](int i, int j, int k) -> int64_t {
        const int gi = wrap1(g.o[0] - 1 + i, B.n[0]), gj = wrap1(g.o[1] - 1 + j, B.n[1]),
                  gk = wrap1(g.o[2] - 1 + k, B.n[2]);
        if ((unsigned)gi >= (unsigned)B.n[0] || (unsigned)gj >= (unsigned)B.n[1] ||
            (unsigned)gk >= (unsigned)B.n[2])   // boxes narrower than the halo
            return wrap_idx(g.o[0] - 1 + i, B.n[0]) + n0 * wrap_idx(g.o[1] - 1 + j, B.n[1]) +
                   n01 * wrap_idx(g.o[2] - 1 + k, B.n[2]);
        return gi + n0 * gj + n01 * gk;
    };

    // 1. stage e^t and b^{t-dt/2} of the tile and its halo
    for (int q = tid; q < g.JN; q += kBlock) {
        const int jk = div_small(q, mJX), i = q - jk * JX;
        const int k = div_small(jk, mJY), j = jk - k * g.JY;
        const int64_t gp = gidx(i, j, k);
#pragma unroll
        for (int c = 0; c < 3; ++c) re[c * g.JN + q] = B.e[c * B.nc + gp];
    }
    for (int q = tid; q < g.BN; q += kBlock) {
        const int jk = div_small(q, mBX), i = q - jk * BX;
        const int k = div_small(jk, mBY), j = jk - k * g.BY;
        const int64_t gp = gidx(i, j, k);
#pragma unroll
        for (int c = 0; c < 3; ++c) rb[c * g.BN + q] = B.b[c * B.nc + gp];
    }
    __syncthreads();

    // the particle loops load each lane's next particle one iteration ahead
    // (lanes past the end load the tile's last particle again and are masked
    // out of every store, claim and deposit by `valid`); the first particle
    // of species 0 is loaded here, so that its HBM latency is covered by the
    // rest of the set-up
    int32_t nx_code = 0, nx_id = 0;
    R nx_d[3] = {R(0.5), R(0.5), R(0.5)}, nx_u[3] = {R(0), R(0), R(0)};
    auto fetch_particle = [&](const PBuf<R> &P, const TileRanges &src, int q) {
        const int at = src.slot(min(q, src.n - 1));
        nx_code = slot_ref(P.lc, at);
        nx_d[0] = slot_ref(P.d[0], at); nx_d[1] = slot_ref(P.d[1], at); nx_d[2] = slot_ref(P.d[2], at);
        nx_u[0] = slot_ref(P.u[0], at); nx_u[1] = slot_ref(P.u[1], at); nx_u[2] = slot_ref(P.u[2], at);
        if (P.id) nx_id = slot_ref(P.id, at);
    };
    auto ranges = [&](int s) {
        TileRanges r;
        r.start = __builtin_amdgcn_readfirstlane(sh_rng[s][0]);
        r.na = __builtin_amdgcn_readfirstlane(sh_rng[s][1]);
        r.bs = __builtin_amdgcn_readfirstlane(sh_rng[s][2]);
        r.n = __builtin_amdgcn_readfirstlane(sh_rng[s][3]);
        return r;
    };
    {
        const TileRanges r0 = ranges(0);
        if (r0.n > 0) fetch_particle(B.sp[0].buf[C.cur], r0, tid);
    }

    // 2. b^t = b^{t-dt/2} - (dt/2) curl e^t (App. A.3.1 item 1), in place;
    //    and for the tile's own cells the full step b^{t+dt/2} = b^{t-dt/2} -
    //    dt curl e^t (App. A.3.1 items 1 and 4 together), written to the other
    //    b buffer, so that no separate b update is launched: every cell
    //    belongs to one tile, and no block reads that buffer in this launch
    const R hdt = R(0.5) * C.dt;
    // raw-b point (i, j, k) is a cell of this tile
    auto own = [&](int i, int j, int k) {
        return (unsigned)(i - 1) < (unsigned)g.ext[0] && (unsigned)(j - 1) < (unsigned)g.ext[1] &&
               (unsigned)(k - 1) < (unsigned)g.ext[2];
    };
    // the new b of own raw-b point (i, j, k), the normal component zero on a
    // conducting wall (App. A.4)
    auto put_b = [&](int i, int j, int k, const R bnew[3]) {
        const int gi = g.o[0] - 1 + i, gj = g.o[1] - 1 + j, gk = g.o[2] - 1 + k;
        const int64_t gp = gi + n0 * gj + n01 * gk;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const bool wall0 = WALLS && B.wall == c && (c == 0 ? gi : (c == 1 ? gj : gk)) == 0;
            B.bn[c * B.nc + gp] = wall0 ? R(0) : bnew[c];
        }
    };
    if (F4) {
        // the fourth-order curl reaches two cells out, past the staged halo:
        // b^t from HBM, exactly as the HBM path forms it
        for (int q = tid; q < g.BN; q += kBlock) {
            const int jk = div_small(q, mBX), i = q - jk * BX;
            const int k = div_small(jk, mBY), j = jk - k * g.BY;
            const int gi = g.o[0] - 1 + i, gj = g.o[1] - 1 + j, gk = g.o[2] - 1 + k;
            if (own(i, j, k)) {
                R bnew[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const R cu = curl4_e(B, c, gi, gj, gk);
                    bnew[c] = rb[c * g.BN + q] - C.dt * cu;
                    rb[c * g.BN + q] = rb[c * g.BN + q] - hdt * cu;
                }
                put_b(i, j, k, bnew);
            } else {
#pragma unroll
                for (int c = 0; c < 3; ++c) rb[c * g.BN + q] = bt_global<R, 1>(B, c, gi, gj, gk, hdt);
            }
        }
    } else {
        const R *ex = re, *ey = re + g.JN, *ez = re + 2 * g.JN;
        for (int q = tid; q < g.BN; q += kBlock) {
            const int jk = div_small(q, mBX), i = q - jk * BX;
            const int k = div_small(jk, mBY), j = jk - k * g.BY;
            const int p = i + JX * j + JXY * k;
            const R cu[3] = {(ez[p + JX] - ez[p]) - (ey[p + JXY] - ey[p]),
                             (ex[p + JXY] - ex[p]) - (ez[p + 1] - ez[p]),
                             (ey[p + 1] - ey[p]) - (ex[p + JX] - ex[p])};
            const R bo[3] = {rb[q], rb[g.BN + q], rb[2 * g.BN + q]};
            rb[q] = bo[0] - hdt * cu[0];
            rb[g.BN + q] = bo[1] - hdt * cu[1];
            rb[2 * g.BN + q] = bo[2] - hdt * cu[2];
            if (own(i, j, k)) {
                const R bnew[3] = {bo[0] - C.dt * cu[0], bo[1] - C.dt * cu[1], bo[2] - C.dt * cu[2]};
                put_b(i, j, k, bnew);
            }
        }
    }
    __syncthreads();

    // 3. node fields on the (ext+1)^3 nodes of the tile (App. A.3.3)
    {
        const R *ex = re, *ey = re + g.JN, *ez = re + 2 * g.JN;
        const R *bx = rb, *by = rb + g.BN, *bz = rb + 2 * g.BN;
        for (int q = tid; q < g.NN; q += kBlock) {
            const int jk = div_small(q, mNX), i = q - jk * NX;
            const int k = div_small(jk, mNY), j = jk - k * g.NY;
            // raw coordinates of node (i,j,k) are (i+1, j+1, k+1)
            const int pe = (i + 1) + JX * (j + 1) + JXY * (k + 1);
            const int pb = (i + 1) + BX * (j + 1) + BXY * (k + 1);
            node[q] = node_avg2(ex[pe - 1], ex[pe]);
            node[g.NN + q] = node_avg2(ey[pe - JX], ey[pe]);
            node[2 * g.NN + q] = node_avg2(ez[pe - JXY], ez[pe]);
            node[3 * g.NN + q] = node_avg4(bx[pb], bx[pb - BX], bx[pb - BX - BXY], bx[pb - BXY]);
            node[4 * g.NN + q] = node_avg4(by[pb], by[pb - BXY], by[pb - 1 - BXY], by[pb - 1]);
            node[5 * g.NN + q] = node_avg4(bz[pb], bz[pb - 1], bz[pb - 1 - BX], bz[pb - BX]);
        }
    }
    __syncthreads();

    // 4. per cell and component, the trilinear interpolant of the eight node
    //    values as c0 + c1 x + c2 y + c3 z + c4 xy + c5 yz + c6 zx + c7 xyz in
    //    the in-cell offsets (the same polynomial, 8 instead of 16 operations
    //    per component at the particle)
    {
        const int ncell = g.ext[0] * g.ext[1] * g.ext[2];
        const int mEX = 65536 / g.ext[0] + 1, mEY = 65536 / g.ext[1] + 1;
        for (int q = tid; q < ncell; q += kBlock) {
            const int jk = div_small(q, mEX), i = q - jk * g.ext[0];
            const int k = div_small(jk, mEY), j = jk - k * g.ext[1];
            R *cf = coef + kCoef * (i | (j << tsx) | (k << tsxy));
            const int m = i + NX * j + NXY * k;
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const R *F = node + c * g.NN + m;
                const R f[8] = {F[0], F[1], F[NX], F[1 + NX], F[NXY], F[1 + NXY], F[NX + NXY], F[1 + NX + NXY]};
                trilinear_coef(f, cf + 8 * c);
            }
        }
    }
    __syncthreads();
    for (int q = tid; q < 3 * g.JN; q += kBlock) jl[q] = JT(0);
    __syncthreads();

    // 5. particles of every species: gather, push, move, deposit, re-bin
    // uniform index offsets of the twelve faces of a piece (see deposit_piece)
    int joff[3][4];
    {
        const int S[3] = {1, JX, JXY};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int b1 = a == 2 ? 0 : a + 1, b2 = a == 0 ? 2 : a - 1;
            joff[a][0] = a * g.JN;
            joff[a][1] = a * g.JN + S[b2];
            joff[a][2] = a * g.JN + S[b1];
            joff[a][3] = a * g.JN + S[b1] + S[b2];
        }
    }
    // this wave's queue of unfinished moves: home-cell index (sign bit =
    // species sign), meta word (move_meta), start of the next piece and end
    // of the move
    const int wave = tid >> 6, lane = __lane_id();
    constexpr int kQCap = QCap<R>::value;
    int32_t *qidx = reinterpret_cast<int32_t *>(qmem) + wave * kQCap;
    int32_t *qmeta = reinterpret_cast<int32_t *>(qmem) + (kWaves + wave) * kQCap;
    R *qval = reinterpret_cast<R *>(qmem + 2 * kWaves * kQCap * sizeof(int32_t)) + wave * 6 * kQCap;
    int qhead = 0, qcount = 0;                    // wave-uniform
    auto put = [&](bool has, int32_t w, int32_t meta, const R ps[3], const R x1[3]) {
        const uint64_t mh = __ballot(has);
        if (has) {
            const int pos = (qhead + qcount + lane_rank(mh)) & (kQCap - 1);
            qidx[pos] = w;
            qmeta[pos] = meta;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                qval[a * kQCap + pos] = ps[a];
                qval[(3 + a) * kQCap + pos] = x1[a];
            }
        }
        qcount += (int)__popcll(mh);
    };
    // deposit the next piece of up to 64 queued moves (whole wave); moves with
    // pieces left go back into the queue
    auto drain = [&]() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int nq = min(qcount, 64);
        int32_t w = 0, meta = 0;
        R ps[3] = {R(0), R(0), R(0)}, x1[3] = {R(0), R(0), R(0)};
        if (lane < nq) {
            const int e = (qhead + lane) & (kQCap - 1);
            w = qidx[e];
            meta = qmeta[e];
#pragma unroll
            for (int a = 0; a < 3; ++a) { ps[a] = qval[a * kQCap + e]; x1[a] = qval[(3 + a) * kQCap + e]; }
        }
        qhead = (qhead + nq) & (kQCap - 1);
        qcount -= nq;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int k = meta & 3, nb = (meta >> 2) & 3;
        bool more = false;
        R pe[3] = {x1[0], x1[1], x1[2]};
        if (lane < nq) {
            int offc[3];
            R sv[3], dd[3];
            chain_piece(ps, x1, meta, k, pe, offc, sv, dd);
            const int cb = (w & 0x7fffffff) + offc[0] + __mul24(JX, offc[1]) + __mul24(JXY, offc[2]);
            const R sc = w < 0 ? -qscale_bits<R>() : qscale_bits<R>();
            deposit_piece<R>(jl, cb, joff, sv, dd, sc);
            more = k < nb;
        }
        put(more, w, meta + 1, pe, x1);
    };
    for (int s = 0; s < C.nsp; ++s) {
        const SpeciesDev<R> &S = B.sp[s];
        const PBuf<R> &P = S.buf[C.cur];
        const TileRanges src = ranges(s);
        const int n = src.n;
        const R hk = R(0.5) * C.kq[s] * C.dt;
        const R scale = -C.qs[s] * qscale_bits<R>();
        const int32_t sgnbit = scale < R(0) ? (int32_t)0x80000000 : 0;
        const int dst = C.cur ^ 1;
        const int dst_start = __builtin_amdgcn_readfirstlane(sh_rng[s][4]);
        const int ovf0 = S.slots - S.ovf_cap;           // first slot of the overflow region
        auto fetch = [&](int q) { fetch_particle(P, src, q); };
        if (n > 0 && s > 0) fetch(tid);                  // species 0: loaded during the set-up
        for (int pb = 0; pb < n; pb += kBlock) {
            const int p = pb + tid;
            const bool valid = p < n;
            const int code = nx_code, id = nx_id;
            R d[3] = {nx_d[0], nx_d[1], nx_d[2]}, u[3] = {nx_u[0], nx_u[1], nx_u[2]};
            if (pb + kBlock < n) fetch(p + kBlock);
            const int lx = code & ((1 << tsx) - 1), ly = (code >> tsx) & ((1 << (tsxy - tsx)) - 1), lz = code >> tsxy;
            const int ix = g.o[0] + lx, iy = g.o[1] + ly, iz = g.o[2] + lz;
            // a particle of the tile's ranges has its cell in the tile; a code
            // past a partial tile's extent would index the tile's LDS out of
            // range, so it takes the HBM path instead
            const bool inside = (unsigned)lx < (unsigned)g.ext[0] && (unsigned)ly < (unsigned)g.ext[1] &&
                                (unsigned)lz < (unsigned)g.ext[2];
            // gather: the cell's trilinear interpolant at the in-cell offset
            R E[3] = {R(0), R(0), R(0)}, Bf[3] = {R(0), R(0), R(0)};
            if (!inside) {
                gather_global<R, F4>(B, ix, iy, iz, d, hdt, E, Bf);
            } else {
                const R *cf = coef + __umul24(kCoef, lx | (ly << tsx) | (lz << tsxy));
                R F[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) F[c] = trilinear_eval(cf + 8 * c, d);
                E[0] = F[0]; E[1] = F[1]; E[2] = F[2];
                Bf[0] = F[3]; Bf[1] = F[4]; Bf[2] = F[5];
            }
            R D[3];
            boris_move(hk, E, Bf, u, C.dt, valid, C.flags, D);

            // node planes crossed by the move (end x1 in the home-cell frame)
            R x1[3], lam[3];
            int dir[3];
            move_crossings(d, D, x1, dir, lam);
            // conducting walls (App. A.4): a move through a wall ends at the
            // mirrored point P2 + D2; its deposit is the piece d -> d + D1
            // (below) and the queued move P2 -> P2 + D2
            bool hitw = false;
            R P2[3], D2[3], D1[3];
            if (WALLS && B.wall >= 0) {
                const int w = B.wall;
                hitw = valid && wall_hit(w, w == 0 ? ix : (w == 1 ? iy : iz), B.n[w], d, D, D1, P2, D2, u);
                if (hitw) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        x1[a] = P2[a] + D2[a];
                        dir[a] = x1[a] < R(0) ? -1 : (x1[a] >= R(1) ? 1 : 0);
                    }
                }
            }

            // new cell and offset, re-binning target, and the slot claims:
            // one returning LDS atomic for the stayers' block of slots and one
            // for the leavers' staging slots, each by the lowest lane of its
            // group, plus a per-direction count for each leaver
            // (the periodic wrap only where a lane may cross the box edge: in
            // a tile on the edge, or when a lane came from outside its tile)
            const bool anyout = __ballot(valid && !inside) != 0;
            int cn[3] = {ix, iy, iz}, lc[3] = {lx, ly, lz};
            R dn[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int f = dir[a];                 // floor(x1)
                dn[a] = offset_in_cell(x1[a]);
                lc[a] += f;
                int ci = cn[a] + f;
                if (edge[a] || anyout) ci = ci < 0 ? ci + bn[a] : (ci >= bn[a] ? ci - bn[a] : ci);
                cn[a] = ci;
            }
            const int32_t ncell = pack_cell(cn[0], cn[1], cn[2]);
            const int ncode = (cn[0] & ((1 << tsx) - 1)) | ((cn[1] & ((1 << (tsxy - tsx)) - 1)) << tsx) |
                              ((cn[2] & ((1 << tsz) - 1)) << tsxy);
            const int tn = tile_of(B, ncell);
            // re-binning: stayers take the next slots at the front of the
            // tile's new A range, leavers into an adjacent tile are staged from
            // the back (both claimed with one LDS atomic per wave); anything
            // else claims its target's B range with a global atomic
            int bin;
            if (FIX && fastbin && !anyout) {
                // every valid lane started in this full 4x4x4 tile and moved at
                // most one cell per axis: its direction code from the local
                // cell, (lc + 4) >> 2 = 0, 1, 2 for lc = -1, 0..3, 4, and 1 on
                // an axis that one tile spans (it wraps into the same tile);
                // the same code as move_bin's
                int code = 0;
#pragma unroll
                for (int a = 0; a < 3; ++a) code += ((span[a] ? 4 : lc[a] + 4) >> 2) * (a == 0 ? 1 : (a == 1 ? 3 : 9));
                bin = valid ? code : -1;
            } else {
                bin = valid ? move_bin(g, rim, cn) : -1;
            }
            const bool stay = bin == 13, lv = bin >= 0 && bin != 13;
            const uint64_t ms = __ballot(stay), ml = __ballot(lv);
            const int sl = ms ? __ffsll((unsigned long long)ms) - 1 : 0;
            const int ll = ml ? __ffsll((unsigned long long)ml) - 1 : 0;
            int fb = 0, bb = 0;
            if (stay && lane == sl) fb = atomicAdd(&sh_front[s], (int)__popcll(ms));
            if (lv && lane == ll) bb = atomicAdd(&sh_back[s], (int)__popcll(ml));
            if (lv) atomicAdd(&sh_bin[s][bin], 1);
            fb = __builtin_amdgcn_readlane(fb, sl);
            bb = __builtin_amdgcn_readlane(bb, ll);
            int at = -1;
            if (stay) {
                at = dst_start + fb + lane_rank(ms);
            } else if (lv) {
                at = dst_start + n - 1 - (bb + lane_rank(ml));
            } else if (valid) {
                const int slot = atomicAdd(&S.nb[dst][tn], 1);
                at = b_range_slot(B, S, dst, tn, S.bs[dst][tn] + slot, C.flags);
            }
            if (at >= 0) write_particle(S.buf[dst], at, lv || at >= ovf0, ncell, ncode, dn, u, id);

            // deposit: the first piece (in the home cell) at once, the move
            // into the wave's queue for its later pieces; the crossings in
            // increasing order of their parameter (axes o0, o1, o2)
            if (WALLS && hitw) {
#pragma unroll
                for (int a = 0; a < 3; ++a) D[a] = D1[a];
                move_crossings(d, D, x1, dir, lam);
            }
            const int nb = (dir[0] != 0) + (dir[1] != 0) + (dir[2] != 0);
            int o0 = 0, o1 = 1, o2 = 2;
            R l0 = lam[0], l1 = lam[1], l2 = lam[2];
            if (l1 < l0) { R t = l0; l0 = l1; l1 = t; int q = o0; o0 = o1; o1 = q; }
            if (l2 < l1) { R t = l1; l1 = l2; l2 = t; int q = o1; o1 = o2; o2 = q; }
            if (l1 < l0) { R t = l0; l0 = l1; l1 = t; int q = o0; o0 = o1; o1 = q; }
            const int jb = (lx + 1) + __mul24(JX, ly + 1) + __mul24(JXY, lz + 1);
            R p1[3];
            if (nb == 0) {
                p1[0] = x1[0]; p1[1] = x1[1]; p1[2] = x1[2];
            } else {
                first_breakpoint(d, D, dir, o0, l0, p1);
            }
            if (valid && inside) {
                const R dd[3] = {p1[0] - d[0], p1[1] - d[1], p1[2] - d[2]};
                deposit_piece<R>(jl, jb, joff, d, dd, scale);
            } else if (valid) {
                PIC_GLOBAL JT *J = B.J;
                deposit_move(d, D, scale, [&](int a, int ox, int oy, int oz, JT q) {
                    if (q == JT(0)) return;
                    const int i = wrap_idx(ix + ox, B.n[0]), j = wrap_idx(iy + oy, B.n[1]),
                              k = wrap_idx(iz + oz, B.n[2]);
                    atomic_add_global(&J[a * B.nc + i + (int64_t)B.n[0] * (j + (int64_t)B.n[1] * k)], q);
                });
            }
            if (kQCap < 128) {
                const int cnt = (int)__popcll(__ballot(valid && inside && nb > 0));
                while (qcount + cnt > kQCap) drain();
            }
            put(valid && inside && nb > 0, jb | sgnbit, move_meta(1, nb, o0, o1, o2, dir), p1, x1);
            while (qcount >= 64) drain();
            if (WALLS && B.wall >= 0 && __ballot(hitw)) {
                // the mirrored rest of the moves that hit a wall: a whole move
                // from its first piece (next piece 0) through the queue
                R y1[3], lb[3];
                int db[3], s2[3];
                wall_rest_start(B.wall, P2, s2);
                move_crossings(P2, D2, y1, db, lb);
                const int nb2 = (db[0] != 0) + (db[1] != 0) + (db[2] != 0);
                int q0 = 0, q1 = 1, q2 = 2;
                R m0 = lb[0], m1 = lb[1], m2 = lb[2];
                if (m1 < m0) { R t = m0; m0 = m1; m1 = t; int q = q0; q0 = q1; q1 = q; }
                if (m2 < m1) { R t = m1; m1 = m2; m2 = t; int q = q1; q1 = q2; q2 = q; }
                if (m1 < m0) { R t = m0; m0 = m1; m1 = t; int q = q0; q0 = q1; q1 = q; }
                const int jb2 = jb + s2[0] + __mul24(JX, s2[1]) + __mul24(JXY, s2[2]);
                if (kQCap < 128) {
                    const int cnt = (int)__popcll(__ballot(hitw && inside));
                    while (qcount + cnt > kQCap) drain();
                }
                put(hitw && inside, jb2 | sgnbit, move_meta(0, nb2, q0, q1, q2, db), P2, y1);
                if (hitw && !inside) {
                    PIC_GLOBAL JT *J = B.J;
                    deposit_rest(P2, D2, scale, [&](int a, int ox, int oy, int oz, JT q) {
                        if (q == JT(0)) return;
                        const int i = wrap_idx(ix + s2[0] + ox, B.n[0]), j = wrap_idx(iy + s2[1] + oy, B.n[1]),
                                  k = wrap_idx(iz + s2[2] + oz, B.n[2]);
                        atomic_add_global(&J[a * B.nc + i + (int64_t)B.n[0] * (j + (int64_t)B.n[1] * k)], q);
                    });
                }
                while (qcount >= 64) drain();
            }
        }
    }
    // 7a. every wave is past its particle loops, so the leaver counts per
    //     (species, direction) are final: claim their slots in the adjacent
    //     tiles' B ranges now, one global atomic each; the replies come back
    //     while the queues drain and the current is flushed
    __syncthreads();
    const int dst = C.cur ^ 1;
    int claim = 0, ctile = 0;
    const bool claimer = tid < C.nsp * 27;
    const int cs = claimer ? tid / 27 : 0, ck = claimer ? tid - 27 * cs : 0;
    const int ccnt = claimer ? sh_bin[cs][ck] : 0;
    int tbs = 0, tseg = 0, tcap = 0;
    if (ccnt > 0) {
        ctile = neighbor_tile(B, g, ck);
        claim = atomicAdd(&B.sp[cs].nb[dst][ctile], ccnt);
        // the target's layout, read while the queues drain
        const SpeciesDev<R> &S = B.sp[cs];
        tbs = S.bs[dst][ctile];
        tseg = S.seg_start[dst][ctile];
        tcap = S.seg_cap[dst][ctile];
    }
    if (tid < C.nsp) {
        const SpeciesDev<R> &S = B.sp[tid];
        S.na[dst][T] = sh_front[tid];
        // staged leavers of species tid: slots [first, first + nl) of copy cur^1
        const int nl = sh_back[tid];
        int before = 0;                                       // leavers of the species before it
        for (int s = 0; s < tid; ++s) before += sh_back[s];
        sh_q[tid] = S.buf[dst];
        sh_loff[tid] = sh_rng[tid][4] + sh_rng[tid][3] - nl - before;
        sh_lend[tid] = before + nl;
    }
    __syncthreads();
    // the staged leavers of all species form one range [0, ntot); a thread
    // loads up to kHand of them before it stores any, so that their HBM round
    // trips overlap instead of following each other.  The first batch is
    // loaded here: its round trips overlap the claims' replies, the drains
    // and the flush.
    constexpr int kHand = 4;
    const int ntot = C.nsp > 0 ? sh_lend[C.nsp - 1] : 0;
    int hsp[kHand], hcell[kHand], hid[kHand];
    R hd[kHand][3], hu[kHand][3];
    auto load_leavers = [&](int q0) {
#pragma unroll
        for (int h = 0; h < kHand; ++h) {
            const int q = q0 + h * kBlock;
            hsp[h] = -1;
            if (q < ntot) {
                int s = 0;
#pragma unroll
                for (int r = 0; r + 1 < kMaxSpecies; ++r) s += (r + 1 < C.nsp && q >= sh_lend[r]) ? 1 : 0;
                const PBuf<R> &Q = sh_q[s];
                const int from = q + sh_loff[s];
                hcell[h] = slot_ref(Q.cell, from);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    hd[h][a] = slot_ref(Q.d[a], from);
                    hu[h][a] = slot_ref(Q.u[a], from);
                }
                hid[h] = Q.id ? slot_ref(Q.id, from) : 0;
                hsp[h] = s;
            }
        }
    };
    load_leavers(tid);
    while (qcount > 0) drain();
    __syncthreads();

    // 6. flush the tile current to HBM (integer sums: order-independent)
    for (int q = tid; q < g.JN; q += kBlock) {
        const JT v0 = jl[q], v1 = jl[g.JN + q], v2 = jl[2 * g.JN + q];
        if (v0 != JT(0) || v1 != JT(0) || v2 != JT(0)) {
            const int jk = div_small(q, mJX), i = q - jk * JX;
            const int k = div_small(jk, mJY), j = jk - k * g.JY;
            const int64_t gp = gidx(i, j, k);
            if (v0 != JT(0)) atomic_add_global(&B.J[gp], v0);
            if (v1 != JT(0)) atomic_add_global(&B.J[B.nc + gp], v1);
            if (v2 != JT(0)) atomic_add_global(&B.J[2 * B.nc + gp], v2);
        }
    }

    // 7b. hand the staged leavers over: the claimed positions and the target
    //     segments go to LDS, so that the copies below read no layout from HBM
    if (claimer) {
        if (ccnt > 0) {
            sh_base[cs][ck] = tbs + claim;                    // position in the target's segment
            sh_tseg[cs][ck] = tseg;
            sh_tend[cs][ck] = tcap;
        }
        sh_bin[cs][ck] = 0;                                   // now the rank counter
    }
    __syncthreads();
    // 7c. store each loaded leaver at its claimed slot, then load the next
    //     batch (tiles with more than kHand * kBlock leavers)
    for (int q0 = tid; q0 < ntot; q0 += kHand * kBlock) {
        if (q0 != tid) load_leavers(q0);
#pragma unroll
        for (int h = 0; h < kHand; ++h) {
            const int s = hsp[h];
            if (s < 0) continue;
            const int c3[3] = {cell_x(hcell[h]), cell_y(hcell[h]), cell_z(hcell[h])};
            const int k = move_bin(g, rim, c3);         // the same bin as at staging
            const int pos = sh_base[s][k] + atomicAdd(&sh_bin[s][k], 1);
            const bool wide = pos >= sh_tend[s][k];
            int at;
            if (!wide) {
                at = sh_tseg[s][k] + pos;
            } else {                                    // the target segment is full: overflow region
                const SpeciesDev<R> &S = B.sp[s];
                const int o = atomicAdd(&S.nb[dst][B.ntiles], 1);
                if (o >= S.ovf_cap) {
                    atomicOr(C.flags, PIC_FLAG_LOST);
                    at = -1;
                } else {
                    at = S.seg_start[dst][B.ntiles] + o;
                }
            }
            if (at >= 0) write_particle(sh_q[s], at, wide, hcell[h], local_code(B, hcell[h]), hd[h], hu[h], hid[h]);
        }
    }
}

// ------------------------------------------------------------- Yee updates

// Between two pushes: copy `old` (just read, written by the next push) gets,
// for tile t, empty A and B ranges with B starting after the particles that
// the tile now holds in copy old ^ 1, and an empty overflow region.
template <typename R>
__device__ inline void next_layout(const BoxDev<R> &B, int nsp, int old, int t)
{
    for (int s = 0; s < nsp; ++s) {
        const SpeciesDev<R> &S = B.sp[s];
        if (t < B.ntiles) {
            S.bs[old][t] = tile_ranges(S, old ^ 1, t).n;
            S.na[old][t] = 0;
        }
        S.nb[old][t] = 0;
    }
}

// Overflow watch, by one whole block: fill of the fullest overflow region
// after a push, over every box and species of copy `copy` (the one just
// written), in thousandths of the smaller of its capacity and kOvfBlocks *
// 1024 particles (the load its sweep blocks take in four rounds).
template <typename R>
__device__ void overflow_watch_block(const BoxDev<R> *__restrict__ boxes, int nboxes, int nsp, int copy,
                                     uint32_t *__restrict__ out)
{
    __shared__ unsigned int best;

    if (threadIdx.x == 0) best = 0;
    __syncthreads();
    unsigned int m = 0;
    for (int b = threadIdx.x; b < nboxes; b += kBlock) {
        const BoxDev<R> &B = boxes[b];
        for (int s = 0; s < nsp; ++s) {
            const SpeciesDev<R> &S = B.sp[s];
            const long long c = S.nb[copy][B.ntiles];
            const long long cap = min((long long)S.ovf_cap, (long long)kOvfBlocks * 1024);
            const unsigned int f = (unsigned int)min(1000LL, c * 1000LL / max(1LL, cap));
            m = max(m, f);
        }
    }
    atomicMax(&best, m);
    __syncthreads();
    if (threadIdx.x == 0) *out = best;
}

// Book-keeping after a push, by the first field kernel that follows it: the
// tile descriptors of copy `old` (the one just read) for the next push, and
// in the grid's last block the overflow watch of copy old ^ 1 (the one just
// written); the whole last block reaches the watch's barriers.
template <typename R>
__device__ inline void after_push(const BoxDev<R> *__restrict__ boxes, const BoxDev<R> &B, int64_t p, int nsp,
                                  int old, int nboxes, uint32_t *__restrict__ watch)
{
    if (p < B.ntiles) next_layout(B, nsp, old, (int)p);
    if (p == 0) next_layout(B, nsp, old, B.ntiles);
    if (watch && blockIdx.x == gridDim.x - 1) overflow_watch_block(boxes, nboxes, nsp, old ^ 1, watch);
}

// Coordinates of cell p of a box with edges n0, n1 (p < n0 n1 n2 <= 2^32, so
// 32-bit divisions are exact).
__device__ inline void cell_coords(int64_t p, int n0, int n1, int &i, int &j, int &k)
{
    const uint32_t q = (uint32_t)p, r = q / (uint32_t)n0;
    i = (int)(q - r * (uint32_t)n0);
    k = (int)(r / (uint32_t)n1);
    j = (int)(r - (uint32_t)k * (uint32_t)n1);
}

// b <- b - h curl e (App. A.3.2), in place.  The steps advance b inside the
// push (its set-up writes b^{t+dt/2} of each tile's cells); this kernel makes
// the half step of the start (h = -dt/2).
template <typename R>
__global__ void __launch_bounds__(kBlock) advance_b_kernel(const BoxDev<R> *__restrict__ boxes,
                                                           const CellBlock *__restrict__ blocks, R h)
{
    const CellBlock cb = blocks[blockIdx.x];
    const BoxDev<R> &B = boxes[cb.box];
    const int64_t p = (int64_t)cb.first + threadIdx.x;
    if (p >= B.nc) return;
    const int n0 = B.n[0], n1 = B.n[1], n2 = B.n[2];
    int i, j, k;
    cell_coords(p, n0, n1, i, j, k);
    const int64_t sx = (i + 1 < n0) ? 1 : 1 - n0;
    const int64_t sy = (j + 1 < n1) ? n0 : (int64_t)n0 * (1 - n1);
    const int64_t sz = (k + 1 < n2) ? (int64_t)n0 * n1 : (int64_t)n0 * n1 * (1 - n2);
    const R *ex = B.e, *ey = B.e + B.nc, *ez = B.e + 2 * B.nc;
    R cx, cy, cz;
    if (B.faraday4) {
        cx = curl4_e(B, 0, i, j, k);
        cy = curl4_e(B, 1, i, j, k);
        cz = curl4_e(B, 2, i, j, k);
    } else {
        cx = (ez[p + sy] - ez[p]) - (ey[p + sz] - ey[p]);
        cy = (ex[p + sz] - ex[p]) - (ez[p + sx] - ez[p]);
        cz = (ey[p + sx] - ey[p]) - (ex[p + sy] - ex[p]);
    }
    B.b[p] -= h * cx;
    B.b[B.nc + p] -= h * cy;
    B.b[2 * B.nc + p] -= h * cz;
    if (B.wall >= 0 && (B.wall == 0 ? i : (B.wall == 1 ? j : k)) == 0)
        B.b[B.wall * B.nc + p] = R(0);           // normal b on a conducting wall (App. A.4)
}

// e <- e + dt curl b + alpha0 J (App. A.3.2 and A.2, eq. max2bis); J <- 0;
// and the book-keeping after the push (after_push).
template <typename R>
__global__ void __launch_bounds__(kBlock) advance_e_kernel(const BoxDev<R> *__restrict__ boxes,
                                                           const CellBlock *__restrict__ blocks, R dt, int nsp,
                                                           int old, int nboxes, uint32_t *__restrict__ watch)
{
    using JT = typename JType<R>::T;
    const CellBlock cb = blocks[blockIdx.x];
    const BoxDev<R> &B = boxes[cb.box];
    const int64_t p = (int64_t)cb.first + threadIdx.x;
    after_push(boxes, B, p, nsp, old, nboxes, watch);
    if (p >= B.nc) return;
    const int n0 = B.n[0], n1 = B.n[1], n2 = B.n[2];
    int i, j, k;
    cell_coords(p, n0, n1, i, j, k);
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
    if (B.wall >= 0 && (B.wall == 0 ? i : (B.wall == 1 ? j : k)) == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c)              // tangential e on a conducting wall (App. A.4)
            if (c != B.wall) B.e[c * B.nc + p] = R(0);
    }
    J[p] = JT(0);
    J[B.nc + p] = JT(0);
    J[2 * B.nc + p] = JT(0);
}

// Sum over the 27 values around cell (i,j,k) of one periodic grid with the
// smoothing weights of App. A.3.4 scaled to integers: 8 for the cell itself,
// 4 per face neighbour, 2 per edge neighbour, 1 per corner neighbour (the
// paper's 1, 1/2, 1/4, 1/8 times 8; they add up to 64).
template <typename T>
__device__ inline T smooth27(const PIC_GLOBAL T *f, const int n[3], int i, int j, int k)
{
    T acc = T(0);
#pragma unroll
    for (int dk = -1; dk <= 1; ++dk) {
        const int64_t kk = wrap1(k + dk, n[2]);
#pragma unroll
        for (int dj = -1; dj <= 1; ++dj) {
            const int64_t row = (int64_t)n[0] * (wrap1(j + dj, n[1]) + (int64_t)n[1] * kk);
#pragma unroll
            for (int di = -1; di <= 1; ++di) {
                const int w = 8 >> ((di != 0) + (dj != 0) + (dk != 0));
                acc += T(w) * f[row + wrap1(i + di, n[0])];
            }
        }
    }
    return acc;
}

// e <- e + dt curl b + alpha0 S J with S the 27-point smoothing of App. A.3.4
// (integer weights in the FP32 form, so the smoothed current stays exact and
// order-independent until its one conversion); J is cleared afterwards by
// clear_current_kernel, since every cell reads its neighbours' J here.
template <typename R>
__global__ void __launch_bounds__(kBlock) advance_e_smoothed_kernel(const BoxDev<R> *__restrict__ boxes,
                                                                    const CellBlock *__restrict__ blocks, R dt,
                                                                    int nsp, int old, int nboxes,
                                                                    uint32_t *__restrict__ watch)
{
    using JT = typename JType<R>::T;
    const CellBlock cb = blocks[blockIdx.x];
    const BoxDev<R> &B = boxes[cb.box];
    const int64_t p = (int64_t)cb.first + threadIdx.x;
    after_push(boxes, B, p, nsp, old, nboxes, watch);
    if (p >= B.nc) return;
    const int n0 = B.n[0], n1 = B.n[1], n2 = B.n[2];
    int i, j, k;
    cell_coords(p, n0, n1, i, j, k);
    const int64_t sx = (i > 0) ? 1 : 1 - n0;
    const int64_t sy = (j > 0) ? n0 : (int64_t)n0 * (1 - n1);
    const int64_t sz = (k > 0) ? (int64_t)n0 * n1 : (int64_t)n0 * n1 * (1 - n2);
    const R *bx = B.b, *by = B.b + B.nc, *bz = B.b + 2 * B.nc;
    const R cx = (bz[p] - bz[p - sy]) - (by[p] - by[p - sz]);
    const R cy = (bx[p] - bx[p - sz]) - (bz[p] - bz[p - sx]);
    const R cz = (by[p] - by[p - sx]) - (bx[p] - bx[p - sy]);
    const double a = B.alpha0 / (double)qscale_bits<R>() / 64.0;
    const R cur[3] = {cx, cy, cz};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const JT s = smooth27<JT>(B.J + c * B.nc, B.n, i, j, k);
        B.e[c * B.nc + p] += dt * cur[c] + (R)(a * (double)s);
    }
}

template <typename R>
__global__ void __launch_bounds__(kBlock) clear_current_kernel(const BoxDev<R> *__restrict__ boxes,
                                                               const CellBlock *__restrict__ blocks)
{
    using JT = typename JType<R>::T;
    const CellBlock cb = blocks[blockIdx.x];
    const BoxDev<R> &B = boxes[cb.box];
    const int64_t p = (int64_t)cb.first + threadIdx.x;
    if (p >= B.nc) return;
    B.J[p] = JT(0);
    B.J[B.nc + p] = JT(0);
    B.J[2 * B.nc + p] = JT(0);
}

// ------------------------------------------------------ counting-sort repack

// The particles of a work item in copy c: a tile's A and B ranges (one block
// striding), or the overflow region (kOvfBlocks blocks striding).
template <typename R>
__device__ inline TileRanges item_range(const BoxDev<R> &B, const SpeciesDev<R> &S, int c, int tile, int &first,
                                        int &stride)
{
    if (tile >= 0) {
        first = threadIdx.x;
        stride = kBlock;
        return tile_ranges(S, c, tile);
    }
    first = (-1 - tile) * kBlock + threadIdx.x;
    stride = kBlock * kOvfBlocks;
    return overflow_range(B, S, c);
}

// Tile counts for the repack: a tile's ranges hold only particles of that
// tile, so they count as a whole; overflow particles one by one.
template <typename R>
__global__ void __launch_bounds__(kBlock) repack_count_kernel(const BoxDev<R> *__restrict__ boxes,
                                                              const Item *__restrict__ items, int nsp, int cur)
{
    const Item it = items[blockIdx.x];
    const BoxDev<R> &B = boxes[it.box];
    for (int s = 0; s < nsp; ++s) {
        const SpeciesDev<R> &S = B.sp[s];
        int first, stride;
        const TileRanges r = item_range(B, S, cur, it.tile, first, stride);
        if (it.tile >= 0) {
            if (threadIdx.x == 0 && r.n > 0) atomicAdd(&S.tcount[it.tile], r.n);
        } else {
            for (int p = first; p < r.n; p += stride) atomicAdd(&S.tcount[tile_of(B, S.buf[cur].cell[r.slot(p)])], 1);
        }
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
        // the counts still start from zero at the next repack
        for (int t = t0; t < t1; ++t) S.tcount[t] = 0;
        if (tid == 0) atomicOr((PIC_GLOBAL uint32_t *)flags, PIC_FLAG_LOST);
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
        S.na[dst][t] = 0;
        S.nb[dst][t] = 0;
        S.bs[dst][t] = 0;
        S.tcount[t] = 0;
        run += cap;
    }
    if (tid == 0) {
        S.seg_start[dst][nt] = S.slots - S.ovf_cap;
        S.seg_cap[dst][nt] = S.ovf_cap;
        S.nb[dst][nt] = 0;
    }
}

template <typename R>
__global__ void __launch_bounds__(kBlock) repack_scatter_kernel(const BoxDev<R> *__restrict__ boxes,
                                                                const Item *__restrict__ items, int nsp, int cur,
                                                                uint32_t *flags)
{
    const Item it = items[blockIdx.x];
    const BoxDev<R> &B = boxes[it.box];
    int o[3] = {0, 0, 0};                               // origin of the tile (tile items)
    if (it.tile >= 0) tile_origin(B, it.tile, o);
    for (int s = 0; s < nsp; ++s) {
        const SpeciesDev<R> &S = B.sp[s];
        int first, stride;
        const TileRanges r = item_range(B, S, cur, it.tile, first, stride);
        const int n = r.n;
        const PBuf<R> &P = S.buf[cur];
        // wave-uniform trip count so that the ballots in store_particle see every lane
        const int trips = n > first - (int)threadIdx.x ? (n - (first - (int)threadIdx.x) + stride - 1) / stride : 0;
        for (int tr = 0; tr < trips; ++tr) {
            const int p = first + tr * stride;
            const bool valid = p < n;
            int32_t cell = 0, id = 0;
            R d[3] = {R(0), R(0), R(0)}, u[3] = {R(0), R(0), R(0)};
            if (valid) {
                const int idx = r.slot(p);
                cell = it.tile >= 0 ? local_cell(B, o, P.lc[idx]) : P.cell[idx];
                for (int a = 0; a < 3; ++a) { d[a] = P.d[a][idx]; u[a] = P.u[a][idx]; }
                if (P.id) id = P.id[idx];
            }
            store_particle(B, S, cur ^ 1, tile_of(B, cell), valid, cell, d, u, id, (PIC_GLOBAL uint32_t *)flags);
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
            S.seg_start[old][t] = S.seg_start[old ^ 1][t];
            S.seg_cap[old][t] = S.seg_cap[old ^ 1][t];
            S.bs[old][t] = t < B.ntiles ? tile_ranges(S, old ^ 1, t).n : 0;
            S.na[old][t] = 0;
            S.nb[old][t] = 0;
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
// k = 0 momentum, the gamma-1 histogram and the CIC charge density.  A tile
// item stages the node-averaged e of its (t+1)^3 nodes in LDS once and sums its
// charge and histogram there (one global atomic per node and bin); the
// overflow items gather from HBM and add to the global sums directly.
constexpr int kDiagNodes = 9 * 9 * 9;   // nodes of the largest tile (8^3 cells)
constexpr int kDiagHist = 512;          // histograms up to this many bins are summed in LDS
template <typename R>
__global__ void __launch_bounds__(kBlock) diag_particles_kernel(const BoxDev<R> *__restrict__ boxes,
                                                                const Item *__restrict__ items, StepConst<R> C,
                                                                DiagBuf out)
{
    __shared__ R sE[3 * kDiagNodes];
    __shared__ double srho[kDiagNodes];
    __shared__ unsigned shist[kDiagHist];
    const Item it = items[blockIdx.x];
    const BoxDev<R> &B = boxes[it.box];
    const R hdt = R(0.5) * C.dt;
    const int tid = threadIdx.x;
    const bool in_tile = it.tile >= 0;
    TileGeom<R> g{};
    if (in_tile) {
        g = tile_geom<R>(B, it.tile);
        // node-averaged e (App. A.3.3)
        for (int q = tid; q < g.NN; q += kBlock) {
            const int i = g.o[0] + q % g.NX, j = g.o[1] + (q / g.NX) % g.NY, k = g.o[2] + q / (g.NX * g.NY);
            sE[q] = node_value_global(B, 0, i, j, k, R(0));
            sE[g.NN + q] = node_value_global(B, 1, i, j, k, R(0));
            sE[2 * g.NN + q] = node_value_global(B, 2, i, j, k, R(0));
            srho[q] = 0.0;
        }
    }
    const bool lhist = C.hist_bins > 0 && C.hist_bins <= kDiagHist;
    for (int s = 0; s < C.nsp; ++s) {
        const SpeciesDev<R> &S = B.sp[s];
        int first, stride;
        const TileRanges r = item_range(B, S, C.cur, it.tile, first, stride);
        const PBuf<R> &P = S.buf[C.cur];
        if (lhist)
            for (int q = tid; q < C.hist_bins; q += kBlock) shist[q] = 0u;
        __syncthreads();
        const double q = (double)C.qs[s] * B.alpha0;
        double acc[6] = {0, 0, 0, 0, 0, 0};
        for (int p = first; p < r.n; p += stride) {
            const int idx = r.slot(p);
            const int32_t cell = in_tile ? local_cell(B, g.o, P.lc[idx]) : P.cell[idx];
            const int ix = cell_x(cell), iy = cell_y(cell), iz = cell_z(cell);
            R d[3] = {P.d[0][idx], P.d[1][idx], P.d[2][idx]};
            R E[3];
            int nb = 0;
            if (in_tile) {
                // the cell's trilinear interpolant, as the push evaluates it
                nb = (ix - g.o[0]) + g.NX * ((iy - g.o[1]) + g.NY * (iz - g.o[2]));

                for (int c = 0; c < 3; ++c) {
                    const R *F = sE + c * g.NN + nb;
                    const int NX = g.NX, NXY = g.NX * g.NY;
                    const R f[8] = {F[0], F[1], F[NX], F[1 + NX], F[NXY], F[1 + NXY], F[NX + NXY], F[1 + NX + NXY]};
                    R cf[8];
                    trilinear_coef(f, cf);
                    E[c] = trilinear_eval(cf, d);
                }
            } else {
                R Bf[3];
                gather_global(B, ix, iy, iz, d, hdt, E, Bf);
            }
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
                if (lhist) atomicAdd(&shist[bin], 1u);
                else atomicAdd(reinterpret_cast<unsigned long long *>(&out.hist[s * C.hist_bins + bin]), 1ull);
            }
            for (int kk = 0; kk < 2; ++kk)
                for (int jj = 0; jj < 2; ++jj)
                    for (int ii = 0; ii < 2; ++ii) {
                        const double w = (ii ? (double)d[0] : 1.0 - (double)d[0]) *
                                         (jj ? (double)d[1] : 1.0 - (double)d[1]) *
                                         (kk ? (double)d[2] : 1.0 - (double)d[2]);
                        if (in_tile) {
                            atomicAdd(&srho[nb + ii + g.NX * (jj + g.NY * kk)], q * w);
                        } else {
                            const int i = wrap_idx(ix + ii, B.n[0]), j = wrap_idx(iy + jj, B.n[1]),
                                      k = wrap_idx(iz + kk, B.n[2]);
                            atomicAdd(&out.rho[i + (int64_t)B.n[0] * (j + (int64_t)B.n[1] * k)], q * w);
                        }
                    }
        }
        for (int k = 0; k < 6; ++k) block_sum_to<R>(&out.acc[kAccSp + 6 * s + k], acc[k]);
        if (lhist) {
            __syncthreads();
            for (int b = tid; b < C.hist_bins; b += kBlock)
                if (shist[b]) atomicAdd(reinterpret_cast<unsigned long long *>(&out.hist[s * C.hist_bins + b]),
                                        (unsigned long long)shist[b]);
            __syncthreads();
        }
    }
    if (in_tile) {
        __syncthreads();
        for (int q = tid; q < g.NN; q += kBlock)
            if (srho[q] != 0.0) {
                const int i = wrap_idx(g.o[0] + q % g.NX, B.n[0]), j = wrap_idx(g.o[1] + (q / g.NX) % g.NY, B.n[1]),
                          k = wrap_idx(g.o[2] + q / (g.NX * g.NY), B.n[2]);
                atomicAdd(&out.rho[i + (int64_t)B.n[0] * (j + (int64_t)B.n[1] * k)], srho[q]);
            }
    }
}

__device__ inline void atomic_max_pos(double *p, double v)
{
    atomicMax(reinterpret_cast<unsigned long long *>(p), (unsigned long long)__double_as_longlong(v));
}

// Field energies (e^t, b^t) and the Gauss-law residual div e - rho at the nodes.
template <typename R>
__global__ void __launch_bounds__(kBlock) diag_fields_kernel(const BoxDev<R> *__restrict__ boxes, int box,
                                                             R dt, int filter, DiagBuf out)
{
    const BoxDev<R> &B = boxes[box];
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    double gmax = 0.0;
    if (p < B.nc) {
        const int n0 = B.n[0], n1 = B.n[1];
        int i, j, k;
        cell_coords(p, n0, n1, i, j, k);
        for (int c = 0; c < 3; ++c) {
            const double ec = (double)B.e[c * B.nc + p];
            const double bc = (double)bt_global(B, c, i, j, k, R(0.5) * dt);
            v[c] = 0.5 * ec * ec;
            v[3 + c] = 0.5 * bc * bc;
        }
        const double div = (double)fld(B.e, B, 0, i, j, k) - (double)fld(B.e, B, 0, i - 1, j, k) +
                           (double)fld(B.e, B, 1, i, j, k) - (double)fld(B.e, B, 1, i, j - 1, k) +
                           (double)fld(B.e, B, 2, i, j, k) - (double)fld(B.e, B, 2, i, j, k - 1);
        // with a smoothed current the conserved charge is the smoothed one
        const double rho = filter ? smooth27<double>(out.rho, B.n, i, j, k) / 64.0 : out.rho[p];
        const bool on_wall = B.wall >= 0 && (B.wall == 0 ? i : (B.wall == 1 ? j : k)) == 0;
        const double r = on_wall ? 0.0 : div - rho;   // a wall plane carries the conductor's surface charge
        v[6] = r * r;
        gmax = fabs(r);
    }
    for (int q = 0; q < 6; ++q) block_sum_to<R>(&out.acc[kAccField + q], v[q]);
    block_sum_to<R>(&out.acc[kAccField + 7], v[6]);
    for (int off = 32; off > 0; off >>= 1) gmax = fmax(gmax, __shfl_down(gmax, off));
    if (__lane_id() == 0) atomic_max_pos(&out.acc[kAccField + 6], gmax);
}

// ----------------------------------------------------------- host launchers

template <typename R>
size_t push_lds_bytes(int t0, int t1, int t2) { return tile_lds_bytes<R>(t0, t1, t2); }

template <typename R>
hipError_t launch_push(const BoxDev<R> *boxes, const Item *items, int nitems, size_t lds, const StepConst<R> &C,
                       int fixed444, int walls, int faraday4, hipStream_t st)
{
    // dynamic LDS beyond 64 KiB has to be allowed per kernel: the limit each
    // variant was last raised to, raised again when a launch needs more
    static size_t raised[6] = {65536, 65536, 65536, 65536, 65536, 65536};
    auto go = [&](auto kern, int v) -> hipError_t {
        if (lds > raised[v]) {
            const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            raised[v] = lds;
        }
        hipLaunchKernelGGL(kern, dim3(nitems), dim3(kBlock), lds, st, boxes, items, C);
        return hipGetLastError();
    };
    // walls and the fourth-order solver are never combined (pic_plan refuses it)
    if (walls) return fixed444 ? go(push_kernel<R, 1, 1, 0>, 3) : go(push_kernel<R, 0, 1, 0>, 2);
    if (faraday4) return fixed444 ? go(push_kernel<R, 1, 0, 1>, 5) : go(push_kernel<R, 0, 0, 1>, 4);
    return fixed444 ? go(push_kernel<R, 1, 0, 0>, 1) : go(push_kernel<R, 0, 0, 0>, 0);
}

template <typename R>
hipError_t launch_fields(const BoxDev<R> *boxes, const CellBlock *blocks, int nblocks, R dt, int nsp, int filter,
                         int clear_copy, int nboxes, uint32_t *watch, hipStream_t st)
{
    if (filter) {
        hipLaunchKernelGGL(advance_e_smoothed_kernel<R>, dim3(nblocks), dim3(kBlock), 0, st, boxes, blocks, dt, nsp,
                           clear_copy, nboxes, watch);
        hipLaunchKernelGGL(clear_current_kernel<R>, dim3(nblocks), dim3(kBlock), 0, st, boxes, blocks);
    } else {
        hipLaunchKernelGGL(advance_e_kernel<R>, dim3(nblocks), dim3(kBlock), 0, st, boxes, blocks, dt, nsp,
                           clear_copy, nboxes, watch);
    }
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

// zero n 8-byte words (a kernel rather than a memset, so that a caller may
// capture the diagnostics into a graph)
// (a plain pointer parameter: an address-space qualifier on a kernel
// parameter would give the device symbol another name than the host's)
__global__ void __launch_bounds__(kBlock) zero_words_kernel(uint64_t *__restrict__ p, int64_t n)
{
    PIC_GLOBAL uint64_t *q = (PIC_GLOBAL uint64_t *)p;
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < n; t += (int64_t)gridDim.x * kBlock) q[t] = 0;
}

template <typename R>
hipError_t launch_diag(const BoxDev<R> *boxes, int box, int64_t nc, const Item *items, int nitems,
                       const StepConst<R> &C, const DiagBuf &out, int hist_len, hipStream_t st)
{
    // the accumulators, the charge density and the histogram start from zero
    const int zb = 1024;
    hipLaunchKernelGGL(zero_words_kernel, dim3(zb), dim3(kBlock), 0, st, (uint64_t *)out.acc, (int64_t)kAccLen);
    hipLaunchKernelGGL(zero_words_kernel, dim3(zb), dim3(kBlock), 0, st, (uint64_t *)out.rho, nc);
    hipLaunchKernelGGL(zero_words_kernel, dim3(zb), dim3(kBlock), 0, st, (uint64_t *)out.hist, (int64_t)hist_len);
    if (nitems)
        hipLaunchKernelGGL(diag_particles_kernel<R>, dim3(nitems), dim3(kBlock), 0, st, boxes, items, C, out);
    const int nb = (int)((nc + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(diag_fields_kernel<R>, dim3(nb), dim3(kBlock), 0, st, boxes, box, C.dt, C.filter, out);
    return hipGetLastError();
}

// The diagnostics' own scratch for callers that cannot allocate device
// memory: one array per GPU, held until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in for
// the symbol); it uses the device address that hipGetSymbolAddress returns,
// taken once per device with that device current.
static __device__ __align__(256) unsigned char scratch[kDiagScratchBytes];

constexpr int kMaxDevices = 64;
static void *scratch_ptr[kMaxDevices];

hipError_t diag_scratch_setup()
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    if (scratch_ptr[dev]) return hipSuccess;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_ptr[dev] = p;
    return hipSuccess;
}

void *diag_scratch()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    return scratch_ptr[dev];
}

// ------------------------------------------------- field Fourier spectra

// Value of field f (0: e^t, 1: b^t = b^{t-dt/2} - (dt/2) curl e^t), component
// c, at grid point (x[0], x[1], x[2]).
template <typename R>
__device__ inline double field_at(const BoxDev<R> &B, int f, int c, const int x[3], R hdt)
{
    if (f == 0) return (double)B.e[c * B.nc + x[0] + (int64_t)B.n[0] * (x[1] + (int64_t)B.n[1] * x[2])];
    return (double)bt_global(B, c, x[0], x[1], x[2], hdt);
}

// First pass of the plane spectra (Sect. 3.2.2): for every plane normal to
// axis an and every line along axis a2 of it, the DFT along axis a1,
// tmp[(p * N2 + i2) * N1 + m1] = sum_i1 f(i1, i2, p) exp(-2 pi i m1 i1 / N1),
// in FP64.  One thread per output value; the block stages the N1 twiddle
// factors in LDS.
template <typename R>
__global__ void __launch_bounds__(kBlock) spectrum_rows_kernel(const BoxDev<R> *__restrict__ boxes, int box,
                                                               int f, int c, int a1, int a2, int an, R hdt,
                                                               double2 *__restrict__ tmp)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double2 *w = reinterpret_cast<double2 *>(smem);
    const BoxDev<R> &B = boxes[box];
    const int N1 = B.n[a1], N2 = B.n[a2], NP = B.n[an];
    for (int q = threadIdx.x; q < N1; q += kBlock) {
        double sn, cs;
        sincospi(-2.0 * q / N1, &sn, &cs);
        w[q] = make_double2(cs, sn);
    }
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)N1 * N2 * NP) return;
    const int m1 = (int)(t % N1);
    const int64_t r = t / N1;
    const int i2 = (int)(r % N2), p = (int)(r / N2);
    int x[3];
    x[a2] = i2;
    x[an] = p;
    double re = 0.0, im = 0.0;
    int k = 0;                                    // (m1 * i1) mod N1
    for (int i1 = 0; i1 < N1; ++i1) {
        x[a1] = i1;
        const double v = field_at(B, f, c, x, hdt);
        re += v * w[k].x;
        im += v * w[k].y;
        k += m1;
        if (k >= N1) k -= N1;
    }
    tmp[t] = make_double2(re, im);
}

// Second pass: the DFT along a2 and the power summed over the planes,
// ps[m1 + N1 m2] = sum_p |sum_i2 tmp[(p N2 + i2) N1 + m1] exp(-2 pi i m2 i2 / N2)|^2.
template <typename R>
__global__ void __launch_bounds__(kBlock) spectrum_cols_kernel(const BoxDev<R> *__restrict__ boxes, int box,
                                                               int a1, int a2, int an,
                                                               const double2 *__restrict__ tmp,
                                                               double *__restrict__ ps)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double2 *w = reinterpret_cast<double2 *>(smem);
    const BoxDev<R> &B = boxes[box];
    const int N1 = B.n[a1], N2 = B.n[a2], NP = B.n[an];
    for (int q = threadIdx.x; q < N2; q += kBlock) {
        double sn, cs;
        sincospi(-2.0 * q / N2, &sn, &cs);
        w[q] = make_double2(cs, sn);
    }
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)N1 * N2) return;
    const int m1 = (int)(t % N1), m2 = (int)(t / N1);
    double pw = 0.0;
    for (int p = 0; p < NP; ++p) {
        double re = 0.0, im = 0.0;
        int k = 0;                                // (m2 * i2) mod N2
        for (int i2 = 0; i2 < N2; ++i2) {
            const double2 a = tmp[((int64_t)p * N2 + i2) * N1 + m1];
            re += a.x * w[k].x - a.y * w[k].y;
            im += a.x * w[k].y + a.y * w[k].x;
            k += m2;
            if (k >= N2) k -= N2;
        }
        pw += re * re + im * im;
    }
    ps[t] = pw;
}

template <typename R>
__global__ void __launch_bounds__(kBlock) fill_zero_kernel(double *__restrict__ p, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < n) p[t] = 0.0;
}

template <typename R>
hipError_t launch_spectrum(const BoxDev<R> *boxes, int box, const int n[3], int f, int c, int an, R hdt,
                           double *scratch, double *ps, hipStream_t st)
{
    const int a1 = an == 0 ? 1 : 0, a2 = an == 2 ? 1 : 2;
    const int64_t rows = (int64_t)n[a1] * n[a2] * n[an], cols = (int64_t)n[a1] * n[a2];
    double2 *tmp = reinterpret_cast<double2 *>(scratch);
    hipLaunchKernelGGL(spectrum_rows_kernel<R>, dim3((unsigned)((rows + kBlock - 1) / kBlock)), dim3(kBlock),
                       n[a1] * sizeof(double2), st, boxes, box, f, c, a1, a2, an, hdt, tmp);
    hipLaunchKernelGGL(spectrum_cols_kernel<R>, dim3((unsigned)((cols + kBlock - 1) / kBlock)), dim3(kBlock),
                       n[a2] * sizeof(double2), st, boxes, box, a1, a2, an, (const double2 *)tmp, ps);
    // the scratch is the current buffer of the box, which the next push expects cleared
    hipLaunchKernelGGL(fill_zero_kernel<R>, dim3((unsigned)((2 * rows + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       st, scratch, 2 * rows);
    return hipGetLastError();
}

#define PIC_INSTANTIATE(R)                                                                                     \
    template size_t push_lds_bytes<R>(int, int, int);                                                         \
    template hipError_t launch_push<R>(const BoxDev<R> *, const Item *, int, size_t, const StepConst<R> &,   \
                                       int, int, int, hipStream_t);                                           \
    template hipError_t launch_fields<R>(const BoxDev<R> *, const CellBlock *, int, R, int, int, int, int,     \
                                         uint32_t *, hipStream_t);                                                        \
    template hipError_t launch_advance_b<R>(const BoxDev<R> *, const CellBlock *, int, R, hipStream_t);       \
    template hipError_t launch_repack<R>(const BoxDev<R> *, int, const Item *, int, const StageItem *, int,    \
                                         const StepConst<R> &, hipStream_t);                                  \
    template hipError_t launch_diag<R>(const BoxDev<R> *, int, int64_t, const Item *, int,                    \
                                       const StepConst<R> &, const DiagBuf &, int, hipStream_t);              \
    template hipError_t launch_spectrum<R>(const BoxDev<R> *, int, const int[3], int, int, int, R, double *,   \
                                           double *, hipStream_t);

PIC_INSTANTIATE(float)
PIC_INSTANTIATE(double)

} // namespace pic
