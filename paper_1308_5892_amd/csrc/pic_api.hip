// Host side of the C ABI declared in include/pic.h: arena layout, context,
// stream-ordered launches of the gfx950 kernels, and host<->device copies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#define PIC_HOST_ONLY_TU   // no kernels here: descriptor pointers stay generic
#include "pic_internal.h"

namespace pic {

constexpr int kTabN = 1 << 16;     // inverse-CDF table intervals
constexpr int kTabM = 1 << 16;     // quadrature intervals behind the table

// ------------------------------------------------------------ arena layout

struct Bump {
    char *base;
    size_t off = 0;
    template <typename T> T *take(size_t n)
    {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += n * sizeof(T);
        return p;
    }
};

static int ilog2(int v)
{
    int s = 0;
    while ((1 << s) < v) ++s;
    return s;
}

struct BoxHost {
    pic_box cfg;
    int tile[3];
    int64_t nc;
    int ntiles;
    int32_t slots[kMaxSpecies], ovf_cap[kMaxSpecies], stage_cap[kMaxSpecies];
};

template <typename R>
static void carve(Bump &A, const pic_config *cfg, std::vector<BoxHost> &bh, std::vector<BoxDev<R>> &bd)
{
    using JT = typename JType<R>::T;
    const bool ids = (cfg->flags & PIC_TRACK_IDS) != 0;
    for (int b = 0; b < cfg->n_boxes; ++b) {
        BoxHost &H = bh[b];
        BoxDev<R> &D = bd[b];
        for (int a = 0; a < 3; ++a) {
            D.n[a] = H.cfg.n[a];
            D.tshift[a] = ilog2(H.tile[a]);
            D.ntile[a] = (H.cfg.n[a] + H.tile[a] - 1) / H.tile[a];
        }
        D.ntiles = H.ntiles;
        D.nc = H.nc;
        D.e = A.take<R>(3 * H.nc);
        D.b = A.take<R>(3 * H.nc);
        D.bn = A.take<R>(3 * H.nc);
        D.J = A.take<JT>(3 * H.nc);
        D.rho = A.take<double>(H.nc);
        D.acc = A.take<double>(kAccLen);
        D.hist = A.take<int64_t>((size_t)std::max(1, cfg->hist_bins) * kMaxSpecies);
        D.alpha0 = 2.0 / (H.cfg.n_x * H.cfg.n_x * H.cfg.rho0);
        D.wall = H.cfg.walls - 1;
        D.faraday4 = (cfg->flags & PIC_FARADAY4) != 0;
        for (int s = 0; s < kMaxSpecies; ++s) {
            SpeciesDev<R> &S = D.sp[s];
            memset(&S, 0, sizeof(S));
            if (s >= cfg->n_species) continue;
            const size_t n = H.slots[s], ns = H.stage_cap[s];
            for (int c = 0; c < 2; ++c) {
                S.buf[c].lc = A.take<uint8_t>(n);
                S.buf[c].cell = A.take<int32_t>(n);
                for (int a = 0; a < 3; ++a) S.buf[c].d[a] = A.take<R>(n);
                for (int a = 0; a < 3; ++a) S.buf[c].u[a] = A.take<R>(n);
                S.buf[c].id = ids ? A.take<int32_t>(n) : nullptr;
            }
            S.stage.cell = A.take<int32_t>(ns);
            for (int a = 0; a < 3; ++a) S.stage.d[a] = A.take<R>(ns);
            for (int a = 0; a < 3; ++a) S.stage.u[a] = A.take<R>(ns);
            S.stage.id = ids ? A.take<int32_t>(ns) : nullptr;
            for (int c = 0; c < 2; ++c) {
                S.seg_start[c] = A.take<int32_t>(H.ntiles + 1);
                S.seg_cap[c] = A.take<int32_t>(H.ntiles + 1);
            }
            for (int c = 0; c < 2; ++c) {
                S.na[c] = A.take<int32_t>(H.ntiles + 1);
                S.nb[c] = A.take<int32_t>(H.ntiles + 1);
                S.bs[c] = A.take<int32_t>(H.ntiles + 1);
            }
            S.tcount = A.take<int32_t>(H.ntiles + 1);
            S.slots = H.slots[s];
            S.ovf_cap = H.ovf_cap[s];
        }
    }
}

// LDS one workgroup may allocate on gfx950 (160 KiB per CU, minus the push
// kernel's static counters and tables)
constexpr size_t kMaxLds = 160 * 1024 - 2176;

static int validate(const pic_config *cfg, std::vector<BoxHost> &bh, std::string &err)
{
    if (!cfg || cfg->n_boxes < 1 || !cfg->boxes) { err = "need at least one box"; return PIC_EINVAL; }
    if (cfg->n_species < 1 || cfg->n_species > kMaxSpecies) { err = "n_species out of range"; return PIC_EINVAL; }
    for (int s = 0; s < cfg->n_species; ++s) {
        if (std::fabs(std::fabs(cfg->species[s].q_over_e) - 1.0) > 0 || !(cfg->species[s].m_over_me > 0)) {
            err = "species charge must be +-e and mass positive";
            return PIC_EINVAL;
        }
    }
    if (!(cfg->dt > 0)) { err = "dt must be positive"; return PIC_EINVAL; }
    if (cfg->flags & ~(uint32_t)(PIC_FP64_FORM | PIC_TRACK_IDS | PIC_FILTER_CURRENT | PIC_FARADAY4)) {
        err = "unknown flag";
        return PIC_EINVAL;
    }
    if (cfg->hist_bins < 0 || (cfg->hist_bins > 0 && !(cfg->hist_hi > cfg->hist_lo))) {
        err = "bad histogram range";
        return PIC_EINVAL;
    }
    const double hr = cfg->headroom > 0 ? cfg->headroom : 1.3;
    if (hr < 1.05) { err = "headroom must be >= 1.05"; return PIC_EINVAL; }
    bh.resize(cfg->n_boxes);
    for (int b = 0; b < cfg->n_boxes; ++b) {
        BoxHost &H = bh[b];
        H.cfg = cfg->boxes[b];
        const int lim[3] = {2048, 2048, 1024};
        for (int a = 0; a < 3; ++a) {
            if (H.cfg.n[a] < 1 || H.cfg.n[a] > lim[a]) { err = "box size out of range"; return PIC_EINVAL; }
            int t = H.cfg.tile[a] ? H.cfg.tile[a] : 4;
            if (t < 1 || t > 8 || (t & (t - 1))) { err = "tile edge must be 1, 2, 4 or 8"; return PIC_EINVAL; }
            H.tile[a] = t;
        }
        const size_t lds = (cfg->flags & PIC_FP64_FORM) ? push_lds_bytes<double>(H.tile[0], H.tile[1], H.tile[2])
                                                        : push_lds_bytes<float>(H.tile[0], H.tile[1], H.tile[2]);
        if (lds > kMaxLds) { err = "tile needs more LDS than a workgroup may use"; return PIC_EINVAL; }
        if (!(H.cfg.n_x > 0) || !(H.cfg.rho0 > 0)) { err = "n_x and rho0 must be positive"; return PIC_EINVAL; }
        if (H.cfg.walls < 0 || H.cfg.walls > 3) { err = "walls must be 0 (periodic) or 1 + axis"; return PIC_EINVAL; }
        if (H.cfg.walls && H.cfg.n[H.cfg.walls - 1] < 2) { err = "walls need two cells along their axis"; return PIC_EINVAL; }
        if (H.cfg.walls && (cfg->flags & PIC_FILTER_CURRENT)) {
            err = "current smoothing is not available with walls";
            return PIC_EINVAL;
        }
        if (H.cfg.walls && (cfg->flags & PIC_FARADAY4)) {
            // its curl reaches two cells out, across the wall plane
            err = "the fourth-order solver is not available with walls";
            return PIC_EINVAL;
        }
        H.nc = (int64_t)H.cfg.n[0] * H.cfg.n[1] * H.cfg.n[2];
        H.ntiles = 1;
        for (int a = 0; a < 3; ++a) H.ntiles *= (H.cfg.n[a] + H.tile[a] - 1) / H.tile[a];
        for (int s = 0; s < cfg->n_species; ++s) {
            const int64_t mp = H.cfg.max_particles[s];
            if (mp < 0) { err = "negative capacity"; return PIC_EINVAL; }
            const int64_t ovf = std::max<int64_t>(1024, mp / 16);
            const int64_t slots = (int64_t)std::ceil(mp * hr) + 32 * (int64_t)H.ntiles + ovf;
            // particle arrays are addressed with 32-bit byte offsets (8-byte elements in the FP64 form)
            if (slots >= (int64_t)1 << 29) { err = "more than 2^29 particle slots in one species"; return PIC_EINVAL; }
            H.slots[s] = (int32_t)slots;
            H.ovf_cap[s] = (int32_t)ovf;
            H.stage_cap[s] = (int32_t)std::max<int64_t>(mp, 1);
        }
    }
    return PIC_OK;
}

struct Layout {
    // the box descriptors twice: [1] has b and bn swapped.  The push reads b
    // and writes bn, so each step flips which array the kernels are given
    void *boxes[2] = {nullptr, nullptr};
    Item *items_push = nullptr, *items_box = nullptr;
    CellBlock *cblocks = nullptr;
    StageItem *sitems = nullptr;
    uint32_t *flags = nullptr;
    double *mj_cum = nullptr, *mj_tab[2] = {nullptr, nullptr};
    int n_items = 0, n_cblocks = 0, max_sitems = 0;
    size_t bytes = 0;
};

template <typename R>
static void make_layout(const pic_config *cfg, std::vector<BoxHost> &bh, char *base, Layout &L,
                        std::vector<BoxDev<R>> &bd)
{
    Bump A{base};
    L.boxes[0] = A.take<BoxDev<R>>(cfg->n_boxes);
    L.boxes[1] = A.take<BoxDev<R>>(cfg->n_boxes);
    L.n_items = 0;
    L.n_cblocks = 0;
    L.max_sitems = 0;
    for (auto &H : bh) {
        L.n_items += H.ntiles + kOvfBlocks;
        L.n_cblocks += (int)((H.nc + kBlock - 1) / kBlock);
        for (int s = 0; s < cfg->n_species; ++s) L.max_sitems += (H.stage_cap[s] + kBlock - 1) / kBlock;
    }
    L.items_push = A.take<Item>(8 * (size_t)L.n_items);   // room for the padding of the push order
    L.items_box = A.take<Item>(L.n_items);
    L.cblocks = A.take<CellBlock>(L.n_cblocks);
    L.sitems = A.take<StageItem>(std::max(1, L.max_sitems));
    L.flags = A.take<uint32_t>(64);
    L.mj_cum = A.take<double>(kTabM + 1);
    L.mj_tab[0] = A.take<double>(kTabN + 1);
    L.mj_tab[1] = A.take<double>(kTabN + 1);
    bd.resize(cfg->n_boxes);
    carve<R>(A, cfg, bh, bd);
    L.bytes = ((A.off + 255) & ~size_t(255)) + 256;
}

} // namespace pic

using namespace pic;

// Overflow watch: after every push the last block of the e update writes the
// fill of the fullest overflow region (thousandths of its capacity) straight
// into a slot of coherent pinned host memory; pic_step reads it kWatchLag steps later
// (waiting for that step only, so the stream stays kWatchLag steps ahead) and
// repacks at once when the fill is above kWatchLimit, instead of letting the
// overflow region - swept by the slow path - fill up or lose particles.
constexpr int kWatch = 4, kWatchLag = 2;
constexpr uint32_t kWatchLimit = 500;

struct pic_ctx {
    pic_config cfg;
    std::vector<pic_box> boxes;
    std::vector<BoxHost> bh;
    bool fp64 = false;
    hipStream_t stream = nullptr;
    char *arena = nullptr;
    Layout L;
    std::vector<BoxDev<float>> bd32;
    std::vector<BoxDev<double>> bd64;
    std::vector<int> box_item_off;          // first item of each box in items_box
    std::vector<int> box_cblock_off;        // first cell block of each box
    std::vector<std::vector<int32_t>> stage_n, stage_half, next_id;
    std::vector<std::vector<int64_t>> binned;   // particles binned per (box, species): capacity and push order
    std::vector<Item> items;                // work items in box order (host copy)
    std::vector<Item> push_perm;            // the push order uploaded last (host copy, kept for the copy)
    int n_push = 0;                         // blocks of a push launch
    int cur = 0;
    int bpar = 0;                           // which descriptor array holds the current b (Layout::boxes)
    int64_t step = 0;
    size_t lds_bytes = 0;
    bool fixed444 = false;             // every tile 4x4x4: the fixed-shape push kernel
    bool walls = false;                // some box has conducting walls
    bool pending = false;
    uint32_t flags_seen = 0;
    std::string err;
    // timing hook: event pairs per kind (0 push, 1 fields, 2 sort)
    int timing = 0;                    // 0 off, 1 every launch kind, 2 the push only
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[3];
    std::vector<hipEvent_t> ev_pool;
    uint32_t *watch_host = nullptr;          // pinned, coherent, kWatch slots
    uint32_t *watch_dev = nullptr;           // the same slots as the device addresses them
    hipEvent_t watch_ev[kWatch] = {};
    int64_t watch_step[kWatch] = {-1, -1, -1, -1};
    int64_t last_repack = 0;
    int64_t early_repacks = 0;
    ~pic_ctx()
    {
        for (auto &v : ev)
            for (auto &p : v) { hipEventDestroy(p.first); hipEventDestroy(p.second); }
        for (auto e : ev_pool) hipEventDestroy(e);
        for (auto e : watch_ev)
            if (e) hipEventDestroy(e);
        if (watch_host) hipHostFree(watch_host);
    }
};

// the device box descriptors in which b is the current b (b^{t-dt/2})
template <typename R>
static const BoxDev<R> *dev_boxes(const pic_ctx *ctx)
{
    return reinterpret_cast<const BoxDev<R> *>(ctx->L.boxes[ctx->bpar]);
}

// the current b of box descriptor D (host side)
template <typename R>
static R *cur_b(const pic_ctx *ctx, const BoxDev<R> &D)
{
    return ctx->bpar ? D.bn : D.b;
}

// An event of the timing hook.  These only take timestamps, so they are made
// without the system-scope fence an event otherwise performs when it is
// recorded (an L2 write-back and invalidation that costs every step it is
// recorded in: 2.6 % of the 64^3 step and 16 us of the 16^3 step's 44 with
// four such events per step).
static hipEvent_t take_event(pic_ctx *ctx)
{
    if (!ctx->ev_pool.empty()) {
        hipEvent_t e = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

// record the start (begin = true) or the end of a timed launch of kind k
// (timing 1: every kind; 2: the push only)
static void mark(pic_ctx *ctx, int k, bool begin)
{
    if (!ctx->timing || (ctx->timing == 2 && k != 0)) return;
    if (begin) {
        hipEvent_t a = take_event(ctx);
        if (!a) return;
        hipEventRecord(a, ctx->stream);
        ctx->ev[k].push_back({a, nullptr});
    } else if (!ctx->ev[k].empty() && !ctx->ev[k].back().second) {
        hipEvent_t b = take_event(ctx);
        if (!b) return;
        hipEventRecord(b, ctx->stream);
        ctx->ev[k].back().second = b;
    }
}

template <typename R> static std::vector<BoxDev<R>> &bdvec(pic_ctx *ctx);
template <> std::vector<BoxDev<float>> &bdvec<float>(pic_ctx *ctx) { return ctx->bd32; }
template <> std::vector<BoxDev<double>> &bdvec<double>(pic_ctx *ctx) { return ctx->bd64; }

#define HIPCHK(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            ctx->err = std::string(#call) + ": " + hipGetErrorString(e_);              \
            return PIC_EDEVICE;                                                        \
        }                                                                              \
    } while (0)

template <typename R>
static StepConst<R> step_const(pic_ctx *ctx)
{
    StepConst<R> C;
    memset(&C, 0, sizeof(C));
    C.dt = (R)ctx->cfg.dt;
    C.nsp = ctx->cfg.n_species;
    for (int s = 0; s < C.nsp; ++s) {
        const pic_species &S = ctx->cfg.species[s];
        C.kq[s] = (R)(S.q_over_e / S.m_over_me);   // (q/e)(m_e/m), App. A.2
        C.qs[s] = (R)(S.q_over_e > 0 ? 1 : -1);
        C.mass[s] = (R)S.m_over_me;
    }
    C.flags = ctx->L.flags;
    C.cur = ctx->cur;
    C.hist_bins = ctx->cfg.hist_bins;
    C.hist_lo = ctx->cfg.hist_lo;
    C.hist_hi = ctx->cfg.hist_hi;
    C.filter = (ctx->cfg.flags & PIC_FILTER_CURRENT) != 0;
    return C;
}

// Push order of the work items.  The items (per box its tiles, then its
// overflow sweeps, boxes in order) are cut into 8 runs of equal cost, one per
// XCD: blocks go round-robin over the 8 XCDs of the MI355X, so block b runs
// item (b / 8) of run (b % 8), and a box's neighbouring tiles meet in one L2.
// A tile costs its share of the box's particles plus a fixed set-up worth
// kTileCost particles; the cut falls on tile boundaries, so the runs differ by
// less than one tile.  Within a run the boxes go in decreasing cost per tile
// (the longest blocks first, so the run does not end on a long one), each box
// with its tiles in order and its sweeps last.  Runs of unequal length are
// padded with idle items (box -1).
constexpr double kTileCost = 256.0;

static void push_order(const pic_ctx *ctx, const std::vector<Item> &items, std::vector<Item> &perm)
{
    const int X = 8;
    const int n = (int)items.size();
    std::vector<double> per_tile(ctx->cfg.n_boxes);
    for (int b = 0; b < ctx->cfg.n_boxes; ++b) {
        double np = 0;
        for (int s = 0; s < ctx->cfg.n_species; ++s) np += (double)ctx->binned[b][s];
        per_tile[b] = np / ctx->bh[b].ntiles + kTileCost;
    }
    double total = 0;
    for (const Item &it : items) total += it.tile >= 0 ? per_tile[it.box] : 0.0;
    // runs: [cut[x], cut[x+1]); a cut goes after the tile that reaches x/X of
    // the total, and after that box's sweeps when the tile is the box's last
    std::vector<int> cut(X + 1, n);
    cut[0] = 0;
    double acc = 0;
    for (int i = 0, x = 1; i < n && x < X; ++i) {
        if (items[i].tile < 0) continue;
        acc += per_tile[items[i].box];
        if (acc >= total * x / X) {
            int j = i + 1;
            while (j < n && items[j].tile < 0 && items[j].box == items[i].box) ++j;
            while (x < X && acc >= total * x / X) cut[x++] = j;
        }
    }
    std::vector<std::vector<Item>> run(X);
    size_t longest = 0;
    for (int x = 0; x < X; ++x) {
        // the run's boxes (or box parts) in decreasing cost per tile
        std::vector<std::pair<int, int>> parts;   // [first item, end) of one box
        for (int i = cut[x]; i < cut[x + 1];) {
            int j = i;
            while (j < cut[x + 1] && items[j].box == items[i].box) ++j;
            parts.push_back({i, j});
            i = j;
        }
        std::stable_sort(parts.begin(), parts.end(), [&](const std::pair<int, int> &a, const std::pair<int, int> &b) {
            return per_tile[items[a.first].box] > per_tile[items[b.first].box];
        });
        for (auto &pr : parts)
            for (int i = pr.first; i < pr.second; ++i) run[x].push_back(items[i]);
        longest = std::max(longest, run[x].size());
    }
    perm.assign(longest * X, Item{-1, 0});
    for (int x = 0; x < X; ++x)
        for (size_t q = 0; q < run[x].size(); ++q) perm[q * X + x] = run[x][q];
}

// bin staged particles (and refresh the layout of the binned ones)
template <typename R>
static int merge_t(pic_ctx *ctx, bool force)
{
    if (!ctx->pending && !force) return PIC_OK;
    std::vector<StageItem> si;
    for (int b = 0; b < ctx->cfg.n_boxes; ++b)
        for (int s = 0; s < ctx->cfg.n_species; ++s)
            for (int f = 0; f < ctx->stage_n[b][s]; f += kBlock)
                si.push_back({b, s, f, std::min(ctx->stage_n[b][s], f + kBlock), ctx->stage_half[b][s]});
    if ((int)si.size() > ctx->L.max_sitems) { ctx->err = "stage item list overflow"; return PIC_ENOMEM; }
    if (!si.empty()) {
        HIPCHK(hipMemcpyAsync(ctx->L.sitems, si.data(), si.size() * sizeof(StageItem), hipMemcpyHostToDevice,
                              ctx->stream));
    }
    StepConst<R> C = step_const<R>(ctx);
    HIPCHK(launch_repack<R>(dev_boxes<R>(ctx), ctx->cfg.n_boxes, ctx->L.items_box,
                            ctx->L.n_items, ctx->L.sitems, (int)si.size(), C, ctx->stream));
    ctx->cur ^= 1;
    for (int b = 0; b < ctx->cfg.n_boxes; ++b)
        for (int s = 0; s < ctx->cfg.n_species; ++s) ctx->binned[b][s] += ctx->stage_n[b][s];
    if (!si.empty()) {
        // the boxes' particle counts changed: balance the push order again
        push_order(ctx, ctx->items, ctx->push_perm);
        HIPCHK(hipMemcpyAsync(ctx->L.items_push, ctx->push_perm.data(), ctx->push_perm.size() * sizeof(Item),
                              hipMemcpyHostToDevice, ctx->stream));
        ctx->n_push = (int)ctx->push_perm.size();
    }
    for (auto &v : ctx->stage_n) std::fill(v.begin(), v.end(), 0);
    ctx->pending = false;
    if (!si.empty()) HIPCHK(hipStreamSynchronize(ctx->stream));   // the host stage list must outlive the copy
    return PIC_OK;
}

static int merge(pic_ctx *ctx, bool force = false)
{
    return ctx->fp64 ? merge_t<double>(ctx, force) : merge_t<float>(ctx, force);
}

template <typename R>
static int init_t(pic_ctx *ctx)
{
    std::vector<BoxDev<R>> &bd = bdvec<R>(ctx);
    make_layout<R>(&ctx->cfg, ctx->bh, ctx->arena, ctx->L, bd);
    HIPCHK(hipMemsetAsync(ctx->arena, 0, ctx->L.bytes - 256, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->L.boxes[0], bd.data(), bd.size() * sizeof(BoxDev<R>), hipMemcpyHostToDevice,
                          ctx->stream));
    std::vector<BoxDev<R>> sw = bd;
    for (auto &D : sw) std::swap(D.b, D.bn);
    HIPCHK(hipMemcpyAsync(ctx->L.boxes[1], sw.data(), sw.size() * sizeof(BoxDev<R>), hipMemcpyHostToDevice,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));   // the host copy of the swapped array is local
    // work items: per box its tiles then its overflow sweeps (box order); the
    // push order (push_order) is balanced again whenever particles are binned
    std::vector<Item> items;
    std::vector<CellBlock> cbs;
    for (int b = 0; b < ctx->cfg.n_boxes; ++b) {
        ctx->box_item_off.push_back((int)items.size());
        for (int t = 0; t < ctx->bh[b].ntiles; ++t) items.push_back({b, t});
        for (int k = 0; k < kOvfBlocks; ++k) items.push_back({b, -1 - k});
        ctx->box_cblock_off.push_back((int)cbs.size());
        for (int64_t f = 0; f < ctx->bh[b].nc; f += kBlock) cbs.push_back({b, (int32_t)f});
    }
    ctx->box_item_off.push_back((int)items.size());
    ctx->box_cblock_off.push_back((int)cbs.size());
    const int n = (int)items.size();
    ctx->items = items;
    push_order(ctx, items, ctx->push_perm);
    ctx->n_push = (int)ctx->push_perm.size();
    HIPCHK(hipMemcpyAsync(ctx->L.items_box, items.data(), n * sizeof(Item), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->L.items_push, ctx->push_perm.data(), ctx->push_perm.size() * sizeof(Item),
                          hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->L.cblocks, cbs.data(), cbs.size() * sizeof(CellBlock), hipMemcpyHostToDevice,
                          ctx->stream));
    size_t lds = 0;
    bool all444 = true;
    for (auto &H : ctx->bh) {
        lds = std::max(lds, push_lds_bytes<R>(H.tile[0], H.tile[1], H.tile[2]));
        all444 = all444 && H.tile[0] == 4 && H.tile[1] == 4 && H.tile[2] == 4;
    }
    ctx->lds_bytes = lds;
    ctx->fixed444 = all444;
    ctx->walls = false;
    for (auto &H : ctx->bh) ctx->walls = ctx->walls || H.cfg.walls != 0;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    // initial segment layout: an empty repack
    return merge_t<R>(ctx, true);
}

// The exported functions take their C linkage from their declarations in pic.h.

int pic_plan(const pic_config *cfg, size_t *arena_bytes)
{
    std::vector<BoxHost> bh;
    std::string err;
    int rc = validate(cfg, bh, err);
    if (rc) return rc;
    if (!arena_bytes) return PIC_EINVAL;
    Layout L;
    if (cfg->flags & PIC_FP64_FORM) {
        std::vector<BoxDev<double>> bd;
        make_layout<double>(cfg, bh, nullptr, L, bd);
    } else {
        std::vector<BoxDev<float>> bd;
        make_layout<float>(cfg, bh, nullptr, L, bd);
    }
    *arena_bytes = L.bytes;
    return PIC_OK;
}

int pic_init(const pic_config *cfg, void *dev_arena, size_t bytes, void *hip_stream, pic_ctx **out)
{
    if (!out) return PIC_EINVAL;
    *out = nullptr;
    pic_ctx *ctx = new (std::nothrow) pic_ctx;
    if (!ctx) return PIC_ENOMEM;
    std::string err;
    int rc = validate(cfg, ctx->bh, err);
    if (rc) { delete ctx; return rc; }
    // stability (App. B): Courant for the 3-D Yee scheme, and omega_pe dt < 2;
    // with the fourth-order Faraday curl the largest mode has (dt/2)^2 sum_a
    // (4 + 2/3) < 1, i.e. dt < 2/sqrt(14)
    const double dt_max = (cfg->flags & PIC_FARADAY4) ? 2.0 / std::sqrt(14.0) : 1.0 / std::sqrt(3.0);
    if (!(cfg->dt < dt_max)) { delete ctx; return PIC_ECOURANT; }
    for (auto &H : ctx->bh)
        if (!(cfg->dt / H.cfg.n_x < 2.0)) { delete ctx; return PIC_ECOURANT; }
    size_t need = 0;
    pic_plan(cfg, &need);
    if (!dev_arena || bytes < need) { delete ctx; return PIC_ENOMEM; }
    if (reinterpret_cast<uintptr_t>(dev_arena) & 255) { delete ctx; return PIC_EINVAL; }
    ctx->cfg = *cfg;
    ctx->boxes.assign(cfg->boxes, cfg->boxes + cfg->n_boxes);
    ctx->cfg.boxes = ctx->boxes.data();
    ctx->fp64 = (cfg->flags & PIC_FP64_FORM) != 0;
    ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
    ctx->arena = reinterpret_cast<char *>(dev_arena);
    ctx->stage_n.assign(cfg->n_boxes, std::vector<int32_t>(kMaxSpecies, 0));
    ctx->binned.assign(cfg->n_boxes, std::vector<int64_t>(kMaxSpecies, 0));
    ctx->stage_half.assign(cfg->n_boxes, std::vector<int32_t>(kMaxSpecies, 0));
    ctx->next_id.assign(cfg->n_boxes, std::vector<int32_t>(kMaxSpecies, 0));
    // the e update writes the watch straight into these slots (coherent, so
    // the host reads it once the step's event has completed): no copy per step
    if (hipHostMalloc(reinterpret_cast<void **>(&ctx->watch_host), kWatch * sizeof(uint32_t),
                      hipHostMallocCoherent) != hipSuccess) {
        ctx->watch_host = nullptr;
        delete ctx;
        return PIC_EDEVICE;
    }
    for (int i = 0; i < kWatch; ++i) ctx->watch_host[i] = 0;
    if (hipHostGetDevicePointer(reinterpret_cast<void **>(&ctx->watch_dev), ctx->watch_host, 0) != hipSuccess) {
        delete ctx;
        return PIC_EDEVICE;
    }
    for (auto &e : ctx->watch_ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            delete ctx;
            return PIC_EDEVICE;
        }
    // device address of pic_diag_noalloc's static scratch on this device (once per device)
    if (diag_scratch_setup() != hipSuccess) {
        delete ctx;
        return PIC_EDEVICE;
    }
    rc = ctx->fp64 ? init_t<double>(ctx) : init_t<float>(ctx);
    if (rc) {
        fprintf(stderr, "pic_init: %s\n", ctx->err.c_str());
        delete ctx;
        return rc;
    }
    *out = ctx;
    return PIC_OK;
}

const char *pic_last_error(const pic_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int64_t pic_steps_done(const pic_ctx *ctx) { return ctx ? ctx->step : -1; }

int pic_free(pic_ctx *ctx)
{
    if (!ctx) return PIC_EINVAL;
    delete ctx;
    return PIC_OK;
}

static int check_box(pic_ctx *ctx, int box)
{
    if (!ctx) return PIC_EINVAL;
    if (box < 0 || box >= ctx->cfg.n_boxes) { ctx->err = "box index out of range"; return PIC_EINVAL; }
    return PIC_OK;
}

static int read_flags(pic_ctx *ctx, uint32_t *out)
{
    uint32_t f = 0;
    HIPCHK(hipMemcpyAsync(&f, ctx->L.flags, sizeof(f), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (f) {
        uint32_t z = 0;
        HIPCHK(hipMemcpyAsync(ctx->L.flags, &z, sizeof(z), hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    *out = f;
    return PIC_OK;
}

int pic_sync(pic_ctx *ctx)
{
    if (!ctx) return PIC_EINVAL;
    uint32_t f = 0;
    int rc = read_flags(ctx, &f);
    if (rc) return rc;
    if (f) {
        ctx->err = "device error flag raised: " + std::to_string(f);
        return PIC_EFLAG;
    }
    return PIC_OK;
}

template <typename R>
static int step_t(pic_ctx *ctx, int n)
{
    for (int i = 0; i < n; ++i) {
        // early repack when the overflow watch of kWatchLag steps ago says so
        const int64_t look = ctx->step - kWatchLag;
        if (look > ctx->last_repack && ctx->watch_step[look % kWatch] == look) {
            HIPCHK(hipEventSynchronize(ctx->watch_ev[look % kWatch]));
            if (ctx->watch_host[look % kWatch] > kWatchLimit) {
                mark(ctx, 2, true);
                int rc = merge_t<R>(ctx, true);
                mark(ctx, 2, false);
                if (rc) return rc;
                ctx->last_repack = ctx->step;
                ctx->early_repacks += 1;
            }
        }
        StepConst<R> C = step_const<R>(ctx);
        mark(ctx, 0, true);
        HIPCHK(launch_push<R>(dev_boxes<R>(ctx), ctx->L.items_push, ctx->n_push, ctx->lds_bytes, C,
                              ctx->fixed444 ? 1 : 0, ctx->walls ? 1 : 0, (ctx->cfg.flags & PIC_FARADAY4) ? 1 : 0,
                              ctx->stream));
        mark(ctx, 0, false);
        // the push wrote b^{t+dt/2} into the other b buffer: it is the current one now
        ctx->bpar ^= 1;
        mark(ctx, 1, true);
        // the e update's last block also takes the overflow watch of the copy
        // just written, into the host slot of the step about to complete
        const int w = (int)((ctx->step + 1) % kWatch);
        HIPCHK(launch_fields<R>(dev_boxes<R>(ctx), ctx->L.cblocks, ctx->L.n_cblocks, (R)ctx->cfg.dt,
                                ctx->cfg.n_species, C.filter, ctx->cur, ctx->cfg.n_boxes, ctx->watch_dev + w,
                                ctx->stream));
        mark(ctx, 1, false);
        ctx->cur ^= 1;
        ctx->step += 1;
        HIPCHK(hipEventRecord(ctx->watch_ev[w], ctx->stream));
        ctx->watch_step[w] = ctx->step;
        if (ctx->cfg.sort_interval > 0 && ctx->step % ctx->cfg.sort_interval == 0) {
            mark(ctx, 2, true);
            int rc = merge_t<R>(ctx, true);
            mark(ctx, 2, false);
            if (rc) return rc;
            ctx->last_repack = ctx->step;
        }
    }
    return PIC_OK;
}

int pic_step(pic_ctx *ctx, int n)
{
    if (!ctx || n < 0) return PIC_EINVAL;
    int rc = merge(ctx);
    if (rc) return rc;
    return ctx->fp64 ? step_t<double>(ctx, n) : step_t<float>(ctx, n);
}

// The diagnostics summed into `buf` (the arena's buffers of the box, or the
// static scratch of pic_diag_noalloc).  Allocates nothing: the histogram goes
// straight into the caller's array.
template <typename R>
static int diag_t(pic_ctx *ctx, int box, pic_diag_out *o, int64_t *hist, const DiagBuf &buf)
{
    const BoxDev<R> *boxes = dev_boxes<R>(ctx);
    const BoxDev<R> &D = bdvec<R>(ctx)[box];
    const int nsp = ctx->cfg.n_species;
    const int hist_len = std::max(1, ctx->cfg.hist_bins) * kMaxSpecies;
    StepConst<R> C = step_const<R>(ctx);
    const int i0 = ctx->box_item_off[box], i1 = ctx->box_item_off[box + 1];
    HIPCHK(launch_diag<R>(boxes, box, D.nc, ctx->L.items_box + i0, i1 - i0, C, buf, hist_len, ctx->stream));
    double acc[kAccLen];
    HIPCHK(hipMemcpyAsync(acc, buf.acc, sizeof(acc), hipMemcpyDeviceToHost, ctx->stream));
    if (hist && ctx->cfg.hist_bins > 0)   // device layout [species][bins], as the caller's
        HIPCHK(hipMemcpyAsync(hist, buf.hist, (size_t)nsp * ctx->cfg.hist_bins * sizeof(int64_t),
                              hipMemcpyDeviceToHost, ctx->stream));
    int32_t novf[kMaxSpecies] = {0, 0, 0, 0};
    for (int s = 0; s < nsp; ++s)
        HIPCHK(hipMemcpyAsync(&novf[s], D.sp[s].nb[ctx->cur] + D.ntiles, sizeof(int32_t), hipMemcpyDeviceToHost,
                              ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    memset(o, 0, sizeof(*o));
    o->t = ctx->step * ctx->cfg.dt;
    o->step = ctx->step;
    for (int c = 0; c < 3; ++c) {
        o->W_E[c] = acc[kAccField + c] / D.alpha0;
        o->W_B[c] = acc[kAccField + 3 + c] / D.alpha0;
    }
    o->gauss_max = acc[kAccField + 6];
    o->gauss_rms = std::sqrt(acc[kAccField + 7] / (double)D.nc);
    for (int s = 0; s < nsp; ++s) {
        const double *a = acc + kAccSp + 6 * s;
        o->K[s] = a[0];
        o->P[s][0] = a[1]; o->P[s][1] = a[2]; o->P[s][2] = a[3];
        o->n_particles[s] = (int64_t)std::llround(a[4]);
        o->sum_gm1[s] = a[5];
        o->n_overflow[s] = std::min(novf[s], D.sp[s].ovf_cap);
    }
    uint32_t f = 0;
    int rc = read_flags(ctx, &f);
    if (rc) return rc;
    o->flags = f;
    if (f) {
        ctx->err = "device error flag raised: " + std::to_string(f);
        return PIC_EFLAG;
    }
    return PIC_OK;
}

int pic_diag(pic_ctx *ctx, int box, pic_diag_out *out, int64_t *hist)
{
    int rc = check_box(ctx, box);
    if (rc) return rc;
    if (!out) return PIC_EINVAL;
    rc = merge(ctx);
    if (rc) return rc;
    if (ctx->fp64) {
        const BoxDev<double> &D = bdvec<double>(ctx)[box];
        return diag_t<double>(ctx, box, out, hist, DiagBuf{D.acc, D.rho, D.hist});
    }
    const BoxDev<float> &D = bdvec<float>(ctx)[box];
    return diag_t<float>(ctx, box, out, hist, DiagBuf{D.acc, D.rho, D.hist});
}

// Bytes of the static scratch that pic_diag_noalloc needs for box `box`:
// accumulators, charge density, histogram, each 256-B aligned.
static size_t noalloc_diag_bytes(const pic_ctx *ctx, int box)
{
    auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
    const size_t hist_len = (size_t)std::max(1, ctx->cfg.hist_bins) * kMaxSpecies;
    return up(kAccLen * sizeof(double)) + up((size_t)ctx->bh[box].nc * sizeof(double)) +
           up(hist_len * sizeof(int64_t));
}

int pic_diag_noalloc(pic_ctx *ctx, int box, pic_diag_out *out, int64_t *hist)
{
    int rc = check_box(ctx, box);
    if (rc) return rc;
    if (!out) return PIC_EINVAL;
    if (ctx->pending) {
        // binning staged particles would copy a host-built list; pic_step or
        // pic_diag bins them
        ctx->err = "pic_diag_noalloc: loaded or set particles are not binned yet (call pic_step or pic_diag first)";
        return PIC_ESTATE;
    }
    const size_t need = noalloc_diag_bytes(ctx, box);
    if (need > kDiagScratchBytes) {
        ctx->err = "pic_diag_noalloc: the box needs more than the static scratch holds (8 bytes per cell plus "
                   "accumulators and histogram, at most 32 MiB)";
        return PIC_ENOMEM;
    }
    char *p = reinterpret_cast<char *>(diag_scratch());
    if (!p) {
        ctx->err = "pic_diag_noalloc: the static scratch is not set up on the current device";
        return PIC_EDEVICE;
    }
    auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
    DiagBuf buf;
    buf.acc = reinterpret_cast<double *>(p);
    buf.rho = reinterpret_cast<double *>(p + up(kAccLen * sizeof(double)));
    buf.hist = reinterpret_cast<int64_t *>(p + up(kAccLen * sizeof(double)) +
                                           up((size_t)ctx->bh[box].nc * sizeof(double)));
    return ctx->fp64 ? diag_t<double>(ctx, box, out, hist, buf) : diag_t<float>(ctx, box, out, hist, buf);
}

template <typename R>
static int spectrum_t(pic_ctx *ctx, int box, int field, int comp, int normal, double *ps)
{
    const BoxDev<R> &D = bdvec<R>(ctx)[box];
    const BoxDev<R> *boxes = dev_boxes<R>(ctx);
    const int a1 = normal == 0 ? 1 : 0, a2 = normal == 2 ? 1 : 2;
    const size_t nps = (size_t)D.n[a1] * D.n[a2];
    // scratch: the box's current (cleared between steps) and its diagnostic charge array
    HIPCHK(launch_spectrum<R>(boxes, box, D.n, field, comp, normal, (R)(0.5 * ctx->cfg.dt),
                              reinterpret_cast<double *>(D.J), D.rho, ctx->stream));
    HIPCHK(hipMemcpyAsync(ps, D.rho, nps * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return PIC_OK;
}

int pic_field_spectrum(pic_ctx *ctx, int box, int field, int comp, int normal_axis, double *ps)
{
    int rc = check_box(ctx, box);
    if (rc) return rc;
    if (field < 0 || field > 1 || comp < 0 || comp > 2 || normal_axis < 0 || normal_axis > 2 || !ps)
        return PIC_EINVAL;
    rc = merge(ctx);
    if (rc) return rc;
    return ctx->fp64 ? spectrum_t<double>(ctx, box, field, comp, normal_axis, ps)
                     : spectrum_t<float>(ctx, box, field, comp, normal_axis, ps);
}

template <typename R>
static int get_particles_t(pic_ctx *ctx, int box, int s, double *x, double *u, int32_t *id, int64_t *n)
{
    const BoxDev<R> &D = bdvec<R>(ctx)[box];
    const SpeciesDev<R> &S = D.sp[s];
    const int nt = D.ntiles;
    std::vector<int32_t> start(nt + 1), cap(nt + 1), na(nt + 1), nb(nt + 1), bs(nt + 1);
    HIPCHK(hipMemcpyAsync(start.data(), S.seg_start[ctx->cur], (nt + 1) * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(cap.data(), S.seg_cap[ctx->cur], (nt + 1) * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(na.data(), S.na[ctx->cur], (nt + 1) * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(nb.data(), S.nb[ctx->cur], (nt + 1) * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(bs.data(), S.bs[ctx->cur], (nt + 1) * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    // slots in use: per tile the A range [0, na) and the B range [bs, bs + nb)
    // (clamped to the segment), then the overflow region
    std::vector<int64_t> order;
    for (int t = 0; t < nt; ++t) {
        for (int k = 0; k < na[t]; ++k) order.push_back(start[t] + k);
        const int nbv = std::max(0, std::min(nb[t], cap[t] - bs[t]));
        for (int k = 0; k < nbv; ++k) order.push_back(start[t] + bs[t] + k);
    }
    for (int k = 0; k < std::min(nb[nt], cap[nt]); ++k) order.push_back(start[nt] + k);
    const int64_t total = (int64_t)order.size();
    if (*n < total) {
        *n = total;
        ctx->err = "output arrays too small";
        return PIC_ENOMEM;
    }
    const size_t ns = S.slots;
    std::vector<int32_t> cell(ns), pid(S.buf[ctx->cur].id ? ns : 0);
    std::vector<R> dd[3], uu[3];
    const PBuf<R> &P = S.buf[ctx->cur];
    std::vector<uint8_t> code(ns);
    HIPCHK(hipMemcpyAsync(cell.data(), P.cell, ns * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(code.data(), P.lc, ns, hipMemcpyDeviceToHost, ctx->stream));
    for (int a = 0; a < 3; ++a) {
        dd[a].resize(ns);
        uu[a].resize(ns);
        HIPCHK(hipMemcpyAsync(dd[a].data(), P.d[a], ns * sizeof(R), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipMemcpyAsync(uu[a].data(), P.u[a], ns * sizeof(R), hipMemcpyDeviceToHost, ctx->stream));
    }
    if (P.id) HIPCHK(hipMemcpyAsync(pid.data(), P.id, ns * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    // a tile's ranges hold tile-local cell codes: the packed cell is the
    // tile's origin plus the code's bits
    for (int t = 0; t < nt; ++t) {
        int o[3];
        tile_origin(D, t, o);
        auto decode = [&](int64_t k) { cell[k] = local_cell(D, o, code[k]); };
        for (int k = 0; k < na[t]; ++k) decode(start[t] + k);
        const int nbv = std::max(0, std::min(nb[t], cap[t] - bs[t]));
        for (int k = 0; k < nbv; ++k) decode(start[t] + bs[t] + k);
    }
    if (P.id) std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return pid[a] < pid[b]; });
    for (int64_t q = 0; q < total; ++q) {
        const int64_t k = order[q];
        const int c[3] = {cell_x(cell[k]), cell_y(cell[k]), cell_z(cell[k])};
        for (int a = 0; a < 3; ++a) {
            if (x) x[3 * q + a] = (double)c[a] + (double)dd[a][k];
            if (u) u[3 * q + a] = (double)uu[a][k];
        }
        if (id) id[q] = P.id ? pid[k] : 0;
    }
    *n = total;
    return PIC_OK;
}

int pic_get_particles(pic_ctx *ctx, int box, int species, double *x, double *u, int32_t *id, int64_t *n)
{
    int rc = check_box(ctx, box);
    if (rc) return rc;
    if (species < 0 || species >= ctx->cfg.n_species || !n) return PIC_EINVAL;
    rc = merge(ctx);
    if (rc) return rc;
    return ctx->fp64 ? get_particles_t<double>(ctx, box, species, x, u, id, n)
                     : get_particles_t<float>(ctx, box, species, x, u, id, n);
}

template <typename R>
static int set_particles_t(pic_ctx *ctx, int box, int s, const double *x, const double *u, const int32_t *id,
                           int64_t n)
{
    const BoxDev<R> &D = bdvec<R>(ctx)[box];
    const SpeciesDev<R> &S = D.sp[s];
    if (n > ctx->bh[box].stage_cap[s]) { ctx->err = "more particles than the species capacity"; return PIC_ENOMEM; }
    // drop the binned particles of (box, s): clear the counters of the current copy
    HIPCHK(hipMemsetAsync(S.na[ctx->cur], 0, (D.ntiles + 1) * sizeof(int32_t), ctx->stream));
    HIPCHK(hipMemsetAsync(S.nb[ctx->cur], 0, (D.ntiles + 1) * sizeof(int32_t), ctx->stream));
    ctx->binned[box][s] = 0;
    std::vector<int32_t> cell(n), pid(S.stage.id ? n : 0);
    std::vector<R> dd[3], uu[3];
    for (int a = 0; a < 3; ++a) { dd[a].resize(n); uu[a].resize(n); }
    for (int64_t p = 0; p < n; ++p) {
        int c[3];
        for (int a = 0; a < 3; ++a) {
            const int N = D.n[a];
            double v = std::fmod(x[3 * p + a], (double)N);
            if (v < 0) v += N;
            if (v >= N) v -= N;
            const double f = std::floor(v);
            R off = (R)(v - f);
            int ci = (int)f;
            if (off >= R(1)) { off = R(0); ci += 1; }
            if (ci >= N) ci -= N;
            c[a] = ci;
            dd[a][p] = off;
            uu[a][p] = (R)u[3 * p + a];
        }
        cell[p] = pack_cell(c[0], c[1], c[2]);
        if (S.stage.id) pid[p] = id ? id[p] : (int32_t)p;
    }
    if (n > 0) {
        HIPCHK(hipMemcpyAsync(S.stage.cell, cell.data(), n * 4, hipMemcpyHostToDevice, ctx->stream));
        for (int a = 0; a < 3; ++a) {
            HIPCHK(hipMemcpyAsync(S.stage.d[a], dd[a].data(), n * sizeof(R), hipMemcpyHostToDevice, ctx->stream));
            HIPCHK(hipMemcpyAsync(S.stage.u[a], uu[a].data(), n * sizeof(R), hipMemcpyHostToDevice, ctx->stream));
        }
        if (S.stage.id) HIPCHK(hipMemcpyAsync(S.stage.id, pid.data(), n * 4, hipMemcpyHostToDevice, ctx->stream));
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->stage_n[box][s] = (int32_t)n;
    ctx->stage_half[box][s] = 0;
    ctx->next_id[box][s] = (int32_t)n;
    ctx->pending = true;
    return PIC_OK;
}

int pic_set_particles(pic_ctx *ctx, int box, int species, const double *x, const double *u, const int32_t *id,
                      int64_t n)
{
    int rc = check_box(ctx, box);
    if (rc) return rc;
    if (species < 0 || species >= ctx->cfg.n_species || n < 0 || (n > 0 && (!x || !u))) return PIC_EINVAL;
    // other pending loads are binned first so that the flags of a stage stay uniform
    if (ctx->pending) {
        rc = merge(ctx);
        if (rc) return rc;
    }
    return ctx->fp64 ? set_particles_t<double>(ctx, box, species, x, u, id, n)
                     : set_particles_t<float>(ctx, box, species, x, u, id, n);
}

template <typename R>
static int get_fields_t(pic_ctx *ctx, int box, double *e, double *b, double *j)
{
    using JT = typename JType<R>::T;
    const BoxDev<R> &D = bdvec<R>(ctx)[box];
    const size_t n3 = 3 * D.nc;
    std::vector<R> tmp(n3);
    if (e) {
        HIPCHK(hipMemcpyAsync(tmp.data(), D.e, n3 * sizeof(R), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        for (size_t q = 0; q < n3; ++q) e[q] = (double)tmp[q];
    }
    if (b) {
        HIPCHK(hipMemcpyAsync(tmp.data(), cur_b(ctx, D), n3 * sizeof(R), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        for (size_t q = 0; q < n3; ++q) b[q] = (double)tmp[q];
    }
    if (j) {
        std::vector<JT> jt(n3);
        HIPCHK(hipMemcpyAsync(jt.data(), D.J, n3 * sizeof(JT), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        const double sc = ctx->fp64 ? 1.0 : std::ldexp(1.0, -kQBits);
        for (size_t q = 0; q < n3; ++q) j[q] = (double)jt[q] * sc;
    }
    return PIC_OK;
}

int pic_get_fields(pic_ctx *ctx, int box, double *e, double *b, double *j)
{
    int rc = check_box(ctx, box);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return ctx->fp64 ? get_fields_t<double>(ctx, box, e, b, j) : get_fields_t<float>(ctx, box, e, b, j);
}

template <typename R>
static int set_fields_t(pic_ctx *ctx, int box, const double *e, const double *b)
{
    const BoxDev<R> &D = bdvec<R>(ctx)[box];
    const size_t n3 = 3 * D.nc;
    std::vector<R> tmp(n3);
    // with conducting walls the given fields take the conductor's condition on
    // the wall plane (index 0 along the wall axis): no tangential e, no
    // normal b (App. A.4)
    auto on_wall = [&](size_t p) {
        const int64_t i = (int64_t)(p % D.n[0]), j = (int64_t)((p / D.n[0]) % D.n[1]),
                      k = (int64_t)(p / ((size_t)D.n[0] * D.n[1]));
        return D.wall >= 0 && (D.wall == 0 ? i : (D.wall == 1 ? j : k)) == 0;
    };
    if (e) {
        for (size_t q = 0; q < n3; ++q)
            tmp[q] = ((int)(q / D.nc) != D.wall && on_wall(q % D.nc)) ? R(0) : (R)e[q];
        HIPCHK(hipMemcpyAsync(D.e, tmp.data(), n3 * sizeof(R), hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    if (b) {
        for (size_t q = 0; q < n3; ++q)
            tmp[q] = ((int)(q / D.nc) == D.wall && on_wall(q % D.nc)) ? R(0) : (R)b[q];
        HIPCHK(hipMemcpyAsync(cur_b(ctx, D), tmp.data(), n3 * sizeof(R), hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    return PIC_OK;
}

int pic_set_fields(pic_ctx *ctx, int box, const double *e, const double *b)
{
    int rc = check_box(ctx, box);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return ctx->fp64 ? set_fields_t<double>(ctx, box, e, b) : set_fields_t<float>(ctx, box, e, b);
}

template <typename R>
static int load_t(pic_ctx *ctx, const pic_load_desc *d)
{
    const int box = d->box;
    const BoxHost &H = ctx->bh[box];
    const BoxDev<R> *boxes = dev_boxes<R>(ctx);
    int64_t npairs;
    if (d->profile == PIC_PROFILE_UNIFORM) {
        npairs = std::llround(d->ppc * (double)H.nc);
    } else {
        const double cross = (double)H.nc / H.cfg.n[d->profile_axis];
        npairs = std::llround(d->ppc * cross * 2.0 * d->thickness * std::tanh(d->half_width / d->thickness));
    }
    const int sa = d->species_a, sb = d->species_b;
    // particles already binned count against the capacity too
    const int64_t need_a = ctx->binned[box][sa] + ctx->stage_n[box][sa] + npairs + (sa == sb ? npairs : 0);
    const int64_t need_b = ctx->binned[box][sb] + ctx->stage_n[box][sb] + npairs;
    if (need_a > H.stage_cap[sa] || need_b > H.stage_cap[sb]) {
        ctx->err = "load exceeds the species capacity";
        return PIC_ENOMEM;
    }
    if (npairs == 0) return PIC_OK;
    const pic_mj *pops[2] = {&d->mj_a, &d->mj_b};
    for (int q = 0; q < 2; ++q)
        HIPCHK(launch_mj_table(pops[q]->theta, pops[q]->gamma_beta, ctx->L.mj_cum, kTabM, kTabN, ctx->L.mj_tab[q],
                               ctx->stream));
    LoadArgs L;
    memset(&L, 0, sizeof(L));
    L.box = box;
    L.sa = sa;
    L.sb = sb;
    L.npairs = npairs;
    L.offa = ctx->stage_n[box][sa];
    L.offb = ctx->stage_n[box][sb] + (sa == sb ? (int32_t)npairs : 0);
    L.ida = ctx->next_id[box][sa];
    L.idb = ctx->next_id[box][sb] + (sa == sb ? (int32_t)npairs : 0);
    L.profile = d->profile;
    L.paxis = d->profile_axis;
    L.centre = d->centre;
    L.thick = d->thickness;
    L.halfw = d->half_width;
    L.seed = d->seed;
    L.stream = d->stream;
    L.N = kTabN;
    for (int q = 0; q < 2; ++q) {
        MJPop &P = q == 0 ? L.A : L.B;
        P.mu = 1.0 / pops[q]->theta;
        P.G = std::sqrt(1.0 + pops[q]->gamma_beta * pops[q]->gamma_beta);
        P.beta0 = pops[q]->gamma_beta / P.G;
        P.axis = pops[q]->axis;
        P.tab = ctx->L.mj_tab[q];
    }
    HIPCHK(launch_load_pairs<R>(boxes, L, ctx->stream));
    ctx->stage_n[box][sa] = (int32_t)(L.offa + npairs);
    ctx->stage_n[box][sb] = (int32_t)(L.offb + npairs);
    ctx->next_id[box][sa] = (int32_t)(L.ida + npairs);
    ctx->next_id[box][sb] = (int32_t)(L.idb + npairs);
    ctx->stage_half[box][sa] = 1;
    ctx->stage_half[box][sb] = 1;
    ctx->pending = true;
    return PIC_OK;
}

int pic_load_maxwell_juttner(pic_ctx *ctx, const pic_load_desc *d)
{
    if (!ctx || !d) return PIC_EINVAL;
    int rc = check_box(ctx, d->box);
    if (rc) return rc;
    const int nsp = ctx->cfg.n_species;
    if (d->species_a < 0 || d->species_a >= nsp || d->species_b < 0 || d->species_b >= nsp) {
        ctx->err = "species index out of range";
        return PIC_EINVAL;
    }
    const pic_mj *pops[2] = {&d->mj_a, &d->mj_b};
    for (auto *p : pops)
        if (!(p->theta > 0) || p->axis < 0 || p->axis > 2 || !std::isfinite(p->gamma_beta)) {
            ctx->err = "bad Maxwell-Juttner parameters";
            return PIC_EINVAL;
        }
    if (!(d->ppc >= 0) || (d->profile != PIC_PROFILE_UNIFORM && d->profile != PIC_PROFILE_HARRIS)) {
        ctx->err = "bad density profile";
        return PIC_EINVAL;
    }
    if (d->profile == PIC_PROFILE_HARRIS &&
        (d->profile_axis < 0 || d->profile_axis > 2 || !(d->thickness > 0) || !(d->half_width > 0))) {
        ctx->err = "bad Harris profile";
        return PIC_EINVAL;
    }
    // a stage holds one kind of batch: bin set_particles batches first
    if (ctx->stage_n[d->box][d->species_a] && !ctx->stage_half[d->box][d->species_a]) merge(ctx);
    if (ctx->stage_n[d->box][d->species_b] && !ctx->stage_half[d->box][d->species_b]) merge(ctx);
    return ctx->fp64 ? load_t<double>(ctx, d) : load_t<float>(ctx, d);
}

int pic_set_harris_field(pic_ctx *ctx, const pic_harris_field *h)
{
    if (!ctx || !h) return PIC_EINVAL;
    int rc = check_box(ctx, h->box);
    if (rc) return rc;
    if (h->grad_axis < 0 || h->grad_axis > 2 || h->field_axis < 0 || h->field_axis > 2 ||
        h->grad_axis == h->field_axis || !(h->thickness > 0) || (h->n_sheets != 1 && h->n_sheets != 2)) {
        ctx->err = "bad Harris field";
        return PIC_EINVAL;
    }
    const int c0 = ctx->box_cblock_off[h->box], c1 = ctx->box_cblock_off[h->box + 1];
    if (ctx->fp64) {
        const BoxDev<double> *boxes = dev_boxes<double>(ctx);
        HIPCHK(launch_harris_field<double>(boxes, ctx->bh[h->box].nc, *h, ctx->stream));
        HIPCHK(launch_advance_b<double>(boxes, ctx->L.cblocks + c0, c1 - c0, -0.5 * ctx->cfg.dt, ctx->stream));
    } else {
        const BoxDev<float> *boxes = dev_boxes<float>(ctx);
        HIPCHK(launch_harris_field<float>(boxes, ctx->bh[h->box].nc, *h, ctx->stream));
        HIPCHK(launch_advance_b<float>(boxes, ctx->L.cblocks + c0, c1 - c0, (float)(-0.5 * ctx->cfg.dt), ctx->stream));
    }
    return PIC_OK;
}


int pic_set_timing(pic_ctx *ctx, int enable)
{
    if (!ctx) return PIC_EINVAL;
    if (enable < 0 || enable > 2) return PIC_EINVAL;
    ctx->timing = enable;
    return PIC_OK;
}

int pic_get_timing(pic_ctx *ctx, pic_timing *out, int reset)
{
    if (!ctx || !out) return PIC_EINVAL;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    int64_t n[3] = {0, 0, 0};
    double ms[3] = {0, 0, 0};
    for (int k = 0; k < 3; ++k)
        for (auto &p : ctx->ev[k]) {
            if (!p.second) continue;
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, p.first, p.second));
            ms[k] += t;
            n[k] += 1;
        }
    out->push_launches = n[0];
    out->push_ms = ms[0];
    out->field_launches = n[1];
    out->field_ms = ms[1];
    out->sort_launches = n[2];
    out->sort_ms = ms[2];
    if (reset)
        for (auto &v : ctx->ev) {
            for (auto &p : v) {
                ctx->ev_pool.push_back(p.first);
                if (p.second) ctx->ev_pool.push_back(p.second);
            }
            v.clear();
        }
    return PIC_OK;
}

// ------------------------------------------------------------------ autotuner

// One trial: a context in the caller's arena, the loads, steps/2 warm-up and
// `steps` timed steps on the stream; ms per step, or a negative value when the
// configuration does not fit the arena or fails.
static double tune_trial(const pic_config *cfg, const pic_load_desc *loads, int n_loads, void *arena, size_t bytes,
                         void *stream, int steps)
{
    size_t need = 0;
    if (pic_plan(cfg, &need) != PIC_OK || need > bytes) return -1.0;
    pic_ctx *ctx = nullptr;
    if (pic_init(cfg, arena, bytes, stream, &ctx) != PIC_OK) return -1.0;
    double ms = -1.0;
    hipEvent_t a = nullptr, b = nullptr;
    bool ok = hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess;
    for (int i = 0; ok && i < n_loads; ++i) ok = pic_load_maxwell_juttner(ctx, &loads[i]) == PIC_OK;
    ok = ok && pic_step(ctx, std::max(1, steps / 2)) == PIC_OK && pic_sync(ctx) == PIC_OK;
    ok = ok && hipEventRecord(a, ctx->stream) == hipSuccess && pic_step(ctx, steps) == PIC_OK &&
         hipEventRecord(b, ctx->stream) == hipSuccess && pic_sync(ctx) == PIC_OK;
    float t = 0.f;
    if (ok && hipEventElapsedTime(&t, a, b) == hipSuccess) ms = t / steps;
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    pic_free(ctx);
    return ms;
}

int pic_autotune(const pic_config *cfg, const pic_load_desc *loads, int n_loads, void *dev_arena, size_t bytes,
                 void *hip_stream, int steps, pic_config *cfg_out, pic_box *boxes_out, pic_tune_result *res)
{
    if (!cfg || !cfg_out || !boxes_out || !res || steps < 1 || n_loads < 0 || (n_loads > 0 && !loads))
        return PIC_EINVAL;
    std::vector<BoxHost> bh;
    std::string err;
    int rc = validate(cfg, bh, err);
    if (rc) return rc;
    const int nb = cfg->n_boxes;
    std::vector<pic_box> boxes(cfg->boxes, cfg->boxes + nb);
    for (auto &b : boxes)
        for (int a = 0; a < 3; ++a)
            if (!b.tile[a]) b.tile[a] = 4;
    pic_config c = *cfg;
    c.boxes = boxes.data();
    // density classes: superparticle capacity per cell below 32, below 128, above
    std::vector<int> cls(nb);
    for (int i = 0; i < nb; ++i) {
        double np = 0;
        for (int s = 0; s < cfg->n_species; ++s) np += (double)boxes[i].max_particles[s];
        const double d = np / ((double)boxes[i].n[0] * boxes[i].n[1] * boxes[i].n[2]);
        cls[i] = d < 32 ? 0 : (d < 128 ? 1 : 2);
    }
    res->trials = 0;
    double best = tune_trial(&c, loads, n_loads, dev_arena, bytes, hip_stream, steps);
    ++res->trials;
    if (best < 0) return PIC_EDEVICE;
    res->ms_per_step_default = best;
    static const int cand[][3] = {{4, 4, 4}, {8, 4, 4}, {8, 8, 4}};
    for (int k = 0; k < 3; ++k) {
        std::vector<int> members;
        for (int i = 0; i < nb; ++i)
            if (cls[i] == k) members.push_back(i);
        if (members.empty()) continue;
        int keep[3] = {boxes[members[0]].tile[0], boxes[members[0]].tile[1], boxes[members[0]].tile[2]};
        for (const auto &t : cand) {
            if (t[0] == keep[0] && t[1] == keep[1] && t[2] == keep[2]) continue;
            for (int i : members)
                for (int a = 0; a < 3; ++a) boxes[i].tile[a] = t[a];
            const double ms = tune_trial(&c, loads, n_loads, dev_arena, bytes, hip_stream, steps);
            ++res->trials;
            if (ms > 0 && ms < best) {
                best = ms;
                for (int a = 0; a < 3; ++a) keep[a] = t[a];
            }
        }
        for (int i : members)
            for (int a = 0; a < 3; ++a) boxes[i].tile[a] = keep[a];
    }
    const int si_keep = c.sort_interval;
    int si_best = si_keep;
    for (int si : {25, 50, 100, 200}) {
        if (si == si_keep) continue;
        c.sort_interval = si;
        const double ms = tune_trial(&c, loads, n_loads, dev_arena, bytes, hip_stream, steps);
        ++res->trials;
        if (ms > 0 && ms < best) {
            best = ms;
            si_best = si;
        }
    }
    c.sort_interval = si_best;
    res->ms_per_step = best;
    std::copy(boxes.begin(), boxes.end(), boxes_out);
    *cfg_out = c;
    cfg_out->boxes = boxes_out;
    return PIC_OK;
}
