// Host side of liblbm: the C ABI of include/lbm.h.  Instances live in
// caller-owned device workspaces; the library allocates no device memory.
// Steps are enqueued as captured HIP graphs of up to MAX_CHUNK steps (two
// kernels per step plus one end-of-chunk kernel), or launched directly when
// the stream is the null stream, which cannot be captured.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "lbm_internal.h"

using namespace lbm;

namespace {

constexpr size_t ALIGN = 256;
constexpr int MAX_SIDE = 65536;
constexpr uint64_t CKPT_MAGIC = 0x314d424c4b504b43ull;   // checkpoint image tag
constexpr int N_STAGE = 4;                               // pinned descriptor staging slots

inline size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t elem_size(int prec) { return prec == LBM_FP64 ? 8 : 4; }

// The population shift reference, rounded to the storage precision so that
// stored deviations and the reconstruction rho = rho_ref + sum g agree.
double storage_value(int prec, double v) { return prec == LBM_FP64 ? v : (double)(float)v; }

// Consecutive population planes are PLANE_SKEW bytes further apart than their
// size.  Grids with power-of-two sides otherwise put the nine planes a
// power-of-two distance apart, so that the nine streams a wavefront reads or
// writes at once start on the same HBM channel; the skew spreads them (8% more
// bandwidth on an 8192 x 4096 grid, measured).
constexpr size_t PLANE_SKEW = 256;

struct Layout {
    size_t desc, tiles, f0, f1, psi, partials, flag, wall_keys, wall_run, result, total;
    long long plane;        // elements from one population plane to the next
    int pitch;
    int64_t max_tiles;
};

// Tiles of an nx x ny grid in the largest work-list any variant builds.
int64_t max_tiles_for(int nx, int ny)
{
    int64_t most = 0;
    for (int v = 0; v < kNumVariants; ++v) {
        const int cols = tile_cols(v), rows = tile_rows(v);
        most = std::max(most, (int64_t)((nx + cols - 1) / cols) * ((ny + rows - 1) / rows));
    }
    return most;
}

Layout layout_of(const lbm_params &p)
{
    Layout L;
    L.pitch = (int)round_up((size_t)p.nx, TILE_X);
    L.max_tiles = max_tiles_for(p.nx, p.ny);
    const size_t es = elem_size(p.precision);
    const size_t plane = (size_t)L.pitch * p.ny + PLANE_SKEW / es;
    L.plane = (long long)plane;
    size_t o = 0;
    L.desc = o; o = round_up(o + sizeof(InstDev), ALIGN);
    L.tiles = o; o = round_up(o + sizeof(Tile) * (size_t)L.max_tiles, ALIGN);
    L.f0 = o; o = round_up(o + 9 * plane * es, ALIGN);
    L.f1 = o; o = round_up(o + 9 * plane * es, ALIGN);
    L.psi = o; o = round_up(o + plane * es, ALIGN);
    L.partials = o; o = round_up(o + sizeof(double) * N_PARTIAL * (size_t)L.max_tiles, ALIGN);
    L.flag = o; o = round_up(o + sizeof(int), ALIGN);
    L.wall_keys = o; o = round_up(o + sizeof(unsigned long long) * MAX_CHUNK, ALIGN);
    L.wall_run = o; o = round_up(o + 2 * sizeof(unsigned long long), ALIGN);
    L.result = o; o = round_up(o + sizeof(double) * (N_PARTIAL + 2), ALIGN);
    L.total = o;
    return L;
}

int check_params(const lbm_params *p)
{
    if (!p) return LBM_EINVAL;
    if (p->nx < 1 || p->ny < 1 || p->nx > MAX_SIDE || p->ny > MAX_SIDE) return LBM_EINVAL;
    if (p->walls_y != 0 && p->walls_y != 1) return LBM_EINVAL;
    if (p->precision < LBM_FP64 || p->precision > LBM_FP32_MIXED) return LBM_EINVAL;
    if (!(p->G < 0) || !(p->T > 0) || !(p->b > 0) || !(p->R > 0) || !(p->a >= 0)) return LBM_EINVAL;
    if (!isfinite(p->eps)) return LBM_EINVAL;
    // kernels address a population plane with 32-bit byte offsets
    const unsigned long long plane_bytes =
        (unsigned long long)round_up((size_t)p->nx, TILE_X) * (unsigned long long)p->ny * elem_size(p->precision) +
        PLANE_SKEW;
    if (plane_bytes >= (1ull << 32)) return LBM_EINVAL;
    const double r[6] = {p->s_rho, p->s_e, p->s_zeta, p->s_j, p->s_q, p->s_nu};
    for (double v : r)
        if (!(v > 0.0 && v < 2.0)) return LBM_EINVAL;
    return LBM_OK;
}

// Pinned staging for descriptor uploads: a ring of slots, each reusable once
// the copy that read it has completed.
struct Stager {
    char *host = nullptr;
    size_t slot_bytes = 0;
    hipEvent_t ev[N_STAGE] = {};
    bool used[N_STAGE] = {};
    int next = 0;

    int init(size_t bytes)
    {
        slot_bytes = round_up(bytes, 64);
        if (hipHostMalloc((void **)&host, slot_bytes * N_STAGE, hipHostMallocDefault) != hipSuccess)
            return LBM_EHIP;
        for (int i = 0; i < N_STAGE; ++i)
            if (hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) != hipSuccess) return LBM_EHIP;
        return LBM_OK;
    }
    void release()
    {
        for (int i = 0; i < N_STAGE; ++i)
            if (ev[i]) (void)hipEventDestroy(ev[i]);
        if (host) (void)hipHostFree(host);
        host = nullptr;
    }
    int upload(void *dst, const void *src, size_t bytes, hipStream_t st)
    {
        if (bytes > slot_bytes) return LBM_EINVAL;
        const int k = next;
        next = (next + 1) % N_STAGE;
        if (used[k] && hipEventSynchronize(ev[k]) != hipSuccess) return LBM_EHIP;
        char *slot = host + (size_t)k * slot_bytes;
        memcpy(slot, src, bytes);
        if (hipMemcpyAsync(dst, slot, bytes, hipMemcpyHostToDevice, st) != hipSuccess) return LBM_EHIP;
        if (hipEventRecord(ev[k], st) != hipSuccess) return LBM_EHIP;
        used[k] = true;
        return LBM_OK;
    }
};

struct GraphKey {
    int variant, K, ntiles, ninst, write_through;
    bool operator<(const GraphKey &o) const
    {
        return std::tie(variant, K, ntiles, ninst, write_through) <
               std::tie(o.variant, o.K, o.ntiles, o.ninst, o.write_through);
    }
};

struct Batch;

struct Instance {
    lbm_params p;
    Layout L;
    char *ws = nullptr;
    hipStream_t stream = nullptr;
    InstDev desc;                 // host mirror of the device descriptor
    InstDev *d_desc = nullptr;
    Tile *d_tiles = nullptr;
    int variant = 0;
    int tiles_variant = -1;       // variant the device tile list was built for
    int ntiles = 0;
    bool tiles_dirty = true;
    bool desc_dirty = true;
    bool has_state = false;
    int sticky = LBM_OK;
    Batch *batch = nullptr;
    Stager stager;
    std::map<GraphKey, hipGraphExec_t> graphs;
    // init record, kept for checkpoints
    int n_bubbles = 0;
    lbm_bubble bubbles[LBM_MAX_BUBBLES];
};

struct Batch {
    int precision;
    hipStream_t stream;
    int max_inst;
    int64_t max_tiles;
    InstDev *d_descs;
    Tile *d_tiles;
    int *d_status;                // latch of each member at the last chunk end
    std::vector<Instance *> members;
    std::vector<InstDev> descs;   // host copies in attach order
    // What the device descriptors hold: the last upload, advanced like the
    // end-of-chunk kernel advances them; an upload happens only when the
    // host copies differ from it.
    std::vector<InstDev> dev;
    bool dev_valid = false;
    int ntiles = 0;
    int variant = 0;
    int write_through = 0;        // fused stores write through L2
    bool dirty = true;
    // Workspace drawn from the library's static scratch array of device
    // static_dev (lbm_batch_create_static): no pinned staging, no graphs.
    int static_dev = -1;
    Stager stager_desc, stager_tiles;
    std::map<GraphKey, hipGraphExec_t> graphs;
};

hipStream_t stream_of(const Instance *h);

template <typename T>
void fill_consts(Consts<T> &c, const InstDev &d)
{
    c.RT = (T)d.RT;
    c.a = (T)d.a;
    c.b4 = (T)d.b4;
    c.two_over_G = (T)d.two_over_G;
    c.mG = (T)(-d.G);
    c.rho_ref = (T)d.rho_ref;
    c.s_e = (T)d.s_e;
    c.s_z = (T)d.s_z;
    c.s_q = (T)d.s_q;
    c.s_nu = (T)d.s_nu;
    c.h_e = (T)(1.0 - 0.5 * d.s_e);
    c.h_z = (T)(1.0 - 0.5 * d.s_z);
    c.h_q = (T)(1.0 - 0.5 * d.s_q);
    c.h_nu = (T)(1.0 - 0.5 * d.s_nu);
    c.li_e = (T)d.li_e;
    c.li_z = (T)d.li_z;
    const double c9 = 1.0 / 36.0, c12 = 1.0 / 12.0, c4 = 0.25;
    c.e_eq = (T)(d.s_e * c9);
    c.e_vf = (T)(6.0 * (1.0 - 0.5 * d.s_e) * c9);
    c.e_li = (T)(d.li_e * c9);
    c.z_eq = (T)(d.s_z * c9);
    c.z_vf = (T)(-6.0 * (1.0 - 0.5 * d.s_z) * c9);
    c.z_li = (T)(-d.li_z * c9);
    c.q_eq = (T)(d.s_q * c12);
    c.q_f = (T)(-(1.0 - 0.5 * d.s_q) * c12);
    c.n_eq = (T)(d.s_nu * c4);
    c.n_xx = (T)(2.0 * (1.0 - 0.5 * d.s_nu) * c4);
    c.n_xy = (T)((1.0 - 0.5 * d.s_nu) * c4);
}

// Refreshes the per-precision constant copies after a descriptor change.
// Sites whose density lies in the spinodal interval of Eq. 15, widened by
// MIX_PAD of its width on each side, evaluate Eqs. 15 and 13 in binary64 under
// LBM_FP32_MIXED.
constexpr double MIX_PAD = 0.1;

void refresh_consts(InstDev &d)
{
    fill_consts(d.cf, d);
    fill_consts(d.cd, d);
    double sg, sl;
    // p depends on R and T only through RT
    if (lbm_spinodals(d.a, 4.0 * d.b4, 1.0, d.RT, &sg, &sl) == LBM_OK) {
        const double pad = MIX_PAD * (sl - sg);
        d.mix_lo = (float)(sg - pad - d.rho_ref);
        d.mix_hi = (float)(sl + pad - d.rho_ref);
    } else {
        d.mix_lo = INFINITY;
        d.mix_hi = -INFINITY;
    }
}

void fill_desc(Instance *h)
{
    const lbm_params &p = h->p;
    InstDev &d = h->desc;
    const size_t es = elem_size(p.precision);
    (void)es;
    d.f[0] = h->ws + h->L.f0;
    d.f[1] = h->ws + h->L.f1;
    d.psi = h->ws + h->L.psi;
    d.partials = (double *)(h->ws + h->L.partials);
    d.flag = (int *)(h->ws + h->L.flag);
    d.wall_keys = (unsigned long long *)(h->ws + h->L.wall_keys);
    d.wall_run = (unsigned long long *)(h->ws + h->L.wall_run);
    d.result = (double *)(h->ws + h->L.result);
    d.plane = h->L.plane;
    d.nx = p.nx;
    d.ny = p.ny;
    d.pitch = h->L.pitch;
    d.walls = p.walls_y;
    d.a = p.a;
    d.b4 = p.b / 4.0;
    d.RT = p.R * p.T;
    d.G = p.G;
    d.two_over_G = 2.0 / p.G;
    d.s_e = p.s_e;
    d.s_z = p.s_zeta;
    d.s_q = p.s_q;
    d.s_nu = p.s_nu;
    d.li_e = p.s_e * 0.75 * p.eps;
    d.li_z = p.s_zeta * 0.75 * p.eps;
    refresh_consts(d);
}

void build_tiles(int inst_index, const lbm_params &p, int variant, std::vector<Tile> &out)
{
    const int rows = tile_rows(variant), cols = tile_cols(variant);
    int k = 0;
    for (int y0 = 0; y0 < p.ny; y0 += rows)
        for (int x0 = 0; x0 < p.nx; x0 += cols) {
            Tile t;
            t.inst = inst_index;
            t.x0 = x0;
            t.y0 = y0;
            t.tile_index = k++;
            out.push_back(t);
        }
}

int hip_ok(hipError_t e) { return e == hipSuccess ? LBM_OK : LBM_EHIP; }

#define TRY(expr)                          \
    do {                                   \
        int rc__ = (expr);                 \
        if (rc__ != LBM_OK) return rc__;   \
    } while (0)

#define TRYHIP(expr) TRY(hip_ok(expr))

hipStream_t stream_of(const Instance *h) { return h->batch ? h->batch->stream : h->stream; }

// Makes the instance's own device descriptor current, and its tile list the
// one of variant v (default: the instance's variant).
int sync_own(Instance *h, int v = -1)
{
    hipStream_t st = stream_of(h);
    if (v < 0) v = h->variant;
    if (h->tiles_dirty || h->tiles_variant != v) {
        std::vector<Tile> tl;
        build_tiles(0, h->p, v, tl);
        h->tiles_variant = v;
        h->ntiles = (int)tl.size();
        h->desc.tiles_x = (h->p.nx + TILE_X - 1) / TILE_X;
        TRYHIP(hipMemcpyAsync(h->d_tiles, tl.data(), sizeof(Tile) * tl.size(), hipMemcpyHostToDevice, st));
        // the pageable copy above is complete when it returns for small sizes,
        // but make sure before the vector goes away
        TRYHIP(hipStreamSynchronize(st));
        h->tiles_dirty = false;
    }
    if (h->desc_dirty) {
        TRY(h->stager.upload(h->d_desc, &h->desc, sizeof(InstDev), st));
        h->desc_dirty = false;
    }
    return LBM_OK;
}

// Enqueues one chunk: K steps of both passes and the end-of-chunk kernel.
int enqueue_chunk(int prec, int variant, const InstDev *d_inst, int ninst, const Tile *d_tiles,
                  int ntiles, int K, hipStream_t st, int *d_status, int write_through)
{
    if (two_step(variant)) {
        // one launch per pair of steps; an instance with an odd count takes
        // its last step alone in launch (n - 1) / 2
        for (int s = 0; s < (K + 1) / 2; ++s)
            TRYHIP(launch_twostep(prec, variant, d_inst, d_tiles, ntiles, s, st, write_through));
        TRYHIP(launch_chunk_end(d_inst, ninst, st, d_status, 1));
        return LBM_OK;
    }
    for (int s = 0; s < K; ++s) {
        if (kVariants[variant].fused == 2) {
            TRYHIP(launch_fused2(prec, variant, d_inst, d_tiles, ntiles, s, st));
        } else if (kVariants[variant].fused == 1) {
            TRYHIP(launch_fused(prec, variant, d_inst, d_tiles, ntiles, s, st, write_through));
        } else {
            TRYHIP(launch_psi_pass(prec, variant, d_inst, d_tiles, ntiles, s, st));
            TRYHIP(launch_collide_stream(prec, variant, d_inst, d_tiles, ntiles, s, st));
        }
    }
    TRYHIP(launch_chunk_end(d_inst, ninst, st, d_status));
    return LBM_OK;
}

// The cached graph of one chunk of K steps, captured, instantiated and
// uploaded to the device the first time it is asked for (st must not be the
// null stream, which cannot be captured).
int chunk_graph(std::map<GraphKey, hipGraphExec_t> &cache, int prec, int variant, const InstDev *d_inst,
                int ninst, const Tile *d_tiles, int ntiles, int K, hipStream_t st, int *d_status,
                int write_through, hipGraphExec_t *out)
{
    GraphKey key{variant, K, ntiles, ninst, write_through};
    auto it = cache.find(key);
    if (it == cache.end()) {
        hipGraph_t g = nullptr;
        TRYHIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        int rc = enqueue_chunk(prec, variant, d_inst, ninst, d_tiles, ntiles, K, st, d_status, write_through);
        hipError_t e = hipStreamEndCapture(st, &g);
        if (rc != LBM_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        TRYHIP(e);
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        TRYHIP(e);
        it = cache.emplace(key, ex).first;
        // the first launch would otherwise copy the graph's launch data
        TRYHIP(hipGraphUpload(ex, st));
    }
    *out = it->second;
    return LBM_OK;
}

// Runs one chunk through a cached graph when the stream can be captured.
int run_chunk(std::map<GraphKey, hipGraphExec_t> &cache, int prec, int variant, const InstDev *d_inst,
              int ninst, const Tile *d_tiles, int ntiles, int K, hipStream_t st, int *d_status = nullptr,
              int write_through = 0)
{
    if (st == nullptr)
        return enqueue_chunk(prec, variant, d_inst, ninst, d_tiles, ntiles, K, st, d_status, write_through);
    hipGraphExec_t ex = nullptr;
    TRY(chunk_graph(cache, prec, variant, d_inst, ninst, d_tiles, ntiles, K, st, d_status, write_through, &ex));
    TRYHIP(hipGraphLaunch(ex, st));
    return LBM_OK;
}

void drop_graphs(std::map<GraphKey, hipGraphExec_t> &cache)
{
    for (auto &kv : cache) (void)hipGraphExecDestroy(kv.second);
    cache.clear();
}

// Host mirror of what the end-of-chunk kernel does to a descriptor.
void advance_mirror(InstDev &d, int n, int variant)
{
    d.step += n;
    d.cur ^= buffer_flips(n, two_step(variant) ? 1 : 0) & 1;
}

int read_latch(Instance *h)
{
    int flag = 0;
    TRYHIP(hipMemcpy(&flag, h->desc.flag, sizeof(int), hipMemcpyDeviceToHost));
    if (flag) h->sticky = LBM_ENONFINITE;
    return h->sticky;
}

// ---------------------------------------------------------------------------
// batch internals
// ---------------------------------------------------------------------------
// Sends bytes from host memory to the batch workspace: through the pinned
// staging ring, or, for a batch on the static scratch array (which has no
// staging), as a copy from the host buffer that is complete before this
// returns, so the buffer may change afterwards.
int batch_upload(Batch *b, Stager &stg, void *dst, const void *src, size_t bytes)
{
    if (b->static_dev < 0) return stg.upload(dst, src, bytes, b->stream);
    TRYHIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, b->stream));
    TRYHIP(hipStreamSynchronize(b->stream));
    return LBM_OK;
}

int batch_sync(Batch *b)
{
    if (b->dirty) {
        // a new composition makes the cached graphs unreachable (their key
        // holds the tile and instance counts); release them once idle
        if (!b->graphs.empty()) {
            TRYHIP(hipStreamSynchronize(b->stream));
            drop_graphs(b->graphs);
        }
        std::vector<Tile> tl;
        b->descs.clear();
        for (size_t i = 0; i < b->members.size(); ++i) {
            Instance *h = b->members[i];
            build_tiles((int)i, h->p, b->variant, tl);
            h->desc.tiles_x = (h->p.nx + TILE_X - 1) / TILE_X;
            b->descs.push_back(h->desc);
        }
        if ((int64_t)tl.size() > b->max_tiles) return LBM_ENOMEM;
        b->ntiles = (int)tl.size();
        // the latch copies belong to the old composition
        TRYHIP(launch_fill_int(b->d_status, b->max_inst, 0, b->stream));
        if (!tl.empty()) TRY(batch_upload(b, b->stager_tiles, b->d_tiles, tl.data(), sizeof(Tile) * tl.size()));
        b->dirty = false;
        b->dev_valid = false;
    } else {
        for (size_t i = 0; i < b->members.size(); ++i) b->descs[i] = b->members[i]->desc;
    }
    // The end-of-chunk kernel advances step and buffer parity on the device
    // as the host mirrors do, so consecutive chunks of the same length need
    // no transfer; anything else (a new chunk length, an instance
    // re-initialised or loaded) differs from the device image and is sent.
    const bool same = b->dev_valid && b->dev.size() == b->descs.size() &&
                      memcmp(b->dev.data(), b->descs.data(), sizeof(InstDev) * b->descs.size()) == 0;
    if (!b->descs.empty() && !same) {
        TRY(batch_upload(b, b->stager_desc, b->d_descs, b->descs.data(), sizeof(InstDev) * b->descs.size()));
        b->dev = b->descs;
        b->dev_valid = true;
    }
    return LBM_OK;
}

// Sets every member's chunk length for the next chunk of a run whose
// remaining counts are rem; returns the chunk's step count K.
int plan_chunk(Batch *b, const std::vector<int64_t> &rem)
{
    int K = 0;
    for (size_t i = 0; i < b->members.size(); ++i) {
        const int ni = (int)std::min<int64_t>(rem[i], MAX_CHUNK);
        b->members[i]->desc.n_chunk = ni;
        K = std::max(K, ni);
    }
    return K;
}

// Steps the members by counts[i] steps each, MAX_CHUNK steps per chunk.
int batch_run(Batch *b, const std::vector<int64_t> &counts, bool timed, float *ms)
{
    const int n = (int)b->members.size();
    for (int i = 0; i < n; ++i) {
        Instance *h = b->members[i];
        if (counts[i] > 0 && !h->has_state) return LBM_ESTATE;
        if (counts[i] > 0 && h->sticky != LBM_OK) return h->sticky;
    }
    std::vector<int64_t> rem(counts);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
        TRYHIP(hipEventCreate(&e0));
        TRYHIP(hipEventCreate(&e1));
        ms[0] = ms[1] = 0.f;
    }
    int rc = LBM_OK;
    for (;;) {
        const int K = plan_chunk(b, rem);
        if (K == 0) break;
        rc = batch_sync(b);
        if (rc != LBM_OK) break;
        if (!timed && b->static_dev >= 0) {
            // no graph: its instantiation may allocate device memory
            rc = enqueue_chunk(b->precision, b->variant, b->d_descs, n, b->d_tiles, b->ntiles, K, b->stream,
                               b->d_status, b->write_through);
        } else if (!timed) {
            rc = run_chunk(b->graphs, b->precision, b->variant, b->d_descs, n, b->d_tiles, b->ntiles, K,
                           b->stream, b->d_status, b->write_through);
        } else {
            const bool fused = kVariants[b->variant].fused;
            const bool pairs = two_step(b->variant);
            // one timed launch per step, or per pair of steps (two-step
            // variants: ms[1] then sums launches of two steps each)
            const int launches = pairs ? (K + 1) / 2 : K;
            for (int s = 0; s < launches && rc == LBM_OK && fused; ++s) {
                float t;
                rc = hip_ok(hipEventRecord(e0, b->stream));
                if (rc == LBM_OK) {
                    if (pairs)
                        rc = hip_ok(launch_twostep(b->precision, b->variant, b->d_descs, b->d_tiles, b->ntiles, s,
                                                   b->stream, b->write_through));
                    else if (kVariants[b->variant].fused == 2)
                        rc = hip_ok(launch_fused2(b->precision, b->variant, b->d_descs, b->d_tiles, b->ntiles, s, b->stream));
                    else
                        rc = hip_ok(launch_fused(b->precision, b->variant, b->d_descs, b->d_tiles, b->ntiles, s, b->stream,
                                                 b->write_through));
                }
                if (rc == LBM_OK) rc = hip_ok(hipEventRecord(e1, b->stream));
                if (rc == LBM_OK) rc = hip_ok(hipEventSynchronize(e1));
                if (rc == LBM_OK) rc = hip_ok(hipEventElapsedTime(&t, e0, e1));
                if (rc == LBM_OK) ms[1] += t;
            }
            for (int s = 0; s < K && rc == LBM_OK && !fused; ++s) {
                float t;
                rc = hip_ok(hipEventRecord(e0, b->stream));
                if (rc == LBM_OK) rc = hip_ok(launch_psi_pass(b->precision, b->variant, b->d_descs, b->d_tiles, b->ntiles, s, b->stream));
                if (rc == LBM_OK) rc = hip_ok(hipEventRecord(e1, b->stream));
                if (rc == LBM_OK) rc = hip_ok(hipEventSynchronize(e1));
                if (rc == LBM_OK) rc = hip_ok(hipEventElapsedTime(&t, e0, e1));
                if (rc == LBM_OK) ms[0] += t;
                if (rc == LBM_OK) rc = hip_ok(hipEventRecord(e0, b->stream));
                if (rc == LBM_OK) rc = hip_ok(launch_collide_stream(b->precision, b->variant, b->d_descs, b->d_tiles, b->ntiles, s, b->stream));
                if (rc == LBM_OK) rc = hip_ok(hipEventRecord(e1, b->stream));
                if (rc == LBM_OK) rc = hip_ok(hipEventSynchronize(e1));
                if (rc == LBM_OK) rc = hip_ok(hipEventElapsedTime(&t, e0, e1));
                if (rc == LBM_OK) ms[1] += t;
            }
            if (rc == LBM_OK) rc = hip_ok(launch_chunk_end(b->d_descs, n, b->stream, b->d_status, pairs ? 1 : 0));
        }
        if (rc != LBM_OK) break;
        for (int i = 0; i < n; ++i) {
            Instance *h = b->members[i];
            const int ni = h->desc.n_chunk;
            advance_mirror(h->desc, ni, b->variant);
            advance_mirror(b->dev[i], ni, b->variant);   // what the end-of-chunk kernel did
            rem[i] -= ni;
            h->desc_dirty = true;    // the instance's own descriptor copy is stale
        }
    }
    for (int i = 0; i < n; ++i) b->members[i]->desc.n_chunk = 0;
    if (timed) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    return rc;
}

// ---------------------------------------------------------------------------
// static scratch for one allocation-free batch per device
// ---------------------------------------------------------------------------
// Layout: descriptors of LBM_STATIC_MAX_INSTANCES instances | tile work-list
// of LBM_STATIC_MAX_TILES tiles | latch copies of LBM_STATIC_MAX_INSTANCES.
constexpr size_t STATIC_DESC_BYTES = (sizeof(InstDev) * LBM_STATIC_MAX_INSTANCES + ALIGN - 1) / ALIGN * ALIGN;
constexpr size_t STATIC_TILE_BYTES = (sizeof(Tile) * (size_t)LBM_STATIC_MAX_TILES + ALIGN - 1) / ALIGN * ALIGN;
constexpr size_t STATIC_STATUS_BYTES = (sizeof(int) * LBM_STATIC_MAX_INSTANCES + ALIGN - 1) / ALIGN * ALIGN;
constexpr size_t STATIC_BYTES = STATIC_DESC_BYTES + STATIC_TILE_BYTES + STATIC_STATUS_BYTES;

// Each device holds its own copy of this array until the process ends.  In
// host code its name is not a device address: host code uses only the
// address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) char scratch[STATIC_BYTES];

constexpr int MAX_DEVICES = 64;
struct StaticSlot {
    void *ptr = nullptr;      // the device's address of `scratch`
    bool in_use = false;      // a static batch holds it
};
std::mutex g_static_mu;
StaticSlot g_static[MAX_DEVICES];

// The current device's address of the scratch array, looked up once per
// device (with that device current) and marked in use; LBM_ESTATE when a
// static batch on this device already holds it.
int acquire_static_scratch(int *dev_out, void **ptr_out)
{
    int dev = -1;
    TRYHIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return LBM_EINVAL;
    std::lock_guard<std::mutex> lock(g_static_mu);
    StaticSlot &sl = g_static[dev];
    if (!sl.ptr) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return LBM_EHIP;
        sl.ptr = p;
    }
    if (sl.in_use) return LBM_ESTATE;
    sl.in_use = true;
    *dev_out = dev;
    *ptr_out = sl.ptr;
    return LBM_OK;
}

void release_static_scratch(int dev)
{
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (dev >= 0 && dev < MAX_DEVICES) g_static[dev].in_use = false;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *lbm_strerror(int status)
{
    switch (status) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOMEM: return "workspace or buffer too small";
    case LBM_EHIP: return "HIP runtime error";
    case LBM_ENONFINITE: return "non-finite density or pseudopotential (psi^2 < 0) latched";
    case LBM_ESTATE: return "call not valid in the current state";
    default: return "unknown status";
    }
}

int lbm_workspace_bytes(const lbm_params *params, size_t *bytes)
{
    TRY(check_params(params));
    if (!bytes) return LBM_EINVAL;
    *bytes = layout_of(*params).total;
    return LBM_OK;
}

int lbm_tile_count(const lbm_params *params, int64_t *max_tiles)
{
    TRY(check_params(params));
    if (!max_tiles) return LBM_EINVAL;
    *max_tiles = layout_of(*params).max_tiles;
    return LBM_OK;
}

int lbm_create(const lbm_params *params, void *d_workspace, size_t ws_bytes, void *hip_stream,
               void **handle)
{
    TRY(check_params(params));
    if (!handle || !d_workspace) return LBM_EINVAL;
    if ((uintptr_t)d_workspace % ALIGN) return LBM_EINVAL;
    const Layout L = layout_of(*params);
    if (ws_bytes < L.total) return LBM_ENOMEM;
    Instance *h = new Instance();
    h->p = *params;
    h->L = L;
    h->ws = (char *)d_workspace;
    h->stream = (hipStream_t)hip_stream;
    memset(&h->desc, 0, sizeof(InstDev));
    h->d_desc = (InstDev *)(h->ws + L.desc);
    h->d_tiles = (Tile *)(h->ws + L.tiles);
    fill_desc(h);
    prime_residency();
    if (h->stager.init(sizeof(InstDev)) != LBM_OK) {
        h->stager.release();
        delete h;
        return LBM_EHIP;
    }
    *handle = h;
    return LBM_OK;
}

void lbm_destroy(void *handle)
{
    Instance *h = (Instance *)handle;
    if (!h) return;
    if (h->batch) lbm_batch_detach(h->batch, h);
    (void)hipStreamSynchronize(h->stream);
    drop_graphs(h->graphs);
    h->stager.release();
    delete h;
}

int lbm_init_bubble(void *handle, const lbm_bubble *b, int nb, int slab_rows, double rho_l,
                    double rho_g, double W, double delta, double noise_amp, uint64_t seed)
{
    Instance *h = (Instance *)handle;
    if (!h) return LBM_EINVAL;
    if (nb < 0 || nb > LBM_MAX_BUBBLES || (nb > 0 && !b) || slab_rows < 0) return LBM_EINVAL;
    if (!(rho_l > 0) || !(rho_g > 0) || !(W > 0) || !isfinite(delta) || !(noise_amp >= 0) ||
        noise_amp >= 1.0)
        return LBM_EINVAL;
    const int nbub = slab_rows > 0 ? 0 : nb;
    h->n_bubbles = nbub;
    for (int k = 0; k < nbub; ++k) h->bubbles[k] = b[k];
    InstDev &d = h->desc;
    d.cur = 0;
    d.step = 0;
    d.n_chunk = 0;
    d.n_bubbles = nbub;
    d.rho_l = rho_l;
    d.rho_g = rho_g;
    d.rho_ref = storage_value(h->p.precision, rho_l);
    refresh_consts(d);
    for (int k = 0; k < LBM_MAX_BUBBLES; ++k) {
        d.bx[k] = k < nbub ? b[k].x0 : 0.0;
        d.by[k] = k < nbub ? b[k].y0 : 0.0;
    }
    h->desc_dirty = true;
    if (h->batch) h->batch->dirty = true;
    TRY(sync_own(h));
    hipStream_t st = stream_of(h);
    TRYHIP(launch_reset_diag(h->d_desc, st));
    TRYHIP(launch_init(h->p.precision, h->d_desc, slab_rows, b, nbub, rho_l, rho_g, W, delta,
                       noise_amp, seed, (long long)h->p.nx * h->p.ny, st));
    h->has_state = true;
    h->sticky = LBM_OK;
    return LBM_OK;
}

int lbm_init_density(void *handle, const void *d_rho, double rho_l, double rho_g)
{
    Instance *h = (Instance *)handle;
    if (!h || !d_rho || !(rho_l > 0) || !(rho_g > 0)) return LBM_EINVAL;
    h->n_bubbles = 0;
    InstDev &d = h->desc;
    d.cur = 0;
    d.step = 0;
    d.n_chunk = 0;
    d.n_bubbles = 0;
    d.rho_l = rho_l;
    d.rho_g = rho_g;
    d.rho_ref = storage_value(h->p.precision, rho_l);
    refresh_consts(d);
    h->desc_dirty = true;
    if (h->batch) h->batch->dirty = true;
    TRY(sync_own(h));
    hipStream_t st = stream_of(h);
    TRYHIP(launch_reset_diag(h->d_desc, st));
    TRYHIP(launch_init_density(h->p.precision, h->d_desc, (const double *)d_rho,
                               (long long)h->p.nx * h->p.ny, st));
    h->has_state = true;
    h->sticky = LBM_OK;
    return LBM_OK;
}

int lbm_step(void *handle, int64_t n)
{
    Instance *h = (Instance *)handle;
    if (!h || n < 0) return LBM_EINVAL;
    if (h->batch) return LBM_ESTATE;
    if (!h->has_state) return LBM_ESTATE;
    if (h->sticky != LBM_OK) return h->sticky;
    TRY(sync_own(h));
    while (n > 0) {
        const int K = (int)std::min<int64_t>(n, MAX_CHUNK);
        if (h->desc.n_chunk != K) {
            h->desc.n_chunk = K;
            h->desc_dirty = true;
        }
        TRY(sync_own(h));
        TRY(run_chunk(h->graphs, h->p.precision, h->variant, h->d_desc, 1, h->d_tiles, h->ntiles, K,
                      h->stream));
        advance_mirror(h->desc, K, h->variant);   // the device advanced its own copy
        n -= K;
    }
    return LBM_OK;
}

int lbm_step_timed(void *handle, int64_t n, float *ms)
{
    Instance *h = (Instance *)handle;
    if (!h || n < 0 || !ms) return LBM_EINVAL;
    if (h->batch) return LBM_ESTATE;
    if (!h->has_state) return LBM_ESTATE;
    if (h->sticky != LBM_OK) return h->sticky;
    // a one-member batch view of the instance, on the instance's stream
    Batch tmp;
    tmp.precision = h->p.precision;
    tmp.stream = h->stream;
    tmp.max_inst = 1;
    tmp.max_tiles = h->L.max_tiles;
    tmp.d_descs = h->d_desc;
    tmp.d_tiles = h->d_tiles;
    tmp.members.push_back(h);
    tmp.variant = h->variant;
    if (tmp.stager_desc.init(sizeof(InstDev)) != LBM_OK || tmp.stager_tiles.init(sizeof(Tile) * h->L.max_tiles) != LBM_OK) {
        tmp.stager_desc.release();
        tmp.stager_tiles.release();
        return LBM_EHIP;
    }
    h->batch = &tmp;
    int rc = batch_run(&tmp, std::vector<int64_t>(1, n), true, ms);
    h->batch = nullptr;
    (void)hipStreamSynchronize(h->stream);
    tmp.stager_desc.release();
    tmp.stager_tiles.release();
    h->tiles_dirty = true;
    h->desc_dirty = true;
    return rc;
}

int lbm_sync(void *handle)
{
    Instance *h = (Instance *)handle;
    if (!h) return LBM_EINVAL;
    TRYHIP(hipStreamSynchronize(stream_of(h)));
    return read_latch(h);
}

static int query_stream(hipStream_t st, int *done)
{
    const hipError_t e = hipStreamQuery(st);
    if (e == hipSuccess) {
        *done = 1;
        return LBM_OK;
    }
    if (e == hipErrorNotReady) {
        (void)hipGetLastError();   // not an error: clear it
        *done = 0;
        return LBM_OK;
    }
    return LBM_EHIP;
}

int lbm_poll(void *handle, int *done)
{
    Instance *h = (Instance *)handle;
    if (!h || !done) return LBM_EINVAL;
    return query_stream(stream_of(h), done);
}

int lbm_macros(void *handle, void *d_rho, void *d_ux, void *d_uy, void *d_p, lbm_diag *out)
{
    Instance *h = (Instance *)handle;
    if (!h) return LBM_EINVAL;
    if (!h->has_state) return LBM_ESTATE;
    // the diagnostics run the two-pass kernels over the 64x4 tiles
    TRY(sync_own(h, 0));
    hipStream_t st = stream_of(h);
    TRYHIP(launch_psi_pass(h->p.precision, 0, h->d_desc, h->d_tiles, h->ntiles, -1, st));
    TRYHIP(launch_macros(h->p.precision, 0, h->d_desc, h->d_tiles, h->ntiles, d_rho, d_ux, d_uy,
                         (double *)d_p, st));
    TRYHIP(launch_reduce(h->d_desc, h->ntiles, st));
    double res[N_PARTIAL];
    unsigned long long run[2];
    int flag = 0;
    TRYHIP(hipMemcpyAsync(res, h->desc.result, sizeof(res), hipMemcpyDeviceToHost, st));
    TRYHIP(hipMemcpyAsync(run, h->desc.wall_run, sizeof(run), hipMemcpyDeviceToHost, st));
    TRYHIP(hipMemcpyAsync(&flag, h->desc.flag, sizeof(int), hipMemcpyDeviceToHost, st));
    TRYHIP(hipStreamSynchronize(st));
    if (flag) h->sticky = LBM_ENONFINITE;
    if (out) {
        memset(out, 0, sizeof(*out));
        out->step = h->desc.step;
        out->mass = res[0];
        out->mom_x = res[1];
        out->mom_y = res[2];
        out->n_bubbles = h->n_bubbles;
        out->nonfinite = flag ? 1 : 0;
        for (int k = 0; k < LBM_MAX_BUBBLES; ++k) {
            out->gas_area[k] = k < h->n_bubbles ? res[3 + k] : 0.0;
            out->radius[k] = k < h->n_bubbles ? sqrt(res[3 + k] / M_PI) : 0.0;
        }
        if (h->p.walls_y && run[0] != 0ull) {
            const unsigned long long u = (run[0] >> 63) ? (run[0] & 0x7fffffffffffffffull) : ~run[0];
            double v;
            memcpy(&v, &u, sizeof v);
            out->wall_p_max = v;
            out->wall_p_step = (int64_t)run[1];
        } else {
            out->wall_p_max = -INFINITY;
            out->wall_p_step = -1;
        }
    }
    return h->sticky;
}

int lbm_get_populations(void *handle, void *d_out)
{
    Instance *h = (Instance *)handle;
    if (!h || !d_out) return LBM_EINVAL;
    if (!h->has_state) return LBM_ESTATE;
    TRY(sync_own(h));
    TRYHIP(launch_pack(h->p.precision, h->d_desc, h->p.nx, h->p.ny, d_out, 1, stream_of(h)));
    return LBM_OK;
}

int lbm_set_populations(void *handle, const void *d_in)
{
    Instance *h = (Instance *)handle;
    if (!h || !d_in) return LBM_EINVAL;
    h->desc.cur = 0;
    h->desc.step = 0;
    h->desc.n_chunk = 0;
    h->desc_dirty = true;
    if (h->batch) h->batch->dirty = true;
    TRY(sync_own(h));
    hipStream_t st = stream_of(h);
    TRYHIP(launch_reset_diag(h->d_desc, st));
    TRYHIP(launch_pack(h->p.precision, h->d_desc, h->p.nx, h->p.ny, const_cast<void *>(d_in), 0, st));
    h->has_state = true;
    h->sticky = LBM_OK;
    return LBM_OK;
}

// ---- checkpoints ------------------------------------------------------------
struct CkptHeader {
    uint64_t magic;
    lbm_params p;
    int64_t step;
    int32_t n_bubbles, pad;
    lbm_bubble bubbles[LBM_MAX_BUBBLES];
    double rho_l, rho_g, rho_ref;
    unsigned long long wall_run[2];
};

int lbm_checkpoint_bytes(void *handle, size_t *bytes)
{
    Instance *h = (Instance *)handle;
    if (!h || !bytes) return LBM_EINVAL;
    *bytes = sizeof(CkptHeader) + 9 * (size_t)h->p.nx * h->p.ny * elem_size(h->p.precision);
    return LBM_OK;
}

int lbm_save(void *handle, void *host_buf, size_t bytes)
{
    Instance *h = (Instance *)handle;
    size_t need = 0;
    TRY(lbm_checkpoint_bytes(handle, &need));
    if (!host_buf) return LBM_EINVAL;
    if (bytes < need) return LBM_ENOMEM;
    if (!h->has_state) return LBM_ESTATE;
    TRY(sync_own(h));
    hipStream_t st = stream_of(h);
    TRYHIP(hipStreamSynchronize(st));
    CkptHeader hd;
    memset(&hd, 0, sizeof hd);
    hd.magic = CKPT_MAGIC;
    hd.p = h->p;
    hd.step = h->desc.step;
    hd.n_bubbles = h->n_bubbles;
    for (int k = 0; k < h->n_bubbles; ++k) hd.bubbles[k] = h->bubbles[k];
    hd.rho_l = h->desc.rho_l;
    hd.rho_g = h->desc.rho_g;
    hd.rho_ref = h->desc.rho_ref;
    TRYHIP(hipMemcpy(hd.wall_run, h->desc.wall_run, sizeof hd.wall_run, hipMemcpyDeviceToHost));
    memcpy(host_buf, &hd, sizeof hd);
    const size_t es = elem_size(h->p.precision);
    char *dst = (char *)host_buf + sizeof hd;
    const char *src = (const char *)h->desc.f[h->desc.cur];
    for (int a = 0; a < 9; ++a)
        TRYHIP(hipMemcpy2D(dst + (size_t)a * h->p.nx * h->p.ny * es, h->p.nx * es,
                           src + (size_t)a * h->desc.plane * es, h->L.pitch * es, h->p.nx * es,
                           h->p.ny, hipMemcpyDeviceToHost));
    return LBM_OK;
}

int lbm_load(void *handle, const void *host_buf, size_t bytes)
{
    Instance *h = (Instance *)handle;
    size_t need = 0;
    TRY(lbm_checkpoint_bytes(handle, &need));
    if (!host_buf) return LBM_EINVAL;
    if (bytes < need) return LBM_ENOMEM;
    CkptHeader hd;
    memcpy(&hd, host_buf, sizeof hd);
    if (hd.magic != CKPT_MAGIC || memcmp(&hd.p, &h->p, sizeof(lbm_params)) != 0) return LBM_EINVAL;
    hipStream_t st = stream_of(h);
    TRYHIP(hipStreamSynchronize(st));
    InstDev &d = h->desc;
    d.cur = 0;
    d.step = hd.step;
    d.n_chunk = 0;
    h->n_bubbles = hd.n_bubbles;
    d.n_bubbles = hd.n_bubbles;
    d.rho_l = hd.rho_l;
    d.rho_g = hd.rho_g;
    d.rho_ref = hd.rho_ref;
    refresh_consts(d);
    for (int k = 0; k < LBM_MAX_BUBBLES; ++k) {
        h->bubbles[k] = hd.bubbles[k];
        d.bx[k] = k < hd.n_bubbles ? hd.bubbles[k].x0 : 0.0;
        d.by[k] = k < hd.n_bubbles ? hd.bubbles[k].y0 : 0.0;
    }
    h->desc_dirty = true;
    if (h->batch) h->batch->dirty = true;
    TRY(sync_own(h));
    TRYHIP(launch_reset_diag(h->d_desc, st));
    TRYHIP(hipStreamSynchronize(st));
    TRYHIP(hipMemcpy(d.wall_run, hd.wall_run, sizeof hd.wall_run, hipMemcpyHostToDevice));
    const size_t es = elem_size(h->p.precision);
    const char *src = (const char *)host_buf + sizeof hd;
    char *dst = (char *)d.f[0];
    for (int a = 0; a < 9; ++a)
        TRYHIP(hipMemcpy2D(dst + (size_t)a * d.plane * es, h->L.pitch * es,
                           src + (size_t)a * h->p.nx * h->p.ny * es, h->p.nx * es, h->p.nx * es,
                           h->p.ny, hipMemcpyHostToDevice));
    h->has_state = true;
    h->sticky = LBM_OK;
    return LBM_OK;
}

// ---- variants ---------------------------------------------------------------
int lbm_variant_count(void) { return kNumVariants; }

const char *lbm_variant_name(int variant)
{
    if (variant < 0 || variant >= kNumVariants) return "";
    return kVariants[variant].name;
}

int lbm_resident_blocks(int precision, int variant, int *blocks)
{
    if (!blocks || variant < 0 || variant >= kNumVariants || precision < LBM_FP64 ||
        precision > LBM_FP32_MIXED)
        return LBM_EINVAL;
    *blocks = resident_blocks(precision, variant);
    return LBM_OK;
}

int lbm_set_variant(void *handle, int variant)
{
    Instance *h = (Instance *)handle;
    if (!h || variant < 0 || variant >= kNumVariants) return LBM_EINVAL;
    if (!variant_fits(variant, h->p.nx)) return LBM_EINVAL;
    if (h->variant != variant) {
        h->variant = variant;
        h->tiles_dirty = true;
    }
    return LBM_OK;
}

// ---- batch ------------------------------------------------------------------
int lbm_batch_workspace_bytes(int max_instances, int64_t max_tiles, size_t *bytes)
{
    if (max_instances < 1 || max_tiles < 1 || !bytes) return LBM_EINVAL;
    *bytes = round_up(sizeof(InstDev) * (size_t)max_instances, ALIGN) +
             round_up(sizeof(Tile) * (size_t)max_tiles, ALIGN) +
             round_up(sizeof(int) * (size_t)max_instances, ALIGN);
    return LBM_OK;
}

int lbm_batch_create(int precision, int max_instances, int64_t max_tiles, void *d_workspace,
                     size_t ws_bytes, void *hip_stream, void **batch)
{
    if (precision < LBM_FP64 || precision > LBM_FP32_MIXED || !batch || !d_workspace) return LBM_EINVAL;
    if ((uintptr_t)d_workspace % ALIGN) return LBM_EINVAL;
    size_t need = 0;
    TRY(lbm_batch_workspace_bytes(max_instances, max_tiles, &need));
    if (ws_bytes < need) return LBM_ENOMEM;
    Batch *b = new Batch();
    b->precision = precision;
    b->stream = (hipStream_t)hip_stream;
    b->max_inst = max_instances;
    b->max_tiles = max_tiles;
    b->d_descs = (InstDev *)d_workspace;
    b->d_tiles = (Tile *)((char *)d_workspace + round_up(sizeof(InstDev) * (size_t)max_instances, ALIGN));
    b->d_status = (int *)((char *)b->d_tiles + round_up(sizeof(Tile) * (size_t)max_tiles, ALIGN));
    prime_residency();
    if (launch_fill_int(b->d_status, max_instances, 0, b->stream) != hipSuccess) {
        delete b;
        return LBM_EHIP;
    }
    if (b->stager_desc.init(sizeof(InstDev) * (size_t)max_instances) != LBM_OK ||
        b->stager_tiles.init(sizeof(Tile) * (size_t)max_tiles) != LBM_OK) {
        b->stager_desc.release();
        b->stager_tiles.release();
        delete b;
        return LBM_EHIP;
    }
    *batch = b;
    return LBM_OK;
}

int lbm_batch_create_static(int precision, int max_instances, int64_t max_tiles, void *hip_stream,
                            void **batch)
{
    if (precision < LBM_FP64 || precision > LBM_FP32_MIXED || !batch || max_instances < 1 || max_tiles < 1)
        return LBM_EINVAL;
    if (max_instances > LBM_STATIC_MAX_INSTANCES || max_tiles > LBM_STATIC_MAX_TILES) return LBM_ENOMEM;
    int dev = -1;
    void *base = nullptr;
    TRY(acquire_static_scratch(&dev, &base));
    Batch *b = new Batch();
    b->precision = precision;
    b->stream = (hipStream_t)hip_stream;
    b->max_inst = max_instances;
    b->max_tiles = max_tiles;
    b->d_descs = (InstDev *)base;
    b->d_tiles = (Tile *)((char *)base + STATIC_DESC_BYTES);
    b->d_status = (int *)((char *)base + STATIC_DESC_BYTES + STATIC_TILE_BYTES);
    b->static_dev = dev;
    // the array keeps the previous batch's contents: the latch copies must
    // start at zero (descriptors and tiles are written before any use)
    if (launch_fill_int(b->d_status, max_instances, 0, b->stream) != hipSuccess) {
        release_static_scratch(dev);
        delete b;
        return LBM_EHIP;
    }
    *batch = b;
    return LBM_OK;
}

int lbm_batch_attach(void *batch, void *handle)
{
    Batch *b = (Batch *)batch;
    Instance *h = (Instance *)handle;
    if (!b || !h) return LBM_EINVAL;
    if (h->batch) return LBM_ESTATE;
    if (h->p.precision != b->precision) return LBM_EINVAL;
    if (!variant_fits(b->variant, h->p.nx)) return LBM_EINVAL;
    if ((int)b->members.size() >= b->max_inst) return LBM_ENOMEM;
    // order the instance's pending work before the batch's
    TRYHIP(hipStreamSynchronize(h->stream));
    h->batch = b;
    b->members.push_back(h);
    b->dirty = true;
    return LBM_OK;
}

int lbm_batch_detach(void *batch, void *handle)
{
    Batch *b = (Batch *)batch;
    Instance *h = (Instance *)handle;
    if (!b || !h || h->batch != b) return LBM_EINVAL;
    TRYHIP(hipStreamSynchronize(b->stream));
    auto it = std::find(b->members.begin(), b->members.end(), h);
    if (it != b->members.end()) b->members.erase(it);
    h->batch = nullptr;
    h->desc_dirty = true;
    b->dirty = true;
    return LBM_OK;
}

int lbm_batch_size(void *batch, int *n_attached)
{
    Batch *b = (Batch *)batch;
    if (!b || !n_attached) return LBM_EINVAL;
    *n_attached = (int)b->members.size();
    return LBM_OK;
}

int lbm_batch_status(void *batch, int *nonfinite, int n)
{
    Batch *b = (Batch *)batch;
    if (!b || !nonfinite || n < (int)b->members.size()) return LBM_EINVAL;
    const int m = (int)b->members.size();
    if (m == 0) return LBM_OK;
    TRYHIP(hipMemcpyAsync(nonfinite, b->d_status, sizeof(int) * (size_t)m, hipMemcpyDeviceToHost, b->stream));
    TRYHIP(hipStreamSynchronize(b->stream));
    for (int i = 0; i < m; ++i) {
        nonfinite[i] = nonfinite[i] != 0;
        if (nonfinite[i]) b->members[i]->sticky = LBM_ENONFINITE;
    }
    return LBM_OK;
}

int lbm_batch_poll(void *batch, int *done)
{
    Batch *b = (Batch *)batch;
    if (!b || !done) return LBM_EINVAL;
    return query_stream(b->stream, done);
}

int lbm_batch_step(void *batch, int64_t n)
{
    Batch *b = (Batch *)batch;
    if (!b || n < 0) return LBM_EINVAL;
    return batch_run(b, std::vector<int64_t>(b->members.size(), n), false, nullptr);
}

int lbm_batch_step_each(void *batch, const int64_t *counts, int n_counts)
{
    Batch *b = (Batch *)batch;
    if (!b || (n_counts > 0 && !counts) || n_counts != (int)b->members.size()) return LBM_EINVAL;
    std::vector<int64_t> c(counts, counts + n_counts);
    for (int64_t v : c)
        if (v < 0) return LBM_EINVAL;
    return batch_run(b, c, false, nullptr);
}

int lbm_batch_prepare(void *batch, int64_t n)
{
    Batch *b = (Batch *)batch;
    if (!b || n < 0) return LBM_EINVAL;
    if (b->stream == nullptr) return LBM_OK;          // the null stream launches directly
    const int m = (int)b->members.size();
    std::vector<int64_t> rem(m, n);
    const int K = plan_chunk(b, rem);
    int rc = K > 0 ? batch_sync(b) : LBM_OK;
    // the graphs of the run's chunk lengths: full chunks and the last one
    // (a batch on the static scratch array launches directly)
    const int tail = b->static_dev >= 0 ? 0 : (int)(n % MAX_CHUNK);
    hipGraphExec_t ex = nullptr;
    if (rc == LBM_OK && n >= MAX_CHUNK && b->static_dev < 0)
        rc = chunk_graph(b->graphs, b->precision, b->variant, b->d_descs, m, b->d_tiles, b->ntiles, MAX_CHUNK,
                         b->stream, b->d_status, b->write_through, &ex);
    if (rc == LBM_OK && tail > 0)
        rc = chunk_graph(b->graphs, b->precision, b->variant, b->d_descs, m, b->d_tiles, b->ntiles, tail,
                         b->stream, b->d_status, b->write_through, &ex);
    for (Instance *h : b->members) h->desc.n_chunk = 0;
    return rc;
}

int lbm_batch_step_timed(void *batch, int64_t n, float *ms)
{
    Batch *b = (Batch *)batch;
    if (!b || n < 0 || !ms) return LBM_EINVAL;
    return batch_run(b, std::vector<int64_t>(b->members.size(), n), true, ms);
}

int lbm_batch_set_write_through(void *batch, int on)
{
    Batch *b = (Batch *)batch;
    if (!b || (on != 0 && on != 1)) return LBM_EINVAL;
    b->write_through = on;
    return LBM_OK;
}

int lbm_batch_set_variant(void *batch, int variant)
{
    Batch *b = (Batch *)batch;
    if (!b || variant < 0 || variant >= kNumVariants) return LBM_EINVAL;
    for (Instance *h : b->members)
        if (!variant_fits(variant, h->p.nx)) return LBM_EINVAL;
    if (b->variant != variant) {
        b->variant = variant;
        b->dirty = true;
    }
    return LBM_OK;
}

int lbm_batch_autotune(void *batch, int reps, int *best_variant, float *ms_per_step)
{
    Batch *b = (Batch *)batch;
    if (!b || reps < 1 || !best_variant) return LBM_EINVAL;
    if (b->members.empty()) return LBM_ESTATE;
    hipEvent_t e0, e1;
    TRYHIP(hipEventCreate(&e0));
    TRYHIP(hipEventCreate(&e1));
    // Three passes over the variants, each variant scored by its fastest
    // pass, so that a single disturbed measurement does not decide.
    constexpr int kPasses = 3;
    std::vector<float> score(kNumVariants, INFINITY);
    int rc = LBM_OK;
    for (int pass = 0; pass < kPasses && rc == LBM_OK; ++pass) {
        for (int v = 0; v < kNumVariants && rc == LBM_OK; ++v) {
            bool fits = true;
            for (Instance *h : b->members) fits = fits && variant_fits(v, h->p.nx);
            if (!fits) continue;
            rc = lbm_batch_set_variant(b, v);
            if (rc == LBM_OK) rc = lbm_batch_step(b, std::min(reps, 8));     // warm-up and capture
            if (rc == LBM_OK) rc = hip_ok(hipEventRecord(e0, b->stream));
            if (rc == LBM_OK) rc = lbm_batch_step(b, reps);
            if (rc == LBM_OK) rc = hip_ok(hipEventRecord(e1, b->stream));
            if (rc == LBM_OK) rc = hip_ok(hipEventSynchronize(e1));
            float t = 0.f;
            if (rc == LBM_OK) rc = hip_ok(hipEventElapsedTime(&t, e0, e1));
            if (rc == LBM_OK) score[v] = std::min(score[v], t);
        }
    }
    int best = b->variant;
    float best_ms = INFINITY;
    for (int v = 0; v < kNumVariants; ++v) {
        if (score[v] < best_ms) {
            best_ms = score[v];
            best = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != LBM_OK) return rc;
    TRY(lbm_batch_set_variant(b, best));
    *best_variant = best;
    if (ms_per_step) *ms_per_step = best_ms / reps;
    return LBM_OK;
}

int lbm_batch_tune_write_through(void *batch, int reps, int *on, float *ms_per_step)
{
    Batch *b = (Batch *)batch;
    if (!b || reps < 1 || !on) return LBM_EINVAL;
    if (b->members.empty()) return LBM_ESTATE;
    const int kind = kVariants[b->variant].fused;
    if (kind != 1 && kind != 3) {                // these variants ignore the setting
        *on = b->write_through;
        if (ms_per_step) *ms_per_step = NAN;
        return LBM_OK;
    }
    hipEvent_t e0, e1;
    TRYHIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return LBM_EHIP;
    }
    // three passes, each setting scored by its fastest pass, as in autotuning
    constexpr int kPasses = 3;
    float score[2] = {INFINITY, INFINITY};
    int rc = LBM_OK;
    for (int pass = 0; pass < kPasses && rc == LBM_OK; ++pass) {
        for (int wt = 0; wt < 2 && rc == LBM_OK; ++wt) {
            b->write_through = wt;
            rc = lbm_batch_step(b, std::min(reps, 8));                         // warm-up and capture
            if (rc == LBM_OK) rc = hip_ok(hipEventRecord(e0, b->stream));
            if (rc == LBM_OK) rc = lbm_batch_step(b, reps);
            if (rc == LBM_OK) rc = hip_ok(hipEventRecord(e1, b->stream));
            if (rc == LBM_OK) rc = hip_ok(hipEventSynchronize(e1));
            float t = 0.f;
            if (rc == LBM_OK) rc = hip_ok(hipEventElapsedTime(&t, e0, e1));
            if (rc == LBM_OK) score[wt] = std::min(score[wt], t);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->write_through = score[1] < score[0] ? 1 : 0;
    if (rc != LBM_OK) return rc;
    *on = b->write_through;
    if (ms_per_step) *ms_per_step = score[b->write_through] / reps;
    return LBM_OK;
}

void lbm_batch_destroy(void *batch)
{
    Batch *b = (Batch *)batch;
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    for (Instance *h : b->members) {
        h->batch = nullptr;
        h->desc_dirty = true;
    }
    drop_graphs(b->graphs);
    b->stager_desc.release();
    b->stager_tiles.release();
    if (b->static_dev >= 0) release_static_scratch(b->static_dev);
    delete b;
}

int lbm_copy_kernel(void *d_dst, const void *d_src, size_t n, void *hip_stream)
{
    if (!d_dst || !d_src || n % 16) return LBM_EINVAL;
    TRYHIP(launch_copy(d_dst, d_src, n, (hipStream_t)hip_stream));
    return LBM_OK;
}

}  // extern "C"

namespace {

// The device's constant-rate clock (the same counter on every CU), read once
// into a variable of the library's own (no allocation, which could disturb the
// timing it serves).
__device__ unsigned long long g_clock_now;

__global__ void clock_now_kernel()
{
    g_clock_now = (unsigned long long)wall_clock64();
}

// Holds its stream until the device clock reaches `until`, or for at most
// `limit` ticks from the kernel's own start, whichever comes first: holds
// launched on several streams with the same `until` end together, however
// far apart the host enqueued them.
__global__ void hold_until_kernel(unsigned long long until, unsigned long long limit)
{
    const unsigned long long t0 = (unsigned long long)wall_clock64();
    for (;;) {
        const unsigned long long t = (unsigned long long)wall_clock64();
        if (t >= until || t - t0 >= limit) break;
    }
}

uint64_t clock_rate_hz()
{
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return 0;
    return (uint64_t)khz * 1000u;
}

}  // namespace

extern "C" {

int lbm_device_clock(uint64_t *tick, uint64_t *rate_hz)
{
    if (!tick || !rate_hz) return LBM_EINVAL;
    const uint64_t rate = clock_rate_hz();
    if (rate == 0) return LBM_EHIP;
    unsigned long long h = 0;
    clock_now_kernel<<<1, 1, 0, nullptr>>>();
    TRYHIP(hipGetLastError());
    TRYHIP(hipMemcpyFromSymbol(&h, HIP_SYMBOL(g_clock_now), sizeof(h), 0, hipMemcpyDeviceToHost));
    *tick = h;
    *rate_hz = rate;
    return LBM_OK;
}

int lbm_hold_until(uint64_t tick, uint64_t max_ticks, void *hip_stream)
{
    const uint64_t rate = clock_rate_hz();
    if (rate == 0) return LBM_EHIP;
    if (max_ticks > rate) return LBM_EINVAL;
    hold_until_kernel<<<1, 1, 0, (hipStream_t)hip_stream>>>(tick, max_ticks);
    TRYHIP(hipGetLastError());
    return LBM_OK;
}

}  // extern "C"
