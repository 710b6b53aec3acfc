// lbell_api.hip - the C ABI declared in include/lbell.h: context set-up over a
// caller-owned device arena, particle management, time stepping (kernel
// launches only; every step of the method runs in the HIP kernels) and
// read-back.  Host code only.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "lbell.h"
#include "lbell_dev.h"
#include "lbell_launch.h"
#include "lbs_internal.h"

using namespace lbd;

namespace {

constexpr size_t ALIGN = 256;
constexpr int FIELDS_CHUNK = 1 << 18;  // sites per read-back chunk
// window bitmask budget: 28 KB, twice (the bitmask and the candidate bits,
// which share the 16 KB link stage when smaller) under the 64 KB of LDS a
// work-group may hold
constexpr int MAX_LDS_WORDS = 7168;
constexpr int NEAR_MARGIN = 2;         // nodes of the near set beyond each particle window

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout {
    size_t f0 = 0, f1 = 0, omap = 0, boxes = 0, rt = 0, tile_box = 0, box_init = 0, parts = 0, links = 0,
           flags = 0, scratch = 0, near_flags = 0, near_list = 0, near_count = 0, warm = 0, step_ctr = 0,
           stamps = 0, cand = 0, band = 0, mon = 0, total = 0;
    long long cells = 0;  // owner-change stamp cells over all boxes
    int near_blocks = 0;  // collide-stream blocks that a near set can name (per slot)
    std::vector<long long> foff, stride, ooff, coff;
    std::vector<int> tile0, ntiles;
    long long pop_elems = 0, omap_elems = 0, link_pool = 0;
    int total_tiles = 0, max_particles = 0, lds_words = 0;
    size_t scratch_bytes = 0;
};

long long link_cap_for(double amax, int q) {
    // 16 (D3Q19) or 24 (D3Q27) links per unit of the circumscribed sphere's
    // area plus a floor: the discrete surface carries about 5.5 (D3Q19) or
    // 9 (D3Q27) links per unit area
    return (long long)((q == 27 ? 24.0 : 16.0) * 4.0 * M_PI * amax * amax) + 1024;
}

int lds_words_for(double amax) {
    // window edge <= 2 ceil(amax) + 6; one bit per window node, whole blocks of PBLOCK
    const int wn = 2 * (int)std::ceil(amax) + 7;
    const long long sites = (long long)wn * wn * wn;
    return (int)(((sites + PBLOCK - 1) / PBLOCK) * (PBLOCK / 32));
}

bool valid_cfg(const lb_config* c, int nboxes, const lb_box* boxes, std::string* why) {
    auto bad = [&](const char* m) {
        if (why) *why = m;
        return false;
    };
    if (!c || !boxes || nboxes <= 0) return bad("null config / boxes or nboxes <= 0");
    if (c->lattice != 19 && c->lattice != 27) return bad("lattice must be 19 (D3Q19) or 27 (D3Q27)");
    if (c->collision < 0 || c->collision > 2) return bad("unknown collision");
    if (!(c->tau > 0.5)) return bad("tau must exceed 1/2");
    if (c->collision == LB_TRT && !(c->magic > 0)) return bad("TRT needs magic > 0");
    if (c->storage < 0 || c->storage > 3) return bad("unknown storage");
    if (c->rho0 != 1.0) return bad("rho0 must be 1");
    if (!(c->max_semi_axis > 0)) return bad("max_semi_axis must be positive");
    // the node map holds id + 1 in 16 bits, 0xFFFF marking walls
    if (c->max_particles < 0 || c->max_particles > 65534) return bad("max_particles must be in 0..65534");
    if (c->rotation < 0 || c->rotation > 2) return bad("rotation must be LB_ROT_ANALYTIC, LB_ROT_FD or LB_ROT_PC");
    if (c->monitor_period < 0) return bad("monitor_period must be >= 0");
    if (lds_words_for(c->max_semi_axis) > MAX_LDS_WORDS) return bad("max_semi_axis too large for the remap window");
    for (int b = 0; b < nboxes; ++b) {
        const lb_box& B = boxes[b];
        if (B.nx < 4 || B.ny < 4 || B.nz < 4) return bad("box edges must be >= 4");
        const long long n = (long long)B.nx * B.ny * B.nz;
        if (n > (1ll << SITE_BITS)) return bad("box larger than 2^27 sites");
        if (B.walls != 0 && B.walls != 1) return bad("walls must be 0 or 1");
        if (B.walls && (B.wall_lo[1] != 0.0 || B.wall_hi[1] != 0.0)) return bad("walls cannot move along y");
        if (B.init == 1 && !B.walls) return bad("Couette start needs walls");
    }
    return true;
}

Layout make_layout(const lb_config* c, int nboxes, const lb_box* boxes) {
    Layout L;
    const int es = storage_bytes(c->storage);
    long long off = 0, ooff = 0;
    int tiles = 0;
    size_t maxpart = 0;
    for (int b = 0; b < nboxes; ++b) {
        const long long n = (long long)boxes[b].nx * boxes[b].ny * boxes[b].nz;
        // direction planes padded so that the 19 streams do not start on the
        // same memory channel
        const long long stride = (long long)align_up((size_t)n, 64) + 64;
        L.foff.push_back(off);
        L.stride.push_back(stride);
        off += (long long)align_up((size_t)(c->lattice * stride), 128);
        L.ooff.push_back(ooff);
        ooff += (long long)align_up((size_t)n, 128);
        const int nt = (int)((n + TILE - 1) / TILE);
        L.tile0.push_back(tiles);
        L.ntiles.push_back(nt);
        tiles += nt;
        maxpart = std::max(maxpart, (size_t)((n + TILE - 1) / TILE) * 6 * sizeof(double));
        L.coff.push_back(L.cells);
        L.cells += (long long)((boxes[b].nx + 7) / 8) * ((boxes[b].ny + 7) / 8) * ((boxes[b].nz + 7) / 8);
    }
    L.pop_elems = off;
    L.omap_elems = ooff;
    L.total_tiles = tiles;
    L.max_particles = c->max_particles > 0 ? c->max_particles : nboxes;
    L.link_pool = (long long)L.max_particles * link_cap_for(c->max_semi_axis, c->lattice);
    L.lds_words = lds_words_for(c->max_semi_axis);
    L.scratch_bytes = std::max(maxpart, (size_t)FIELDS_CHUNK * 4 * sizeof(double));
    size_t p = 0;
    auto take = [&](size_t bytes) {
        const size_t at = p;
        p = align_up(p + bytes, ALIGN);
        return at;
    };
    L.f0 = take((size_t)off * es);
    L.f1 = take((size_t)off * es);
    L.omap = take((size_t)ooff * sizeof(uint16_t));
    L.boxes = take(sizeof(BoxDesc) * nboxes);
    L.rt = take(sizeof(BoxRT) * nboxes);
    L.tile_box = take(sizeof(int) * tiles);
    L.box_init = take(sizeof(int) * nboxes);
    L.parts = take(sizeof(PartDev) * L.max_particles);
    L.links = take(sizeof(uint32_t) * L.link_pool);
    L.flags = take(sizeof(int) * 4);
    L.scratch = take(L.scratch_bytes);
    L.near_blocks = std::max(tiles, (boxes[0].ny * boxes[0].nz + 3) / 4);
    L.near_flags = take(sizeof(uint32_t) * 2 * L.near_blocks);
    L.near_list = take(sizeof(int) * 2 * L.near_blocks);
    L.near_count = take(sizeof(int) * 4);
    // the step counter the collide-stream kernels read (one slot per buffer
    // parity: a launch reads its slot and writes step + 1 to the other), so
    // that graph replays see the true step; slot 2 holds the epoch of the
    // particle being added (set-up epochs count down from 2^32 - 1, step
    // epochs up from 1)
    L.step_ctr = take(sizeof(uint32_t) * 4);
    // warm start: per particle load scale (1), prediction (6) and training
    // sample (8 + 6 floats = 7 doubles); then the start field's scratch
    L.warm = take(sizeof(double) * (14 * (size_t)L.max_particles + stokes_scratch_doubles(nboxes, tiles)));
    // boxes with several particles: owner-change stamps per cell of 8^3
    // nodes, and each particle's remap claim candidates (one window bitmask)
    L.stamps = take(sizeof(uint32_t) * (size_t)L.cells);
    L.cand = take(sizeof(uint32_t) * (size_t)L.max_particles * L.lds_words);
    // the narrow band of each particle's last full remap scan (a window bitmask)
    L.band = take(sizeof(uint32_t) * (size_t)L.max_particles * L.lds_words);
    // warm-start monitor: a record per box, each particle's velocity at the
    // last check (6 doubles), a flow-energy partial per tile
    L.mon = take(sizeof(BoxMon) * nboxes + sizeof(double) * (6 * (size_t)L.max_particles + tiles));
    L.total = p;
    return L;
}

struct PartHost {
    int box;
    double Fext[3], Text[3];
    double axes[3];
};

}  // namespace

struct lb_ctx {
    lb_config cfg;
    std::vector<lb_box> boxes;
    Layout L;
    hipStream_t stream = nullptr;
    char* arena = nullptr;
    std::vector<BoxDesc> hbox;
    std::vector<PartHost> hpart;
    int np = 0;
    long long link_used = 0;
    // Population storage.  Pull variants: ping-pong buffers, cur = buffer
    // holding the current state (0 -> f0, 1 -> f1).  In-place variants (aa):
    // buffer aa_buf only, cur = parity of the state (0: after an odd step,
    // convention CV_ODD; 1: after an even step, CV_EVEN).  cur also selects
    // the device step counter slot and the cached graph.
    int cur = 0;
    bool aa = false;
    int aa_buf = 0;
    long long step = 0;
    uint32_t setup_epoch = 0xFFFFFFFFu;  // owner-change stamps of the next lb_add_ellipsoid
    KParams kp{};
    bool any_walls = false;
    int k1_variant = 0;  // collide-stream variant in use (index into K1_SHAPES)
    int n_cu = 256;      // compute units of the device (persistent grid size)
    int rows_k = 0;      // row-wave width, 0 when the box shape does not allow it
    // second stream: particle phase concurrent with the far blocks (off by
    // default: measured slower when the particle kernels' dependent loads
    // queue behind the streaming kernel; LBELL_OVERLAP=1 turns it on)
    bool overlap = false;
    bool fused = true;  // one particle kernel per step when no box holds two particles (LBELL_FUSED=0: two kernels)
    bool use_band = true;  // remap rescans within the narrow band test only its nodes (LBELL_BAND=0: full scans)
    int opb_np = -1;    // particle count for which opb was computed
    bool opb = true;    // no box holds two particles
    hipStream_t nstream = nullptr;
    hipEvent_t evK = nullptr, evP = nullptr, evStart = nullptr;
    // graph replay of whole groups of steps (0 = off); one cached executable
    // per buffer parity, keyed by what the captured launch arguments depend on
    int graph_steps = 0;
    struct GraphSlot {
        hipGraphExec_t exec = nullptr;
        int np = -1, variant = -1, steps = 0;
    } graph[2];
    // warm-start monitor: checks every monitor_period steps from mon_next
    // while mon_active, until mon_until (every watched box decided by then)
    bool mon_active = false;
    long long mon_next = 0, mon_until = 0;
    std::string err;

    template <typename T>
    T* at(size_t off) { return reinterpret_cast<T*>(arena + off); }
    void* fbuf(int which) { return arena + ((aa ? aa_buf : which) ? L.f1 : L.f0); }
    // the population buffer not holding the state
    void* spare_buf() { return arena + ((aa ? aa_buf : cur) ? L.f0 : L.f1); }
    // every change of cur goes through here so the convention in kp follows
    void set_cur(int c) {
        cur = c;
        kp.conv = aa ? (c ? CV_EVEN : CV_ODD) : CV_PULL;
    }
};

namespace {

// Collide-stream variants the tuner chooses from (the index is the variant
// number of the ABI).  Row-wave kinds need a single box with nx = 64, 128 or
// 256; the near-set schedule needs kinds 0-2.  Variants 11-14 update one
// buffer in place (even / odd steps): half the population memory, so a
// lattice whose two buffers overflow the last-level cache may fit with one.
struct K1Shape {
    int kind;      // 0 generic tiles, 1 row-wave, 2 row-wave with non-temporal stores
    int spt;       // tiles per block (generic)
    int xcd;       // block order (generic): 0 plain, 1 XCD-chunked, 2 XCD-grouped
    bool persist;  // grid of a few blocks per CU walking the tiles (generic)
    bool nt;       // non-temporal stores (generic)
    bool aa;       // in place (generic)
};
constexpr K1Shape K1_SHAPES[] = {
    {0, 1, false, false, false, false}, {1, 1, false, false, false, false}, {2, 1, false, false, false, false},
    {0, 1, true, false, false, false},  {0, 2, false, false, false, false}, {0, 2, true, false, false, false},
    {0, 1, true, true, false, false},   {0, 2, true, true, false, false},   {0, 4, true, false, false, false},
    {0, 1, true, false, true, false},   {0, 2, true, false, true, false},
    {0, 1, false, false, false, true},  {0, 1, true, false, false, true},   {0, 2, true, false, false, true},
    {0, 1, true, false, true, true},   {0, 1, 2, false, true, false},
};
constexpr int K1_NSHAPES = (int)(sizeof(K1_SHAPES) / sizeof(K1_SHAPES[0]));

bool k1_applicable(const lb_ctx* ctx, int v) {
    if (v < 0 || v >= K1_NSHAPES) return false;
    // D3Q27: one tile per block, plain or XCD-chunked, pull or in place
    if (ctx->cfg.lattice == 27 && v != 0 && v != 3 && v != 11 && v != 12) return false;
    if (K1_SHAPES[v].kind != 0 && ctx->rows_k == 0) return false;
    if (ctx->overlap && v > 2) return false;
    return true;
}

lb_status fail(lb_ctx* c, lb_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

lb_status hip_check(lb_ctx* c, hipError_t e, const char* what) {
    if (e == hipSuccess) return LB_OK;
    return fail(c, LB_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPC(expr)                                              \
    do {                                                        \
        lb_status _s = hip_check(ctx, (expr), #expr);           \
        if (_s != LB_OK) return _s;                             \
    } while (0)

lb_status flags_status(lb_ctx* ctx) {
    int fl[4] = {0, 0, 0, 0};
    HIPC(hipMemcpyAsync(fl, ctx->at<int>(ctx->L.flags), sizeof fl, hipMemcpyDeviceToHost, ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    if (fl[0] == 0) return LB_OK;
    int z[4] = {0, 0, 0, 0};
    HIPC(hipMemcpyAsync(ctx->at<int>(ctx->L.flags), z, sizeof z, hipMemcpyHostToDevice, ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    if (fl[0] & F_OVERLAP) return fail(ctx, LB_EOVERLAP, "a node was claimed by two particles or a particle and a wall");
    if (fl[0] & F_NONFINITE) return fail(ctx, LB_ENONFINITE, "singular system, non-finite or |U| > 0.5 particle velocity");
    if (fl[0] & F_LINKS) return fail(ctx, LB_ENOMEM, "boundary-link capacity exceeded");
    return fail(ctx, LB_ENOMEM, "remap window exceeds the LDS budget");
}

LaunchPart part_launch(lb_ctx* ctx, int first, int count, int mode) {
    LaunchPart a{};
    a.boxes = ctx->at<BoxDesc>(ctx->L.boxes);
    a.rt = ctx->at<BoxRT>(ctx->L.rt);
    a.parts = ctx->at<PartDev>(ctx->L.parts);
    a.links = ctx->at<uint32_t>(ctx->L.links);
    a.omap = ctx->at<uint16_t>(ctx->L.omap);
    a.f = ctx->fbuf(ctx->cur);
    a.flags = ctx->at<int>(ctx->L.flags);
    a.first = first;
    a.count = count;
    a.kp = ctx->kp;
    a.lds_words = ctx->L.lds_words;
    a.mode = mode;
    a.stamps = ctx->at<uint32_t>(ctx->L.stamps);
    // after the collide launch of a step, the counter slot of the current
    // parity holds step + 1: unique to the step, also in graph replays
    a.epoch = ctx->at<uint32_t>(ctx->L.step_ctr) + ctx->cur;
    a.cand = ctx->at<uint32_t>(ctx->L.cand);
    a.force_box = -1;
    a.band = ctx->at<uint32_t>(ctx->L.band);
    a.use_band = ctx->use_band ? 1 : 0;
    return a;
}

lb_status upload_box(lb_ctx* ctx, int b) {
    HIPC(hipMemcpyAsync(ctx->at<BoxDesc>(ctx->L.boxes) + b, &ctx->hbox[b], sizeof(BoxDesc), hipMemcpyHostToDevice,
                        ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    return LB_OK;
}

template <typename T>
lb_status write_part_field(lb_ctx* ctx, int id, size_t offset, const T* src, size_t count) {
    char* dst = reinterpret_cast<char*>(ctx->at<PartDev>(ctx->L.parts) + id) + offset;
    HIPC(hipMemcpyAsync(dst, src, sizeof(T) * count, hipMemcpyHostToDevice, ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    return LB_OK;
}

lb_status read_part(lb_ctx* ctx, int id, PartDev* out) {
    HIPC(hipMemcpyAsync(out, ctx->at<PartDev>(ctx->L.parts) + id, sizeof(PartDev), hipMemcpyDeviceToHost,
                        ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    return LB_OK;
}

void set_mass(PartDev& P, double rho_p) {
    const double a = P.axes[0], b = P.axes[1], c = P.axes[2];
    P.M = rho_p * 4.0 / 3.0 * M_PI * a * b * c;
    P.Ib[0] = P.M * (b * b + c * c) / 5.0;
    P.Ib[1] = P.M * (a * a + c * c) / 5.0;
    P.Ib[2] = P.M * (a * a + b * b) / 5.0;
}

lb_status check_id(lb_ctx* ctx, int id) {
    if (!ctx) return LB_EINVAL;
    if (id < 0 || id >= ctx->np) return fail(ctx, LB_EINVAL, "no such particle id");
    return LB_OK;
}

lb_status box_fext_update(lb_ctx* ctx, int b) {
    double s[3] = {0, 0, 0};
    for (int p = 0; p < ctx->np; ++p)
        if (ctx->hpart[p].box == b)
            for (int k = 0; k < 3; ++k) s[k] += ctx->hpart[p].Fext[k];
    BoxDesc& D = ctx->hbox[b];
    for (int k = 0; k < 3; ++k) {
        D.fext[k] = s[k];
        // the uniform force density of the counter-force (the expression the
        // kernels used to evaluate per site)
        D.gcf[k] = D.counterforce ? -D.fext[k] / (double)(D.n - D.n_wall) : 0.0;
    }
    return upload_box(ctx, b);
}

lb_status moments(lb_ctx* ctx, int box, double out[6]) {
    const BoxDesc& B = ctx->hbox[box];
    const int nb = (B.n + TILE - 1) / TILE;
    double* partial = ctx->at<double>(ctx->L.scratch);
    HIPC(launch_moments(ctx->at<BoxDesc>(ctx->L.boxes), box, B.n, ctx->at<uint16_t>(ctx->L.omap), ctx->fbuf(ctx->cur),
                        partial, ctx->kp, ctx->stream));
    std::vector<double> h((size_t)nb * 6);
    HIPC(hipMemcpyAsync(h.data(), partial, h.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    // Neumaier summation of the per-block partials, in block order
    for (int k = 0; k < 6; ++k) {
        double s = 0, c = 0;
        for (int b = 0; b < nb; ++b) {
            const double v = h[(size_t)b * 6 + k], t = s + v;
            c += std::fabs(s) >= std::fabs(v) ? (s - t) + v : (v - t) + s;
            s = t;
        }
        out[k] = s + c;
    }
    return LB_OK;
}

lb_status near_rebuild(lb_ctx* ctx);

}  // namespace

extern "C" {

lb_status lb_config_default(lb_config* cfg) {
    if (!cfg) return LB_EINVAL;
    std::memset(cfg, 0, sizeof *cfg);
    cfg->lattice = 19;
    cfg->collision = LB_BGK;
    cfg->tau = 1.0;
    cfg->magic = 3.0 / 16.0;
    cfg->storage = LB_FP32;
    cfg->scale_log2 = 0;
    cfg->velocity_scale = 1e-3;
    cfg->rho0 = 1.0;
    cfg->counterforce = 0;
    cfg->max_particles = 0;
    cfg->max_semi_axis = 8.0;
    cfg->rotation = LB_ROT_ANALYTIC;
    cfg->monitor_period = 25;
    return LB_OK;
}

size_t lb_arena_bytes(const lb_config* cfg, int nboxes, const lb_box* boxes) {
    if (!valid_cfg(cfg, nboxes, boxes, nullptr)) return 0;
    return make_layout(cfg, nboxes, boxes).total;
}

namespace {
lb_status switch_layout(lb_ctx* ctx, bool to_aa);
}  // namespace

lb_status lb_init(const lb_config* cfg, int nboxes, const lb_box* boxes, void* dev_arena, size_t arena_bytes,
                  void* hip_stream, lb_ctx** out) {
    if (!out) return LB_EINVAL;
    *out = nullptr;
    std::string why;
    if (!valid_cfg(cfg, nboxes, boxes, &why)) {
        std::fprintf(stderr, "lb_init: %s\n", why.c_str());
        return LB_EINVAL;
    }
    if (!dev_arena || ((uintptr_t)dev_arena % ALIGN) != 0) return LB_EINVAL;
    lb_ctx* ctx = new lb_ctx();
    ctx->cfg = *cfg;
    ctx->boxes.assign(boxes, boxes + nboxes);
    ctx->L = make_layout(cfg, nboxes, boxes);
    if (arena_bytes < ctx->L.total) {
        delete ctx;
        return LB_ENOMEM;
    }
    ctx->arena = (char*)dev_arena;
    ctx->stream = (hipStream_t)hip_stream;
    ctx->hpart.resize(ctx->L.max_particles);
    // relaxation rates and storage scale
    KParams& kp = ctx->kp;
    kp.omega = 1.0 / cfg->tau;
    kp.omega_m = cfg->collision == LB_TRT ? 1.0 / (0.5 + cfg->magic / (cfg->tau - 0.5)) : kp.omega;
    kp.rho0 = cfg->rho0;
    kp.collision = cfg->collision;
    kp.storage = cfg->storage;
    kp.q = cfg->lattice;
    kp.rot = cfg->rotation;
    int e = 0;
    if (cfg->storage == LB_FP16 || cfg->storage == LB_BF16) {
        e = cfg->scale_log2;
        if (e == 0) {
            const double dmax = (cfg->velocity_scale > 0 ? cfg->velocity_scale : 1e-3) / 6.0;
            e = (int)std::floor(std::log2(0.25 / dmax));
        }
    }
    kp.scale = std::ldexp(1.0, e);
    kp.inv_scale = std::ldexp(1.0, -e);
    // box descriptors and tile table
    ctx->hbox.resize(nboxes);
    std::vector<int> tile_box(ctx->L.total_tiles), init(nboxes);
    for (int b = 0; b < nboxes; ++b) {
        BoxDesc& D = ctx->hbox[b];
        std::memset(&D, 0, sizeof D);
        const lb_box& X = boxes[b];
        D.nx = X.nx;
        D.ny = X.ny;
        D.nz = X.nz;
        D.n = X.nx * X.ny * X.nz;
        D.foff = ctx->L.foff[b];
        D.stride = ctx->L.stride[b];
        D.ooff = ctx->L.ooff[b];
        D.walls = X.walls;
        D.n_wall = X.walls ? 2 * X.nx * X.nz : 0;
        D.tile0 = ctx->L.tile0[b];
        D.ntiles = ctx->L.ntiles[b];
        D.counterforce = cfg->counterforce;
        magic_div(X.nx, D.mnx, D.lnx);
        magic_div(X.ny, D.mny, D.lny);
        D.coff = ctx->L.coff[b];
        D.cnx = (X.nx + 7) / 8;
        D.cny = (X.ny + 7) / 8;
        for (int k = 0; k < 3; ++k) {
            D.wall_lo[k] = X.wall_lo[k];
            D.wall_hi[k] = X.wall_hi[k];
        }
        for (int t = 0; t < D.ntiles; ++t) tile_box[D.tile0 + t] = b;
        init[b] = X.init;
        ctx->any_walls = ctx->any_walls || X.walls;
    }
    // node map: walls 0xFFFF, everything else fluid
    std::vector<uint16_t> om((size_t)ctx->L.omap_elems, 0);
    for (int b = 0; b < nboxes; ++b) {
        const BoxDesc& D = ctx->hbox[b];
        if (!D.walls) continue;
        for (int z = 0; z < D.nz; ++z)
            for (int x = 0; x < D.nx; ++x) {
                om[D.ooff + x + (size_t)D.nx * (0 + (size_t)D.ny * z)] = 0xFFFF;
                om[D.ooff + x + (size_t)D.nx * ((D.ny - 1) + (size_t)D.ny * z)] = 0xFFFF;
            }
    }
    std::vector<BoxRT> rt(nboxes);
    std::memset(rt.data(), 0, sizeof(BoxRT) * nboxes);
    hipError_t he = hipSuccess;
    auto H = [&](hipError_t x) {
        if (he == hipSuccess) he = x;
    };
    H(hipMemcpyAsync(ctx->at<BoxDesc>(ctx->L.boxes), ctx->hbox.data(), sizeof(BoxDesc) * nboxes,
                     hipMemcpyHostToDevice, ctx->stream));
    H(hipMemcpyAsync(ctx->at<BoxRT>(ctx->L.rt), rt.data(), sizeof(BoxRT) * nboxes, hipMemcpyHostToDevice,
                     ctx->stream));
    H(hipMemcpyAsync(ctx->at<int>(ctx->L.tile_box), tile_box.data(), sizeof(int) * tile_box.size(),
                     hipMemcpyHostToDevice, ctx->stream));
    H(hipMemcpyAsync(ctx->at<int>(ctx->L.box_init), init.data(), sizeof(int) * nboxes, hipMemcpyHostToDevice,
                     ctx->stream));
    H(hipMemcpyAsync(ctx->at<uint16_t>(ctx->L.omap), om.data(), sizeof(uint16_t) * om.size(), hipMemcpyHostToDevice,
                     ctx->stream));
    H(hipMemsetAsync(ctx->at<int>(ctx->L.flags), 0, sizeof(int) * 4, ctx->stream));
    H(launch_init(ctx->at<BoxDesc>(ctx->L.boxes), ctx->at<int>(ctx->L.tile_box), ctx->L.total_tiles, ctx->fbuf(0),
                  ctx->fbuf(1), ctx->at<int>(ctx->L.box_init), kp, ctx->stream));
    H(hipStreamSynchronize(ctx->stream));
    if (he != hipSuccess) {
        std::fprintf(stderr, "lb_init: %s\n", hipGetErrorString(he));
        delete ctx;
        return LB_EDEVICE;
    }
    // collide-stream variant: the row-wave kernel needs a single box whose x
    // edge is 64, 128 or 256 sites
    if (nboxes == 1 && cfg->lattice == 19 && (boxes[0].nx == 64 || boxes[0].nx == 128 || boxes[0].nx == 256)) {
        ctx->rows_k = boxes[0].nx / 64;
        ctx->k1_variant = 1;
    }
    if (const char* v = std::getenv("LBELL_OVERLAP")) ctx->overlap = std::atoi(v) != 0;
    if (const char* v = std::getenv("LBELL_FUSED")) ctx->fused = std::atoi(v) != 0;
    if (const char* v = std::getenv("LBELL_BAND")) ctx->use_band = std::atoi(v) != 0;
    if (const char* v = std::getenv("LBELL_K1_VARIANT")) {
        if (!k1_applicable(ctx, std::atoi(v))) {
            std::fprintf(stderr, "lb_init: LBELL_K1_VARIANT=%s does not apply to these boxes\n", v);
            delete ctx;
            return LB_EINVAL;
        }
        ctx->k1_variant = std::atoi(v);
    }
    {
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
            ctx->n_cu = ncu;
    }
    {
        hipError_t e2 = hipStreamCreateWithFlags(&ctx->nstream, hipStreamNonBlocking);
        if (e2 == hipSuccess) e2 = hipEventCreateWithFlags(&ctx->evK, hipEventDisableTiming);
        if (e2 == hipSuccess) e2 = hipEventCreateWithFlags(&ctx->evP, hipEventDisableTiming);
        if (e2 == hipSuccess) e2 = hipEventCreateWithFlags(&ctx->evStart, hipEventDisableTiming);
        if (e2 == hipSuccess)
            e2 = hipMemsetAsync(ctx->arena + ctx->L.near_flags, 0, ctx->L.near_count + 4 * sizeof(int) - ctx->L.near_flags,
                                ctx->stream);
        if (e2 == hipSuccess) e2 = hipMemsetAsync(ctx->arena + ctx->L.step_ctr, 0, sizeof(uint32_t) * 4, ctx->stream);
        if (e2 == hipSuccess) e2 = hipMemsetAsync(ctx->arena + ctx->L.stamps, 0, sizeof(uint32_t) * ctx->L.cells, ctx->stream);
        if (e2 == hipSuccess) e2 = hipMemsetAsync(ctx->arena + ctx->L.mon, 0, sizeof(BoxMon) * nboxes, ctx->stream);
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(ctx->stream);
        if (e2 != hipSuccess) {
            std::fprintf(stderr, "lb_init: %s\n", hipGetErrorString(e2));
            lb_destroy(ctx);
            return LB_EDEVICE;
        }
    }
    if (K1_SHAPES[ctx->k1_variant].aa && switch_layout(ctx, true) != LB_OK) {
        std::fprintf(stderr, "lb_init: %s\n", ctx->err.c_str());
        lb_destroy(ctx);
        return LB_EDEVICE;
    }
    *out = ctx;
    return LB_OK;
}

lb_status lb_add_ellipsoid(lb_ctx* ctx, int box, const double centre[3], const double semi_axes[3],
                           const double quat[4], int* id) {
    if (!ctx || !centre || !semi_axes || !quat) return LB_EINVAL;
    if (box < 0 || box >= (int)ctx->boxes.size()) return fail(ctx, LB_EINVAL, "no such box");
    if (ctx->np >= ctx->L.max_particles) return fail(ctx, LB_ENOMEM, "particle capacity exhausted");
    const BoxDesc& B = ctx->hbox[box];
    const double amax = std::max(semi_axes[0], std::max(semi_axes[1], semi_axes[2]));
    for (int k = 0; k < 3; ++k)
        if (!(semi_axes[k] > 0) || !std::isfinite(centre[k])) return fail(ctx, LB_EINVAL, "bad axes or centre");
    const int dmin = std::min(B.nx, std::min(B.ny, B.nz));
    if (2 * amax + 2 > dmin) return fail(ctx, LB_EINVAL, "particle does not fit the box");
    if (amax > ctx->cfg.max_semi_axis) return fail(ctx, LB_EINVAL, "semi-axis above cfg.max_semi_axis");
    const double nq = std::sqrt(quat[0] * quat[0] + quat[1] * quat[1] + quat[2] * quat[2] + quat[3] * quat[3]);
    if (!(std::fabs(nq - 1.0) <= 1e-6)) return fail(ctx, LB_EINVAL, "quaternion is not unit");
    const long long cap = link_cap_for(amax, ctx->cfg.lattice);
    if (ctx->link_used + cap > ctx->L.link_pool) return fail(ctx, LB_ENOMEM, "link pool exhausted");
    PartDev P;
    std::memset(&P, 0, sizeof P);
    const int n3[3] = {B.nx, B.ny, B.nz};
    for (int k = 0; k < 4; ++k) P.q[k] = P.qprev[k] = quat[k] / nq;
    for (int k = 0; k < 3; ++k) {
        double c = centre[k];
        if (c >= n3[k]) c -= n3[k] * std::floor(c / n3[k]);
        if (c < 0) c += n3[k] * std::ceil(-c / n3[k]);
        P.xc[k] = c;
        P.xu[k] = centre[k];
        P.axes[k] = semi_axes[k];
        P.ia2[k] = 1.0 / (semi_axes[k] * semi_axes[k]);
    }
    set_mass(P, ctx->cfg.rho0);
    P.box = box;
    P.lcap = (int)cap;
    P.lbase = ctx->link_used;
    const int pid = ctx->np;
    uint32_t* ep_slot = ctx->at<uint32_t>(ctx->L.step_ctr) + 2;
    const uint32_t ep = ctx->setup_epoch--;
    HIPC(hipMemcpyAsync(ep_slot, &ep, sizeof ep, hipMemcpyHostToDevice, ctx->stream));
    HIPC(hipMemcpyAsync(ctx->at<PartDev>(ctx->L.parts) + pid, &P, sizeof P, hipMemcpyHostToDevice, ctx->stream));
    {
        LaunchPart a = part_launch(ctx, pid, 1, 1);
        a.epoch = ep_slot;
        HIPC(launch_particle_remap(a, ctx->stream));
    }
    lb_status s = flags_status(ctx);
    if (s != LB_OK) {
        HIPC(launch_particle_remap(part_launch(ctx, pid, 1, 2), ctx->stream));
        HIPC(hipStreamSynchronize(ctx->stream));
        return s;
    }
    ctx->link_used += cap;
    PartHost& h = ctx->hpart[pid];
    std::memset(&h, 0, sizeof h);
    h.box = box;
    for (int k = 0; k < 3; ++k) h.axes[k] = semi_axes[k];
    ctx->np++;
    if (id) *id = pid;
    bool shared = false;
    for (int p = 0; p < pid; ++p) shared = shared || ctx->hpart[p].box == box;
    if (shared) {
        // the new nodes may have been fluid neighbours of another particle of
        // the box: the particles there whose window meets a cell the add
        // stamped rebuild their links from the node map
        LaunchPart a = part_launch(ctx, 0, ctx->np, 0);
        a.force_box = box;
        a.epoch = ep_slot;
        HIPC(launch_particle_links(a, ctx->stream));
        s = flags_status(ctx);
        if (s != LB_OK) return s;
    }
    return near_rebuild(ctx);
}

lb_status lb_set_external(lb_ctx* ctx, int id, const double F[3], const double T[3]) {
    lb_status s = check_id(ctx, id);
    if (s != LB_OK) return s;
    if (!F || !T) return LB_EINVAL;
    for (int k = 0; k < 3; ++k) {
        ctx->hpart[id].Fext[k] = F[k];
        ctx->hpart[id].Text[k] = T[k];
    }
    s = write_part_field(ctx, id, offsetof(PartDev, Fext), F, 3);
    if (s != LB_OK) return s;
    s = write_part_field(ctx, id, offsetof(PartDev, Text), T, 3);
    if (s != LB_OK) return s;
    return box_fext_update(ctx, ctx->hpart[id].box);
}

lb_status lb_set_squirmer(lb_ctx* ctx, int id, double B1, double B2) {
    lb_status s = check_id(ctx, id);
    if (s != LB_OK) return s;
    const double* ax = ctx->hpart[id].axes;
    if ((B1 != 0 || B2 != 0) && (std::fabs(ax[1] - ax[2]) > 1e-12 * ax[1] || ax[0] < ax[1]))
        return fail(ctx, LB_EINVAL, "squirmer needs a prolate spheroid, a >= b == c");
    const double v[2] = {B1, B2};
    return write_part_field(ctx, id, offsetof(PartDev, B1), v, 2);
}

lb_status lb_set_velocity(lb_ctx* ctx, int id, const double U[3], const double W[3]) {
    lb_status s = check_id(ctx, id);
    if (s != LB_OK) return s;
    if (!U || !W) return LB_EINVAL;
    {
        const double* ax = ctx->hpart[id].axes;
        const double amax = std::max(ax[0], std::max(ax[1], ax[2]));
        const double sp = std::sqrt(U[0] * U[0] + U[1] * U[1] + U[2] * U[2]) +
                          std::sqrt(W[0] * W[0] + W[1] * W[1] + W[2] * W[2]) * amax;
        if (!(sp <= 0.5)) return fail(ctx, LB_EINVAL, "velocity above the surface-speed limit");
    }
    s = write_part_field(ctx, id, offsetof(PartDev, U), U, 3);
    if (s != LB_OK) return s;
    return write_part_field(ctx, id, offsetof(PartDev, W), W, 3);
}

lb_status lb_set_particle_density(lb_ctx* ctx, int id, double rho_p) {
    lb_status s = check_id(ctx, id);
    if (s != LB_OK) return s;
    if (!(rho_p > 0)) return LB_EINVAL;
    PartDev P;
    s = read_part(ctx, id, &P);
    if (s != LB_OK) return s;
    set_mass(P, rho_p);
    s = write_part_field(ctx, id, offsetof(PartDev, M), &P.M, 1);
    if (s != LB_OK) return s;
    return write_part_field(ctx, id, offsetof(PartDev, Ib), P.Ib, 3);
}

namespace {
LaunchCS collide_args(lb_ctx* ctx, int variant) {
    LaunchCS cs{};
    cs.boxes = ctx->at<BoxDesc>(ctx->L.boxes);
    cs.rt = ctx->at<BoxRT>(ctx->L.rt);
    cs.tile_box = ctx->at<int>(ctx->L.tile_box);
    cs.ntiles = ctx->L.total_tiles;
    cs.fin = ctx->fbuf(ctx->cur);
    cs.fout = ctx->fbuf(ctx->cur ^ 1);  // the same buffer in place
    cs.kp = ctx->kp;
    cs.step_in = ctx->at<uint32_t>(ctx->L.step_ctr) + ctx->cur;
    cs.step_out = ctx->at<uint32_t>(ctx->L.step_ctr) + (ctx->cur ^ 1);
    cs.walls = ctx->any_walls;
    const K1Shape& sh = K1_SHAPES[k1_applicable(ctx, variant) ? variant : 0];
    cs.variant = sh.kind;
    cs.aa = sh.aa;
    cs.spt = sh.spt;
    cs.xcd = sh.xcd;
    cs.nt = sh.nt;
    cs.grid = sh.persist ? 8 * ctx->n_cu : 0;
    cs.rows_k = ctx->rows_k;
    cs.rows_ny = ctx->hbox[0].ny;
    cs.rows_nz = ctx->hbox[0].nz;
    cs.part = 0;
    return cs;
}

// Near set of step t: slot t % 2, tagged with epoch t + 1.
NearSet near_set(lb_ctx* ctx, long long t) {
    NearSet ns{};
    const int slot = (int)(t & 1);
    ns.flags = ctx->at<uint32_t>(ctx->L.near_flags) + (size_t)slot * ctx->L.near_blocks;
    ns.list = ctx->at<int>(ctx->L.near_list) + (size_t)slot * ctx->L.near_blocks;
    ns.count = ctx->at<int>(ctx->L.near_count) + slot;
    ns.epoch = (uint32_t)(t + 1);
    ns.rows_geom = (ctx->rows_k > 0 && K1_SHAPES[ctx->k1_variant].kind != 0) ? 1 : 0;
    ns.margin = NEAR_MARGIN;
    return ns;
}

// Upper bound of the near-set size, the launch size of the near part.
int near_grid(lb_ctx* ctx) {
    const int R = 2 * (int)std::ceil(ctx->cfg.max_semi_axis) + 6 + 2 * NEAR_MARGIN;
    const long long per = ctx->rows_k > 0 && K1_SHAPES[ctx->k1_variant].kind != 0 ? (long long)R * (R / 4 + 2)
                                                                  : (long long)R * R * (R / TILE + 2);
    return (int)std::min<long long>(ctx->L.near_blocks, per * std::max(ctx->np, 1));
}

lb_status launch_collide(lb_ctx* ctx, hipStream_t st, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr) {
    LaunchCS cs = collide_args(ctx, ctx->k1_variant);
    cs.ev_start = t0;
    cs.ev_stop = t1;
    cs.next_count = ctx->overlap && ctx->np > 0 ? near_set(ctx, ctx->step + 1).count : nullptr;
    HIPC(launch_collide_stream(cs, st));
    ctx->set_cur(ctx->cur ^ 1);
    return LB_OK;
}

// Particle phase of the step whose collide-stream output is the current
// buffer; also builds the near set of the next step from x(t + 1).
bool one_particle_per_box(lb_ctx* ctx) {
    if (ctx->opb_np != ctx->np) {  // recomputed when the particle count changes
        std::vector<int> cnt(ctx->boxes.size(), 0);
        ctx->opb = true;
        for (int p = 0; p < ctx->np; ++p)
            if (++cnt[ctx->hpart[p].box] > 1) ctx->opb = false;
        ctx->opb_np = ctx->np;
    }
    return ctx->opb;
}

lb_status launch_particles(lb_ctx* ctx, hipStream_t st) {
    if (ctx->np == 0) return LB_OK;
    LaunchPart a = part_launch(ctx, 0, ctx->np, 0);
    if (ctx->overlap) a.near = near_set(ctx, ctx->step + 1);  // only the two-stream schedule reads it
    if (ctx->fused && one_particle_per_box(ctx)) {
        // a box with one particle has no other writer, so solve and remap
        // can share a work-group
        HIPC(launch_particle_step(a, st));
    } else {
        // kernel boundaries order, over all particles: every bounce-back and
        // release before any claim (and its covered-node reads), every claim
        // before any link rebuild
        HIPC(launch_particle_solve_map(a, st));
        HIPC(launch_particle_claim(a, st));
        HIPC(launch_particle_links(a, st));
    }
    return LB_OK;
}

// Rebuilds the near set of the coming step from the current positions.
// Both slots' tags are cleared first: a tag left from another step count (a
// checkpoint load can move the counter back) must never match a new epoch.
lb_status near_rebuild(lb_ctx* ctx) {
    if (!ctx->overlap) return LB_OK;
    LaunchPart a = part_launch(ctx, 0, ctx->np, 0);
    a.near = near_set(ctx, ctx->step);
    HIPC(hipMemsetAsync(ctx->arena + ctx->L.near_flags, 0, sizeof(uint32_t) * 2 * ctx->L.near_blocks, ctx->stream));
    HIPC(hipMemsetAsync(ctx->arena + ctx->L.near_count, 0, sizeof(int) * 4, ctx->stream));
    HIPC(launch_near_mark(a, ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    return LB_OK;
}

// One step in two streams.  Caller's stream: near blocks, then far blocks.
// Particle stream: after the near blocks, the particle phase of the same
// step, concurrent with the far blocks.  The next step's near blocks wait for
// the particle phase.  The near set of step t holds every block within a
// margin of the particle windows at x(t) (built by the remap of step t - 1),
// which covers all nodes the particle phase reads or writes at step t.
lb_status step_overlapped(lb_ctx* ctx) {
    LaunchCS far = collide_args(ctx, ctx->k1_variant), nr = far;
    const NearSet ns = near_set(ctx, ctx->step);
    far.part = 1;
    nr.part = 2;
    far.near_flags = nr.near_flags = ns.flags;
    far.near_list = nr.near_list = ns.list;
    far.near_count = nr.near_count = ns.count;
    far.near_epoch = nr.near_epoch = ns.epoch;
    nr.near_grid = near_grid(ctx);
    nr.next_count = near_set(ctx, ctx->step + 1).count;  // emptied before the particle phase fills it
    HIPC(hipStreamWaitEvent(ctx->stream, ctx->evP, 0));
    HIPC(launch_collide_stream(nr, ctx->stream));
    HIPC(hipEventRecord(ctx->evK, ctx->stream));
    HIPC(launch_collide_stream(far, ctx->stream));
    HIPC(hipStreamWaitEvent(ctx->nstream, ctx->evK, 0));
    ctx->set_cur(ctx->cur ^ 1);
    lb_status s = launch_particles(ctx, ctx->nstream);
    if (s != LB_OK) return s;
    HIPC(hipEventRecord(ctx->evP, ctx->nstream));
    return LB_OK;
}

void graph_drop(lb_ctx* ctx) {
    for (auto& g : ctx->graph) {
        if (g.exec) hipGraphExecDestroy(g.exec);
        g = lb_ctx::GraphSlot{};
    }
}

// Moves the populations between the two-buffer pull layout and the in-place
// layout (to_aa).  Every slot is permuted exactly, nothing is recomputed, so
// the run continues bit for bit.  The state lands in the other buffer; the
// device step counter moves to the slot of the new cur.
lb_status switch_layout(lb_ctx* ctx, bool to_aa) {
    if (ctx->aa == to_aa) return LB_OK;
    graph_drop(ctx);
    const int src_buf = ctx->aa ? ctx->aa_buf : ctx->cur, dst_buf = src_buf ^ 1;
    HIPC(launch_relayout(ctx->at<BoxDesc>(ctx->L.boxes), ctx->at<int>(ctx->L.tile_box), ctx->L.total_tiles,
                         ctx->arena + (src_buf ? ctx->L.f1 : ctx->L.f0), ctx->arena + (dst_buf ? ctx->L.f1 : ctx->L.f0),
                         ctx->kp.conv, to_aa ? CV_EVEN : CV_PULL, ctx->cfg.storage, ctx->cfg.lattice, ctx->stream));
    ctx->aa = to_aa;
    ctx->aa_buf = dst_buf;
    const int c = to_aa ? 1 : dst_buf;
    const uint32_t st32 = (uint32_t)ctx->step;
    HIPC(hipMemcpyAsync(ctx->at<uint32_t>(ctx->L.step_ctr) + c, &st32, sizeof st32, hipMemcpyHostToDevice,
                        ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    ctx->set_cur(c);
    return LB_OK;
}

// Makes v the collide-stream variant: the population layout follows it, and
// the near set is rebuilt when the block geometry changes.
lb_status use_variant(lb_ctx* ctx, int v) {
    const bool kind_changed = K1_SHAPES[v].kind != K1_SHAPES[ctx->k1_variant].kind;
    lb_status s = switch_layout(ctx, K1_SHAPES[v].aa);
    if (s != LB_OK) return s;
    ctx->k1_variant = v;
    return kind_changed ? near_rebuild(ctx) : LB_OK;
}

// One replay of a group of graph_steps steps; captures the group first if
// the cached executable does not match the current launch arguments.
lb_status step_graph(lb_ctx* ctx) {
    lb_ctx::GraphSlot& g = ctx->graph[ctx->cur];
    if (!g.exec || g.np != ctx->np || g.variant != ctx->k1_variant || g.steps != ctx->graph_steps) {
        if (g.exec) hipGraphExecDestroy(g.exec);
        g = lb_ctx::GraphSlot{};
        const int cur0 = ctx->cur;
        const long long step0 = ctx->step;
        HIPC(hipStreamBeginCapture(ctx->nstream, hipStreamCaptureModeThreadLocal));
        lb_status s = LB_OK;
        for (int k = 0; k < ctx->graph_steps && s == LB_OK; ++k) {
            s = launch_collide(ctx, ctx->nstream);
            if (s == LB_OK) s = launch_particles(ctx, ctx->nstream);
            ctx->step++;
        }
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(ctx->nstream, &graph);
        ctx->set_cur(cur0);
        ctx->step = step0;
        if (s != LB_OK) {
            if (graph) hipGraphDestroy(graph);
            return s;
        }
        HIPC(ec);
        const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        HIPC(ei);
        g.np = ctx->np;
        g.variant = ctx->k1_variant;
        g.steps = ctx->graph_steps;
    }
    HIPC(hipGraphLaunch(g.exec, ctx->stream));
    ctx->set_cur(ctx->cur ^ (ctx->graph_steps & 1));
    ctx->step += ctx->graph_steps;
    return LB_OK;
}

}  // namespace

lb_status lb_set_graph(lb_ctx* ctx, int steps) {
    if (!ctx || steps < 0) return LB_EINVAL;
    if (steps > 0 && ctx->overlap) return fail(ctx, LB_ESTATE, "graph replay is not available with two streams");
    graph_drop(ctx);
    ctx->graph_steps = steps;
    return LB_OK;
}

namespace {
int monitor_period(const lb_ctx* ctx) { return ctx->cfg.monitor_period > 0 ? ctx->cfg.monitor_period : 25; }

// The warm-start check of every watched box, when one is due (after the
// step or group of steps just enqueued); enqueued on the stream like a step.
lb_status monitor_if_due(lb_ctx* ctx) {
    if (!ctx->mon_active || ctx->step < ctx->mon_next) return LB_OK;
    const int nb = (int)ctx->boxes.size();
    BoxMon* mon = ctx->at<BoxMon>(ctx->L.mon);
    double* vref = reinterpret_cast<double*>(mon + nb);
    double* partial = vref + 6 * (size_t)ctx->L.max_particles;
    const double* pred = ctx->at<double>(ctx->L.warm) + ctx->L.max_particles;
    HIPC(launch_box_energy(ctx->at<BoxDesc>(ctx->L.boxes), ctx->at<int>(ctx->L.tile_box), ctx->L.total_tiles,
                           ctx->at<uint16_t>(ctx->L.omap), ctx->fbuf(ctx->cur), mon, partial, ctx->kp, ctx->stream));
    HIPC(launch_warm_monitor(ctx->at<BoxDesc>(ctx->L.boxes), nb, ctx->at<int>(ctx->L.tile_box), ctx->L.total_tiles,
                             mon, partial, ctx->at<PartDev>(ctx->L.parts), ctx->np, pred, vref, ctx->step,
                             ctx->fbuf(ctx->cur), ctx->cfg.storage, ctx->cfg.lattice, ctx->stream));
    ctx->mon_next = ctx->step + monitor_period(ctx);
    if (ctx->step > ctx->mon_until) ctx->mon_active = false;
    return LB_OK;
}
}  // namespace

lb_status lb_step(lb_ctx* ctx, int n) {
    if (!ctx || n < 0) return LB_EINVAL;
    if (n == 0) return LB_OK;
    const bool ov = ctx->overlap && ctx->np > 0;
    if (ov) {  // the particle stream starts after everything already on the caller's stream
        HIPC(hipEventRecord(ctx->evStart, ctx->stream));
        HIPC(hipStreamWaitEvent(ctx->nstream, ctx->evStart, 0));
        HIPC(hipEventRecord(ctx->evP, ctx->stream));
    }
    int k = 0;
    if (!ov && ctx->graph_steps > 0) {
        for (; k + ctx->graph_steps <= n; k += ctx->graph_steps) {
            lb_status s = step_graph(ctx);
            if (s == LB_OK) s = monitor_if_due(ctx);
            if (s != LB_OK) return s;
        }
    }
    for (; k < n; ++k) {
        lb_status s = ov ? step_overlapped(ctx) : launch_collide(ctx, ctx->stream);
        if (s == LB_OK && !ov) s = launch_particles(ctx, ctx->stream);
        if (s != LB_OK) return s;
        ctx->step++;
        if (!ov && (s = monitor_if_due(ctx)) != LB_OK) return s;
    }
    if (ov) HIPC(hipStreamWaitEvent(ctx->stream, ctx->evP, 0));  // join
    return LB_OK;
}

lb_status lb_profile_step(lb_ctx* ctx, int n, double* ms_collide, double* ms_particle) {
    if (!ctx || n < 0) return LB_EINVAL;
    // collide-stream: events bound to the kernel's own start and end; particle
    // phase: events on the stream around its launches
    std::vector<hipEvent_t> ev((size_t)4 * n);
    for (auto& e : ev) HIPC(hipEventCreate(&e));
    lb_status s = LB_OK;
    for (int k = 0; k < n && s == LB_OK; ++k) {
        s = launch_collide(ctx, ctx->stream, ev[4 * k], ev[4 * k + 1]);
        HIPC(hipEventRecord(ev[4 * k + 2], ctx->stream));
        if (s == LB_OK) s = launch_particles(ctx, ctx->stream);
        HIPC(hipEventRecord(ev[4 * k + 3], ctx->stream));
        ctx->step++;
    }
    HIPC(hipStreamSynchronize(ctx->stream));
    double c = 0, p = 0;
    for (int k = 0; k < n; ++k) {
        float a = 0, b = 0;
        HIPC(hipEventElapsedTime(&a, ev[4 * k], ev[4 * k + 1]));
        HIPC(hipEventElapsedTime(&b, ev[4 * k + 2], ev[4 * k + 3]));
        c += a;
        p += b;
    }
    for (auto& e : ev) hipEventDestroy(e);
    if (ms_collide) *ms_collide = c;
    if (ms_particle) *ms_particle = p;
    return s;
}

lb_status lb_autotune(lb_ctx* ctx, int reps, int* variant, double* ms_best) {
    if (!ctx || reps <= 0) return LB_EINVAL;
    // Every variant is timed inside real time steps (collide-stream, then the
    // particle phase), so each launch reads the buffer the previous step
    // wrote, as in production; timing a kernel against the same input again
    // and again would let the last-level cache serve part of it.  The events
    // take the kernel's own start and end.  All variants compute
    // bit-identical results, so the steps taken here are ordinary steps of
    // the simulation.
    std::vector<hipEvent_t> ev((size_t)2 * reps);
    for (auto& e : ev) HIPC(hipEventCreate(&e));
    const int keep = ctx->k1_variant;
    // Two sweeps over the variants; each variant counts with the smaller of
    // its two means.  In a single sweep the variants timed first would also
    // carry the clock ramp-up of an idle GPU.
    constexpr int SWEEPS = 2;
    double tv[K1_NSHAPES];
    for (double& t : tv) t = 1e300;
    lb_status s = LB_OK;
    for (int sw = 0; sw < SWEEPS && s == LB_OK; ++sw) {
        for (int v = 0; v < K1_NSHAPES && s == LB_OK; ++v) {
            if (!k1_applicable(ctx, v)) continue;
            if ((s = use_variant(ctx, v)) != LB_OK) break;
            // two untimed steps first: after a layout switch the first step
            // finds the populations out of the last-level cache
            for (int r = -2; r < reps && s == LB_OK; ++r) {
                s = r >= 0 ? launch_collide(ctx, ctx->stream, ev[2 * r], ev[2 * r + 1]) : launch_collide(ctx, ctx->stream);
                if (s == LB_OK) s = launch_particles(ctx, ctx->stream);
                ctx->step++;
            }
            if (s != LB_OK) break;
            HIPC(hipStreamSynchronize(ctx->stream));
            double t = 0;
            for (int r = 0; r < reps; ++r) {
                float ms = 0;
                HIPC(hipEventElapsedTime(&ms, ev[2 * r], ev[2 * r + 1]));
                t += ms;
            }
            tv[v] = std::min(tv[v], t / reps);
        }
    }
    int best = keep;
    double tbest = 1e300;
    for (int v = 0; v < K1_NSHAPES; ++v)
        if (tv[v] < tbest) {
            tbest = tv[v];
            best = v;
        }
    for (auto& e : ev) hipEventDestroy(e);
    if (s != LB_OK) return s;
    if ((s = use_variant(ctx, best)) != LB_OK) return s;
    if (variant) *variant = best;
    if (ms_best) *ms_best = tbest;
    return flags_status(ctx);
}

lb_status lb_bandwidth_probe(void* dst, const void* src, size_t bytes, void* hip_stream, int reps, double* gbs) {
    if (!dst || !src || bytes < 16 || (bytes % 16) != 0 || reps <= 0 || !gbs) return LB_EINVAL;
    if (((uintptr_t)dst | (uintptr_t)src) % 16 != 0) return LB_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return LB_EDEVICE;
    (void)cus;
    const size_t nblk = (bytes / 16 + 255) / 256;  // one 16-byte element per thread
    if (nblk > (size_t)INT32_MAX) return LB_EINVAL;
    const int blocks = (int)nblk;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return LB_EDEVICE;
    bool ok = launch_copy_probe(src, dst, bytes, blocks, st) == hipSuccess;  // warm-up
    ok = ok && hipEventRecord(e0, st) == hipSuccess;
    for (int r = 0; r < reps && ok; ++r) ok = launch_copy_probe(src, dst, bytes, blocks, st) == hipSuccess;
    ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
    float ms = 0;
    ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (!ok) return LB_EDEVICE;
    *gbs = 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9;
    return LB_OK;
}

lb_status lb_sync(lb_ctx* ctx) {
    if (!ctx) return LB_EINVAL;
    HIPC(hipStreamSynchronize(ctx->stream));
    return flags_status(ctx);
}

lb_status lb_get_force_torque(lb_ctx* ctx, int id, double F[3], double T[3]) {
    lb_status s = check_id(ctx, id);
    if (s != LB_OK) return s;
    PartDev P;
    s = read_part(ctx, id, &P);
    if (s != LB_OK) return s;
    for (int k = 0; k < 3; ++k) {
        if (F) F[k] = P.F[k];
        if (T) T[k] = P.T[k];
    }
    return flags_status(ctx);
}

lb_status lb_get_particle(lb_ctx* ctx, int id, double x[3], double q[4], double U[3], double W[3]) {
    lb_status s = check_id(ctx, id);
    if (s != LB_OK) return s;
    PartDev P;
    s = read_part(ctx, id, &P);
    if (s != LB_OK) return s;
    for (int k = 0; k < 3; ++k) {
        if (x) x[k] = P.xu[k];
        if (U) U[k] = P.U[k];
        if (W) W[k] = P.W[k];
    }
    if (q)
        for (int k = 0; k < 4; ++k) q[k] = P.q[k];
    return flags_status(ctx);
}

lb_status lb_get_particle_aux(lb_ctx* ctx, int id, double* M, double* dm, double P3[3], double L3[3], int* nlinks) {
    lb_status s = check_id(ctx, id);
    if (s != LB_OK) return s;
    PartDev P;
    s = read_part(ctx, id, &P);
    if (s != LB_OK) return s;
    if (M) *M = P.M;
    if (dm) *dm = P.dm;
    for (int k = 0; k < 3; ++k) {
        if (P3) P3[k] = P.Pp[k];
        if (L3) L3[k] = P.Lp[k];
    }
    if (nlinks) *nlinks = P.nlinks;
    return LB_OK;
}

lb_status lb_get_links(lb_ctx* ctx, int id, uint32_t* site, uint8_t* dir, int cap, int* n) {
    lb_status s = check_id(ctx, id);
    if (s != LB_OK) return s;
    PartDev P;
    s = read_part(ctx, id, &P);
    if (s != LB_OK) return s;
    if (n) *n = P.nlinks;
    if (cap < P.nlinks) return LB_ERANGE;
    std::vector<uint32_t> codes((size_t)std::max(P.nlinks, 1));
    if (P.nlinks > 0) {
        HIPC(hipMemcpyAsync(codes.data(), ctx->at<uint32_t>(ctx->L.links) + P.lbase, sizeof(uint32_t) * P.nlinks,
                            hipMemcpyDeviceToHost, ctx->stream));
        HIPC(hipStreamSynchronize(ctx->stream));
    }
    for (int k = 0; k < P.nlinks; ++k) {
        if (site) site[k] = codes[k] & SITE_MASK;
        if (dir) dir[k] = (uint8_t)(codes[k] >> SITE_BITS);
    }
    return LB_OK;
}

lb_status lb_get_mask(lb_ctx* ctx, int box, uint16_t* owner) {
    if (!ctx || !owner || box < 0 || box >= (int)ctx->boxes.size()) return LB_EINVAL;
    const BoxDesc& B = ctx->hbox[box];
    HIPC(hipMemcpyAsync(owner, ctx->at<uint16_t>(ctx->L.omap) + B.ooff, sizeof(uint16_t) * B.n, hipMemcpyDeviceToHost,
                        ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    return LB_OK;
}

lb_status lb_get_fields(lb_ctx* ctx, int box, double* rho, double* u) {
    if (!ctx || box < 0 || box >= (int)ctx->boxes.size()) return LB_EINVAL;
    const BoxDesc& B = ctx->hbox[box];
    double* tmp = ctx->at<double>(ctx->L.scratch);
    std::vector<double> h((size_t)FIELDS_CHUNK * 4);
    for (int s0 = 0; s0 < B.n; s0 += FIELDS_CHUNK) {
        const int cnt = std::min(FIELDS_CHUNK, B.n - s0);
        HIPC(launch_fields(ctx->at<BoxDesc>(ctx->L.boxes), box, ctx->at<uint16_t>(ctx->L.omap), ctx->fbuf(ctx->cur),
                           s0, cnt, tmp, ctx->kp, ctx->stream));
        HIPC(hipMemcpyAsync(h.data(), tmp, sizeof(double) * 4 * cnt, hipMemcpyDeviceToHost, ctx->stream));
        HIPC(hipStreamSynchronize(ctx->stream));
        for (int k = 0; k < cnt; ++k) {
            if (rho) rho[s0 + k] = h[4 * (size_t)k];
            if (u)
                for (int c = 0; c < 3; ++c) u[3 * (size_t)(s0 + k) + c] = h[4 * (size_t)k + 1 + c];
        }
    }
    return LB_OK;
}

lb_status lb_get_mass(lb_ctx* ctx, int box, double* mass) {
    if (!ctx || !mass || box < 0 || box >= (int)ctx->boxes.size()) return LB_EINVAL;
    double m[6];
    lb_status s = moments(ctx, box, m);
    if (s != LB_OK) return s;
    // every non-wall node counted at rho0 (particle nodes carry rho0 through
    // their transitions), plus the fluid's excess and the pending excess
    const BoxDesc& B = ctx->hbox[box];
    double tot = (double)(B.n - B.n_wall) * ctx->cfg.rho0 + m[1];
    for (int p = 0; p < ctx->np; ++p)
        if (ctx->hpart[p].box == box) {
            double dm = 0;
            s = lb_get_particle_aux(ctx, p, nullptr, &dm, nullptr, nullptr, nullptr);
            if (s != LB_OK) return s;
            tot += dm;
        }
    *mass = tot;
    return LB_OK;
}

lb_status lb_get_momentum(lb_ctx* ctx, int box, double P[3]) {
    if (!ctx || !P || box < 0 || box >= (int)ctx->boxes.size()) return LB_EINVAL;
    double m[6];
    lb_status s = moments(ctx, box, m);
    if (s != LB_OK) return s;
    for (int k = 0; k < 3; ++k) P[k] = m[2 + k];
    return LB_OK;
}

lb_status lb_check_finite(lb_ctx* ctx, int box, long long* count) {
    if (!ctx || !count || box < 0 || box >= (int)ctx->boxes.size()) return LB_EINVAL;
    double m[6];
    lb_status s = moments(ctx, box, m);
    if (s != LB_OK) return s;
    *count = (long long)m[5];
    return LB_OK;
}

lb_status lb_get_step(lb_ctx* ctx, long long* step) {
    if (!ctx || !step) return LB_EINVAL;
    *step = ctx->step;
    return LB_OK;
}

namespace {
// 3: the particle record carries the previous orientation and the remap
// skip reference, and no drag matrix (rebuilt from the link moments);
// 4: and the remap change flags of boxes with several particles
constexpr int CKPT_VERSION = 5;
struct CkptHeader {
    char magic[8];
    int version, nboxes, storage, np, cur, pad;  // version: CKPT_VERSION
    long long step, pop_elems, omap_elems, link_used;
    size_t part_bytes;
};
}  // namespace

lb_status lb_save(lb_ctx* ctx, const char* path) {
    if (!ctx || !path) return LB_EINVAL;
    HIPC(hipStreamSynchronize(ctx->stream));
    FILE* fp = std::fopen(path, "wb");
    if (!fp) return fail(ctx, LB_EIO, "cannot open checkpoint for writing");
    CkptHeader h{};
    std::memcpy(h.magic, "LBELLCK1", 8);
    h.version = CKPT_VERSION;
    h.pad = ctx->aa ? 1 : 0;  // populations in the in-place layout (cur = parity)
    h.nboxes = (int)ctx->boxes.size();
    h.storage = ctx->cfg.storage;
    h.np = ctx->np;
    h.cur = ctx->cur;
    h.step = ctx->step;
    h.pop_elems = ctx->L.pop_elems;
    h.omap_elems = ctx->L.omap_elems;
    h.link_used = ctx->link_used;
    h.part_bytes = sizeof(PartDev);
    const size_t es = storage_bytes(ctx->cfg.storage);
    std::vector<char> buf;
    bool ok = std::fwrite(&h, sizeof h, 1, fp) == 1;
    auto dump = [&](const void* dptr, size_t bytes) {
        if (!ok) return;
        buf.resize(std::max(bytes, (size_t)1));
        if (hipMemcpy(buf.data(), dptr, bytes, hipMemcpyDeviceToHost) != hipSuccess) ok = false;
        if (ok && bytes && std::fwrite(buf.data(), 1, bytes, fp) != bytes) ok = false;
    };
    dump(ctx->fbuf(ctx->cur), (size_t)ctx->L.pop_elems * es);
    dump(ctx->at<char>(ctx->L.omap), (size_t)ctx->L.omap_elems * sizeof(uint16_t));
    dump(ctx->at<char>(ctx->L.rt), sizeof(BoxRT) * ctx->boxes.size());
    dump(ctx->at<char>(ctx->L.parts), sizeof(PartDev) * ctx->np);
    dump(ctx->at<char>(ctx->L.links), sizeof(uint32_t) * ctx->link_used);
    if (ok) ok = std::fwrite(ctx->hpart.data(), sizeof(PartHost), ctx->np, fp) == (size_t)ctx->np;
    if (std::fclose(fp) != 0) ok = false;
    return ok ? LB_OK : fail(ctx, LB_EIO, "checkpoint write failed");
}

lb_status lb_load(lb_ctx* ctx, const char* path) {
    if (!ctx || !path) return LB_EINVAL;
    FILE* fp = std::fopen(path, "rb");
    if (!fp) return fail(ctx, LB_EIO, "cannot open checkpoint");
    CkptHeader h{};
    bool ok = std::fread(&h, sizeof h, 1, fp) == 1;
    if (!ok || std::memcmp(h.magic, "LBELLCK1", 8) != 0) {
        std::fclose(fp);
        return fail(ctx, LB_EIO, "not a checkpoint");
    }
    if (h.version != CKPT_VERSION || h.nboxes != (int)ctx->boxes.size() || h.storage != ctx->cfg.storage ||
        h.pop_elems != ctx->L.pop_elems ||
        h.omap_elems != ctx->L.omap_elems || h.np > ctx->L.max_particles || h.link_used > ctx->L.link_pool ||
        h.part_bytes != sizeof(PartDev)) {
        std::fclose(fp);
        return fail(ctx, LB_EINVAL, "checkpoint does not match this context");
    }
    HIPC(hipStreamSynchronize(ctx->stream));
    const size_t es = storage_bytes(ctx->cfg.storage);
    std::vector<char> buf;
    auto load = [&](void* dptr, size_t bytes) {
        if (!ok) return;
        buf.resize(std::max(bytes, (size_t)1));
        if (bytes && std::fread(buf.data(), 1, bytes, fp) != bytes) ok = false;
        if (ok && hipMemcpy(dptr, buf.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) ok = false;
    };
    graph_drop(ctx);
    ctx->aa = h.pad != 0;
    ctx->aa_buf = 0;
    ctx->set_cur(h.cur);
    load(ctx->fbuf(ctx->cur), (size_t)h.pop_elems * es);
    load(ctx->at<char>(ctx->L.omap), (size_t)h.omap_elems * sizeof(uint16_t));
    load(ctx->at<char>(ctx->L.rt), sizeof(BoxRT) * ctx->boxes.size());
    {   // the particle records; their narrow bands are not part of a checkpoint
        std::vector<PartDev> parts((size_t)h.np);
        if (ok && h.np && std::fread(parts.data(), sizeof(PartDev), h.np, fp) != (size_t)h.np) ok = false;
        for (auto& P : parts) P.bvalid = 0;
        if (ok && h.np &&
            hipMemcpy(ctx->at<PartDev>(ctx->L.parts), parts.data(), sizeof(PartDev) * h.np, hipMemcpyHostToDevice) !=
                hipSuccess)
            ok = false;
    }
    load(ctx->at<char>(ctx->L.links), sizeof(uint32_t) * h.link_used);
    if (ok) ok = std::fread(ctx->hpart.data(), sizeof(PartHost), h.np, fp) == (size_t)h.np;
    std::fclose(fp);
    if (!ok) return fail(ctx, LB_EIO, "checkpoint read failed");
    ctx->np = h.np;
    ctx->opb_np = -1;  // which boxes hold several particles is recomputed
    ctx->step = h.step;
    ctx->link_used = h.link_used;
    // stamps of the steps after the checkpoint must not match an epoch again;
    // the warm-start monitor is not part of a checkpoint
    HIPC(hipMemsetAsync(ctx->arena + ctx->L.stamps, 0, sizeof(uint32_t) * ctx->L.cells, ctx->stream));
    HIPC(hipMemsetAsync(ctx->arena + ctx->L.mon, 0, sizeof(BoxMon) * ctx->boxes.size(), ctx->stream));
    ctx->mon_active = false;
    {
        const uint32_t st32 = (uint32_t)h.step;  // the device step counter of the restored parity
        HIPC(hipMemcpyAsync(ctx->at<uint32_t>(ctx->L.step_ctr) + ctx->cur, &st32, sizeof st32, hipMemcpyHostToDevice,
                            ctx->stream));
        HIPC(hipStreamSynchronize(ctx->stream));
    }
    for (int b = 0; b < (int)ctx->boxes.size(); ++b) {
        lb_status s = box_fext_update(ctx, b);
        if (s != LB_OK) return s;
    }
    // the checkpoint's layout, converted to the one this context's variant uses
    lb_status s = switch_layout(ctx, K1_SHAPES[ctx->k1_variant].aa);
    if (s != LB_OK) return s;
    return near_rebuild(ctx);
}

lb_status lb_debug_poke(lb_ctx* ctx, int box, int site, int dir, double value) {
    if (!ctx || box < 0 || box >= (int)ctx->boxes.size() || dir < 0 || dir >= ctx->cfg.lattice) return LB_EINVAL;
    if (site < 0 || site >= ctx->hbox[box].n) return LB_EINVAL;
    HIPC(launch_poke(ctx->at<BoxDesc>(ctx->L.boxes), box, ctx->fbuf(ctx->cur), site, dir, value, ctx->kp,
                     ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    return LB_OK;
}

lb_status lb_get_particles(lb_ctx* ctx, int first, int count, double* x, double* q, double* U, double* W) {
    if (!ctx || first < 0 || count < 0 || first + count > ctx->np) return LB_EINVAL;
    if (count == 0) return LB_OK;
    std::vector<PartDev> P((size_t)count);
    HIPC(hipMemcpyAsync(P.data(), ctx->at<PartDev>(ctx->L.parts) + first, sizeof(PartDev) * count,
                        hipMemcpyDeviceToHost, ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    for (int i = 0; i < count; ++i)
        for (int k = 0; k < 4; ++k) {
            if (k < 3) {
                if (x) x[3 * i + k] = P[i].xu[k];
                if (U) U[3 * i + k] = P[i].U[k];
                if (W) W[3 * i + k] = P[i].W[k];
            }
            if (q) q[4 * i + k] = P[i].q[k];
        }
    return flags_status(ctx);
}

namespace {
double viscosity(const lb_ctx* ctx) { return (1.0 / ctx->kp.omega - 0.5) / 3.0; }

lb_status stokes_start(lb_ctx* ctx, int only_box = -1) {
    for (size_t b = 0; b < ctx->boxes.size(); ++b)
        if ((only_box < 0 || (int)b == only_box) && ctx->boxes[b].walls)
            return fail(ctx, LB_EINVAL, "the start field is defined for periodic boxes only");
    double* scratch = ctx->at<double>(ctx->L.warm) + 14 * (size_t)ctx->L.max_particles;
    // the nodes' free flow and pressure go to the population buffer that does
    // not hold the state (the next step's output, or unused in place): 4
    // doubles per node fit in the Q >= 19 populations of >= 2 bytes each.
    // One box: into that box's own block of it, so other boxes' blocks (a
    // walled box's never-written wall rows among them) keep their contents.
    const size_t es = storage_bytes(ctx->cfg.storage), need = stokes_free_doubles() * sizeof(double);
    char* spare = (char*)ctx->spare_buf();
    long long base = 0;
    if (only_box >= 0) {
        const BoxDesc& B = ctx->hbox[only_box];
        if ((size_t)B.n * need > (size_t)ctx->cfg.lattice * B.stride * es)
            return fail(ctx, LB_EINVAL, "population block too small for the start field's scratch");
        spare += (size_t)B.foff * es;  // foff is a multiple of 128 elements: 8-byte aligned
        base = B.ooff;
    } else if ((size_t)ctx->L.omap_elems * need > (size_t)ctx->L.pop_elems * es) {
        return fail(ctx, LB_EINVAL, "population buffer too small for the start field's scratch");
    }
    HIPC(launch_stokes_start(ctx->at<BoxDesc>(ctx->L.boxes), (int)ctx->boxes.size(), ctx->at<int>(ctx->L.tile_box),
                             ctx->L.total_tiles, ctx->at<uint16_t>(ctx->L.omap), ctx->at<PartDev>(ctx->L.parts),
                             ctx->np, viscosity(ctx) * ctx->kp.rho0, scratch, (double*)spare, base,
                             ctx->fbuf(ctx->cur), ctx->kp, only_box, ctx->stream));
    return LB_OK;
}
}  // namespace

lb_status lb_stokes_start(lb_ctx* ctx) {
    if (!ctx) return LB_EINVAL;
    lb_status s = stokes_start(ctx);
    if (s != LB_OK) return s;
    HIPC(hipStreamSynchronize(ctx->stream));
    return flags_status(ctx);
}

lb_status lb_warm_start(lb_ctx* ctx, int box, lbs* sur, double tol, double* pred) {
    if (!ctx || !sur) return LB_EINVAL;
    const int nb = (int)ctx->boxes.size();
    if (box < -1 || box >= nb) return fail(ctx, LB_EINVAL, "no such box");
    if (ctx->np == 0) return LB_OK;
    if (ctx->np > sur->max_n) return fail(ctx, LB_EINVAL, "more particles than the surrogate's sample capacity");
    for (int b = 0; b < nb; ++b)
        if ((box < 0 || b == box) && ctx->boxes[b].walls)
            return fail(ctx, LB_EINVAL, "the warm start is defined for periodic boxes only");
    // the surrogate's work goes on the context's stream, after the steps already queued there
    double* sc = ctx->at<double>(ctx->L.warm);
    double* pr = sc + ctx->L.max_particles;
    PartDev* parts = ctx->at<PartDev>(ctx->L.parts);
    const double nu = viscosity(ctx), mu = ctx->kp.rho0 * nu;
    HIPC(launch_warm_features(ctx->at<BoxDesc>(ctx->L.boxes), parts, ctx->np, mu, sur->X, sc, ctx->stream));
    MlpArgs a{sur->P, sur->X, nullptr, sur->out, nullptr, nullptr, ctx->np, 0.f, 0};
    HIPC(launch_mlp(a, ctx->stream));
    HIPC(launch_warm_apply(parts, ctx->np, sur->out, sc, mu, pr, box, ctx->stream));
    lb_status s = stokes_start(ctx, box);
    if (s != LB_OK) return s;
    // the monitor of the warm-started boxes
    BoxMon* mon = ctx->at<BoxMon>(ctx->L.mon);
    std::vector<BoxMon> hm((size_t)nb);
    HIPC(hipMemcpyAsync(hm.data(), mon, sizeof(BoxMon) * nb, hipMemcpyDeviceToHost, ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    long long maxW0 = 0;
    for (int b = 0; b < nb; ++b) {
        if (box >= 0 && b != box) continue;
        BoxMon& M = hm[b];
        std::memset(&M, 0, sizeof M);
        // W0: the viscous time of the box's largest particle, 2 a^2 / nu
        int W0 = -1;
        for (int p = 0; p < ctx->np; ++p)
            if (ctx->hpart[p].box == b) {
                const double* ax = ctx->hpart[p].axes;
                const double am = std::max(ax[0], std::max(ax[1], ax[2]));
                W0 = std::max(W0, (int)std::ceil(2.0 * am * am / nu));
            }
        M.status = (tol > 0 && W0 >= 0) ? MON_PENDING : MON_OFF;
        M.W0 = std::max(W0, 1);
        M.Wref = M.W0 / 4;
        M.tol = tol;
        M.t0 = ctx->step;
        M.t_ref = -1;
        M.t_decided = -1;
        if (M.status == MON_PENDING) maxW0 = std::max(maxW0, (long long)M.W0);
    }
    HIPC(hipMemcpyAsync(mon, hm.data(), sizeof(BoxMon) * nb, hipMemcpyHostToDevice, ctx->stream));
    if (maxW0 > 0 || tol > 0) {
        const long long until = ctx->step + maxW0 + 2 * monitor_period(ctx);
        ctx->mon_until = ctx->mon_active ? std::max(ctx->mon_until, until) : until;
        if (!ctx->mon_active) ctx->mon_next = ctx->step + monitor_period(ctx);
        ctx->mon_active = tol > 0 || ctx->mon_active;
    }
    if (pred)
        HIPC(hipMemcpyAsync(pred, pr, sizeof(double) * 6 * ctx->np, hipMemcpyDeviceToHost, ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    return flags_status(ctx);
}

lb_status lb_warm_status(lb_ctx* ctx, int* status, long long* decided_step) {
    if (!ctx) return LB_EINVAL;
    const int nb = (int)ctx->boxes.size();
    std::vector<BoxMon> hm((size_t)nb);
    HIPC(hipMemcpyAsync(hm.data(), ctx->at<BoxMon>(ctx->L.mon), sizeof(BoxMon) * nb, hipMemcpyDeviceToHost,
                        ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    for (int b = 0; b < nb; ++b) {
        if (status) status[b] = hm[b].status;
        if (decided_step) decided_step[b] = hm[b].t_decided;
    }
    return LB_OK;
}

lb_status lb_surrogate_sample(lb_ctx* ctx, float* X, float* Y) {
    if (!ctx || !X || !Y) return LB_EINVAL;
    if (ctx->np == 0) return LB_OK;
    double* sc = ctx->at<double>(ctx->L.warm);
    float* xy = reinterpret_cast<float*>(sc + 7 * (size_t)ctx->L.max_particles);  // after the scales and predictions
    const PartDev* parts = ctx->at<PartDev>(ctx->L.parts);
    const double mu = ctx->kp.rho0 * viscosity(ctx);
    HIPC(launch_warm_features(ctx->at<BoxDesc>(ctx->L.boxes), parts, ctx->np, mu, xy, sc, ctx->stream));
    HIPC(launch_warm_targets(parts, ctx->np, sc, mu, xy + (size_t)MLP_IN * ctx->np, ctx->stream));
    HIPC(hipMemcpyAsync(X, xy, sizeof(float) * MLP_IN * ctx->np, hipMemcpyDeviceToHost, ctx->stream));
    HIPC(hipMemcpyAsync(Y, xy + (size_t)MLP_IN * ctx->np, sizeof(float) * MLP_OUT * ctx->np, hipMemcpyDeviceToHost,
                        ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    return flags_status(ctx);
}

lb_status lb_destroy(lb_ctx* ctx) {
    if (!ctx) return LB_EINVAL;
    hipStreamSynchronize(ctx->stream);
    if (ctx->nstream) {
        hipStreamSynchronize(ctx->nstream);
        hipStreamDestroy(ctx->nstream);
    }
    for (hipEvent_t e : {ctx->evK, ctx->evP, ctx->evStart})
        if (e) hipEventDestroy(e);
    graph_drop(ctx);
    delete ctx;
    return LB_OK;
}

const char* lb_status_str(lb_status s) {
    switch (s) {
        case LB_OK: return "ok";
        case LB_EINVAL: return "invalid argument";
        case LB_ENOMEM: return "capacity exhausted";
        case LB_EDEVICE: return "HIP runtime error";
        case LB_ESTATE: return "invalid state";
        case LB_EOVERLAP: return "particle overlap";
        case LB_ENONFINITE: return "non-finite or singular particle update";
        case LB_ERANGE: return "buffer too small";
        case LB_EIO: return "checkpoint I/O error";
        default: return "unknown status";
    }
}

const char* lb_last_error(lb_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

}  // extern "C"
