// lbdem_api.cpp -- host side of the C interface declared in include/lbdem.h.
//
// Validates arguments, lays the device buffers of a set out in one workspace, uploads
// the per-lattice tables, and queues the five step kernels, either one by one or as
// replays of a HIP graph built from kernel nodes.  No step arithmetic happens here: the
// host only prepares tables (waveform values, probe maps) and copies data in and out.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/lbdem.h"
#include "lbdem_internal.hpp"

using namespace lbdem;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) return fail(LBDEM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

size_t elem_size(int prec)
{
    switch (prec) {
    case PREC_FP64: return 8;
    case PREC_FP32: return 4;
    default: return 2;
    }
}

// Carves aligned sub-buffers out of a base pointer; with base == nullptr it only sizes.
struct Carver {
    char *base = nullptr;
    size_t off = 0;
    template <class T> T *take(size_t n)
    {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += n * sizeof(T);
        return p;
    }
};

struct Geometry {
    std::vector<MemberDev> mem;
    long long cells = 0;
    int tiles = 0;
    int tiles_max = 0;        // the fluid grid's largest size (probe partials are sized for it)
    int ptot = 0;
    int nprobe = 0;
    long long ring_doubles = 0;
    long long wave_doubles = 0;
    long long pz = 0;
    int nzt = 4;
    int listmode = 1;
    int compact = 0;
    int list_margin = 2;
    int fluid_off = 0;
    long long rt_words = 0;
    int ring_len = 1;
    int pv_ring = 0;
    int chg_cap = 0;
    int lcap = 1;
    int bcap = 1;
    int prec = PREC_FP32;
};

bool is_pow2_tile(int v) { return v == 8 || v == 16 || v == 32 || v == 64; }

int validate(int32_t n, const lbdem_params *lat, const lbdem_config *cfg)
{
    if (n < 1 || n > 4096 || !lat) return fail(LBDEM_EINVAL, "need 1..4096 lattices, got %d", n);
    if (cfg->precision < 0 || cfg->precision > 3) return fail(LBDEM_EINVAL, "unknown precision %d", cfg->precision);
    if (cfg->probe_ring < 1) return fail(LBDEM_EINVAL, "probe_ring must be >= 1");
    if (cfg->tile_x != 0 && !is_pow2_tile(cfg->tile_x)) return fail(LBDEM_EINVAL, "tile_x must be 0, 8, 16, 32 or 64");
    if (cfg->z_per_thread < 0 || cfg->z_per_thread > 16) return fail(LBDEM_EINVAL, "z_per_thread must be 0..16");
    if (cfg->graph_steps < 0 || cfg->graph_steps > 64) return fail(LBDEM_EINVAL, "graph_steps must be 0..64");
    if (cfg->node_lists < -1 || cfg->node_lists > 2) return fail(LBDEM_EINVAL, "node_lists must be -1, 0, 1 or 2");
    if (cfg->list_margin < 0 || cfg->list_margin > 8) return fail(LBDEM_EINVAL, "list_margin must be 0..8");
    if (cfg->fluid_off != 0 && cfg->fluid_off != 1) return fail(LBDEM_EINVAL, "fluid_off must be 0 or 1");
    if (cfg->particle_ring < 0 || cfg->particle_ring > (1 << 24))
        return fail(LBDEM_EINVAL, "particle_ring must be 0..2^24");
    for (int m = 0; m < n; ++m) {
        const lbdem_params &p = lat[m];
        if (cfg->node_lists == 2 && (long long)p.ny * ((p.nx + 31) / 32) > kMaxPlaneWords)
            return fail(LBDEM_EINVAL, "lattice %d: an x-y plane is too large for compact storage", m);
        if (p.nx < 1 || p.ny < 1 || p.nz < 1) return fail(LBDEM_EINVAL, "lattice %d: sizes must be >= 1", m);
        const long long nc = (long long)p.nx * p.ny * p.nz;
        if (nc * kQ >= (1LL << 31)) return fail(LBDEM_EINVAL, "lattice %d: more than 113M cells", m);
        const long long pop_bytes = nc * kQ * (cfg->precision == LBDEM_FP64 ? 8 : cfg->precision == LBDEM_FP32 ? 4 : 2);
        if (pop_bytes >= (1LL << 32))
            return fail(LBDEM_EINVAL, "lattice %d: its 19 population arrays must stay below 4 GiB", m);
        if (!(p.tau > 0.5)) return fail(LBDEM_EINVAL, "lattice %d: tau must exceed 1/2 (got %g)", m, p.tau);
        if (!(p.rho_f > 0.0)) return fail(LBDEM_EINVAL, "lattice %d: rho_f must be positive", m);
        for (int f = 0; f < 6; ++f)
            if (p.face_bc[f] < 0 || p.face_bc[f] > 2) return fail(LBDEM_EINVAL, "lattice %d: face %d kind", m, f);
        for (int a = 0; a < 3; ++a)
            if ((p.face_bc[2 * a] == LBDEM_PERIODIC) != (p.face_bc[2 * a + 1] == LBDEM_PERIODIC))
                return fail(LBDEM_EINVAL, "lattice %d: axis %d mixes periodic and non-periodic faces", m, a);
        for (int f = 0; f < 4; ++f)
            if (p.face_bc[f] == LBDEM_PRESSURE) return fail(LBDEM_EINVAL, "lattice %d: density faces must be z faces", m);
        if ((p.face_bc[4] == LBDEM_PRESSURE || p.face_bc[5] == LBDEM_PRESSURE) && p.nz < 2)
            return fail(LBDEM_EINVAL, "lattice %d: density faces need nz >= 2", m);
        if (p.wave < 0 || p.wave > 3) return fail(LBDEM_EINVAL, "lattice %d: wave kind", m);
        if (p.t_n < 0 || p.t_n > (1LL << 28)) return fail(LBDEM_EINVAL, "lattice %d: t_n out of range", m);
        if (p.n_probe < 0 || p.n_probe > LBDEM_MAX_PROBES) return fail(LBDEM_EINVAL, "lattice %d: n_probe", m);
        for (int k = 0; k < p.n_probe; ++k) {
            if (p.probe_z[k] < 0 || p.probe_z[k] >= p.nz) return fail(LBDEM_EINVAL, "lattice %d: probe %d outside", m, k);
            for (int k2 = 0; k2 < k; ++k2)
                if (p.probe_z[k2] == p.probe_z[k]) return fail(LBDEM_EINVAL, "lattice %d: duplicate probe plane", m);
        }
        if (p.tile_x != 0 && !is_pow2_tile(p.tile_x)) return fail(LBDEM_EINVAL, "lattice %d: tile_x must be 0, 8, 16, 32 or 64", m);
        if (p.rest_free != 0 && p.rest_free != 1) return fail(LBDEM_EINVAL, "lattice %d: rest_free must be 0 or 1", m);
        if (p.max_particles < 0 || p.max_particles > kMaxLocal) return fail(LBDEM_EINVAL, "lattice %d: max_particles", m);
        if (p.max_particles > 0 && !(p.max_radius > 0.0 && p.max_radius < 1024.0))
            return fail(LBDEM_EINVAL, "lattice %d: max_radius must be positive when particles are allowed", m);
        if (!(p.young_E >= 0.0) || !(p.poisson_nu > -1.0 && p.poisson_nu < 1.0) || !(p.friction_mu >= 0.0) ||
            !(p.rho_p > 0.0))
            return fail(LBDEM_EINVAL, "lattice %d: material constants out of range", m);
    }
    return LBDEM_OK;
}

int choose_tile_x(int nx, int req)
{
    if (req) return req;
    int best = 64;
    long long waste_best = -1;
    for (int bx : {64, 32, 16, 8}) {
        long long waste = (long long)((nx + bx - 1) / bx) * bx - nx;
        if (waste_best < 0 || waste < waste_best) { waste_best = waste; best = bx; }
    }
    return best;
}

void build_geometry(int32_t n, const lbdem_params *lat, const lbdem_config *cfg, Geometry &G)
{
    G.mem.assign(n, MemberDev{});
    G.prec = cfg->precision;
    // automatic: dense tiles when the particles can cover at most a quarter of the cells
    // (lists would skip little, and rebuilding the lists of a large, mostly fluid lattice
    // costs more than they save); else node lists with compact storage (the fastest
    // mapping measured at every precision), unless an x-y plane has too many row-table
    // words for it; then node lists for 16-bit storage, where partial-line writes cost
    // less than the idle lanes of dense tiles, and dense tiles with whole-line writes
    // otherwise
    int mode = cfg->node_lists;
    if (mode < 0) {
        bool fits = true;
        double solid = 0.0, cells = 0.0;
        for (int m = 0; m < n; ++m) {
            fits = fits && (long long)lat[m].ny * ((lat[m].nx + 31) / 32) <= kMaxPlaneWords;
            const double r = lat[m].max_radius;
            solid += (double)lat[m].max_particles * (4.0 / 3.0) * 3.14159265358979323846 * r * r * r;
            cells += (double)lat[m].nx * lat[m].ny * lat[m].nz;
        }
        if (solid <= 0.25 * cells) mode = 0;
        else mode = fits ? 2 : ((cfg->precision == LBDEM_FP16DEV || cfg->precision == LBDEM_BF16DEV) ? 1 : 0);
    }
    G.listmode = mode != 0 ? 1 : 0;
    G.compact = mode == 2 ? 1 : 0;
    G.list_margin = cfg->list_margin;
    G.fluid_off = cfg->fluid_off;
    int nzt = cfg->z_per_thread ? cfg->z_per_thread : 2;
    int nzmin = lat[0].nz;
    for (int m = 1; m < n; ++m) nzmin = std::min(nzmin, lat[m].nz);
    G.nzt = G.listmode ? 1 : std::max(1, std::min(nzt, nzmin));
    G.ring_len = cfg->probe_ring;
    G.pv_ring = cfg->particle_ring;
    long long cells = 0, ring = 0, wave = 0, pz = 0;
    int tiles = 0, pt = 0, npr = 0;
    for (int m = 0; m < n; ++m) {
        const lbdem_params &p = lat[m];
        MemberDev &M = G.mem[m];
        M.nx = p.nx; M.ny = p.ny; M.nz = p.nz;
        M.bx = choose_tile_x(p.nx, p.tile_x ? p.tile_x : cfg->tile_x);
        M.bx_log2 = (int)std::lround(std::log2((double)M.bx));
        M.by = 256 / M.bx;
        if (G.listmode) {
            // one workgroup per 256 listed nodes of a z plane (at most nx*ny of them)
            M.ntx = (int)(((long long)p.nx * p.ny + 255) / 256);
            M.nty = 1;
            M.ntz = p.nz;
        } else {
            M.ntx = (p.nx + M.bx - 1) / M.bx;
            M.nty = (p.ny + M.by - 1) / M.by;
            M.ntz = (p.nz + G.nzt - 1) / G.nzt;
        }
        M.tile_off = tiles;
        tiles += M.ntx * M.nty * M.ntz;
        for (int f = 0; f < 6; ++f) M.bc[f] = p.face_bc[f];
        const int dims[3] = {p.nx, p.ny, p.nz};
        M.narrow = 0;
        M.rest_free = p.rest_free ? 1 : 0;
        for (int a = 0; a < 3; ++a) {
            M.per[a] = p.face_bc[2 * a] == LBDEM_PERIODIC;
            M.box[a] = (double)dims[a];
            if (M.per[a] && dims[a] < 2.0 * p.max_radius + 4.0) M.narrow = 1;
        }
        M.ncell = (long long)p.nx * p.ny * p.nz;
        M.cell_off = cells;
        M.pop_off = cells * kQ;
        cells += M.ncell;
        M.omega = 1.0 / p.tau;
        M.rho_f = p.rho_f;
        M.wave_off = wave;
        M.t_n = p.t_n;
        wave += p.t_n + 2;
        M.pz_off = (int)pz;
        pz += p.nz;
        M.nw = (p.nx + 31) / 32;
        M.rt_off = G.rt_words;
        G.rt_words += (long long)p.nz * p.ny * M.nw;
        M.plist_off = npr;
        M.n_probe = p.n_probe;
        npr += p.n_probe;
        M.ring_off = ring;
        ring += (long long)G.ring_len * std::max(p.n_probe, 1) * 4;
        M.p_off = pt;
        M.p_cap = p.max_particles;
        M.np = 0;
        pt += p.max_particles;
        M.E = p.young_E; M.nu = p.poisson_nu; M.mu = p.friction_mu; M.rho_p = p.rho_p;
    }
    G.cells = cells;
    G.tiles = tiles;
    G.tiles_max = tiles;
    G.ptot = pt;
    G.nprobe = npr;
    G.ring_doubles = ring;
    G.wave_doubles = wave;
    G.pz = pz;
    G.chg_cap = (int)std::min<long long>(std::max<long long>(65536, 256LL * pt), 1LL << 26);
    // shell-list capacity: lattice nodes with -kShell < d - R <= sqrt(2) + kShell are within
    // the shell thickened by half a cell diagonal on both sides
    double rmax = 0.0;
    for (int m = 0; m < n; ++m)
        if (lat[m].max_particles > 0) rmax = std::max(rmax, lat[m].max_radius);
    if (rmax > 0.0) {
        const double ro = rmax + std::sqrt(2.0) + kShell + 0.8661, ri = std::max(0.0, rmax - kShell - 0.8661);
        G.lcap = (int)std::ceil(4.0 / 3.0 * M_PI * (ro * ro * ro - ri * ri * ri)) + 64;
        const double bo = rmax + kBandOut + 0.8661, bi = std::max(0.0, rmax - kBandIn - 0.8661);
        G.bcap = (int)std::ceil(4.0 / 3.0 * M_PI * (bo * bo * bo - bi * bi * bi)) + 64;
    }
}

// Lays out (or sizes, when base is null) every device buffer; fills the pointers of s.
size_t carve(const Geometry &G, char *base, DevSet &s)
{
    Carver c;
    c.base = base;
    const size_t es = elem_size(G.prec);
    const int P = std::max(G.ptot, 1);
    s.nmem = (int)G.mem.size();
    s.mem = c.take<MemberDev>(G.mem.size());
    s.tiles_total = G.tiles;
    s.nzt = G.nzt;
    s.listmode = G.listmode;
    s.compact = G.compact;
    s.list_margin = (double)G.list_margin;
    s.fluid_off = G.fluid_off;
    s.narrow = 0;
    for (const MemberDev &M : G.mem) s.narrow |= M.narrow;
    s.es = (int)es;
    s.rt = c.take<uint2>((size_t)std::max<long long>(G.compact ? G.rt_words : 1, 1));
    s.popC = c.take<char>(G.compact ? es * kQ * (size_t)G.cells : 1);
    s.nplanes = (int)G.pz;
    s.clist = c.take<int>((size_t)G.cells);
    s.ccnt = c.take<int>((size_t)std::max<long long>(G.pz, 1));
    s.relist_at = c.take<long long>(1);
    s.skin = c.take<double>(G.mem.size());
    s.pend = c.take<int>((size_t)G.cells);
    s.pbuf[0] = c.take<double>(4 * (size_t)kPendCap);
    s.pbuf[1] = c.take<double>(4 * (size_t)kPendCap);
    s.pcnt = c.take<int>(2);
    s.popA = c.take<char>(es * kQ * (size_t)G.cells);
    s.popB = c.take<char>(es * kQ * (size_t)G.cells);
    s.own[0] = c.take<int>(G.cells);
    s.own[1] = c.take<int>(G.cells);
    s.lw = c.take<unsigned long long>(2 * (size_t)G.cells);
    s.lwc = c.take<unsigned long long>((size_t)G.cells);
    s.lwc_bad = c.take<long long>(1);
    s.ncell_total = G.cells;
    s.frec = c.take<char>(4 * (size_t)G.cells * (G.prec == PREC_FP64 ? 32 : 16));
    s.rec_step = c.take<long long>(1);
    s.chg_cap = G.chg_cap;
    s.chg[0] = c.take<int>(2 * (size_t)G.chg_cap);
    s.chg[1] = c.take<int>(2 * (size_t)G.chg_cap);
    s.chgcnt = c.take<int>(2);
    s.pprt = c.take<double>((size_t)G.tiles_max * G.nzt * 4);
    s.ring = c.take<double>(G.ring_doubles);
    s.ring_len = G.ring_len;
    s.pzmap = c.take<short>(G.pz);
    s.plist = c.take<int>(std::max(G.nprobe, 1));
    s.nprobe_total = G.nprobe;
    s.wave = c.take<double>(G.wave_doubles);
    s.ptot = G.ptot;
    for (int k = 0; k < 2; ++k) {
        s.X[k] = c.take<double>(3 * (size_t)P);
        s.V[k] = c.take<double>(3 * (size_t)P);
        s.W[k] = c.take<double>(3 * (size_t)P);
    }
    s.R = c.take<double>(P);
    s.m = c.take<double>(P);
    s.I = c.take<double>(P);
    s.Fg = c.take<double>(3 * (size_t)P);
    s.Fh = c.take<double>(3 * (size_t)P);
    s.Th = c.take<double>(3 * (size_t)P);
    s.Ph = c.take<double>(3 * (size_t)P);
    s.Lh = c.take<double>(3 * (size_t)P);
    s.Xref = c.take<double>(3 * (size_t)P);
    s.Xl = c.take<double>(3 * (size_t)P);
    s.pspd = c.take<double>((size_t)P);
    s.pf[0] = c.take<float>(12 * (size_t)P);
    s.pf[1] = c.take<float>(12 * (size_t)P);
    s.margin = c.take<double>(P);
    s.fixed = c.take<int>(P);
    s.pmem = c.take<int>(P);
    s.ppart = c.take<double>((size_t)P * kChunks * kLinkComp);
    s.pv_ring = G.pv_ring;
    s.pvring = c.take<double>(G.pv_ring > 0 ? (size_t)G.pv_ring * P * 3 : 1);
    s.zcache = c.take<double>((size_t)P * kChunks * kZComp);
    s.nearl = c.take<int>((size_t)P * kNearCap);
    s.nnear = c.take<int>(P);
    s.near_at = c.take<long long>(P);
    s.lcap = G.lcap;
    s.lcell = c.take<int>((size_t)P * G.lcap);
    s.ldr = c.take<float>((size_t)P * G.lcap);
    s.lmask = c.take<unsigned>((size_t)P * G.lcap);
    s.lcnt = c.take<int>(P);
    s.xcell = c.take<int>((size_t)P * G.lcap);
    s.xslot = c.take<int>((size_t)P * G.lcap);
    s.xgrp = c.take<unsigned>((size_t)P * G.lcap);
    s.xcnt = c.take<int>((size_t)P * kChunks);
    s.lreb = c.take<long long>(P);
    s.ldirty = c.take<long long>((size_t)P * kChunks);
    s.lzr = c.take<int>(2 * (size_t)P);
    s.lchunk = c.take<int>((size_t)P * (kChunks + 1));
    s.rdisp = c.take<double>((size_t)P);
    s.rlens = c.take<double>((size_t)P);
    s.bcap = G.bcap;
    s.bcell = c.take<int>((size_t)P * G.bcap);
    s.bdr = c.take<float>((size_t)P * G.bcap);
    s.bcnt = c.take<int>(P);
    for (int k = 0; k < 2; ++k) {
        s.hj[k] = c.take<int>((size_t)P * kHistCap);
        s.hf[k] = c.take<double>((size_t)P * kHistCap * 3);
        s.hn[k] = c.take<int>(P);
    }
    s.tstep = c.take<long long>(1);
    s.tcopy = c.take<long long>(1);
    s.flags = c.take<unsigned int>(1);
    return (c.off + 255) & ~size_t(255);
}

uint16_t f32_to_bf16_host(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
float bf16_to_f32_host(uint16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float x;
    std::memcpy(&x, &u, 4);
    return x;
}

const double kWh[kQ] = {1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 36, 1.0 / 36,
                        1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                        1.0 / 36, 1.0 / 36, 1.0 / 3};
const float kInvWh[kQ] = {18, 18, 18, 18, 18, 18, 36, 36, 36, 36, 36, 36, 36, 36, 36, 36, 36, 36, 3};

constexpr int kKernels = 5; // links, motion, fluid, re-projection, refresh

} // namespace

struct lbdem_set {
    Geometry G;
    DevSet ds{};
    std::vector<lbdem_params> params;
    lbdem_config cfg{};
    hipStream_t stream = nullptr;
    void *ws = nullptr;
    size_t ws_bytes = 0;      // bytes of the workspace the set uses
    bool owns_ws = false;
    int64_t t_host = 0;
    // compact storage: populations currently held at their nodes (after creation or an
    // expansion, until the next step's list rebuild compacts them again)
    bool node_layout = true;
    // graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int graph_steps = 0;
    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, int>> ev_pending[kKernels];
    double ms_acc[kKernels] = {0, 0, 0, 0, 0};
    int64_t ms_cnt[kKernels] = {0, 0, 0, 0, 0};
    size_t ev_next = 0;
};

namespace {

int sync_set(lbdem_set *S)
{
    HIPCHK(hipStreamSynchronize(S->stream));
    return LBDEM_OK;
}

// Compact storage: moves the populations of every lattice back to their nodes (the row
// tables become the identity) and has the next step rebuild the lists, which compacts
// them again.  Host access to populations and particle set-up work on the node layout.
int node_layout(lbdem_set *S)
{
    if (!S->G.compact || S->node_layout) return LBDEM_OK;
    int rc = sync_set(S);
    if (rc) return rc;
    HIPCHK(launch_expand(S->G.prec, S->ds, S->stream));
    HIPCHK(hipMemcpyAsync(S->ds.relist_at, S->ds.tstep, sizeof(long long), hipMemcpyDeviceToDevice, S->stream));
    S->node_layout = true;
    return sync_set(S);
}

int upload_member(lbdem_set *S, int m)
{
    HIPCHK(hipMemcpyAsync((void *)(S->ds.mem + m), &S->G.mem[m], sizeof(MemberDev), hipMemcpyHostToDevice, S->stream));
    return LBDEM_OK;
}

int build_graph(lbdem_set *S, int steps);

// Node lists: workgroups per plane of a lattice from the listed nodes its particles leave.
// A plane's cross-sections of the spheres shrunk by the widest list skin and half a node
// bound its solid non-listed area from below (overlaps aside), so nx*ny minus that area
// bounds its listed nodes from above.  The fluid kernel gives a plane with more listed
// nodes than its workgroups hold further chunks per workgroup, so the estimate sets the
// speed, and the result only through the grouping of the probes' partial sums.
int retile_lists(lbdem_set *S, int lattice, int n, const double *X, const double *Rv)
{
    if (!S->G.listmode) return LBDEM_OK;
    MemberDev &M = S->G.mem[lattice];
    const long long nxy = (long long)M.nx * M.ny;
    std::vector<double> solid((size_t)M.nz, 0.0);
    for (int q = 0; q < n; ++q) {
        const double r = Rv[q] - kListSkin - 0.5, zc = X[3 * q + 2];
        if (r <= 0.0) continue;
        for (int z = (int)std::ceil(zc - r); z <= (int)std::floor(zc + r); ++z) {
            int zz = z;
            if (M.per[2]) zz = ((z % M.nz) + M.nz) % M.nz;
            else if (z < 0 || z >= M.nz) continue;
            const double h = (double)z - zc;
            solid[(size_t)zz] += M_PI * std::max(r * r - h * h, 0.0);
        }
    }
    // workgroups per plane: midway between the mean and the largest estimated count of a
    // plane's listed nodes (a larger plane gives its workgroups further chunks; sizing for
    // the largest left two thirds of the FCC case's workgroups empty, and measured slower)
    double worst = 0.0, mean = 0.0;
    for (int z = 0; z < M.nz; ++z) {
        worst = std::max(worst, (double)nxy - solid[(size_t)z]);
        mean += (double)nxy - solid[(size_t)z];
    }
    mean /= (double)M.nz;
    const int full = (int)((nxy + 255) / 256);
    const int ntx = std::min(std::max((int)std::ceil(0.5 * (mean + worst) / 256.0) + 1, 1), full);
    if (ntx == M.ntx) return LBDEM_OK;
    M.ntx = ntx;
    int tiles = 0;
    for (MemberDev &Mm : S->G.mem) {
        Mm.tile_off = tiles;
        tiles += Mm.ntx * Mm.nty * Mm.ntz;
    }
    S->G.tiles = tiles;
    S->ds.tiles_total = tiles;
    HIPCHK(hipMemcpyAsync((void *)S->ds.mem, S->G.mem.data(), sizeof(MemberDev) * S->G.mem.size(),
                          hipMemcpyHostToDevice, S->stream));
    HIPCHK(hipStreamSynchronize(S->stream));
    if (S->gexec) return build_graph(S, S->graph_steps);
    return LBDEM_OK;
}

int destroy_graph(lbdem_set *S)
{
    if (S->gexec) { (void)hipGraphExecDestroy(S->gexec); S->gexec = nullptr; }
    if (S->graph) { (void)hipGraphDestroy(S->graph); S->graph = nullptr; }
    return LBDEM_OK;
}

int build_graph(lbdem_set *S, int steps)
{
    destroy_graph(S);
    HIPCHK(hipGraphCreate(&S->graph, 0));
    static int mode0 = 0, only_all = -1;
    void *fluid_args[] = {(void *)&S->ds};
    void *part_args[] = {(void *)&S->ds, (void *)&mode0, (void *)&only_all};
    hipGraphNode_t prev = nullptr;
    for (int k = 0; k < steps; ++k) {
        hipKernelNodeParams kp{};
        hipGraphNode_t n0, n1, n2, n3, n4;
        kp.blockDim = dim3(256);
        kp.sharedMemBytes = 0;
        kp.extra = nullptr;
        // refresh -> link records -> link pass -> motion -> fluid -> re-projection
        kp.func = refresh_kernel_ptr(S->G.prec);
        kp.gridDim = dim3(refresh_grid(S->ds));
        kp.kernelParams = fluid_args;
        HIPCHK(hipGraphAddKernelNode(&n4, S->graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp));
        if (S->G.fluid_off) {
            // hydrodynamics switched off: no link pass and no fluid step
            n0 = n4;
        } else {
            hipGraphNode_t nr;
            kp.func = records_kernel_ptr(S->G.prec, S->G.compact, S->ds.narrow);
            kp.gridDim = dim3(records_grid(S->ds));
            kp.kernelParams = fluid_args;
            HIPCHK(hipGraphAddKernelNode(&nr, S->graph, &n4, 1, &kp));
            kp.func = links_kernel_ptr(S->G.prec, S->ds.narrow);
            kp.gridDim = dim3(links_grid(S->ds));
            kp.blockDim = dim3(links_block());
            kp.kernelParams = part_args;
            HIPCHK(hipGraphAddKernelNode(&n0, S->graph, &nr, 1, &kp));
        }
        kp.blockDim = dim3(256);
        kp.kernelParams = part_args;
        kp.func = motion_kernel_ptr();
        kp.gridDim = dim3(motion_grid(S->ds));
        HIPCHK(hipGraphAddKernelNode(&n1, S->graph, &n0, 1, &kp));
        if (S->G.fluid_off) {
            n2 = n1;
        } else {
            kp.func = fluid_kernel_ptr(S->G.prec, S->G.compact, S->ds.narrow);
            kp.gridDim = dim3(S->ds.tiles_total);
            kp.kernelParams = fluid_args;
            HIPCHK(hipGraphAddKernelNode(&n2, S->graph, &n1, 1, &kp));
        }
        kp.func = remap_kernel_ptr_prec(S->G.prec);
        kp.gridDim = dim3(remap_grid(S->ds));
        kp.kernelParams = part_args;
        HIPCHK(hipGraphAddKernelNode(&n3, S->graph, &n2, 1, &kp));
        prev = n3;
    }
    HIPCHK(hipGraphInstantiate(&S->gexec, S->graph, nullptr, nullptr, 0));
    S->graph_steps = steps;
    return LBDEM_OK;
}

int harvest_events(lbdem_set *S)
{
    for (int k = 0; k < kKernels; ++k) {
        for (auto &pr : S->ev_pending[k]) {
            float ms = 0.0f;
            HIPCHK(hipEventSynchronize(S->ev_pool[pr.second]));
            HIPCHK(hipEventElapsedTime(&ms, S->ev_pool[pr.first], S->ev_pool[pr.second]));
            S->ms_acc[k] += ms;
            S->ms_cnt[k] += 1;
        }
        S->ev_pending[k].clear();
    }
    S->ev_next = 0;
    return LBDEM_OK;
}

int launch_step_eager(lbdem_set *S)
{
    // launch order refresh, links, motion, fluid, re-projection; timing slots keep the
    // order links, motion, fluid, re-projection, refresh of lbdem_timing_read
    static const int order[kKernels] = {4, 0, 1, 2, 3};
    for (int o = 0; o < kKernels; ++o) {
        const int k = order[o];
        if (S->G.fluid_off && (k == 0 || k == 2)) continue;  // no link forces, no fluid step
        int e0 = -1, e1 = -1;
        if (S->timing) {
            if (S->ev_next + 2 > S->ev_pool.size()) {
                int rc = harvest_events(S);
                if (rc) return rc;
            }
            e0 = (int)S->ev_next++;
            e1 = (int)S->ev_next++;
            HIPCHK(hipEventRecord(S->ev_pool[e0], S->stream));
        }
        hipError_t err;
        if (k == 4) err = launch_refresh(S->G.prec, S->ds, S->stream);
        else if (k == 0) {
            // the link records and the link pass share the links timing slot
            err = launch_records(S->G.prec, S->ds, S->stream);
            if (err == hipSuccess) err = launch_links(S->G.prec, S->ds, S->stream);
        }
        else if (k == 1) err = launch_motion(S->ds, 0, -1, S->stream);
        else if (k == 2) err = launch_fluid(S->G.prec, S->ds, S->stream);
        else err = launch_remap_prec(S->G.prec, S->ds, 0, -1, S->stream);
        if (err != hipSuccess) return fail(LBDEM_EDEVICE, "kernel launch %d: %s", k, hipGetErrorString(err));
        if (S->timing) {
            HIPCHK(hipEventRecord(S->ev_pool[e1], S->stream));
            S->ev_pending[k].push_back({e0, e1});
        }
    }
    return LBDEM_OK;
}

int check_lattice(lbdem_set *S, int32_t lattice)
{
    if (!S) return fail(LBDEM_EINVAL, "null set");
    if (lattice < 0 || lattice >= (int)S->G.mem.size()) return fail(LBDEM_EINVAL, "lattice index %d out of range", lattice);
    return LBDEM_OK;
}

} // namespace

extern "C" {

const char *lbdem_last_error(void) { return g_err.c_str(); }

int lbdem_default_config(lbdem_config *cfg)
{
    if (!cfg) return fail(LBDEM_EINVAL, "null config");
    cfg->precision = LBDEM_FP32;
    cfg->probe_ring = 4096;
    cfg->tile_x = 0;
    cfg->node_lists = -1;
    cfg->list_margin = 2;
    cfg->fluid_off = 0;
    cfg->z_per_thread = 0;
    cfg->graph_steps = 8;
    cfg->particle_ring = 0;
    return LBDEM_OK;
}

int lbdem_workspace_size(int32_t n_lat, const lbdem_params *lat, const lbdem_config *cfg, size_t *bytes)
{
    lbdem_config c;
    if (cfg) c = *cfg; else lbdem_default_config(&c);
    if (!bytes) return fail(LBDEM_EINVAL, "null output");
    int rc = validate(n_lat, lat, &c);
    if (rc) return rc;
    Geometry G;
    build_geometry(n_lat, lat, &c, G);
    DevSet s{};
    *bytes = carve(G, nullptr, s);
    return LBDEM_OK;
}

int lbdem_create(int32_t n_lat, const lbdem_params *lat, const lbdem_config *cfg, void *device_workspace,
                 size_t workspace_bytes, void *hip_stream, lbdem_set **out)
{
    if (!out) return fail(LBDEM_EINVAL, "null output");
    *out = nullptr;
    lbdem_config c;
    if (cfg) c = *cfg; else lbdem_default_config(&c);
    int rc = validate(n_lat, lat, &c);
    if (rc) return rc;
    lbdem_set *S = new (std::nothrow) lbdem_set();
    if (!S) return fail(LBDEM_ENOMEM, "host allocation failed");
    S->cfg = c;
    S->params.assign(lat, lat + n_lat);
    S->stream = (hipStream_t)hip_stream;
    build_geometry(n_lat, lat, &c, S->G);
    DevSet probe{};
    const size_t need = carve(S->G, nullptr, probe);
    if (device_workspace) {
        if (workspace_bytes < need) {
            delete S;
            return fail(LBDEM_ENOMEM, "workspace of %zu bytes, %zu needed", workspace_bytes, need);
        }
        if (((uintptr_t)device_workspace & 255u) != 0) {
            delete S;
            return fail(LBDEM_EINVAL, "workspace must be 256-byte aligned");
        }
        S->ws = device_workspace;
    } else {
        hipError_t e = hipMalloc(&S->ws, need);
        if (e != hipSuccess) {
            delete S;
            return fail(LBDEM_ENOMEM, "hipMalloc(%zu): %s", need, hipGetErrorString(e));
        }
        S->owns_ws = true;
    }
    carve(S->G, (char *)S->ws, S->ds);
    S->ws_bytes = need;
    DevSet &s = S->ds;
    hipStream_t st = S->stream;
    auto cleanup = [&](int code) {
        lbdem_destroy(S);
        return code;
    };
#define CHK(expr)                                                                            \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return cleanup(fail(LBDEM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_))); \
    } while (0)
    // tables
    CHK(hipMemcpyAsync((void *)s.mem, S->G.mem.data(), sizeof(MemberDev) * n_lat, hipMemcpyHostToDevice, st));
    std::vector<short> pz(S->G.pz, (short)-1);
    std::vector<int> plist(std::max(S->G.nprobe, 1), 0);
    std::vector<double> wave(S->G.wave_doubles);
    std::vector<int> pmem(std::max(S->G.ptot, 1), 0);
    for (int m = 0; m < n_lat; ++m) {
        const lbdem_params &p = lat[m];
        const MemberDev &M = S->G.mem[m];
        for (int k = 0; k < p.n_probe; ++k) {
            pz[M.pz_off + p.probe_z[k]] = (short)k;
            plist[M.plist_off + k] = p.probe_z[k];
        }
        // waveform values rho(t) of Eq. (source) / Table (tab:source) for t = 0..t_n,
        // then rho_f for every later time level
        for (long long tt = 0; tt <= p.t_n; ++tt) {
            double v = p.rho_f;
            if (p.wave != LBDEM_WAVE_NONE) {
                const double wt = p.omega * (double)tt;
                if (p.wave == LBDEM_WAVE_SINE) v = p.rho_f + p.rho_amp * sin(wt);
                else if (p.wave == LBDEM_WAVE_COSINE) v = p.rho_f + p.rho_amp * (1.0 - cos(wt));
                else v = p.rho_f + p.rho_amp;
            }
            wave[M.wave_off + tt] = v;
        }
        wave[M.wave_off + p.t_n + 1] = p.rho_f;
        for (int q = 0; q < M.p_cap; ++q) pmem[M.p_off + q] = m;
    }
    CHK(hipMemcpyAsync((void *)s.pzmap, pz.data(), sizeof(short) * pz.size(), hipMemcpyHostToDevice, st));
    CHK(hipMemcpyAsync((void *)s.plist, plist.data(), sizeof(int) * plist.size(), hipMemcpyHostToDevice, st));
    CHK(hipMemcpyAsync((void *)s.wave, wave.data(), sizeof(double) * wave.size(), hipMemcpyHostToDevice, st));
    CHK(hipMemcpyAsync(s.pmem, pmem.data(), sizeof(int) * pmem.size(), hipMemcpyHostToDevice, st));
    if (S->G.compact) {
        // before the first list build every node is listed: slot = cell
        std::vector<uint2> rt((size_t)S->G.rt_words);
        for (int m = 0; m < n_lat; ++m) {
            const MemberDev &M = S->G.mem[m];
            for (int k = 0; k < M.nz; ++k)
                for (int j = 0; j < M.ny; ++j)
                    for (int w = 0; w < M.nw; ++w) {
                        const int lo = 32 * w, n_in = std::min(32, M.nx - lo);
                        const unsigned bits = n_in == 32 ? 0xffffffffu : ((1u << n_in) - 1u);
                        rt[(size_t)(M.rt_off + ((long long)k * M.ny + j) * M.nw + w)] =
                            make_uint2(bits, (unsigned)(j * M.nx + lo));
                    }
        }
        CHK(hipMemcpyAsync(s.rt, rt.data(), sizeof(uint2) * rt.size(), hipMemcpyHostToDevice, st));
        CHK(hipStreamSynchronize(st)); // rt is a local vector
    }
    // state
    const int P = std::max(S->G.ptot, 1);
    CHK(hipMemsetAsync(s.own[0], 0xff, sizeof(int) * S->G.cells, st));
    CHK(hipMemsetAsync(s.own[1], 0xff, sizeof(int) * S->G.cells, st));
    CHK(hipMemsetAsync(s.lw, 0, sizeof(unsigned long long) * 2 * S->G.cells, st));
    CHK(hipMemsetAsync(s.lwc_bad, 0x80, sizeof(long long), st)); // (the first step rebuilds the lists)
    CHK(hipMemsetAsync(s.relist_at, 0, sizeof(long long), st)); // lists are built by the first step
    {
        std::vector<double> sk(S->G.mem.size(), kListSkin);
        CHK(hipMemcpyAsync(s.skin, sk.data(), sizeof(double) * sk.size(), hipMemcpyHostToDevice, st));
        CHK(hipStreamSynchronize(st)); // sk is a local vector
    }
    CHK(hipMemsetAsync(s.pend, 0xff, sizeof(int) * S->G.cells, st));
    CHK(hipMemsetAsync(s.pcnt, 0, sizeof(int) * 2, st));
    // -1: no list yet, so the first rebuild lays out every plane
    CHK(hipMemsetAsync(s.ccnt, 0xff, sizeof(int) * std::max<long long>(S->G.pz, 1), st));
    CHK(hipMemsetAsync(s.chgcnt, 0, sizeof(int) * 2, st));
    CHK(hipMemsetAsync(s.pprt, 0, sizeof(double) * S->G.tiles_max * S->G.nzt * 4, st));
    CHK(hipMemsetAsync(s.ring, 0, sizeof(double) * S->G.ring_doubles, st));
    for (int k = 0; k < 2; ++k) {
        CHK(hipMemsetAsync(s.X[k], 0, sizeof(double) * 3 * P, st));
        CHK(hipMemsetAsync(s.V[k], 0, sizeof(double) * 3 * P, st));
        CHK(hipMemsetAsync(s.W[k], 0, sizeof(double) * 3 * P, st));
        CHK(hipMemsetAsync(s.hn[k], 0, sizeof(int) * P, st));
    }
    double *zero3[] = {s.Fg, s.Fh, s.Th, s.Ph, s.Lh, s.Xref};
    for (double *z : zero3) CHK(hipMemsetAsync(z, 0, sizeof(double) * 3 * P, st));
    CHK(hipMemsetAsync(s.margin, 0, sizeof(double) * P, st));
    CHK(hipMemsetAsync(s.pspd, 0, sizeof(double) * P, st));
    CHK(hipMemsetAsync(s.rdisp, 0, sizeof(double) * P, st));
    CHK(hipMemsetAsync(s.rlens, 0, sizeof(double) * P, st));
    CHK(hipMemsetAsync(s.pf[0], 0, sizeof(float) * 12 * P, st));
    CHK(hipMemsetAsync(s.pf[1], 0, sizeof(float) * 12 * P, st));
    CHK(hipMemsetAsync(s.nnear, 0, sizeof(int) * P, st));
    CHK(hipMemsetAsync(s.near_at, 0xff, sizeof(long long) * P, st)); // -1: build at the first step
    CHK(hipMemsetAsync(s.lcnt, 0, sizeof(int) * P, st));
    CHK(hipMemsetAsync(s.xcnt, 0, sizeof(int) * P * kChunks, st));
    CHK(hipMemsetAsync(s.bcnt, 0, sizeof(int) * P, st));
    CHK(hipMemsetAsync(s.lreb, 0xff, sizeof(long long) * P, st));
    CHK(hipMemsetAsync(s.ldirty, 0xff, sizeof(long long) * P * kChunks, st));
    CHK(hipMemsetAsync(s.lzr, 0, sizeof(int) * 2 * P, st));
    CHK(hipMemsetAsync(s.lchunk, 0, sizeof(int) * P * (kChunks + 1), st));
    CHK(hipMemsetAsync(s.tstep, 0, sizeof(long long), st));
    CHK(hipMemsetAsync(s.rec_step, 0x80, sizeof(long long), st)); // no link records yet
    CHK(hipMemsetAsync(s.tcopy, 0, sizeof(long long), st));
    CHK(hipMemsetAsync(s.flags, 0, sizeof(unsigned), st));
    CHK(launch_init_pops(S->G.prec, s, S->G.cells, st));
    CHK(hipStreamSynchronize(st));
#undef CHK
    if (c.graph_steps > 0) {
        rc = build_graph(S, c.graph_steps);
        if (rc) return cleanup(rc);
    }
    S->ev_pool.resize(6 * 1024);
    for (auto &e : S->ev_pool) {
        hipError_t er = hipEventCreate(&e);
        if (er != hipSuccess) return cleanup(fail(LBDEM_EDEVICE, "hipEventCreate: %s", hipGetErrorString(er)));
    }
    *out = S;
    return LBDEM_OK;
}

int lbdem_destroy(lbdem_set *S)
{
    if (!S) return LBDEM_OK;
    (void)hipStreamSynchronize(S->stream);
    destroy_graph(S);
    for (auto &e : S->ev_pool)
        if (e) (void)hipEventDestroy(e);
    if (S->owns_ws && S->ws) (void)hipFree(S->ws);
    delete S;
    return LBDEM_OK;
}

int lbdem_set_stream(lbdem_set *S, void *hip_stream)
{
    if (!S) return fail(LBDEM_EINVAL, "null set");
    HIPCHK(hipStreamSynchronize(S->stream));
    S->stream = (hipStream_t)hip_stream;
    return LBDEM_OK;
}

int lbdem_particles_set(lbdem_set *S, int32_t lattice, int32_t n, const double *x, const double *v, const double *w,
                        const double *radius, const double *fg, const uint8_t *fixed)
{
    int rc = check_lattice(S, lattice);
    if (rc) return rc;
    MemberDev &M = S->G.mem[lattice];
    if (n < 0 || n > M.p_cap) return fail(LBDEM_EINVAL, "lattice %d holds at most %d particles, got %d", lattice, M.p_cap, n);
    if (n > 0 && (!x || !radius)) return fail(LBDEM_EINVAL, "positions and radii are required");
    const int dims[3] = {M.nx, M.ny, M.nz};
    std::vector<double> X(3 * (size_t)n), Vv(3 * (size_t)n, 0.0), Wv(3 * (size_t)n, 0.0), F(3 * (size_t)n, 0.0);
    std::vector<double> Rv(n), mv(n), Iv(n);
    std::vector<int> fx(n, 0);
    for (int q = 0; q < n; ++q) {
        const double R = radius[q];
        if (!(R > 0.0) || !std::isfinite(R)) return fail(LBDEM_EINVAL, "particle %d: radius must be positive", q);
        if (R > S->params[lattice].max_radius)
            return fail(LBDEM_EINVAL, "particle %d: radius %g exceeds max_radius %g", q, R, S->params[lattice].max_radius);
        for (int a = 0; a < 3; ++a) {
            double c = x[3 * q + a];
            if (!std::isfinite(c)) return fail(LBDEM_EINVAL, "particle %d: non-finite position", q);
            if (M.per[a]) {
                // a node lies inside at most one image of a sphere, and the midpoint of a
                // link into an image (at most R + 1/2 from its centre along an axis) lies
                // less than half a period from that image's centre, which identifies it
                if (!(dims[a] > 2.0 * R + 1.5))
                    return fail(LBDEM_EINVAL, "particle %d: periodic axis %d not longer than 2R + 1.5", q, a);
                c = std::fmod(c, (double)dims[a]);
                if (c < 0.0) c += dims[a];
            } else if (c < 0.0 || c > dims[a] - 1) {
                return fail(LBDEM_EINVAL, "particle %d: centre outside the non-periodic extent of axis %d", q, a);
            }
            X[3 * q + a] = c;
            if (fg) F[3 * q + a] = fg[3 * q + a];
        }
        fx[q] = fixed ? (fixed[q] != 0) : 0;
        if (!fx[q]) {
            for (int a = 0; a < 3; ++a) {
                if (v) Vv[3 * q + a] = v[3 * q + a];
                if (w) Wv[3 * q + a] = w[3 * q + a];
            }
        }
        Rv[q] = R;
        mv[q] = M.rho_p * (4.0 / 3.0) * M_PI * R * R * R;
        Iv[q] = 0.4 * mv[q] * R * R;
    }
    rc = node_layout(S);
    if (rc) return rc;
    rc = sync_set(S);
    if (rc) return rc;
    long long t = 0;
    HIPCHK(hipMemcpy(&t, S->ds.tstep, sizeof(long long), hipMemcpyDeviceToHost));
    const int par = (int)(t & 1);
    M.pv_from = t;
    DevSet &s = S->ds;
    hipStream_t st = S->stream;
    const size_t o3 = 3 * (size_t)M.p_off, o1 = M.p_off;
    if (n > 0) {
        HIPCHK(hipMemcpyAsync(s.X[par] + o3, X.data(), 8 * 3 * n, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(s.V[par] + o3, Vv.data(), 8 * 3 * n, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(s.W[par] + o3, Wv.data(), 8 * 3 * n, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(s.Xref + o3, X.data(), 8 * 3 * n, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(s.Fg + o3, F.data(), 8 * 3 * n, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(s.R + o1, Rv.data(), 8 * n, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(s.m + o1, mv.data(), 8 * n, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(s.I + o1, Iv.data(), 8 * n, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(s.fixed + o1, fx.data(), 4 * n, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemsetAsync(s.Fh + o3, 0, 8 * 3 * n, st));
        HIPCHK(hipMemsetAsync(s.Th + o3, 0, 8 * 3 * n, st));
        HIPCHK(hipMemsetAsync(s.Ph + o3, 0, 8 * 3 * n, st));
        HIPCHK(hipMemsetAsync(s.Lh + o3, 0, 8 * 3 * n, st));
        HIPCHK(hipMemsetAsync(s.hn[0] + o1, 0, 4 * n, st));
        HIPCHK(hipMemsetAsync(s.hn[1] + o1, 0, 4 * n, st));
    }
    // fresh projection: clear both node maps of this lattice, then classify
    HIPCHK(hipMemsetAsync(s.own[0] + M.cell_off, 0xff, sizeof(int) * M.ncell, st));
    HIPCHK(hipMemsetAsync(s.own[1] + M.cell_off, 0xff, sizeof(int) * M.ncell, st));
    M.np = n;
    rc = upload_member(S, lattice);
    if (rc) return rc;
    rc = retile_lists(S, lattice, n, X.data(), Rv.data());
    if (rc) return rc;
    hipError_t e = launch_motion(s, 1, lattice, st);
    if (e != hipSuccess) return fail(LBDEM_EDEVICE, "near-list kernel: %s", hipGetErrorString(e));
    e = launch_remap_prec(S->G.prec, s, 1, lattice, st);
    if (e != hipSuccess) return fail(LBDEM_EDEVICE, "projection kernel: %s", hipGetErrorString(e));
    // both node maps of this lattice now agree; a pending change list may still name its
    // old cells, so the next fluid pass copies the current maps whole instead of applying it
    int cnt[2];
    HIPCHK(hipMemcpyAsync(cnt, s.chgcnt, sizeof(cnt), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    cnt[par ^ 1] = s.chg_cap + 1;
    HIPCHK(hipMemcpyAsync(s.chgcnt, cnt, sizeof(cnt), hipMemcpyHostToDevice, st));
    return sync_set(S);
}

int lbdem_particles_get(lbdem_set *S, int32_t lattice, int32_t n, double *x, double *v, double *w, double *force,
                        double *torque)
{
    int rc = check_lattice(S, lattice);
    if (rc) return rc;
    const MemberDev &M = S->G.mem[lattice];
    if (n != M.np) return fail(LBDEM_EINVAL, "lattice %d has %d particles, asked for %d", lattice, M.np, n);
    rc = sync_set(S);
    if (rc) return rc;
    if (n == 0) return LBDEM_OK;
    long long t = 0;
    HIPCHK(hipMemcpy(&t, S->ds.tstep, sizeof(long long), hipMemcpyDeviceToHost));
    const int par = (int)(t & 1);
    const size_t o3 = 3 * (size_t)M.p_off, b = 8 * 3 * (size_t)n;
    if (x) HIPCHK(hipMemcpy(x, S->ds.X[par] + o3, b, hipMemcpyDeviceToHost));
    if (v) HIPCHK(hipMemcpy(v, S->ds.V[par] + o3, b, hipMemcpyDeviceToHost));
    if (w) HIPCHK(hipMemcpy(w, S->ds.W[par] + o3, b, hipMemcpyDeviceToHost));
    if (force) HIPCHK(hipMemcpy(force, S->ds.Fh + o3, b, hipMemcpyDeviceToHost));
    if (torque) HIPCHK(hipMemcpy(torque, S->ds.Th + o3, b, hipMemcpyDeviceToHost));
    return LBDEM_OK;
}

int lbdem_step(lbdem_set *S, int64_t nsteps)
{
    if (!S) return fail(LBDEM_EINVAL, "null set");
    if (nsteps < 0) return fail(LBDEM_EINVAL, "negative step count");
    int64_t left = nsteps;
    if (!S->timing && S->gexec && S->graph_steps > 0) {
        while (left >= S->graph_steps) {
            HIPCHK(hipGraphLaunch(S->gexec, S->stream));
            left -= S->graph_steps;
        }
    }
    for (; left > 0; --left) {
        int rc = launch_step_eager(S);
        if (rc) return rc;
    }
    S->t_host += nsteps;
    if (nsteps > 0) S->node_layout = false;
    return LBDEM_OK;
}

int lbdem_time(lbdem_set *S, int64_t *t)
{
    if (!S || !t) return fail(LBDEM_EINVAL, "null argument");
    int rc = sync_set(S);
    if (rc) return rc;
    long long tt = 0;
    HIPCHK(hipMemcpy(&tt, S->ds.tstep, sizeof(long long), hipMemcpyDeviceToHost));
    *t = tt;
    return LBDEM_OK;
}

int lbdem_synchronize(lbdem_set *S)
{
    if (!S) return fail(LBDEM_EINVAL, "null set");
    return sync_set(S);
}

int lbdem_status(lbdem_set *S, uint32_t *bits, int clear)
{
    if (!S || !bits) return fail(LBDEM_EINVAL, "null argument");
    int rc = sync_set(S);
    if (rc) return rc;
    unsigned f = 0;
    HIPCHK(hipMemcpy(&f, S->ds.flags, sizeof(unsigned), hipMemcpyDeviceToHost));
    *bits = f;
    if (clear) HIPCHK(hipMemset(S->ds.flags, 0, sizeof(unsigned)));
    const unsigned errs = LBDEM_STATUS_NEAR_OVERFLOW | LBDEM_STATUS_HISTORY_OVERFLOW | LBDEM_STATUS_TOO_FAST |
                          LBDEM_STATUS_SHELL_OVERFLOW | LBDEM_STATUS_LINK_OVERFLOW | LBDEM_STATUS_LIST_MISS;
    if (f & LBDEM_STATUS_NONFINITE) return fail(LBDEM_ENUMERIC, "device status 0x%x: non-finite fluid density", f);
    if (f & errs) return fail(LBDEM_ECAPACITY, "device status 0x%x", f);
    return LBDEM_OK;
}

int lbdem_probe_read(lbdem_set *S, int32_t lattice, int64_t first, int64_t n, double *out)
{
    int rc = check_lattice(S, lattice);
    if (rc) return rc;
    if (n < 0 || (n > 0 && !out)) return fail(LBDEM_EINVAL, "bad output");
    int64_t t = 0;
    rc = lbdem_time(S, &t);
    if (rc) return rc;
    const MemberDev &M = S->G.mem[lattice];
    if (first < 0 || first + n > t || first < t - S->G.ring_len)
        return fail(LBDEM_ERANGE, "steps [%lld, %lld) not held (t = %lld, ring %d)", (long long)first,
                    (long long)(first + n), (long long)t, S->G.ring_len);
    if (M.n_probe == 0 || n == 0) return LBDEM_OK;
    const size_t rec = (size_t)M.n_probe * 4;
    for (int64_t k = 0; k < n; ++k) {
        const int64_t slot = (first + k) % S->G.ring_len;
        HIPCHK(hipMemcpy(out + k * rec, S->ds.ring + M.ring_off + slot * rec, rec * 8, hipMemcpyDeviceToHost));
    }
    return LBDEM_OK;
}

int lbdem_probe_signal(lbdem_set *S, int32_t lattice, int64_t first, int64_t n, int32_t quantity, double *x)
{
    int rc = check_lattice(S, lattice);
    if (rc) return rc;
    if (n < 0 || (n > 0 && !x)) return fail(LBDEM_EINVAL, "bad output");
    if (quantity != 0 && quantity != 1) return fail(LBDEM_EINVAL, "quantity must be 0 (density) or 1 (momentum)");
    int64_t t = 0;
    rc = lbdem_time(S, &t);
    if (rc) return rc;
    const MemberDev &M = S->G.mem[lattice];
    if (first < 0 || first + n > t || first < t - S->G.ring_len)
        return fail(LBDEM_ERANGE, "steps [%lld, %lld) not held (t = %lld, ring %d)", (long long)first,
                    (long long)(first + n), (long long)t, S->G.ring_len);
    if (M.n_probe == 0 || n == 0) return LBDEM_OK;
    HIPCHK(launch_probe_signal(S->ds.ring + M.ring_off, S->G.ring_len, M.n_probe, first, n, quantity, x, S->stream));
    return LBDEM_OK;
}

int lbdem_particle_signal(lbdem_set *S, int32_t lattice, int64_t first, int64_t n, const int32_t *layer,
                          int32_t n_layers, int32_t component, double *x)
{
    int rc = check_lattice(S, lattice);
    if (rc) return rc;
    if (n < 0 || (n > 0 && !x)) return fail(LBDEM_EINVAL, "bad output");
    if (component < 0 || component > 2) return fail(LBDEM_EINVAL, "component must be 0, 1 or 2");
    if (n_layers < 1 || n_layers > (1 << 20)) return fail(LBDEM_EINVAL, "n_layers must be 1..2^20");
    const MemberDev &M = S->G.mem[lattice];
    if (M.np > 0 && !layer) return fail(LBDEM_EINVAL, "null layer array");
    int64_t t = 0;
    rc = lbdem_time(S, &t);
    if (rc) return rc;
    const int ring = S->G.pv_ring;
    if (ring < 1) return fail(LBDEM_ERANGE, "the set keeps no particle velocities (particle_ring 0)");
    if (first < 0 || first + n > t || first < t - ring || first < M.pv_from)
        return fail(LBDEM_ERANGE, "steps [%lld, %lld) not held (t = %lld, ring %d, particles set at %lld)",
                    (long long)first, (long long)(first + n), (long long)t, ring, M.pv_from);
    // the members of each layer in index order: members[start[l] .. start[l + 1])
    std::vector<int> start(n_layers + 1, 0);
    for (int q = 0; q < M.np; ++q) {
        const int l = layer[q];
        if (l < -1 || l >= n_layers)
            return fail(LBDEM_EINVAL, "particle %d: layer %d outside -1..%d", q, l, n_layers - 1);
        if (l >= 0) ++start[l + 1];
    }
    for (int l = 0; l < n_layers; ++l) start[l + 1] += start[l];
    std::vector<int> members(std::max(start[n_layers], 1), 0);
    {
        std::vector<int> fill(start.begin(), start.end() - 1);
        for (int q = 0; q < M.np; ++q)
            if (layer[q] >= 0) members[fill[layer[q]]++] = q;
    }
    if (n == 0) return LBDEM_OK;
    int *dev = nullptr;
    const size_t words = start.size() + members.size();
    if (hipMalloc((void **)&dev, words * sizeof(int)) != hipSuccess)
        return fail(LBDEM_ENOMEM, "no device memory for %zu layer words", words);
    hipError_t e = hipMemcpyAsync(dev, start.data(), start.size() * sizeof(int), hipMemcpyHostToDevice, S->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dev + start.size(), members.data(), members.size() * sizeof(int), hipMemcpyHostToDevice,
                           S->stream);
    if (e == hipSuccess)
        e = launch_particle_signal(S->ds.pvring, ring, S->G.ptot, M.p_off, first, n, dev, dev + start.size(),
                                   n_layers, component, x, S->stream);
    // the host arrays and the device copy live until the copies and the kernel are done
    if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
    const hipError_t ef = hipFree(dev);
    if (e != hipSuccess) return fail(LBDEM_EDEVICE, "particle signal: %s", hipGetErrorString(e));
    if (ef != hipSuccess) return fail(LBDEM_EDEVICE, "particle signal: %s", hipGetErrorString(ef));
    return LBDEM_OK;
}

int lbdem_biot_velocities(double k_dry, double g_dry, double phi, double k_p, double k_f, double rho_p,
                          double rho_f, double r, double *out)
{
    if (!out) return fail(LBDEM_EINVAL, "null output");
    if (!(phi > 0.0 && phi < 1.0) || !(k_p > 0.0) || !(k_f > 0.0) || !(rho_p > 0.0) || !(rho_f > 0.0) ||
        !(k_dry >= 0.0) || !(g_dry >= 0.0) || !std::isfinite(k_dry + g_dry + k_p + k_f + rho_p + rho_f + r))
        return fail(LBDEM_EINVAL, "moduli and densities must be positive (k_dry, g_dry >= 0), 0 < phi < 1");
    // Biot's elastic coefficients of the saturated packing, with c = 1 - phi - k_dry / k_p
    // and d = c + phi k_p / k_f: P = ((1 - phi) c k_p + phi k_p k_dry / k_f) / d + 4/3 g_dry,
    // Q = phi c k_p / d, R = phi^2 k_p / d
    const double c = 1.0 - phi - k_dry / k_p;
    const double d = c + phi * k_p / k_f;
    const double P = ((1.0 - phi) * c * k_p + phi * k_p * k_dry / k_f) / d + 4.0 / 3.0 * g_dry;
    const double Q = phi * c * k_p / d;
    const double R = phi * phi * k_p / d;
    // inertial coupling through the tortuosity alpha = 1 - r (1 - 1 / phi)
    const double alpha = 1.0 - r * (1.0 - 1.0 / phi);
    const double r12 = (1.0 - alpha) * phi * rho_f;
    const double r11 = (1.0 - phi) * rho_p - r12;
    const double r22 = phi * rho_f - r12;
    const double det = r11 * r22 - r12 * r12;
    // Eq. (vp): v^2 are the roots of det v^4 - (P r22 + R r11 - 2 Q r12) v^2 + (P R - Q^2) = 0
    const double bsum = P * r22 + R * r11 - 2.0 * Q * r12;
    const double disc = bsum * bsum - 4.0 * det * (P * R - Q * Q);
    if (!(det > 0.0) || !(disc >= 0.0) || !(bsum > 0.0))
        return fail(LBDEM_EINVAL, "these inputs give no real wave speeds");
    const double v2f = (bsum + std::sqrt(disc)) / (2.0 * det);
    // the smaller root without cancellation: the product of the roots over the larger one
    const double v2s = (P * R - Q * Q) / det / v2f;
    // Eq. (vs): the shear wave moves the solid with the fluid mass the coupling drags along
    const double v2t = g_dry / (r11 - r12 * r12 / r22);
    if (!(v2s >= 0.0) || !(v2t >= 0.0)) return fail(LBDEM_EINVAL, "these inputs give no real wave speeds");
    out[0] = std::sqrt(v2f);
    out[1] = std::sqrt(v2s);
    out[2] = std::sqrt(v2t);
    return LBDEM_OK;
}

namespace {

int check_dft_sizes(int64_t nt, int32_t nz, int32_t nw, int32_t nk)
{
    const long long lim = 1ll << 28;
    if (nt < 1 || nt > (1ll << 31) || nz < 1 || nz > 65536 || nw < 1 || nw > (1 << 20) || nk < 1 || nk > (1 << 20))
        return fail(LBDEM_EINVAL, "sizes out of range (nt %lld, nz %d, nw %d, nk %d)", (long long)nt, nz, nw, nk);
    if ((long long)nw * nz > lim || (long long)nz * nk > lim || (long long)nw * nk > lim)
        return fail(LBDEM_EINVAL, "spectrum too large (nw %d, nz %d, nk %d)", nw, nz, nk);
    return LBDEM_OK;
}

size_t dft_bytes(int64_t nt, int32_t nz, int32_t nw, int32_t nk)
{
    const DftPlan p = dft_plan(nt, nz, nw, nk);
    return p.part_bytes + p.g_bytes + p.e_bytes;
}

}  // namespace

int lbdem_dft_workspace_size(int64_t nt, int32_t nz, int32_t nw, int32_t nk, size_t *bytes)
{
    if (!bytes) return fail(LBDEM_EINVAL, "null output");
    int rc = check_dft_sizes(nt, nz, nw, nk);
    if (rc) return rc;
    *bytes = dft_bytes(nt, nz, nw, nk);
    return LBDEM_OK;
}

int lbdem_st_dft(const double *x, int64_t nt, int32_t nz, const double *zpos, double t0, double w0, double dw,
                 int32_t nw, double k0, double dk, int32_t nk, double *F, int32_t *ridge, void *work,
                 size_t work_bytes, void *stream)
{
    int rc = check_dft_sizes(nt, nz, nw, nk);
    if (rc) return rc;
    if (!x || !zpos || !F || !work) return fail(LBDEM_EINVAL, "null pointer");
    if ((uintptr_t)work % 256) return fail(LBDEM_EINVAL, "workspace not 256-byte aligned");
    const DftPlan p = dft_plan(nt, nz, nw, nk);
    if (work_bytes < p.part_bytes + p.g_bytes + p.e_bytes)
        return fail(LBDEM_ENOMEM, "workspace of %zu bytes, %zu needed", work_bytes, p.part_bytes + p.g_bytes + p.e_bytes);
    HIPCHK(launch_st_dft(p, x, nt, nz, zpos, t0, w0, dw, nw, k0, dk, nk, F, ridge, work, (hipStream_t)stream));
    return LBDEM_OK;
}

int lbdem_wave_fit(const double *x, int64_t nt, int32_t nz, const double *zpos, double t0, double omega,
                   double *out, void *work, size_t work_bytes, void *stream)
{
    int rc = check_dft_sizes(nt, nz, 1, 1);
    if (rc) return rc;
    if (!x || !zpos || !out || !work) return fail(LBDEM_EINVAL, "null pointer");
    if (!(omega != 0.0) || !std::isfinite(omega)) return fail(LBDEM_EINVAL, "omega must be finite and non-zero");
    if ((uintptr_t)work % 256) return fail(LBDEM_EINVAL, "workspace not 256-byte aligned");
    if (work_bytes < dft_bytes(nt, nz, 1, 1))
        return fail(LBDEM_ENOMEM, "workspace of %zu bytes, %zu needed", work_bytes, dft_bytes(nt, nz, 1, 1));
    HIPCHK(launch_wave_fit(x, nt, nz, zpos, t0, omega, out, work, (hipStream_t)stream));
    return LBDEM_OK;
}

int lbdem_wave_fit_noalloc(const double *x, int64_t nt, int32_t nz, const double *zpos, double t0, double omega,
                           double *out, void *stream)
{
    int rc = check_dft_sizes(nt, nz, 1, 1);
    if (rc) return rc;
    if (!x || !zpos || !out) return fail(LBDEM_EINVAL, "null pointer");
    if (!(omega != 0.0) || !std::isfinite(omega)) return fail(LBDEM_EINVAL, "omega must be finite and non-zero");
    const size_t need = dft_bytes(nt, nz, 1, 1);
    if (need > kNoAllocScratchBytes)
        return fail(LBDEM_ENOMEM, "the fit needs %zu bytes of scratch, more than the %zu-byte static scratch", need,
                    kNoAllocScratchBytes);
    void *work = nullptr;
    HIPCHK(noalloc_scratch(&work));
    HIPCHK(launch_wave_fit(x, nt, nz, zpos, t0, omega, out, work, (hipStream_t)stream));
    return LBDEM_OK;
}

int lbdem_populations_get(lbdem_set *S, int32_t lattice, double *f)
{
    int rc = check_lattice(S, lattice);
    if (rc) return rc;
    if (!f) return fail(LBDEM_EINVAL, "null output");
    rc = node_layout(S);
    if (rc) return rc;
    int64_t t = 0;
    rc = lbdem_time(S, &t);
    if (rc) return rc;
    const MemberDev &M = S->G.mem[lattice];
    const size_t es = elem_size(S->G.prec), cnt = (size_t)kQ * M.ncell;
    const char *src = (const char *)((t & 1) ? S->ds.popB : S->ds.popA) + es * M.pop_off;
    std::vector<char> raw(es * cnt);
    HIPCHK(hipMemcpy(raw.data(), src, raw.size(), hipMemcpyDeviceToHost));
    const float rf = (float)M.rho_f;
    for (size_t k = 0; k < cnt; ++k) {
        const int d = (int)(k / M.ncell);
        switch (S->G.prec) {
        case PREC_FP64: f[k] = ((const double *)raw.data())[k]; break;
        case PREC_FP32: f[k] = (double)(((const float *)raw.data())[k] + (float)(kWh[d] * M.rho_f)); break;
        case PREC_FP16DEV: f[k] = (double)((float)kWh[d] * (rf + (float)((const _Float16 *)raw.data())[k])); break;
        default: f[k] = (double)((float)kWh[d] * (rf + bf16_to_f32_host(((const uint16_t *)raw.data())[k]))); break;
        }
    }
    return LBDEM_OK;
}

int lbdem_populations_set(lbdem_set *S, int32_t lattice, const double *f)
{
    int rc = check_lattice(S, lattice);
    if (rc) return rc;
    if (!f) return fail(LBDEM_EINVAL, "null input");
    rc = node_layout(S);
    if (rc) return rc;
    int64_t t = 0;
    rc = lbdem_time(S, &t);
    if (rc) return rc;
    const MemberDev &M = S->G.mem[lattice];
    const size_t es = elem_size(S->G.prec), cnt = (size_t)kQ * M.ncell;
    char *dst = (char *)((t & 1) ? S->ds.popB : S->ds.popA) + es * M.pop_off;
    std::vector<char> raw(es * cnt);
    const float rf = (float)M.rho_f;
    for (size_t k = 0; k < cnt; ++k) {
        const int d = (int)(k / M.ncell);
        switch (S->G.prec) {
        case PREC_FP64: ((double *)raw.data())[k] = f[k]; break;
        case PREC_FP32: ((float *)raw.data())[k] = (float)f[k] - (float)(kWh[d] * M.rho_f); break;
        case PREC_FP16DEV: ((_Float16 *)raw.data())[k] = (_Float16)((float)f[k] * kInvWh[d] - rf); break;
        default: ((uint16_t *)raw.data())[k] = f32_to_bf16_host((float)f[k] * kInvWh[d] - rf); break;
        }
    }
    HIPCHK(hipMemcpy(dst, raw.data(), raw.size(), hipMemcpyHostToDevice));
    // the link records no longer describe the populations
    HIPCHK(hipMemset(S->ds.rec_step, 0x80, sizeof(long long)));
    return LBDEM_OK;
}

int lbdem_owner_get(lbdem_set *S, int32_t lattice, int32_t *owner)
{
    int rc = check_lattice(S, lattice);
    if (rc) return rc;
    if (!owner) return fail(LBDEM_EINVAL, "null output");
    int64_t t = 0;
    rc = lbdem_time(S, &t);
    if (rc) return rc;
    const MemberDev &M = S->G.mem[lattice];
    HIPCHK(hipMemcpy(owner, S->ds.own[t & 1] + M.cell_off, sizeof(int) * M.ncell, hipMemcpyDeviceToHost));
    for (long long k = 0; k < M.ncell; ++k)
        if (owner[k] >= 0) owner[k] -= M.p_off;
    return LBDEM_OK;
}

int lbdem_fields_get(lbdem_set *S, int32_t lattice, double *rho, double *u, int32_t *owner)
{
    int rc = check_lattice(S, lattice);
    if (rc) return rc;
    if (owner) {
        rc = lbdem_owner_get(S, lattice, owner);
        if (rc) return rc;
    }
    if (!rho && !u) return LBDEM_OK;
    rc = node_layout(S);
    if (rc) return rc;
    const MemberDev &M = S->G.mem[lattice];
    double *dev = nullptr;
    hipError_t e = hipMalloc(&dev, sizeof(double) * 4 * (size_t)M.ncell);
    if (e != hipSuccess) return fail(LBDEM_ENOMEM, "hipMalloc of the field scratch: %s", hipGetErrorString(e));
    std::vector<double> host(4 * (size_t)M.ncell);
    e = launch_fields(S->G.prec, S->ds, lattice, M.ncell, dev, S->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
    if (e == hipSuccess) e = hipMemcpy(host.data(), dev, sizeof(double) * host.size(), hipMemcpyDeviceToHost);
    (void)hipFree(dev);
    if (e != hipSuccess) return fail(LBDEM_EDEVICE, "fields: %s", hipGetErrorString(e));
    const size_t n = (size_t)M.ncell;
    if (rho) std::memcpy(rho, host.data(), sizeof(double) * n);
    if (u) std::memcpy(u, host.data() + n, sizeof(double) * 3 * n);
    return LBDEM_OK;
}

} // extern "C"

namespace {

// Checkpoint layout: header, the host copy of the per-lattice constants, then the
// workspace image without the scratch population buffer of compact storage (it holds
// nothing between kernels).
struct CkptHeader {
    char magic[8];
    uint32_t version, n_lat;
    uint64_t ws_bytes, skip_off, skip_bytes, digest;
    int64_t t_host;
    int32_t node_layout, reserved;
};
constexpr uint32_t kCkptVersion = 1;

void fnv(uint64_t &h, const void *p, size_t n)
{
    const unsigned char *b = (const unsigned char *)p;
    for (size_t k = 0; k < n; ++k) { h ^= b[k]; h *= 1099511628211ull; }
}

// Digest of everything a checkpoint depends on: every parameter field and the set-wide
// configuration except graph_steps (field by field, so padding bytes do not enter).
uint64_t set_digest(const lbdem_set *S)
{
    uint64_t h = 1469598103934665603ull;
    for (const lbdem_params &p : S->params) {
        fnv(h, &p.nx, 12); fnv(h, p.face_bc, sizeof(p.face_bc)); fnv(h, &p.tau, 8); fnv(h, &p.rho_f, 8);
        fnv(h, &p.wave, 4); fnv(h, &p.rho_amp, 8); fnv(h, &p.omega, 8); fnv(h, &p.t_n, 8); fnv(h, &p.young_E, 8);
        fnv(h, &p.poisson_nu, 8); fnv(h, &p.friction_mu, 8); fnv(h, &p.rho_p, 8); fnv(h, &p.n_probe, 4);
        fnv(h, p.probe_z, 4 * (size_t)std::max(0, std::min(p.n_probe, LBDEM_MAX_PROBES)));
        fnv(h, &p.max_particles, 4); fnv(h, &p.max_radius, 8); fnv(h, &p.tile_x, 4); fnv(h, &p.rest_free, 4);
    }
    const lbdem_config &c = S->cfg;
    fnv(h, &c.precision, 4); fnv(h, &c.probe_ring, 4); fnv(h, &c.tile_x, 4); fnv(h, &c.z_per_thread, 4);
    fnv(h, &c.node_lists, 4); fnv(h, &c.list_margin, 4); fnv(h, &c.fluid_off, 4);
    fnv(h, &c.particle_ring, 4);
    const uint64_t ws = S->ws_bytes;
    fnv(h, &ws, 8);
    return h;
}

void ckpt_ranges(const lbdem_set *S, uint64_t &skip_off, uint64_t &skip_bytes)
{
    skip_off = (uint64_t)((const char *)S->ds.popC - (const char *)S->ws);
    skip_bytes = S->G.compact ? (uint64_t)elem_size(S->G.prec) * kQ * (uint64_t)S->G.cells : 0;
}

} // namespace

extern "C" {

int lbdem_state_size(lbdem_set *S, size_t *bytes)
{
    if (!S || !bytes) return fail(LBDEM_EINVAL, "null argument");
    uint64_t so, sb;
    ckpt_ranges(S, so, sb);
    *bytes = sizeof(CkptHeader) + sizeof(MemberDev) * S->G.mem.size() + (S->ws_bytes - sb);
    return LBDEM_OK;
}

int lbdem_state_save(lbdem_set *S, void *buf, size_t cap, size_t *used)
{
    if (!S || !buf) return fail(LBDEM_EINVAL, "null argument");
    size_t need = 0;
    int rc = lbdem_state_size(S, &need);
    if (rc) return rc;
    if (cap < need) return fail(LBDEM_ENOMEM, "checkpoint needs %zu bytes, buffer holds %zu", need, cap);
    rc = sync_set(S);
    if (rc) return rc;
    CkptHeader h{};
    std::memcpy(h.magic, "LBDEMCKP", 8);
    h.version = kCkptVersion;
    h.n_lat = (uint32_t)S->G.mem.size();
    h.ws_bytes = S->ws_bytes;
    ckpt_ranges(S, h.skip_off, h.skip_bytes);
    h.digest = set_digest(S);
    h.t_host = S->t_host;
    h.node_layout = S->node_layout ? 1 : 0;
    char *o = (char *)buf;
    std::memcpy(o, &h, sizeof(h));
    o += sizeof(h);
    std::memcpy(o, S->G.mem.data(), sizeof(MemberDev) * S->G.mem.size());
    o += sizeof(MemberDev) * S->G.mem.size();
    const char *ws = (const char *)S->ws;
    HIPCHK(hipMemcpy(o, ws, h.skip_off, hipMemcpyDeviceToHost));
    o += h.skip_off;
    const uint64_t tail = h.ws_bytes - h.skip_off - h.skip_bytes;
    HIPCHK(hipMemcpy(o, ws + h.skip_off + h.skip_bytes, tail, hipMemcpyDeviceToHost));
    if (used) *used = need;
    return LBDEM_OK;
}

int lbdem_state_load(lbdem_set *S, const void *buf, size_t size)
{
    if (!S || !buf) return fail(LBDEM_EINVAL, "null argument");
    CkptHeader h;
    if (size < sizeof(h)) return fail(LBDEM_EINVAL, "not a checkpoint (too short)");
    std::memcpy(&h, buf, sizeof(h));
    if (std::memcmp(h.magic, "LBDEMCKP", 8) != 0 || h.version != kCkptVersion)
        return fail(LBDEM_EINVAL, "not a checkpoint of this library");
    uint64_t so, sb;
    ckpt_ranges(S, so, sb);
    if (h.n_lat != S->G.mem.size() || h.ws_bytes != S->ws_bytes || h.skip_off != so || h.skip_bytes != sb ||
        h.digest != set_digest(S))
        return fail(LBDEM_EINVAL, "checkpoint of a set with other parameters");
    size_t need = 0;
    int rc = lbdem_state_size(S, &need);
    if (rc) return rc;
    if (size != need) return fail(LBDEM_EINVAL, "checkpoint of %zu bytes, %zu expected", size, need);
    rc = sync_set(S);
    if (rc) return rc;
    const char *in = (const char *)buf + sizeof(h);
    std::vector<MemberDev> mem(h.n_lat);
    std::memcpy(mem.data(), in, sizeof(MemberDev) * h.n_lat);
    in += sizeof(MemberDev) * h.n_lat;
    char *ws = (char *)S->ws;
    HIPCHK(hipMemcpy(ws, in, h.skip_off, hipMemcpyHostToDevice));
    in += h.skip_off;
    HIPCHK(hipMemcpy(ws + h.skip_off + h.skip_bytes, in, h.ws_bytes - h.skip_off - h.skip_bytes,
                     hipMemcpyHostToDevice));
    // the host's copy of the per-lattice constants (particle counts, fluid-kernel grid)
    S->G.mem = mem;
    int tiles = 0;
    for (const MemberDev &M : S->G.mem) tiles = std::max(tiles, M.tile_off + M.ntx * M.nty * M.ntz);
    S->G.tiles = tiles;
    S->ds.tiles_total = tiles;
    S->t_host = h.t_host;
    S->node_layout = h.node_layout != 0;
    if (S->gexec) return build_graph(S, S->graph_steps);
    return LBDEM_OK;
}

int lbdem_timing_enable(lbdem_set *S, int enable)
{
    if (!S) return fail(LBDEM_EINVAL, "null set");
    int rc = sync_set(S);
    if (rc) return rc;
    rc = harvest_events(S);
    if (rc) return rc;
    S->timing = enable != 0;
    for (int k = 0; k < kKernels; ++k) { S->ms_acc[k] = 0.0; S->ms_cnt[k] = 0; }
    return LBDEM_OK;
}

int lbdem_timing_read(lbdem_set *S, double *ms, int64_t *count)
{
    if (!S || !ms || !count) return fail(LBDEM_EINVAL, "null argument");
    int rc = sync_set(S);
    if (rc) return rc;
    rc = harvest_events(S);
    if (rc) return rc;
    for (int k = 0; k < kKernels; ++k) { ms[k] = S->ms_acc[k]; count[k] = S->ms_cnt[k]; }
    return LBDEM_OK;
}

int lbdem_tile_info(lbdem_set *S, int32_t lattice, int32_t *tile_x, int32_t *tile_y, int32_t *z_per_thread)
{
    int rc = check_lattice(S, lattice);
    if (rc) return rc;
    const MemberDev &M = S->G.mem[lattice];
    if (tile_x) *tile_x = M.bx;
    if (tile_y) *tile_y = M.by;
    if (z_per_thread) *z_per_thread = S->G.nzt;
    return LBDEM_OK;
}

} // extern "C"

// ---------------------------------------------------------------------------
// Adjoint window over frozen geometry
// ---------------------------------------------------------------------------
struct lbdem_adj {
    lbdem_set *set = nullptr;
    int lattice = 0, prec = 0;
    size_t es = 0, cs = 0;      // storage / arithmetic element sizes
    int64_t nsteps = 0;
    int ck = 1, nck = 0;
    int64_t t0 = 0;
    double tau = 1.0;
    bool have_forward = false;
    AdjDev a{};
    hipStream_t stream = nullptr;
    char *f0 = nullptr, *ckp = nullptr, *seg = nullptr, *lam0 = nullptr, *lam1 = nullptr, *mu = nullptr;
    double *vdev = nullptr, *shape = nullptr, *P = nullptr, *dLdP = nullptr, *accw = nullptr, *acca = nullptr;
    double *macc = nullptr, *gv = nullptr, *nfl = nullptr, *X = nullptr, *W = nullptr, *R = nullptr;
    int *own = nullptr, *pz = nullptr;
    std::vector<double> v_host;
};

extern "C" {

static size_t adj_layout(lbdem_adj *J, int64_t ncell, int64_t np, int nprobe, int nblk, int64_t nsteps, int ck,
                         size_t es, size_t cs, char *base)
{
    Carver c;
    c.base = base;
    const size_t st = (size_t)kQ * ncell;
    const int nck = (int)((nsteps + ck - 1) / ck);
    char *f0 = c.take<char>(es * st);
    char *ckp = c.take<char>(es * st * (size_t)nck);
    char *seg = c.take<char>(es * st * (size_t)std::max(ck, 2));
    char *lam0 = c.take<char>(cs * st), *lam1 = c.take<char>(cs * st), *mu = c.take<char>(cs * st);
    double *macc = c.take<double>((size_t)(kQ - 1) * ncell);
    int *own = c.take<int>((size_t)ncell);
    double *X = c.take<double>(3 * (size_t)std::max<int64_t>(np, 1));
    double *W = c.take<double>(3 * (size_t)std::max<int64_t>(np, 1));
    double *R = c.take<double>((size_t)std::max<int64_t>(np, 1));
    double *V = c.take<double>(3 * (size_t)std::max<int64_t>(np, 1));
    double *gv = c.take<double>(3 * (size_t)std::max<int64_t>(np, 1));
    double *shape = c.take<double>((size_t)std::max<int64_t>(nsteps, 1));
    double *P = c.take<double>((size_t)std::max<int64_t>(nsteps * nprobe, 1));
    double *dLdP = c.take<double>((size_t)std::max<int64_t>(nsteps * nprobe, 1));
    double *accw = c.take<double>((size_t)nblk), *acca = c.take<double>((size_t)nblk);
    double *nfl = c.take<double>((size_t)std::max(nprobe, 1));
    int *pz = c.take<int>((size_t)std::max(nprobe, 1));
    if (J) {
        J->f0 = f0; J->ckp = ckp; J->seg = seg; J->lam0 = lam0; J->lam1 = lam1; J->mu = mu; J->macc = macc;
        J->own = own; J->X = X; J->W = W; J->R = R; J->vdev = V; J->gv = gv; J->shape = shape; J->P = P;
        J->dLdP = dLdP; J->accw = accw; J->acca = acca; J->nfl = nfl; J->pz = pz; J->nck = nck;
    }
    return (c.off + 255) & ~size_t(255);
}

int lbdem_adj_workspace_size(lbdem_set *S, int32_t lattice, int64_t nsteps, int32_t ckpt_every, size_t *bytes)
{
    int rc = check_lattice(S, lattice);
    if (rc) return rc;
    if (!bytes) return fail(LBDEM_EINVAL, "null argument");
    if (nsteps < 1 || ckpt_every < 1) return fail(LBDEM_EINVAL, "nsteps and ckpt_every must be >= 1");
    const MemberDev &M = S->G.mem[lattice];
    const size_t es = elem_size(S->G.prec), cs = S->G.prec == PREC_FP64 ? 8 : 4;
    const int nblk = (int)((M.ncell + 255) / 256);
    *bytes = adj_layout(nullptr, M.ncell, M.np, S->params[lattice].n_probe, nblk, nsteps, ckpt_every, es, cs, nullptr);
    return LBDEM_OK;
}

int lbdem_adj_create(lbdem_set *S, int32_t lattice, int64_t nsteps, int32_t ckpt_every, void *workspace,
                     size_t workspace_bytes, lbdem_adj **out)
{
    if (!out) return fail(LBDEM_EINVAL, "null output");
    *out = nullptr;
    size_t need = 0;
    int rc = lbdem_adj_workspace_size(S, lattice, nsteps, ckpt_every, &need);
    if (rc) return rc;
    if (!workspace || workspace_bytes < need) return fail(LBDEM_ENOMEM, "adjoint workspace needs %zu bytes", need);
    if (((uintptr_t)workspace & 255) != 0) return fail(LBDEM_EINVAL, "workspace must be 256-byte aligned");
    const MemberDev &M = S->G.mem[lattice];
    const lbdem_params &p = S->params[lattice];
    if (M.ncell > (1LL << 31) / kQ) return fail(LBDEM_EINVAL, "lattice too large for the adjoint window");
    std::unique_ptr<lbdem_adj> J(new lbdem_adj());
    J->set = S;
    J->lattice = lattice;
    J->prec = S->G.prec;
    J->es = elem_size(S->G.prec);
    J->cs = S->G.prec == PREC_FP64 ? 8 : 4;
    J->nsteps = nsteps;
    J->ck = ckpt_every;
    J->stream = S->stream;
    const int nblk = (int)((M.ncell + 255) / 256);
    adj_layout(J.get(), M.ncell, M.np, p.n_probe, nblk, nsteps, ckpt_every, J->es, J->cs, (char *)workspace);
    rc = lbdem_time(S, &J->t0);
    if (rc) return rc;
    rc = node_layout(S);
    if (rc) return rc;
    rc = sync_set(S);
    if (rc) return rc;
    // frozen geometry: node map (local particle indices), particle state, start populations
    std::vector<int32_t> own((size_t)M.ncell);
    rc = lbdem_owner_get(S, lattice, own.data());
    if (rc) return rc;
    const int np = M.np;
    std::vector<double> x(3 * (size_t)std::max(np, 1)), v(x.size()), w(x.size()), fh(x.size()), th(x.size());
    rc = lbdem_particles_get(S, lattice, np, x.data(), v.data(), w.data(), fh.data(), th.data());
    if (rc) return rc;
    J->v_host.assign(v.begin(), v.begin() + 3 * np);
    HIPCHK(hipMemcpy(J->own, own.data(), sizeof(int32_t) * own.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(J->X, x.data(), sizeof(double) * x.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(J->W, w.data(), sizeof(double) * w.size(), hipMemcpyHostToDevice));
    if (np > 0) HIPCHK(hipMemcpy(J->R, S->ds.R + M.p_off, sizeof(double) * np, hipMemcpyDeviceToDevice));
    const char *src = (const char *)((J->t0 & 1) ? S->ds.popB : S->ds.popA) + J->es * M.pop_off;
    HIPCHK(hipMemcpy(J->f0, src, J->es * kQ * M.ncell, hipMemcpyDeviceToDevice));
    // unit-amplitude waveform at the time levels t0+1 .. t0+nsteps, Eq. (source)
    std::vector<double> shape((size_t)nsteps);
    for (int64_t n = 0; n < nsteps; ++n) {
        const int64_t tt = J->t0 + n + 1;
        double sv = 0.0;
        if (p.wave != LBDEM_WAVE_NONE && tt <= p.t_n) {
            const double wt = p.omega * (double)tt;
            sv = p.wave == LBDEM_WAVE_SINE ? sin(wt) : (p.wave == LBDEM_WAVE_COSINE ? 1.0 - cos(wt) : 1.0);
        }
        shape[(size_t)n] = sv;
    }
    HIPCHK(hipMemcpy(J->shape, shape.data(), sizeof(double) * shape.size(), hipMemcpyHostToDevice));
    if (p.n_probe > 0) HIPCHK(hipMemcpy(J->pz, p.probe_z, sizeof(int) * p.n_probe, hipMemcpyHostToDevice));
    AdjDev &a = J->a;
    a.M = M;
    a.ncell = (int)M.ncell;
    a.own = J->own;
    a.X = J->X; a.W = J->W; a.R = J->R; a.V = J->vdev;
    a.np = np;
    a.rho_f = p.rho_f;
    a.omega = 1.0 / p.tau;
    a.amp = p.rho_amp;
    a.shape = J->shape;
    a.n_probe = p.n_probe;
    a.probe_z = J->pz;
    a.probe_nfl = J->nfl;
    a.P = J->P;
    a.dLdP = J->dLdP;
    a.acc_w = J->accw; a.acc_a = J->acca;
    a.macc = J->macc;
    a.gv = J->gv;
    HIPCHK(launch_adj_nfl(a, J->nfl, J->stream));
    HIPCHK(hipStreamSynchronize(J->stream));
    *out = J.release();
    return LBDEM_OK;
}

int lbdem_adj_forward(lbdem_adj *J, double tau, double amp, const double *v, double *probes)
{
    if (!J) return fail(LBDEM_EINVAL, "null adjoint window");
    if (!(tau > 0.5)) return fail(LBDEM_EINVAL, "tau must exceed 1/2");
    AdjDev &a = J->a;
    const size_t st = (size_t)kQ * a.ncell * J->es;
    J->tau = tau;
    a.omega = 1.0 / tau;
    a.amp = amp;
    const std::vector<double> &vv = v ? std::vector<double>(v, v + 3 * a.np) : J->v_host;
    if (a.np > 0) HIPCHK(hipMemcpyAsync(J->vdev, vv.data(), sizeof(double) * 3 * a.np, hipMemcpyHostToDevice, J->stream));
    char *cur = J->seg, *nxt = J->seg + st;
    HIPCHK(hipMemcpyAsync(cur, J->f0, st, hipMemcpyDeviceToDevice, J->stream));
    for (int64_t n = 0; n < J->nsteps; ++n) {
        if (n % J->ck == 0)
            HIPCHK(hipMemcpyAsync(J->ckp + st * (size_t)(n / J->ck), cur, st, hipMemcpyDeviceToDevice, J->stream));
        if (a.n_probe > 0) HIPCHK(launch_adj_probe(J->prec, a, cur, (int)n, J->stream));
        HIPCHK(launch_adj_step(J->prec, a, cur, nxt, (int)n, J->stream));
        std::swap(cur, nxt);
    }
    if (probes && a.n_probe > 0)
        HIPCHK(hipMemcpyAsync(probes, J->P, sizeof(double) * J->nsteps * a.n_probe, hipMemcpyDeviceToHost, J->stream));
    HIPCHK(hipStreamSynchronize(J->stream));
    J->have_forward = true;
    return LBDEM_OK;
}

int lbdem_adj_backward(lbdem_adj *J, const double *dL_dP, double *dL_dtau, double *dL_damp, double *dL_dv)
{
    if (!J) return fail(LBDEM_EINVAL, "null adjoint window");
    if (!J->have_forward) return fail(LBDEM_ESTATE, "lbdem_adj_forward must run first");
    AdjDev &a = J->a;
    const size_t st = (size_t)kQ * a.ncell * J->es, sl = (size_t)kQ * a.ncell * J->cs;
    const int nblk = adj_blocks(a);
    if (a.n_probe > 0) {
        if (!dL_dP) return fail(LBDEM_EINVAL, "null loss gradient");
        HIPCHK(hipMemcpyAsync(J->dLdP, dL_dP, sizeof(double) * J->nsteps * a.n_probe, hipMemcpyHostToDevice, J->stream));
    }
    HIPCHK(hipMemsetAsync(J->lam0, 0, sl, J->stream));
    HIPCHK(hipMemsetAsync(J->accw, 0, sizeof(double) * nblk, J->stream));
    HIPCHK(hipMemsetAsync(J->acca, 0, sizeof(double) * nblk, J->stream));
    HIPCHK(hipMemsetAsync(J->macc, 0, sizeof(double) * (kQ - 1) * (size_t)a.ncell, J->stream));
    char *lam = J->lam0, *lam_next = J->lam1;
    for (int s = J->nck - 1; s >= 0; --s) {
        const int64_t start = (int64_t)s * J->ck;
        const int64_t len = std::min<int64_t>(J->ck, J->nsteps - start);
        // recompute the segment's states from its checkpoint
        HIPCHK(hipMemcpyAsync(J->seg, J->ckp + st * (size_t)s, st, hipMemcpyDeviceToDevice, J->stream));
        for (int64_t m = 0; m + 1 < len; ++m)
            HIPCHK(launch_adj_step(J->prec, a, J->seg + st * (size_t)m, J->seg + st * (size_t)(m + 1), (int)(start + m),
                                   J->stream));
        for (int64_t m = len - 1; m >= 0; --m) {
            HIPCHK(launch_adj_mu(J->prec, a, J->seg + st * (size_t)m, lam, J->mu, (int)(start + m), J->stream));
            HIPCHK(launch_adj_pull(J->prec, a, J->mu, lam_next, J->stream));
            std::swap(lam, lam_next);
        }
    }
    HIPCHK(launch_adj_vgrad(a, J->stream));
    std::vector<double> aw(nblk), aa(nblk);
    HIPCHK(hipMemcpyAsync(aw.data(), J->accw, sizeof(double) * nblk, hipMemcpyDeviceToHost, J->stream));
    HIPCHK(hipMemcpyAsync(aa.data(), J->acca, sizeof(double) * nblk, hipMemcpyDeviceToHost, J->stream));
    if (dL_dv && a.np > 0)
        HIPCHK(hipMemcpyAsync(dL_dv, J->gv, sizeof(double) * 3 * a.np, hipMemcpyDeviceToHost, J->stream));
    HIPCHK(hipStreamSynchronize(J->stream));
    double gw = 0.0, ga = 0.0;
    for (int b = 0; b < nblk; ++b) { gw += aw[b]; ga += aa[b]; }
    // omega = 1/tau
    if (dL_dtau) *dL_dtau = gw * (-1.0 / (J->tau * J->tau));
    if (dL_damp) *dL_damp = ga;
    return LBDEM_OK;
}

int lbdem_adj_destroy(lbdem_adj *J)
{
    if (!J) return LBDEM_OK;
    (void)hipStreamSynchronize(J->stream);
    delete J;
    return LBDEM_OK;
}

} // extern "C"
