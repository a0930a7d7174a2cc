// dfhm_api.hip -- host runtime behind include/dfhm.h.
//
// The host only validates descriptors, lays out device memory, packs walls
// into workgroups and enqueues kernels; every step of the method (grid
// constants, layer ids, start-up, DF updates, fluxes, zone balance) runs on
// the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/dfhm.h"
#include "df_kernels.hpp"
#include "df_resident.hpp"
#include "df_implicit.hpp"

using namespace dfhm;

struct dfhm_ctx {
    dfhm_config cfg{};
    RunConst rc{};
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t nw = 0, nr = 0, N = 0;
    int64_t n = 0;                 // host copy of the step index
    int precision = DFHM_FP64;
    size_t esize = 8;
    // device memory
    bool own_arena = false;
    void *arena = nullptr;
    size_t arena_bytes = 0;
    WallDev *d_walls = nullptr;
    int2 *d_tiles = nullptr;
    int ntiles = 0;
    void *d_T[2] = {nullptr, nullptr};
    void *d_P[2] = {nullptr, nullptr};
    uint8_t *d_lay = nullptr;
    double *d_flux = nullptr;
    int *d_bad = nullptr;
    int64_t *d_step = nullptr;
    ResIO *d_io = nullptr;         // write-back pointers of the resident kernel
    ResIO io_host{};               // what d_io holds
    bool io_valid = false;
    // zones
    void *room_mem = nullptr;
    RoomDev *d_rooms = nullptr;
    int32_t *d_room_walls = nullptr;
    double *d_roomT = nullptr, *d_roomP = nullptr, *d_go = nullptr, *d_qh = nullptr;
    // resident packing
    void *pack_mem = nullptr;
    ResBlock *d_blocks = nullptr;
    ResSlot *d_slots = nullptr;
    int32_t *d_block_rooms = nullptr;
    int n_blocks = 0, max_wpb = 0, max_rpb = 0;
    double pack_eff = 0.0;
    int res_threads = 0, res_npt = 0;
    bool packed = false;
    // some wall has an incident or long-wave source, or zones are linked: the
    // resident kernel then runs its extended variant
    bool extended = false;
    // inter-zone links
    void *link_mem = nullptr;
    ZoneLinkDev *d_links = nullptr;   // per receiving zone (RoomDev l_begin..l_end)
    double *d_inz = nullptr;          // per zone: heat, vapour gained (streaming)
    int64_t n_links = 0;
    std::vector<RoomDev> rooms_host;
    std::vector<double> sched_go, sched_qh;            // zone schedules (host copies)
    std::vector<ZoneLinkDev> links_host;               // per receiving zone, as on the device
    std::vector<std::vector<int32_t>> zone_partners;   // linked zones of each zone
    std::vector<double> zone_mass, zone_cma, zone_sT, zone_sM;   // stability sums
    // captured chunk of streaming steps
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int graph_steps = 0;
    // law shape shared by all walls (required by the resident kernel)
    bool shape_uniform = false;
    Shape shape{};
    int max_group_nodes = 0;
    // autotuned choice
    bool tuned = false;
    int tuned_sched = DFHM_SCHED_RESIDENT;
    // host copies
    std::vector<WallDev> walls;
    std::vector<int64_t> wall_room;
    std::vector<int8_t> room_side;
    std::string err;
    dfhm_status latched = DFHM_OK;
};

namespace {

dfhm_status fail(dfhm_ctx *c, dfhm_status s, const std::string &msg)
{
    if (c) c->err = msg;
    return s;
}

#define HIP_TRY(ctx, call)                                                                  \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((ctx), DFHM_E_DEVICE,                                               \
                        std::string(#call) + ": " + hipGetErrorString(e_));                 \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
    size_t walls, tiles, T0, T1, P0, P1, lay, flux, bad, step, total;
};

int count_tiles(const dfhm_wall *w, int64_t nw)
{
    int64_t t = 0;
    for (int64_t i = 0; i < nw; ++i) t += (w[i].nx + kStreamTile - 1) / kStreamTile;
    return (int)t;
}

Layout layout_of(int precision, const dfhm_wall *w, int64_t nw)
{
    size_t es = precision == DFHM_FP32 ? 4 : 8;
    int64_t N = 0;
    for (int64_t i = 0; i < nw; ++i) N += w[i].nx;
    Layout L{};
    size_t o = 0;
    L.walls = o; o = align256(o + sizeof(WallDev) * nw);
    L.tiles = o; o = align256(o + sizeof(int2) * (size_t)count_tiles(w, nw));
    L.T0 = o; o = align256(o + es * N);
    L.T1 = o; o = align256(o + es * N);
    L.P0 = o; o = align256(o + es * N);
    L.P1 = o; o = align256(o + es * N);
    L.lay = o; o = align256(o + (size_t)N);
    L.flux = o; o = align256(o + sizeof(double) * 12 * nw);
    L.bad = o; o = align256(o + sizeof(int));
    L.step = o; o = align256(o + sizeof(int64_t));
    L.total = o;
    return L;
}

bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0; }

std::string check_wall(const dfhm_wall &w, int64_t i)
{
    char b[160];
    if (w.nx < 3 || w.nx > kMaxNx) {
        snprintf(b, sizeof b, "wall %lld: nx=%d outside [3, %d]", (long long)i, w.nx, kMaxNx);
        return b;
    }
    if (w.n_layers < 1 || w.n_layers > kMaxLayers) {
        snprintf(b, sizeof b, "wall %lld: n_layers=%d outside [1, 3]", (long long)i, w.n_layers);
        return b;
    }
    for (int l = 0; l < w.n_layers; ++l) {
        const dfhm_layer &m = w.layer[l];
        if (!(std::isfinite(m.thickness_m) && m.thickness_m > 0.0) || !finite_nonneg(m.k0) ||
            !finite_nonneg(m.kM0) || !(std::isfinite(m.c0) && m.c0 > 0.0) ||
            !(std::isfinite(m.cM0) && m.cM0 > 0.0) || !std::isfinite(m.a_T) ||
            !std::isfinite(m.a_M) || !std::isfinite(m.b_TM) || !std::isfinite(m.c_T) ||
            !std::isfinite(m.c_M) || !std::isfinite(m.e_TM) || !std::isfinite(m.f_TM)) {
            snprintf(b, sizeof b, "wall %lld layer %d: bad thickness or coefficients",
                     (long long)i, l);
            return b;
        }
    }
    for (int s = 0; s < 2; ++s) {
        if (!finite_nonneg(w.h_T[s]) || !finite_nonneg(w.h_M[s]) || !std::isfinite(w.q_inf[s]) ||
            !std::isfinite(w.g_inf[s])) {
            snprintf(b, sizeof b, "wall %lld side %d: bad surface coefficients", (long long)i, s);
            return b;
        }
        const dfhm_sine *ss[3] = {&w.T_amb[s], &w.RH_amb[s], &w.q_sun[s]};
        for (const dfhm_sine *q : ss)
            if (!(std::isfinite(q->period_s) && q->period_s > 0.0) || !std::isfinite(q->mean) ||
                !std::isfinite(q->amp) || !std::isfinite(q->phase)) {
                snprintf(b, sizeof b, "wall %lld side %d: bad ambient or radiation sinusoid",
                         (long long)i, s);
                return b;
            }
        if (!(w.emissivity[s] >= 0.0 && w.emissivity[s] <= 1.0)) {
            snprintf(b, sizeof b, "wall %lld side %d: emissivity outside [0, 1]", (long long)i, s);
            return b;
        }
    }
    if (!(std::isfinite(w.T0) && w.T0 > 0.0) || !(std::isfinite(w.RH0) && w.RH0 > 0.0) ||
        !finite_nonneg(w.area_m2)) {
        snprintf(b, sizeof b, "wall %lld: bad initial state or area", (long long)i);
        return b;
    }
    return "";
}

void fill_wall(WallDev &d, const dfhm_wall &w, int32_t off)
{
    std::memset(&d, 0, sizeof d);
    d.off = off;
    d.nx = w.nx;
    d.n_layers = w.n_layers;
    d.room = -1;
    d.room_side = 1;
    d.area = w.area_m2;
    d.T0 = w.T0;
    d.RH0 = w.RH0;
    for (int s = 0; s < 2; ++s) {
        d.hT[s] = w.h_T[s];
        d.hM[s] = w.h_M[s];
        d.qinf[s] = w.q_inf[s];
        d.ginf[s] = w.g_inf[s];
        const dfhm_sine &a = w.T_amb[s], &b = w.RH_amb[s];
        d.Tamb[s][0] = a.mean; d.Tamb[s][1] = a.amp; d.Tamb[s][2] = a.period_s; d.Tamb[s][3] = a.phase;
        d.RHamb[s][0] = b.mean; d.RHamb[s][1] = b.amp; d.RHamb[s][2] = b.period_s; d.RHamb[s][3] = b.phase;
        const dfhm_sine &q = w.q_sun[s];
        d.qsun[s][0] = q.mean; d.qsun[s][1] = q.amp; d.qsun[s][2] = q.period_s; d.qsun[s][3] = q.phase;
        d.emis[s] = w.emissivity[s];
    }
    d.esig = 0.0;          // set when a zone is coupled
    d.room_walls = 0;
    for (int l = 0; l < kMaxLayers; ++l) {
        const dfhm_layer &m = w.layer[l];
        double *p = d.lay[l];
        if (l >= w.n_layers) {
            // unused slots mirror layer 0 so that no lane ever reads garbage
            std::memcpy(p, d.lay[0], sizeof(double) * L_COUNT);
            continue;
        }
        p[L_THICK] = m.thickness_m; p[L_K0] = m.k0; p[L_AT] = m.a_T; p[L_KM0] = m.kM0;
        p[L_AM] = m.a_M; p[L_BTM] = m.b_TM; p[L_C0] = m.c0; p[L_CT] = m.c_T;
        p[L_CM0] = m.cM0; p[L_AC] = m.c_M; p[L_ETM] = m.e_TM; p[L_FTM] = m.f_TM;
    }
}

double orz(double v, double d) { return v == 0.0 ? d : v; }

dfhm_status check_bad(dfhm_ctx *c)
{
    int bad = 0;
    HIP_TRY(c, hipMemcpyAsync(&bad, c->d_bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (bad) {
        c->latched = DFHM_E_STATE;
        return fail(c, DFHM_E_NONFINITE, "a step produced a non-finite value");
    }
    return DFHM_OK;
}

template <typename R>
void launch_stream_step(dfhm_ctx *c, int off)
{
    auto kern = c->cfg.law == DFHM_LAW_TABLE1
                    ? (c->extended ? k_df_stream<R, true, 1> : k_df_stream<R, false, 1>)
                    : (c->extended ? k_df_stream<R, true, 0> : k_df_stream<R, false, 0>);
    hipLaunchKernelGGL(kern, dim3(c->ntiles), dim3(kStreamBlock), 0, c->stream,
                       c->d_walls, c->d_tiles, (R *)c->d_T[0], (R *)c->d_T[1], (R *)c->d_P[0],
                       (R *)c->d_P[1], c->d_lay, c->d_roomT, c->d_roomP, c->d_rooms,
                       c->d_room_walls, c->d_flux, c->d_bad, c->d_step, off, c->rc);
}

template <typename R>
dfhm_status launch_room_step(dfhm_ctx *c, int off)
{
    if (c->nr == 0) return DFHM_OK;
    int nb = (int)((c->nr + 63) / 64);
    if (c->n_links > 0)
        hipLaunchKernelGGL(k_zone_exchange, dim3(nb), dim3(64), 0, c->stream, c->d_rooms,
                           c->d_links, c->d_roomT, c->d_roomP, c->d_inz, (int)c->nr, c->rc);
    hipLaunchKernelGGL(k_room_step<R>, dim3(nb), dim3(64), 0, c->stream, c->d_rooms,
                       c->d_room_walls, c->d_walls, (const R *)c->d_T[0], (const R *)c->d_T[1],
                       (const R *)c->d_P[0], (const R *)c->d_P[1], c->d_roomT, c->d_roomP,
                       c->d_go, c->d_qh, c->n_links > 0 ? c->d_inz : nullptr, (int)c->nr,
                       c->d_step, off, c->rc);
    return DFHM_OK;
}

template <typename R>
dfhm_status launch_startup(dfhm_ctx *c)
{
    hipLaunchKernelGGL(k_startup<R>, dim3((unsigned)c->nw), dim3(kStartBlock), 0, c->stream,
                       c->d_walls, (R *)c->d_T[0], (R *)c->d_T[1], (R *)c->d_P[0],
                       (R *)c->d_P[1], c->d_lay, c->d_roomT, c->d_roomP, c->d_rooms,
                       c->d_room_walls, c->d_flux, c->d_bad, c->rc, c->cfg.law);
    return DFHM_OK;
}

void tick(dfhm_ctx *c, int k)
{
    hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, c->stream, c->d_step, k);
}

// Enqueue `k` streaming steps starting at host step c->n (n >= 1, or n == 0
// with the repeat start), with one device tick at the end.
template <typename R>
void enqueue_stream_chunk(dfhm_ctx *c, int k)
{
    for (int i = 0; i < k; ++i) {
        launch_stream_step<R>(c, i);
        launch_room_step<R>(c, i);
    }
    tick(c, k);
}

template <typename R>
dfhm_status step_stream(dfhm_ctx *c, int64_t nsteps)
{
    while (nsteps > 0) {
        if (c->n == 0 && c->cfg.startup == DFHM_START_FTCS) {
            launch_startup<R>(c);
            launch_room_step<R>(c, 0);
            tick(c, 1);
            c->n += 1;
            nsteps -= 1;
            continue;
        }
        int chunk = c->cfg.chunk_steps > 0 ? c->cfg.chunk_steps : 100;
        if (c->cfg.use_graph && nsteps >= chunk) {
            if (!c->graph_exec || c->graph_steps != chunk) {
                if (c->graph_exec) { (void)hipGraphExecDestroy(c->graph_exec); c->graph_exec = nullptr; }
                if (c->graph) { (void)hipGraphDestroy(c->graph); c->graph = nullptr; }
                // capture on a private stream (the caller's may be the legacy
                // default stream, which cannot be captured); replay on theirs
                hipStream_t cap = nullptr;
                HIP_TRY(c, hipStreamSynchronize(c->stream));
                HIP_TRY(c, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
                hipStream_t user = c->stream;
                c->stream = cap;
                hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
                if (e == hipSuccess) {
                    enqueue_stream_chunk<R>(c, chunk);
                    e = hipStreamEndCapture(cap, &c->graph);
                }
                c->stream = user;
                (void)hipStreamDestroy(cap);
                if (e != hipSuccess)
                    return fail(c, DFHM_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
                HIP_TRY(c, hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
                c->graph_steps = chunk;
            }
            HIP_TRY(c, hipGraphLaunch(c->graph_exec, c->stream));
            c->n += chunk;
            nsteps -= chunk;
            continue;
        }
        int k = (int)std::min<int64_t>(nsteps, chunk);
        if (c->n == 0) k = 1;   // repeat start: the first step on its own
        enqueue_stream_chunk<R>(c, k);
        HIP_TRY(c, hipGetLastError());
        c->n += k;
        nsteps -= k;
    }
    return DFHM_OK;
}

// ----------------------------------------------------------- resident path

struct Cand { int nt, npt; };
// launch shapes the library is built for (threads, nodes per lane)
const Cand kCands[] = {{256, 4}, {256, 2}, {128, 4}, {512, 2}, {128, 8}, {512, 4}, {256, 8}};

int effective_schedule(const dfhm_ctx *c)
{
    if (c->cfg.schedule != DFHM_SCHED_AUTO) return c->cfg.schedule;
    if (c->tuned) return c->tuned_sched;
    return c->shape_uniform ? DFHM_SCHED_RESIDENT : DFHM_SCHED_STREAM;
}

// Groups that must share a workgroup: a set of linked zones with all of
// their walls, or one wall without a zone (walls and zones ascending).
struct Group {
    std::vector<int32_t> walls, rooms;
};
void groups_of(const dfhm_ctx *c, std::vector<Group> &groups)
{
    groups.clear();
    std::vector<int64_t> root(c->nr);
    for (int64_t r = 0; r < c->nr; ++r) root[r] = r;
    auto find = [&](int64_t x) {
        while (root[x] != x) { root[x] = root[root[x]]; x = root[x]; }
        return x;
    };
    for (int64_t r = 0; r < (int64_t)c->zone_partners.size(); ++r)
        for (int32_t p : c->zone_partners[r]) {
            int64_t a = find(r), b = find(p);
            if (a != b) root[std::max(a, b)] = std::min(a, b);
        }
    std::vector<int64_t> gid(c->nr, -1);
    for (int64_t w = 0; w < c->nw; ++w) {
        int64_t r = c->wall_room[w];
        if (r < 0) { groups.push_back({{(int32_t)w}, {}}); continue; }
        int64_t z = find(r);
        if (gid[z] < 0) { gid[z] = (int64_t)groups.size(); groups.push_back({}); }
        groups[gid[z]].walls.push_back((int32_t)w);
    }
    for (int64_t r = 0; r < c->nr; ++r) groups[gid[find(r)]].rooms.push_back((int32_t)r);
}

// LDS of a resident workgroup of this context with mw walls and mr zones.
size_t res_lds(const dfhm_ctx *c, int nt, int npt, int mw, int mr)
{
    const bool ext = c->extended;
    const int law = c->cfg.law == DFHM_LAW_TABLE1;
    return c->precision == DFHM_FP32 ? res_lds_bytes<float>(nt, npt, mw, mr, ext, law)
                                     : res_lds_bytes<double>(nt, npt, mw, mr, ext, law);
}

// The LDS one workgroup may take so that LDS does not cut the number of
// resident workgroups below what the register budget allows.  Every
// workgroup of a launch gets the LDS of the launch's largest one (records for
// its wall and zone counts), so one crowded workgroup would set the
// occupancy of all: a batch with many small walls packs up to 54 walls into
// a 2048-node workgroup, 84 KB of FP64 tables against the 80 KB that two
// workgroups per CU leave.  Batches that do not fill every CU once are not
// limited (their workgroups do not share CUs).
size_t res_lds_budget(const dfhm_ctx *c, int nt, int npt)
{
    int dev = 0, ncu = 0, lds_cu = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) !=
            hipSuccess || ncu <= 0 || lds_cu <= 0)
        return SIZE_MAX;
    if (c->N <= (int64_t)ncu * nt * npt) return SIZE_MAX;
    const int waves = res_waves(c->precision == DFHM_FP32 ? 4 : 8, npt, nt);
    const int wg_per_cu = std::max(1, waves * 4 / std::max(1, nt / 64));
    return (size_t)lds_cu / (size_t)wg_per_cu;
}

dfhm_status pack(dfhm_ctx *c, int nt, int npt)
{
    const int cap = nt * npt;
    const size_t lds_budget = res_lds_budget(c, nt, npt);
    int wcap = kResMaxWalls;   // walls per workgroup within the LDS budget
    while (wcap > 1 && res_lds(c, nt, npt, wcap, 1) > lds_budget) --wcap;
    std::vector<Group> groups;
    groups_of(c, groups);
    std::vector<int> gsize(groups.size());
    for (size_t g = 0; g < groups.size(); ++g) {
        int s = 0;
        for (int32_t w : groups[g].walls) s += c->walls[w].nx;
        gsize[g] = s;
        if (s > cap)
            return fail(c, DFHM_E_INVAL, "a wall or zone group of " + std::to_string(s) +
                                             " nodes exceeds the workgroup capacity " + std::to_string(cap));
        if ((int)groups[g].walls.size() > kResMaxWalls)
            return fail(c, DFHM_E_INVAL, "a zone group has more walls than a workgroup holds");
        if ((int)groups[g].rooms.size() > kResMaxRooms)
            return fail(c, DFHM_E_INVAL, "a set of linked zones has more zones than a workgroup holds");
        for (int32_t r : groups[g].rooms)
            if ((int)c->zone_partners[r].size() > kResMaxLinks)
                return fail(c, DFHM_E_INVAL, "zone " + std::to_string(r) + " has more than " +
                                                 std::to_string(kResMaxLinks) +
                                                 " links (resident schedule)");
    }
    std::vector<int> order(groups.size());
    for (size_t g = 0; g < order.size(); ++g) order[g] = (int)g;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return gsize[a] > gsize[b]; });
    // best-fit decreasing: smallest remaining capacity that still fits
    struct Bin { int used, walls, rooms; std::vector<int> gs; };
    std::vector<Bin> bins;
    std::multimap<int, int> free_cap;   // remaining -> bin
    for (int g : order) {
        const int need = gsize[g];
        const int gw = (int)groups[g].walls.size();
        const int gr = (int)groups[g].rooms.size();
        int chosen = -1;
        for (auto it = free_cap.lower_bound(need); it != free_cap.end(); ++it) {
            Bin &b = bins[it->second];
            if (b.walls + gw <= wcap && b.rooms + gr <= kResMaxRooms &&
                (gr == 0 || res_lds(c, nt, npt, b.walls + gw, b.rooms + gr) <= lds_budget)) {
                chosen = it->second;
                free_cap.erase(it);
                break;
            }
        }
        if (chosen < 0) {
            chosen = (int)bins.size();
            bins.push_back({0, 0, 0, {}});
        }
        Bin &b = bins[chosen];
        b.used += need;
        b.walls += gw;
        b.rooms += gr;
        b.gs.push_back(g);
        // a bin at its wall limit takes nothing more (every group has a wall)
        if (cap - b.used > 0 && b.walls < wcap) free_cap.emplace(cap - b.used, chosen);
    }
    std::vector<ResBlock> blocks(bins.size());
    std::vector<ResSlot> bw;
    std::vector<int32_t> br;
    int maxw = 0, maxr = 0;
    for (size_t i = 0; i < bins.size(); ++i) {
        std::vector<int32_t> ws;
        std::vector<int32_t> rs;
        for (int g : bins[i].gs) {
            for (int32_t w : groups[g].walls) ws.push_back(w);
            for (int32_t r : groups[g].rooms) rs.push_back(r);
        }
        std::sort(ws.begin(), ws.end());
        std::sort(rs.begin(), rs.end());
        ResBlock &B = blocks[i];
        B.w_begin = (int32_t)bw.size();
        int32_t at = 0;
        for (int32_t w : ws) {
            const int32_t nx = c->walls[w].nx;
            bw.push_back({w, at, at + nx, c->walls[w].off});
            at += nx;
        }
        B.w_end = (int32_t)bw.size();
        B.r_begin = (int32_t)br.size();
        br.insert(br.end(), rs.begin(), rs.end());
        B.r_end = (int32_t)br.size();
        B.n_nodes = bins[i].used;
        B.pad = 0;
        maxw = std::max(maxw, (int)ws.size());
        maxr = std::max(maxr, (int)rs.size());
    }
    if (br.empty()) br.push_back(0);
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
    size_t ob = take(sizeof(ResBlock) * blocks.size());
    size_t ow = take(sizeof(ResSlot) * bw.size());
    size_t orr = take(sizeof(int32_t) * br.size());
    size_t oio = take(sizeof(ResIO));
    if (c->pack_mem) { (void)hipStreamSynchronize(c->stream); (void)hipFree(c->pack_mem); c->pack_mem = nullptr; }
    void *mem = nullptr;
    if (hipMalloc(&mem, o) != hipSuccess) return fail(c, DFHM_E_NOMEM, "packing tables");
    c->pack_mem = mem;
    c->d_blocks = (ResBlock *)((char *)mem + ob);
    c->d_slots = (ResSlot *)((char *)mem + ow);
    c->d_block_rooms = (int32_t *)((char *)mem + orr);
    c->d_io = (ResIO *)((char *)mem + oio);
    c->io_valid = false;
    HIP_TRY(c, hipMemcpyAsync(c->d_blocks, blocks.data(), sizeof(ResBlock) * blocks.size(), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->d_slots, bw.data(), sizeof(ResSlot) * bw.size(), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->d_block_rooms, br.data(), sizeof(int32_t) * br.size(), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->n_blocks = (int)blocks.size();
    c->max_wpb = maxw;
    c->max_rpb = maxr;
    c->pack_eff = (double)c->N / ((double)blocks.size() * cap);
    c->res_threads = nt;
    c->res_npt = npt;
    c->packed = true;
    return DFHM_OK;
}

int max_group(const dfhm_ctx *c)
{
    std::vector<Group> groups;
    groups_of(c, groups);
    int m = 0;
    for (auto &g : groups) {
        int s = 0;
        for (int32_t w : g.walls) s += c->walls[w].nx;
        m = std::max(m, s);
    }
    return m;
}

// Default launch shape: the first candidate whose capacity holds the largest
// group (nodes per lane >= 2 keeps the halo exchange small).
Cand default_shape(const dfhm_ctx *c)
{
    int need = max_group(c);
    for (const Cand &k : kCands)
        if (k.nt * k.npt >= need) return k;
    return {256, 8};
}

dfhm_status ensure_packing(dfhm_ctx *c)
{
    if (!c->shape_uniform)
        return fail(c, DFHM_E_INVAL, "the resident schedule needs one law shape for all walls");
    int nt = c->res_threads, npt = c->res_npt;
    if (c->cfg.block_threads > 0 && c->cfg.nodes_per_thread > 0) {
        nt = c->cfg.block_threads;
        npt = c->cfg.nodes_per_thread;
    } else if (!nt || !npt) {
        Cand k = default_shape(c);
        nt = k.nt;
        npt = k.npt;
    }
    bool known = false;
    for (const Cand &k : kCands) known |= (k.nt == nt && k.npt == npt);
    if (!known) return fail(c, DFHM_E_INVAL, "unsupported resident launch shape");
    if (c->packed && c->res_threads == nt && c->res_npt == npt) return DFHM_OK;
    return pack(c, nt, npt);
}

// The resident kernel reads its write-back pointers from device memory;
// refresh them when the level buffers or the zone arrays have moved.
void refresh_io(dfhm_ctx *c)
{
    ResIO io{};
    io.T[0] = c->d_T[0]; io.T[1] = c->d_T[1];
    io.P[0] = c->d_P[0]; io.P[1] = c->d_P[1];
    io.flux = c->d_flux;
    io.roomT = c->d_roomT;
    io.roomP = c->d_roomP;
    io.bad = c->d_bad;
    if (c->io_valid && std::memcmp(&io, &c->io_host, sizeof io) == 0) return;
    c->io_host = io;
    (void)hipMemcpyAsync(c->d_io, &c->io_host, sizeof io, hipMemcpyHostToDevice, c->stream);
    c->io_valid = true;
}

template <typename R, int NPT, int NT, int MODE, int LAW>
void launch_res(dfhm_ctx *c, int k)
{
    refresh_io(c);
    // the largest tables need more than 64 KB of LDS; set on every launch (a
    // host-side call, once per chunk), so that every device the library runs
    // on and every thread sees it
    (void)hipFuncSetAttribute((const void *)k_df_resident<R, NPT, NT, MODE, LAW>,
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)res_lds_bytes<R>(NT, NPT, kResMaxWalls, kResMaxRooms,
                                                    MODE == kModeExt, LAW));
    // LDS records sized by the largest wall / zone count of a workgroup of
    // this packing (at least one of each)
    const int mw = std::max(1, c->max_wpb), mr = std::max(1, c->max_rpb);
    hipLaunchKernelGGL((k_df_resident<R, NPT, NT, MODE, LAW>), dim3(c->n_blocks), dim3(NT),
                       res_lds_bytes<R>(NT, NPT, mw, mr, MODE == kModeExt, LAW), c->stream, c->d_blocks,
                       c->d_slots,
                       c->d_block_rooms, c->d_walls, (const R *)c->d_T[0], (const R *)c->d_T[1],
                       (const R *)c->d_P[0], (const R *)c->d_P[1], c->d_lay, c->d_rooms,
                       c->d_roomT, c->d_roomP, c->d_go, c->d_qh, c->d_flux, c->d_step, c->d_io,
                       c->d_links, k, mw, c->rc, c->shape);
}

template <typename R>
void launch_resident(dfhm_ctx *c, int k)
{
    const int nt = c->res_threads, npt = c->res_npt;
    // zones and radiative sources / links compile into variants of their
    // own, so that runs without them keep the leaner step loop
    const int mode = c->extended ? kModeExt : (c->nr > 0 ? kModeZones : kModePlain);
#define DFHM_RES_LAW(T_, P_, L_)                                                     \
    {                                                                                \
        if (mode == kModeExt) launch_res<R, P_, T_, kModeExt, L_>(c, k);             \
        else if (mode == kModeZones) launch_res<R, P_, T_, kModeZones, L_>(c, k);    \
        else launch_res<R, P_, T_, kModePlain, L_>(c, k);                            \
    }
#define DFHM_RES_CASE(T_, P_)                                                        \
    if (nt == T_ && npt == P_) {                                                     \
        if (c->cfg.law == DFHM_LAW_TABLE1) DFHM_RES_LAW(T_, P_, 1)                   \
        else DFHM_RES_LAW(T_, P_, 0)                                                 \
        return;                                                                      \
    }
    DFHM_RES_CASE(256, 4) DFHM_RES_CASE(128, 8) DFHM_RES_CASE(256, 2) DFHM_RES_CASE(512, 2)
    DFHM_RES_CASE(128, 4) DFHM_RES_CASE(512, 4) DFHM_RES_CASE(256, 8)
#undef DFHM_RES_CASE
#undef DFHM_RES_LAW
}

template <typename R>
dfhm_status step_resident(dfhm_ctx *c, int64_t nsteps)
{
    while (nsteps > 0) {
        if (c->n == 0 && c->cfg.startup == DFHM_START_FTCS) {
            launch_startup<R>(c);
            launch_room_step<R>(c, 0);
            tick(c, 1);
            HIP_TRY(c, hipGetLastError());
            c->n += 1;
            nsteps -= 1;
            continue;
        }
        dfhm_status st = ensure_packing(c);
        if (st) return st;
        const int chunk = c->cfg.chunk_steps > 0 ? c->cfg.chunk_steps : 1000;
        const int k = (int)std::min<int64_t>(nsteps, chunk);
        launch_resident<R>(c, k);
        tick(c, k);
        HIP_TRY(c, hipGetLastError());
        c->n += k;
        nsteps -= k;
    }
    return DFHM_OK;
}

bool shape_of(const dfhm_wall *w, int64_t nw, Shape &sh)
{
    const dfhm_layer &m0 = w[0].layer[0];
    sh = {m0.a_T, m0.a_M, m0.b_TM, m0.c_T, m0.c_M, m0.e_TM, m0.f_TM};
    for (int64_t i = 0; i < nw; ++i)
        for (int l = 0; l < w[i].n_layers; ++l) {
            const dfhm_layer &m = w[i].layer[l];
            if (m.a_T != sh.aT || m.a_M != sh.aM || m.b_TM != sh.bTM || m.c_T != sh.cT ||
                m.c_M != sh.aC || m.e_TM != sh.eTM || m.f_TM != sh.fTM)
                return false;
        }
    return true;
}

} // namespace

// ===================================================================== API

extern "C" {

const char *dfhm_status_string(dfhm_status s)
{
    switch (s) {
    case DFHM_OK: return "ok";
    case DFHM_E_INVAL: return "invalid argument";
    case DFHM_E_NOMEM: return "out of device memory";
    case DFHM_E_DEVICE: return "device error";
    case DFHM_E_NONFINITE: return "non-finite state";
    case DFHM_E_STATE: return "invalid state";
    case DFHM_E_UNSTABLE: return "unstable explicit zone step";
    }
    return "unknown";
}

size_t dfhm_arena_bytes(const dfhm_config *cfg, const dfhm_wall *walls, int64_t n_walls)
{
    if (!cfg || !walls || n_walls < 1) return 0;
    return layout_of(cfg->precision, walls, n_walls).total;
}

dfhm_status dfhm_create(const dfhm_config *cfg, const dfhm_wall *walls, int64_t n_walls,
                        void *arena, size_t arena_bytes, dfhm_ctx **out)
{
    if (!out) return DFHM_E_INVAL;
    *out = nullptr;
    if (!cfg || !walls || n_walls < 1) return DFHM_E_INVAL;
    if (!(std::isfinite(cfg->dt_s) && cfg->dt_s > 0.0)) return DFHM_E_INVAL;
    if (cfg->precision != DFHM_FP64 && cfg->precision != DFHM_FP32) return DFHM_E_INVAL;
    if (cfg->startup != DFHM_START_FTCS && cfg->startup != DFHM_START_REPEAT) return DFHM_E_INVAL;
    if (cfg->schedule < DFHM_SCHED_AUTO || cfg->schedule > DFHM_SCHED_RESIDENT) return DFHM_E_INVAL;
    if (cfg->chunk_steps < 0 || cfg->block_threads < 0 || cfg->nodes_per_thread < 0) return DFHM_E_INVAL;
    if (cfg->law != DFHM_LAW_SHAPE && cfg->law != DFHM_LAW_TABLE1) return DFHM_E_INVAL;
    int64_t N = 0;
    for (int64_t i = 0; i < n_walls; ++i) {
        if (!check_wall(walls[i], i).empty()) return DFHM_E_INVAL;
        N += walls[i].nx;
    }
    if (N >= (int64_t(1) << 31)) return DFHM_E_INVAL;
    Layout L = layout_of(cfg->precision, walls, n_walls);
    if (arena && arena_bytes < L.total) return DFHM_E_NOMEM;

    dfhm_ctx *c = new (std::nothrow) dfhm_ctx();
    if (!c) return DFHM_E_NOMEM;
    c->cfg = *cfg;
    c->precision = cfg->precision;
    c->esize = cfg->precision == DFHM_FP32 ? 4 : 8;
    c->stream = (hipStream_t)cfg->stream;
    c->nw = n_walls;
    c->N = N;
    c->rc.dt = cfg->dt_s;
    c->rc.Lv = orz(cfg->Lv, 2.5e6);
    c->rc.cw = orz(cfg->cw, 4180.0);
    c->rc.rho_a = orz(cfg->rho_a, 1.2);
    c->rc.c_pa = orz(cfg->c_pa, 1006.0);
    c->rc.c_pv = orz(cfg->c_pv, 1860.0);
    c->rc.Pv_ref = orz(cfg->Pv_ref, 1.61e5);
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; return DFHM_E_DEVICE; }

    if (arena) {
        c->arena = arena;
        c->arena_bytes = arena_bytes;
    } else {
        if (hipMalloc(&c->arena, L.total) != hipSuccess) { delete c; return DFHM_E_NOMEM; }
        c->own_arena = true;
        c->arena_bytes = L.total;
    }
    char *base = (char *)c->arena;
    c->d_walls = (WallDev *)(base + L.walls);
    c->d_tiles = (int2 *)(base + L.tiles);
    c->d_T[0] = base + L.T0; c->d_T[1] = base + L.T1;
    c->d_P[0] = base + L.P0; c->d_P[1] = base + L.P1;
    c->d_lay = (uint8_t *)(base + L.lay);
    c->d_flux = (double *)(base + L.flux);
    c->d_bad = (int *)(base + L.bad);
    c->d_step = (int64_t *)(base + L.step);

    c->walls.resize(n_walls);
    std::vector<int2> tiles;
    tiles.reserve(count_tiles(walls, n_walls));
    int32_t off = 0;
    for (int64_t i = 0; i < n_walls; ++i) {
        fill_wall(c->walls[i], walls[i], off);
        for (int sd = 0; sd < 2; ++sd)    // can the clipped incident flux be nonzero?
            if (walls[i].q_sun[sd].mean + std::fabs(walls[i].q_sun[sd].amp) > 0.0) c->extended = true;
        for (int j0 = 0; j0 < walls[i].nx; j0 += kStreamTile) tiles.push_back(make_int2((int)i, j0));
        off += walls[i].nx;
    }
    c->ntiles = (int)tiles.size();
    c->wall_room.assign(n_walls, -1);
    c->room_side.assign(n_walls, 1);
    // the resident kernel needs one shape for the shape law (the Table 1 law
    // has a fixed one)
    c->shape_uniform = cfg->law == DFHM_LAW_TABLE1 || shape_of(walls, n_walls, c->shape);
    if (cfg->schedule == DFHM_SCHED_RESIDENT && !c->shape_uniform) {
        delete c;
        return DFHM_E_INVAL;
    }

    auto bail = [&](dfhm_status s) {
        dfhm_destroy(c);
        return s;
    };
    std::vector<double> zeros(12 * n_walls, 0.0);
    int zero = 0;
    int64_t zero64 = 0;
    if (hipMemcpyAsync(c->d_walls, c->walls.data(), sizeof(WallDev) * n_walls,
                       hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(c->d_tiles, tiles.data(), sizeof(int2) * tiles.size(),
                       hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(c->d_flux, zeros.data(), sizeof(double) * zeros.size(),
                       hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(c->d_bad, &zero, sizeof(int), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(c->d_step, &zero64, sizeof(int64_t), hipMemcpyHostToDevice, c->stream) != hipSuccess)
        return bail(DFHM_E_DEVICE);
    hipLaunchKernelGGL(k_init_walls, dim3((unsigned)((n_walls + 63) / 64)), dim3(64), 0, c->stream,
                       c->d_walls, (int)n_walls, c->rc.dt);
    if (c->precision == DFHM_FP64)
        hipLaunchKernelGGL(k_init_nodes<double>, dim3(c->ntiles), dim3(kStreamBlock), 0, c->stream,
                           c->d_walls, c->d_tiles, c->d_lay, (double *)c->d_T[0], (double *)c->d_T[1],
                           (double *)c->d_P[0], (double *)c->d_P[1]);
    else
        hipLaunchKernelGGL(k_init_nodes<float>, dim3(c->ntiles), dim3(kStreamBlock), 0, c->stream,
                           c->d_walls, c->d_tiles, c->d_lay, (float *)c->d_T[0], (float *)c->d_T[1],
                           (float *)c->d_P[0], (float *)c->d_P[1]);
    if (hipGetLastError() != hipSuccess) return bail(DFHM_E_DEVICE);
    // keep the device-computed grid constants and initial vapour pressure
    if (hipMemcpyAsync(c->walls.data(), c->d_walls, sizeof(WallDev) * n_walls,
                       hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return bail(DFHM_E_DEVICE);
    *out = c;
    return DFHM_OK;
}

namespace {
// Forward Euler of zone r is stable and monotone when a dt < 1 for both
// fields, a = (sum of its exchange conductances) / (its capacity).
dfhm_status zone_stable(dfhm_ctx *c, int64_t r, double sT = -1.0, double sM = -1.0)
{
    if (sT < 0.0) sT = c->zone_sT[r];
    if (sM < 0.0) sM = c->zone_sM[r];
    const RunConst &rc = c->rc;
    const double aT = sT / (c->zone_mass[r] * c->zone_cma[r]);
    const double aM = sM / (c->zone_mass[r] / rc.Pv_ref);
    if (!(aT * rc.dt < 1.0) || !(aM * rc.dt < 1.0)) {
        char b[200];
        snprintf(b, sizeof b, "zone %lld: explicit step unstable (a_T dt = %.3g, a_M dt = %.3g)",
                 (long long)r, aT * rc.dt, aM * rc.dt);
        return fail(c, DFHM_E_UNSTABLE, b);
    }
    return DFHM_OK;
}
} // namespace

dfhm_status dfhm_room_couple(dfhm_ctx *c, const dfhm_room *rooms, int64_t n_rooms,
                             const int64_t *wall_room, const int8_t *room_side)
{
    if (!c) return DFHM_E_INVAL;
    if (c->n != 0 || c->nr != 0) return fail(c, DFHM_E_STATE, "zones must be coupled once, at step 0");
    if (!rooms || n_rooms < 1 || !wall_room || !room_side)
        return fail(c, DFHM_E_INVAL, "rooms, wall_room and room_side are required");
    for (int64_t w = 0; w < c->nw; ++w) {
        if (wall_room[w] < -1 || wall_room[w] >= n_rooms)
            return fail(c, DFHM_E_INVAL, "wall_room index out of range");
        if (wall_room[w] >= 0 && room_side[w] != 0 && room_side[w] != 1)
            return fail(c, DFHM_E_INVAL, "room_side must be 0 or 1");
    }
    int64_t total_sched = 0;
    for (int64_t r = 0; r < n_rooms; ++r) {
        const dfhm_room &m = rooms[r];
        if (!(m.volume_m3 > 0.0) || !(m.ach_per_h >= 0.0) || !(m.T0 > 0.0) || !(m.RH0 > 0.0) ||
            m.n_sched < 1 || !(m.sched_dt_s > 0.0) || !m.g_o_kg_s || !m.Q_h_W ||
            !(m.T_out.period_s > 0.0) || !(m.RH_out.period_s > 0.0) ||
            !(m.view_factor >= 0.0 && m.view_factor <= 1.0))
            return fail(c, DFHM_E_INVAL, "bad zone descriptor " + std::to_string(r));
        total_sched += m.n_sched;
    }
    // room -> walls lists in ascending wall order
    std::vector<std::vector<int32_t>> lists(n_rooms);
    for (int64_t w = 0; w < c->nw; ++w)
        if (wall_room[w] >= 0) lists[wall_room[w]].push_back((int32_t)w);
    for (int64_t r = 0; r < n_rooms; ++r)
        if (lists[r].empty()) return fail(c, DFHM_E_INVAL, "zone " + std::to_string(r) + " has no wall");
    // explicit zone step stability (forward Euler): a dt < 1 for both fields
    const RunConst &rc = c->rc;
    c->zone_mass.assign(n_rooms, 0.0);
    c->zone_cma.assign(n_rooms, 0.0);
    c->zone_sT.assign(n_rooms, 0.0);
    c->zone_sM.assign(n_rooms, 0.0);
    for (int64_t r = 0; r < n_rooms; ++r) {
        const dfhm_room &m = rooms[r];
        double mass = rc.rho_a * m.volume_m3;
        double gv = m.ach_per_h * mass / 3600.0;
        double Pa0 = m.RH0 * 610.94 * std::exp(17.625 * (m.T0 - 273.15) / (m.T0 - 273.15 + 243.04));
        double cma = rc.c_pa + rc.c_pv * Pa0 / rc.Pv_ref;
        double sT = gv * cma, sM = gv / rc.Pv_ref;
        for (int32_t w : lists[r]) {
            const WallDev &W = c->walls[w];
            int side = room_side[w];
            sT += W.area * W.hT[side];
            sM += W.area * W.hM[side];
        }
        c->zone_mass[r] = mass; c->zone_cma[r] = cma; c->zone_sT[r] = sT; c->zone_sM[r] = sM;
        dfhm_status st = zone_stable(c, r);
        if (st) return st;
    }
    std::vector<RoomDev> rd(n_rooms);
    std::vector<int32_t> rw;
    std::vector<double> go(total_sched), qh(total_sched), Ta(n_rooms), Pa(n_rooms);
    int32_t so = 0;
    for (int64_t r = 0; r < n_rooms; ++r) {
        const dfhm_room &m = rooms[r];
        RoomDev &d = rd[r];
        std::memset(&d, 0, sizeof d);
        d.volume = m.volume_m3; d.ach = m.ach_per_h; d.T0 = m.T0; d.RH0 = m.RH0;
        d.Tout[0] = m.T_out.mean; d.Tout[1] = m.T_out.amp; d.Tout[2] = m.T_out.period_s; d.Tout[3] = m.T_out.phase;
        d.RHout[0] = m.RH_out.mean; d.RHout[1] = m.RH_out.amp; d.RHout[2] = m.RH_out.period_s; d.RHout[3] = m.RH_out.phase;
        d.sched_dt = m.sched_dt_s;
        d.n_sched = m.n_sched;
        d.sched_off = so;
        std::memcpy(&go[so], m.g_o_kg_s, sizeof(double) * m.n_sched);
        std::memcpy(&qh[so], m.Q_h_W, sizeof(double) * m.n_sched);
        so += m.n_sched;
        d.w_begin = (int32_t)rw.size();
        for (int32_t w : lists[r]) rw.push_back(w);
        d.w_end = (int32_t)rw.size();
        d.view = m.view_factor;
        d.l_begin = d.l_end = 0;
        Ta[r] = m.T0;
        Pa[r] = m.RH0;   // converted to Pv on the device
    }
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
    size_t o_rooms = take(sizeof(RoomDev) * n_rooms);
    size_t o_rw = take(sizeof(int32_t) * std::max<size_t>(rw.size(), 1));
    size_t o_T = take(sizeof(double) * n_rooms);
    size_t o_P = take(sizeof(double) * n_rooms);
    size_t o_go = take(sizeof(double) * total_sched);
    size_t o_qh = take(sizeof(double) * total_sched);
    void *mem = nullptr;
    if (hipMalloc(&mem, o) != hipSuccess) return fail(c, DFHM_E_NOMEM, "zone buffers");
    char *b = (char *)mem;
    c->room_mem = mem;
    c->d_rooms = (RoomDev *)(b + o_rooms);
    c->d_room_walls = (int32_t *)(b + o_rw);
    c->d_roomT = (double *)(b + o_T);
    c->d_roomP = (double *)(b + o_P);
    c->d_go = (double *)(b + o_go);
    c->d_qh = (double *)(b + o_qh);
    for (int64_t w = 0; w < c->nw; ++w) {
        c->wall_room[w] = wall_room[w];
        c->room_side[w] = wall_room[w] >= 0 ? room_side[w] : 1;
        c->walls[w].room = (int32_t)wall_room[w];
        c->walls[w].room_side = c->room_side[w];
        if (wall_room[w] >= 0) {
            // long-wave exchange factor of the zone side: s eps sigma
            const int64_t r = wall_room[w];
            c->walls[w].esig = rooms[r].view_factor * c->walls[w].emis[c->room_side[w]] * kSigma;
            c->walls[w].room_walls = (int32_t)lists[r].size();
            if (c->walls[w].esig != 0.0) c->extended = true;
        }
    }
    HIP_TRY(c, hipMemcpyAsync(c->d_rooms, rd.data(), sizeof(RoomDev) * n_rooms, hipMemcpyHostToDevice, c->stream));
    if (!rw.empty())
        HIP_TRY(c, hipMemcpyAsync(c->d_room_walls, rw.data(), sizeof(int32_t) * rw.size(), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->d_roomT, Ta.data(), sizeof(double) * n_rooms, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->d_roomP, Pa.data(), sizeof(double) * n_rooms, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->d_go, go.data(), sizeof(double) * total_sched, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->d_qh, qh.data(), sizeof(double) * total_sched, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->d_walls, c->walls.data(), sizeof(WallDev) * c->nw, hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_init_rooms, dim3((unsigned)((n_rooms + 63) / 64)), dim3(64), 0, c->stream,
                       c->d_rooms, c->d_roomP, (int)n_rooms);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->nr = n_rooms;
    c->rooms_host = rd;
    c->sched_go = go;
    c->sched_qh = qh;
    c->zone_partners.assign(n_rooms, {});
    c->packed = false;   // the resident packing must keep zones whole
    return DFHM_OK;
}

dfhm_status dfhm_zone_links(dfhm_ctx *c, const dfhm_zone_link *links, int64_t n_links)
{
    if (!c) return DFHM_E_INVAL;
    if (c->nr == 0) return fail(c, DFHM_E_INVAL, "no zones are coupled");
    if (c->n != 0 || c->n_links != 0) return fail(c, DFHM_E_STATE, "zones are linked once, at step 0");
    if (!links || n_links < 1) return fail(c, DFHM_E_INVAL, "links are required");
    for (int64_t l = 0; l < n_links; ++l) {
        const dfhm_zone_link &k = links[l];
        if (k.zone_a < 0 || k.zone_a >= c->nr || k.zone_b < 0 || k.zone_b >= c->nr ||
            k.zone_a == k.zone_b || !(std::isfinite(k.g_kg_s) && k.g_kg_s >= 0.0))
            return fail(c, DFHM_E_INVAL, "bad zone link " + std::to_string(l));
    }
    // stability with the link flows added to both zones (zone i loses
    // g c_i to its temperature and g / Pv_ref to its humidity ratio)
    std::vector<double> sT = c->zone_sT, sM = c->zone_sM;
    for (int64_t l = 0; l < n_links; ++l)
        for (int32_t z : {links[l].zone_a, links[l].zone_b}) {
            sT[z] += links[l].g_kg_s * c->zone_cma[z];
            sM[z] += links[l].g_kg_s / c->rc.Pv_ref;
        }
    for (int64_t r = 0; r < c->nr; ++r) {
        dfhm_status st = zone_stable(c, r, sT[r], sM[r]);
        if (st) return st;
    }
    // per receiving zone, in link order
    std::vector<std::vector<ZoneLinkDev>> per(c->nr);
    for (int64_t l = 0; l < n_links; ++l) {
        const dfhm_zone_link &k = links[l];
        per[k.zone_a].push_back({k.zone_b, 0, k.g_kg_s});
        per[k.zone_b].push_back({k.zone_a, 0, k.g_kg_s});
    }
    std::vector<ZoneLinkDev> flat;
    std::vector<RoomDev> rd = c->rooms_host;
    for (int64_t r = 0; r < c->nr; ++r) {
        rd[r].l_begin = (int32_t)flat.size();
        for (const ZoneLinkDev &d : per[r]) {
            flat.push_back(d);
            c->zone_partners[r].push_back(d.partner);
        }
        rd[r].l_end = (int32_t)flat.size();
    }
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
    size_t o_l = take(sizeof(ZoneLinkDev) * flat.size());
    size_t o_x = take(sizeof(double) * 2 * c->nr);
    void *mem = nullptr;
    if (hipMalloc(&mem, o) != hipSuccess) return fail(c, DFHM_E_NOMEM, "zone links");
    c->link_mem = mem;
    c->d_links = (ZoneLinkDev *)((char *)mem + o_l);
    c->d_inz = (double *)((char *)mem + o_x);
    HIP_TRY(c, hipMemcpyAsync(c->d_links, flat.data(), sizeof(ZoneLinkDev) * flat.size(), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->d_rooms, rd.data(), sizeof(RoomDev) * c->nr, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->rooms_host = rd;
    c->links_host = flat;
    c->n_links = n_links;
    c->extended = true;
    c->packed = false;   // linked zones share a workgroup
    return DFHM_OK;
}

dfhm_status dfhm_step_n(dfhm_ctx *c, int64_t nsteps)
{
    if (!c) return DFHM_E_INVAL;
    if (nsteps < 0) return fail(c, DFHM_E_INVAL, "negative step count");
    if (c->latched != DFHM_OK) return fail(c, DFHM_E_STATE, "context holds a non-finite state");
    if (nsteps == 0) return DFHM_OK;
    int sched = effective_schedule(c);
    if (sched == DFHM_SCHED_RESIDENT) {
        return c->precision == DFHM_FP64 ? step_resident<double>(c, nsteps)
                                          : step_resident<float>(c, nsteps);
    }
    return c->precision == DFHM_FP64 ? step_stream<double>(c, nsteps) : step_stream<float>(c, nsteps);
}

dfhm_status dfhm_sync(dfhm_ctx *c)
{
    if (!c) return DFHM_E_INVAL;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->latched != DFHM_OK) return fail(c, DFHM_E_STATE, "context holds a non-finite state");
    return check_bad(c);
}

dfhm_status dfhm_fluxes(dfhm_ctx *c, double *now, double *integral)
{
    if (!c) return DFHM_E_INVAL;
    std::vector<double> f(12 * c->nw);
    HIP_TRY(c, hipMemcpyAsync(f.data(), c->d_flux, sizeof(double) * f.size(), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int64_t w = 0; w < c->nw; ++w)
        for (int k = 0; k < 4; ++k) {
            if (now) now[4 * w + k] = f[12 * w + k];
            if (integral) integral[4 * w + k] = f[12 * w + 4 + k] + f[12 * w + 8 + k];
        }
    return DFHM_OK;
}

static dfhm_status copy_level(dfhm_ctx *c, int level, int64_t off, int64_t cnt, void *host)
{
    int b = (int)((c->n + (level == 0 ? 0 : 1)) & 1);
    char *T = (char *)c->d_T[b] + c->esize * off;
    char *P = (char *)c->d_P[b] + c->esize * off;
    HIP_TRY(c, hipMemcpyAsync(host, T, c->esize * cnt, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync((char *)host + c->esize * cnt, P, c->esize * cnt, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return DFHM_OK;
}

static void to_abs(const dfhm_ctx *c, const WallDev &W, const void *raw, int64_t cnt, int64_t at,
                   double *T, double *P)
{
    if (c->precision == DFHM_FP64) {
        const double *t = (const double *)raw;
        std::memcpy(T, t + at, sizeof(double) * W.nx);
        std::memcpy(P, t + cnt + at, sizeof(double) * W.nx);
    } else {
        const float *t = (const float *)raw;
        double pref = (double)(float)W.P0;
        for (int j = 0; j < W.nx; ++j) {
            T[j] = W.T0 + (double)t[at + j];
            P[j] = pref + (double)t[cnt + at + j];
        }
    }
}

dfhm_status dfhm_get_fields(dfhm_ctx *c, int64_t wall, int level, double *T, double *Pv)
{
    if (!c) return DFHM_E_INVAL;
    if (wall < 0 || wall >= c->nw || (level != 0 && level != 1) || !T || !Pv)
        return fail(c, DFHM_E_INVAL, "bad wall index, level or buffer");
    const WallDev &W = c->walls[wall];
    std::vector<char> raw(c->esize * 2 * W.nx);
    dfhm_status s = copy_level(c, level, W.off, W.nx, raw.data());
    if (s) return s;
    to_abs(c, W, raw.data(), W.nx, 0, T, Pv);
    return DFHM_OK;
}

dfhm_status dfhm_get_all_fields(dfhm_ctx *c, int level, double *T, double *Pv)
{
    if (!c) return DFHM_E_INVAL;
    if ((level != 0 && level != 1) || !T || !Pv) return fail(c, DFHM_E_INVAL, "bad level or buffer");
    std::vector<char> raw(c->esize * 2 * c->N);
    dfhm_status s = copy_level(c, level, 0, c->N, raw.data());
    if (s) return s;
    for (int64_t w = 0; w < c->nw; ++w) {
        const WallDev &W = c->walls[w];
        to_abs(c, W, raw.data(), c->N, W.off, T + W.off, Pv + W.off);
    }
    return DFHM_OK;
}

dfhm_status dfhm_set_fields(dfhm_ctx *c, int64_t wall, int level, const double *T, const double *Pv)
{
    if (!c) return DFHM_E_INVAL;
    if (wall < 0 || wall >= c->nw || (level != 0 && level != 1) || !T || !Pv)
        return fail(c, DFHM_E_INVAL, "bad wall index, level or buffer");
    const WallDev &W = c->walls[wall];
    for (int j = 0; j < W.nx; ++j)
        if (!std::isfinite(T[j]) || !std::isfinite(Pv[j]))
            return fail(c, DFHM_E_INVAL, "non-finite field value");
    int b = (int)((c->n + (level == 0 ? 0 : 1)) & 1);
    std::vector<char> raw(c->esize * 2 * W.nx);
    if (c->precision == DFHM_FP64) {
        std::memcpy(raw.data(), T, 8 * W.nx);
        std::memcpy(raw.data() + 8 * W.nx, Pv, 8 * W.nx);
    } else {
        float *t = (float *)raw.data();
        double pref = (double)(float)W.P0;
        for (int j = 0; j < W.nx; ++j) {
            t[j] = (float)(T[j] - W.T0);
            t[W.nx + j] = (float)(Pv[j] - pref);
        }
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy((char *)c->d_T[b] + c->esize * W.off, raw.data(), c->esize * W.nx, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy((char *)c->d_P[b] + c->esize * W.off, raw.data() + c->esize * W.nx, c->esize * W.nx, hipMemcpyHostToDevice));
    int zero = 0;
    HIP_TRY(c, hipMemcpy(c->d_bad, &zero, sizeof(int), hipMemcpyHostToDevice));
    c->latched = DFHM_OK;
    return DFHM_OK;
}

dfhm_status dfhm_set_step_index(dfhm_ctx *c, int64_t n)
{
    if (!c) return DFHM_E_INVAL;
    if (n < 0) return fail(c, DFHM_E_INVAL, "negative step index");
    // level buffers follow the parity of n: move data if the parity changes
    if ((n & 1) != (c->n & 1)) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        std::swap(c->d_T[0], c->d_T[1]);
        std::swap(c->d_P[0], c->d_P[1]);
        if (c->graph_exec) { (void)hipGraphExecDestroy(c->graph_exec); c->graph_exec = nullptr; }
        if (c->graph) { (void)hipGraphDestroy(c->graph); c->graph = nullptr; }
    }
    HIP_TRY(c, hipMemcpy(c->d_step, &n, sizeof(int64_t), hipMemcpyHostToDevice));
    c->n = n;
    return DFHM_OK;
}

dfhm_status dfhm_get_rooms(dfhm_ctx *c, double *Ta, double *Pva)
{
    if (!c) return DFHM_E_INVAL;
    if (c->nr == 0) return fail(c, DFHM_E_STATE, "no zones coupled");
    if (!Ta || !Pva) return fail(c, DFHM_E_INVAL, "null buffer");
    HIP_TRY(c, hipMemcpyAsync(Ta, c->d_roomT, sizeof(double) * c->nr, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(Pva, c->d_roomP, sizeof(double) * c->nr, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return DFHM_OK;
}

dfhm_status dfhm_get_info(const dfhm_ctx *c, dfhm_info *info)
{
    if (!c || !info) return DFHM_E_INVAL;
    std::memset(info, 0, sizeof *info);
    int sched = effective_schedule(c);
    info->schedule = sched;
    info->precision = c->precision;
    info->block_threads = sched == DFHM_SCHED_RESIDENT ? c->res_threads : kStreamBlock;
    info->nodes_per_thread = sched == DFHM_SCHED_RESIDENT ? c->res_npt : 1;
    info->chunk_steps = c->cfg.chunk_steps > 0 ? c->cfg.chunk_steps
                                               : (sched == DFHM_SCHED_RESIDENT ? 1000 : 100);
    info->n_blocks = sched == DFHM_SCHED_RESIDENT ? c->n_blocks : c->ntiles;
    info->max_walls_per_block = c->max_wpb;
    info->max_rooms_per_block = c->max_rpb;
    info->reserved = 0;
    info->n_links = c->n_links;
    info->use_graph = c->cfg.use_graph;
    info->n_walls = c->nw;
    info->n_rooms = c->nr;
    info->total_nodes = c->N;
    info->step_index = c->n;
    info->pack_efficiency = c->pack_eff;
    return DFHM_OK;
}

// ------------------------------------------------------ implicit comparator

struct dfhm_implicit {
    dfhm_implicit_config cfg{};
    hipStream_t stream = nullptr;
    int64_t nw = 0, n = 0, slots = 0;
    int ngroups = 0;
    std::vector<WallDev> walls;
    std::vector<ImpGroup> groups;
    void *mem = nullptr;
    WallDev *d_walls = nullptr;
    ImpGroup *d_groups = nullptr;
    ImpArrays A{};
    int64_t *d_iters = nullptr;
    std::string err;
};

dfhm_status dfhm_implicit_create(const dfhm_implicit_config *cfg, const dfhm_wall *walls,
                                 int64_t n_walls, dfhm_implicit **out)
{
    if (!out) return DFHM_E_INVAL;
    *out = nullptr;
    if (!cfg || !walls || n_walls < 1) return DFHM_E_INVAL;
    if (!(std::isfinite(cfg->dt_s) && cfg->dt_s > 0.0) || !(cfg->theta >= 0.5 && cfg->theta <= 1.0) ||
        !(cfg->eta > 0.0) || cfg->max_iters < 1 ||
        (cfg->law != DFHM_LAW_SHAPE && cfg->law != DFHM_LAW_TABLE1))
        return DFHM_E_INVAL;
    for (int64_t i = 0; i < n_walls; ++i)
        if (!check_wall(walls[i], i).empty()) return DFHM_E_INVAL;
    dfhm_implicit *ic = new (std::nothrow) dfhm_implicit();
    if (!ic) return DFHM_E_NOMEM;
    ic->cfg = *cfg;
    ic->cfg.Lv = orz(cfg->Lv, 2.5e6);
    ic->cfg.cw = orz(cfg->cw, 4180.0);
    ic->stream = (hipStream_t)cfg->stream;
    ic->nw = n_walls;
    ic->walls.resize(n_walls);
    for (int64_t i = 0; i < n_walls; ++i) fill_wall(ic->walls[i], walls[i], 0);
    // groups of 32 consecutive walls (one wave, two lanes per wall), each a
    // node-major block padded to its longest wall
    int64_t base = 0;
    for (int64_t w0 = 0; w0 < n_walls; w0 += kImpWalls) {
        ImpGroup g;
        g.base = base;
        g.w0 = (int32_t)w0;
        g.nw = (int32_t)std::min<int64_t>(kImpWalls, n_walls - w0);
        int maxnx = 0;
        for (int k = 0; k < g.nw; ++k) maxnx = std::max(maxnx, (int)walls[w0 + k].nx);
        base += (int64_t)maxnx * kImpWalls;
        ic->groups.push_back(g);
    }
    ic->slots = base;
    ic->ngroups = (int)ic->groups.size();
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
    const size_t ow = take(sizeof(WallDev) * n_walls), og = take(sizeof(ImpGroup) * ic->ngroups);
    size_t oa[7];
    for (int k = 0; k < 7; ++k) oa[k] = take(sizeof(double) * (size_t)base);
    const size_t oi = take(sizeof(int64_t) * n_walls);
    if (hipMalloc(&ic->mem, o) != hipSuccess) { delete ic; return DFHM_E_NOMEM; }
    char *m = (char *)ic->mem;
    ic->d_walls = (WallDev *)(m + ow);
    ic->d_groups = (ImpGroup *)(m + og);
    ic->A.T[0] = (double *)(m + oa[0]); ic->A.T[1] = (double *)(m + oa[1]);
    ic->A.P[0] = (double *)(m + oa[2]); ic->A.P[1] = (double *)(m + oa[3]);
    ic->A.Pn = (double *)(m + oa[4]); ic->A.cp = (double *)(m + oa[5]); ic->A.dp = (double *)(m + oa[6]);
    ic->d_iters = (int64_t *)(m + oi);
    auto bail = [&]() { dfhm_implicit_destroy(ic); return DFHM_E_DEVICE; };
    if (hipMemcpyAsync(ic->d_walls, ic->walls.data(), sizeof(WallDev) * n_walls, hipMemcpyHostToDevice, ic->stream) != hipSuccess ||
        hipMemcpyAsync(ic->d_groups, ic->groups.data(), sizeof(ImpGroup) * ic->ngroups, hipMemcpyHostToDevice, ic->stream) != hipSuccess ||
        hipMemsetAsync(ic->d_iters, 0, sizeof(int64_t) * n_walls, ic->stream) != hipSuccess)
        return bail();
    hipLaunchKernelGGL(k_init_walls, dim3((unsigned)((n_walls + 63) / 64)), dim3(64), 0, ic->stream,
                       ic->d_walls, (int)n_walls, cfg->dt_s);
    hipLaunchKernelGGL(k_imp_init, dim3(ic->ngroups), dim3(kImpLanes), 0, ic->stream, ic->d_walls,
                       ic->d_groups, ic->A);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(ic->stream) != hipSuccess) return bail();
    *out = ic;
    return DFHM_OK;
}

dfhm_status dfhm_implicit_step_n(dfhm_implicit *ic, int64_t n_steps)
{
    if (!ic || n_steps < 0) return DFHM_E_INVAL;
    for (int64_t k = 0; k < n_steps; ++k) {
        auto kern = ic->cfg.law == DFHM_LAW_TABLE1 ? k_imp_step<1> : k_imp_step<0>;
        hipLaunchKernelGGL(kern, dim3(ic->ngroups), dim3(kImpLanes), 0, ic->stream, ic->d_walls,
                           ic->d_groups, ic->A, ic->n, ic->cfg.dt_s, ic->cfg.theta, ic->cfg.eta,
                           (int)ic->cfg.max_iters, ic->cfg.Lv, ic->cfg.cw, ic->d_iters);
        ic->n += 1;
    }
    if (hipGetLastError() != hipSuccess) { ic->err = "kernel launch failed"; return DFHM_E_DEVICE; }
    return DFHM_OK;
}

dfhm_status dfhm_implicit_get_fields(dfhm_implicit *ic, int64_t wall, double *T, double *Pv)
{
    if (!ic || !T || !Pv || wall < 0 || wall >= ic->nw) return DFHM_E_INVAL;
    const ImpGroup &g = ic->groups[wall / kImpWalls];
    const int slot = (int)(wall % kImpWalls), nx = ic->walls[wall].nx;
    const int p = (int)(ic->n & 1);
    // one strided copy per field: element j of the wall is at base + 32 j + slot
    if (hipMemcpy2DAsync(T, sizeof(double), ic->A.T[p] + g.base + slot, sizeof(double) * kImpWalls,
                         sizeof(double), nx, hipMemcpyDeviceToHost, ic->stream) != hipSuccess ||
        hipMemcpy2DAsync(Pv, sizeof(double), ic->A.P[p] + g.base + slot, sizeof(double) * kImpWalls,
                         sizeof(double), nx, hipMemcpyDeviceToHost, ic->stream) != hipSuccess ||
        hipStreamSynchronize(ic->stream) != hipSuccess) {
        ic->err = "copy failed";
        return DFHM_E_DEVICE;
    }
    return DFHM_OK;
}

dfhm_status dfhm_implicit_iterations(dfhm_implicit *ic, double *mean_per_step)
{
    if (!ic || !mean_per_step) return DFHM_E_INVAL;
    std::vector<int64_t> it(ic->nw);
    if (hipMemcpyAsync(it.data(), ic->d_iters, sizeof(int64_t) * ic->nw, hipMemcpyDeviceToHost, ic->stream) != hipSuccess ||
        hipStreamSynchronize(ic->stream) != hipSuccess)
        return DFHM_E_DEVICE;
    double s = 0.0;
    for (int64_t v : it) s += (double)v;
    *mean_per_step = ic->n > 0 ? s / ((double)ic->nw * (double)ic->n) : 0.0;
    return DFHM_OK;
}

int64_t dfhm_implicit_step_index(const dfhm_implicit *ic) { return ic ? ic->n : -1; }

void dfhm_implicit_destroy(dfhm_implicit *ic)
{
    if (!ic) return;
    if (ic->stream) (void)hipStreamSynchronize(ic->stream);
    else (void)hipDeviceSynchronize();
    if (ic->mem) (void)hipFree(ic->mem);
    delete ic;
}

// ------------------------------------------------------------ checkpoints

namespace {
constexpr uint64_t kCkptMagic = 0x31504b434d484644ull;   // "DFHMCKP1"

struct CkptHeader {
    uint64_t magic;
    int32_t version, precision;
    int64_t n_walls, n_nodes, n_rooms, step;
    uint64_t digest;                 // of the wall and zone descriptors
    uint64_t payload;                // bytes after the header
};

// FNV-1a over everything a run's future depends on besides its evolving
// state: the run constants (dt above all: levels n and n-1 of the three-level
// recurrence are one dt apart), the law, every input field of the wall
// descriptors, the zone descriptors with their schedules, and the links.
uint64_t describe(const dfhm_ctx *c)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void *p, size_t n) {
        const unsigned char *b = (const unsigned char *)p;
        for (size_t i = 0; i < n; ++i) { h ^= b[i]; h *= 1099511628211ull; }
    };
    const RunConst &rc = c->rc;
    for (double v : {rc.dt, rc.Lv, rc.cw, rc.rho_a, rc.c_pa, rc.c_pv, rc.Pv_ref}) mix(&v, sizeof v);
    mix(&c->cfg.law, sizeof c->cfg.law);
    mix(&c->cfg.startup, sizeof c->cfg.startup);
    for (const WallDev &W : c->walls) {
        mix(&W.nx, sizeof W.nx);
        mix(&W.n_layers, sizeof W.n_layers);
        mix(&W.room, sizeof W.room);
        mix(&W.room_side, sizeof W.room_side);
        mix(&W.area, sizeof W.area);
        mix(&W.T0, sizeof W.T0);
        mix(&W.RH0, sizeof W.RH0);
        mix(W.hT, sizeof W.hT);
        mix(W.hM, sizeof W.hM);
        mix(W.qinf, sizeof W.qinf);
        mix(W.ginf, sizeof W.ginf);
        mix(W.Tamb, sizeof W.Tamb);
        mix(W.RHamb, sizeof W.RHamb);
        mix(W.lay, sizeof W.lay);
        mix(W.qsun, sizeof W.qsun);
        mix(W.emis, sizeof W.emis);
        mix(&W.esig, sizeof W.esig);
    }
    mix(c->wall_room.data(), sizeof(int64_t) * c->wall_room.size());
    mix(&c->nr, sizeof c->nr);
    for (const RoomDev &R : c->rooms_host) {
        mix(&R.volume, sizeof R.volume);
        mix(&R.ach, sizeof R.ach);
        mix(&R.T0, sizeof R.T0);
        mix(&R.RH0, sizeof R.RH0);
        mix(R.Tout, sizeof R.Tout);
        mix(R.RHout, sizeof R.RHout);
        mix(&R.sched_dt, sizeof R.sched_dt);
        mix(&R.n_sched, sizeof R.n_sched);
        mix(&R.view, sizeof R.view);
    }
    if (!c->sched_go.empty()) mix(c->sched_go.data(), sizeof(double) * c->sched_go.size());
    if (!c->sched_qh.empty()) mix(c->sched_qh.data(), sizeof(double) * c->sched_qh.size());
    mix(&c->n_links, sizeof c->n_links);
    for (const ZoneLinkDev &L : c->links_host) {
        mix(&L.partner, sizeof L.partner);
        mix(&L.g, sizeof L.g);
    }
    return h;
}

size_t ckpt_payload(const dfhm_ctx *c)
{
    return 4 * c->esize * (size_t)c->N + sizeof(double) * (12 * (size_t)c->nw + 2 * (size_t)c->nr);
}
} // namespace

dfhm_status dfhm_save(dfhm_ctx *c, void *buf, size_t *bytes)
{
    if (!c || !bytes) return DFHM_E_INVAL;
    const size_t need = sizeof(CkptHeader) + ckpt_payload(c);
    if (!buf) { *bytes = need; return DFHM_OK; }
    if (*bytes < need) return fail(c, DFHM_E_INVAL, "checkpoint buffer too small");
    CkptHeader h{};
    h.magic = kCkptMagic;
    h.version = 2;
    h.precision = c->precision;
    h.n_walls = c->nw;
    h.n_nodes = c->N;
    h.n_rooms = c->nr;
    h.step = c->n;
    h.digest = describe(c);
    h.payload = ckpt_payload(c);
    char *o = (char *)buf;
    std::memcpy(o, &h, sizeof h);
    o += sizeof h;
    // level n then level n-1, each T then P, in the storage format
    const size_t lv = c->esize * (size_t)c->N;
    for (int level = 0; level < 2; ++level) {
        const int b = (int)((c->n + level) & 1);
        HIP_TRY(c, hipMemcpyAsync(o, c->d_T[b], lv, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipMemcpyAsync(o + lv, c->d_P[b], lv, hipMemcpyDeviceToHost, c->stream));
        o += 2 * lv;
    }
    HIP_TRY(c, hipMemcpyAsync(o, c->d_flux, sizeof(double) * 12 * c->nw, hipMemcpyDeviceToHost, c->stream));
    o += sizeof(double) * 12 * c->nw;
    if (c->nr) {
        HIP_TRY(c, hipMemcpyAsync(o, c->d_roomT, sizeof(double) * c->nr, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipMemcpyAsync(o + sizeof(double) * c->nr, c->d_roomP, sizeof(double) * c->nr,
                                  hipMemcpyDeviceToHost, c->stream));
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    *bytes = need;
    return DFHM_OK;
}

dfhm_status dfhm_load(dfhm_ctx *c, const void *buf, size_t bytes)
{
    if (!c || !buf) return DFHM_E_INVAL;
    CkptHeader h;
    if (bytes < sizeof h) return fail(c, DFHM_E_INVAL, "checkpoint too short");
    std::memcpy(&h, buf, sizeof h);
    if (h.magic != kCkptMagic || h.version != 2) return fail(c, DFHM_E_INVAL, "not a dfhm checkpoint");
    if (h.precision != c->precision || h.n_walls != c->nw || h.n_nodes != c->N || h.n_rooms != c->nr ||
        h.digest != describe(c) || h.payload != ckpt_payload(c) || bytes < sizeof h + h.payload)
        return fail(c, DFHM_E_INVAL, "checkpoint of different walls, zones or precision");
    if (h.step < 0) return fail(c, DFHM_E_INVAL, "negative step index in checkpoint");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    dfhm_status st = dfhm_set_step_index(c, h.step);
    if (st) return st;
    const char *o = (const char *)buf + sizeof h;
    const size_t lv = c->esize * (size_t)c->N;
    for (int level = 0; level < 2; ++level) {
        const int b = (int)((c->n + level) & 1);
        HIP_TRY(c, hipMemcpy(c->d_T[b], o, lv, hipMemcpyHostToDevice));
        HIP_TRY(c, hipMemcpy(c->d_P[b], o + lv, lv, hipMemcpyHostToDevice));
        o += 2 * lv;
    }
    HIP_TRY(c, hipMemcpy(c->d_flux, o, sizeof(double) * 12 * c->nw, hipMemcpyHostToDevice));
    o += sizeof(double) * 12 * c->nw;
    if (c->nr) {
        HIP_TRY(c, hipMemcpy(c->d_roomT, o, sizeof(double) * c->nr, hipMemcpyHostToDevice));
        HIP_TRY(c, hipMemcpy(c->d_roomP, o + sizeof(double) * c->nr, sizeof(double) * c->nr,
                             hipMemcpyHostToDevice));
    }
    int zero = 0;
    HIP_TRY(c, hipMemcpy(c->d_bad, &zero, sizeof(int), hipMemcpyHostToDevice));
    c->latched = DFHM_OK;
    return DFHM_OK;
}

int64_t dfhm_step_index(const dfhm_ctx *c) { return c ? c->n : -1; }

const char *dfhm_last_error(const dfhm_ctx *c) { return c ? c->err.c_str() : "null context"; }

void dfhm_destroy(dfhm_ctx *c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->own_arena && c->arena) (void)hipFree(c->arena);
    if (c->room_mem) (void)hipFree(c->room_mem);
    if (c->link_mem) (void)hipFree(c->link_mem);
    if (c->pack_mem) (void)hipFree(c->pack_mem);
    delete c;
}

} // extern "C"

// ---------------------------------------------------------------- autotune

namespace {

struct Snapshot {
    void *mem = nullptr;
    size_t lev = 0, flux = 0, rooms = 0;
};

dfhm_status snap_save(dfhm_ctx *c, Snapshot &sn)
{
    sn.lev = c->esize * c->N;
    sn.flux = sizeof(double) * 12 * c->nw;
    sn.rooms = sizeof(double) * c->nr;
    size_t total = 4 * sn.lev + sn.flux + 2 * sn.rooms + sizeof(int64_t);
    if (hipMalloc(&sn.mem, total) != hipSuccess) return fail(c, DFHM_E_NOMEM, "autotune snapshot");
    char *b = (char *)sn.mem;
    HIP_TRY(c, hipMemcpyAsync(b, c->d_T[0], sn.lev, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(b + sn.lev, c->d_T[1], sn.lev, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(b + 2 * sn.lev, c->d_P[0], sn.lev, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(b + 3 * sn.lev, c->d_P[1], sn.lev, hipMemcpyDeviceToDevice, c->stream));
    b += 4 * sn.lev;
    HIP_TRY(c, hipMemcpyAsync(b, c->d_flux, sn.flux, hipMemcpyDeviceToDevice, c->stream));
    b += sn.flux;
    if (c->nr) {
        HIP_TRY(c, hipMemcpyAsync(b, c->d_roomT, sn.rooms, hipMemcpyDeviceToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(b + sn.rooms, c->d_roomP, sn.rooms, hipMemcpyDeviceToDevice, c->stream));
    }
    b += 2 * sn.rooms;
    HIP_TRY(c, hipMemcpyAsync(b, c->d_step, sizeof(int64_t), hipMemcpyDeviceToDevice, c->stream));
    return DFHM_OK;
}

dfhm_status snap_restore(dfhm_ctx *c, const Snapshot &sn)
{
    char *b = (char *)sn.mem;
    HIP_TRY(c, hipMemcpyAsync(c->d_T[0], b, sn.lev, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->d_T[1], b + sn.lev, sn.lev, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->d_P[0], b + 2 * sn.lev, sn.lev, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->d_P[1], b + 3 * sn.lev, sn.lev, hipMemcpyDeviceToDevice, c->stream));
    b += 4 * sn.lev;
    HIP_TRY(c, hipMemcpyAsync(c->d_flux, b, sn.flux, hipMemcpyDeviceToDevice, c->stream));
    b += sn.flux;
    if (c->nr) {
        HIP_TRY(c, hipMemcpyAsync(c->d_roomT, b, sn.rooms, hipMemcpyDeviceToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->d_roomP, b + sn.rooms, sn.rooms, hipMemcpyDeviceToDevice, c->stream));
    }
    b += 2 * sn.rooms;
    HIP_TRY(c, hipMemcpyAsync(c->d_step, b, sizeof(int64_t), hipMemcpyDeviceToDevice, c->stream));
    int zero = 0;
    HIP_TRY(c, hipMemcpyAsync(c->d_bad, &zero, sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return DFHM_OK;
}

// Time `steps` steps of one candidate (sched, nt, npt); returns ms or < 0.
template <typename R>
double probe(dfhm_ctx *c, int sched, int nt, int npt, int steps)
{
    if (sched == DFHM_SCHED_RESIDENT) {
        if (!c->packed || c->res_threads != nt || c->res_npt != npt)
            if (pack(c, nt, npt) != DFHM_OK) return -1.0;
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.0;
    (void)hipEventRecord(e0, c->stream);
    if (sched == DFHM_SCHED_RESIDENT) {
        launch_resident<R>(c, steps);
        tick(c, steps);
    } else {
        enqueue_stream_chunk<R>(c, steps);
    }
    (void)hipEventRecord(e1, c->stream);
    float ms = -1.0f;
    if (hipEventSynchronize(e1) == hipSuccess) (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (hipGetLastError() != hipSuccess) return -1.0;
    return ms;
}

std::string tune_key(const dfhm_ctx *c)
{
    hipDeviceProp_t p;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&p, c->device) == hipSuccess) arch = p.gcnArchName;
    int64_t nb = 1;
    while (nb < c->N) nb <<= 1;   // size bucket: next power of two of the node count
    char b[256];
    // kernel variant: walls only, zones, or the extended variant (radiative
    // sources, linked zones); the law changes the node work about twofold
    const int mode = c->extended ? 2 : (c->nr > 0 ? 1 : 0);
    snprintf(b, sizeof b, "%s p%d s%d g%d n%lld m%d L%d", arch.c_str(), c->precision, c->cfg.schedule,
             max_group(c), (long long)nb, mode, (int)c->cfg.law);
    for (char *q = b; *q; ++q)
        if (*q == ' ' || *q == ':') *q = '_';
    return b;
}

bool cache_lookup(const std::string &key, int &sched, int &nt, int &npt)
{
    const char *path = std::getenv("DFHM_AUTOTUNE_CACHE");
    if (!path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char k[256];
    int a, b, d;
    bool hit = false;
    while (std::fscanf(f, "%255s %d %d %d", k, &a, &b, &d) == 4)
        if (key == k) { sched = a; nt = b; npt = d; hit = true; }
    std::fclose(f);
    return hit;
}

void cache_store(const std::string &key, int sched, int nt, int npt)
{
    const char *path = std::getenv("DFHM_AUTOTUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %d\n", key.c_str(), sched, nt, npt);
    std::fclose(f);
}

template <typename R>
dfhm_status autotune_impl(dfhm_ctx *c, int probe_steps)
{
    const std::string key = tune_key(c);
    int sched = 0, nt = 0, npt = 0;
    if (cache_lookup(key, sched, nt, npt)) {
        c->tuned = true;
        c->tuned_sched = sched;
        if (sched == DFHM_SCHED_RESIDENT) return pack(c, nt, npt);
        return DFHM_OK;
    }
    Snapshot sn;
    dfhm_status st = snap_save(c, sn);
    if (st) return st;
    const int need = max_group(c);
    double best = 1e300;
    int bs = -1, bnt = 0, bnpt = 0;
    const bool try_stream = c->cfg.schedule != DFHM_SCHED_RESIDENT;
    const bool try_res = c->cfg.schedule != DFHM_SCHED_STREAM && c->shape_uniform;
    if (try_stream) {
        (void)probe<R>(c, DFHM_SCHED_STREAM, 0, 0, 1);   // warm-up
        snap_restore(c, sn);
        double ms = probe<R>(c, DFHM_SCHED_STREAM, 0, 0, probe_steps);
        snap_restore(c, sn);
        if (ms >= 0 && ms < best) { best = ms; bs = DFHM_SCHED_STREAM; }
    }
    if (try_res) {
        for (const Cand &k : kCands) {
            if (k.nt * k.npt < need) continue;
            // skip shapes that leave most lanes idle on the largest group
            if (k.nt * k.npt >= 4 * std::max(need, 64)) continue;
            (void)probe<R>(c, DFHM_SCHED_RESIDENT, k.nt, k.npt, 2);   // warm-up + packing
            snap_restore(c, sn);
            double ms = probe<R>(c, DFHM_SCHED_RESIDENT, k.nt, k.npt, probe_steps);
            snap_restore(c, sn);
            if (ms >= 0 && ms < best) { best = ms; bs = DFHM_SCHED_RESIDENT; bnt = k.nt; bnpt = k.npt; }
        }
    }
    (void)hipFree(sn.mem);
    if (bs < 0) return fail(c, DFHM_E_DEVICE, "autotune: no candidate ran");
    c->tuned = true;
    c->tuned_sched = bs;
    cache_store(key, bs, bnt, bnpt);
    if (bs == DFHM_SCHED_RESIDENT) return pack(c, bnt, bnpt);
    return DFHM_OK;
}

} // namespace

extern "C" dfhm_status dfhm_autotune(dfhm_ctx *c, int32_t probe_steps)
{
    if (!c) return DFHM_E_INVAL;
    if (probe_steps < 1) return fail(c, DFHM_E_INVAL, "probe_steps must be >= 1");
    if (c->latched != DFHM_OK) return fail(c, DFHM_E_STATE, "context holds a non-finite state");
    if (c->cfg.block_threads > 0 && c->cfg.nodes_per_thread > 0)
        return fail(c, DFHM_E_STATE, "launch shape fixed by the configuration");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const int64_t n_saved = c->n;
    dfhm_status st = c->precision == DFHM_FP64 ? autotune_impl<double>(c, probe_steps)
                                               : autotune_impl<float>(c, probe_steps);
    c->n = n_saved;
    return st;
}
