// fdlb_api.cpp -- host runtime behind the C interface of include/fdlb.h.
//
// A context owns: the per-instance descriptors (device copy), the tile table of the step
// launch, the non-physical flag, reduction scratch and the captured step graphs.  The
// distributions, pressures and wall rows live in the caller's arena.
//
// Model constants are computed here once in float64 with every expression written in the
// order of the equations of the paper (compiled without contraction): the diagonal
// component v_k * sqrt(2)/2, |v|^2 / 2, the weight-polynomial constants of Eq. (fk_eq1)
// with the cyclic index of Eq. (kl_eq), and the line coefficients c/2, c^2/2 and
// c (1 - c^2) / 12 of Eq. (dis_eq1) with c = v dt / dr (Eq. add3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fdlb.h"
#include "fdlb_internal.h"

using fdlb::Inst;
using fdlb::Tile;

namespace {

constexpr double kHalfSqrt2 = 0.70710678118654757;  // nearest double to sqrt(2)/2
constexpr int kGraphSteps = 32;                      // steps per captured graph (even)
constexpr size_t kAlign = 256;
constexpr size_t kPlanePad = 256;                    // see plane_pad_bytes

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
int round_up(int v, int a) { return (v + a - 1) / a * a; }

struct Layout {
    int fpitch, ppitch, wlen;
    int64_t fplane, mplane;
    size_t esize;
    size_t f_bytes, p_bytes, m_bytes, w_bytes, total;
};

// Bytes between the end of one plane and the start of the next (f planes and moment
// planes).  Rows are padded to 32 elements, so on large grids the plane stride is a power
// of two, and a cell's values in the 33 planes then fall into the same cache sets and
// memory channels.  FDLB_PLANE_PAD (bytes, a multiple of 256) overrides the measured
// default.
size_t plane_pad_bytes() {
    const char *e = std::getenv("FDLB_PLANE_PAD");
    if (e) {
        const long v = std::atol(e);
        if (v >= 0 && v % 256 == 0) return (size_t)v;
    }
    return kPlanePad;
}

// Buffer slots a context borrows: the two ping-pong halves, and with two steps per pass the
// intermediate step's buffer.
int nslots(const fdlb_params &p) { return p.tblock == 2 ? 3 : 2; }

Layout layout_of(const fdlb_params &p) {
    Layout L{};
    L.esize = p.precision == FDLB_F64 ? 8 : 4;
    L.fpitch = round_up(p.nx, 32);
    L.ppitch = round_up(p.nx, 32);
    L.wlen = round_up(std::max(p.nx, p.ny), 32);
    const size_t pad = plane_pad_bytes();
    L.fplane = (int64_t)p.ny * L.fpitch + (int64_t)(pad / L.esize);
    L.mplane = (int64_t)p.ny * L.ppitch + (int64_t)(pad / 8);
    L.f_bytes = align_up((size_t)fdlb::NQ * (size_t)L.fplane * L.esize, kAlign);
    L.p_bytes = align_up((size_t)p.ny * L.ppitch * 8, kAlign);
    L.m_bytes = align_up((size_t)4 * L.mplane * 8, kAlign);
    L.w_bytes = align_up((size_t)4 * L.wlen * 8, kAlign);
    L.total = (size_t)nslots(p) * (L.f_bytes + L.p_bytes + L.m_bytes + L.w_bytes);
    return L;
}

bool finite_pos(double a) { return std::isfinite(a) && a > 0.0; }

// 0 = valid
int validate(const fdlb_params &p) {
    if (p.nx < 1 || p.ny < 1) return 1;
    if ((int64_t)p.nx * p.ny > (int64_t)1 << 28) return 1;  // a plane stays below 2 GiB
    // interior tiles address a plane with 32-bit byte offsets: the padded plane must fit
    {
        const int64_t esize = p.precision == FDLB_F64 ? 8 : 4;
        if ((int64_t)round_up(p.nx, 32) * p.ny * esize > (int64_t)INT32_MAX) return 1;
    }
    if (!finite_pos(p.dx) || !finite_pos(p.dy) || !finite_pos(p.dt) || !finite_pos(p.tau)) return 1;
    if (!std::isfinite(p.lambda) || p.lambda < 0.0) return 1;
    if (p.precision != FDLB_F64 && p.precision != FDLB_F32 && p.precision != FDLB_F32_DEV) return 1;
    if (p.tile < 0 || p.tile > fdlb::kNumTileShapes) return 1;
    if (p.lines < 0 || p.lines > 15) return 1;
    if (p.tblock < 0 || p.tblock > 2) return 1;
    if (p.tblock == 2 && p.precision != FDLB_F64) return 1;  // two-step passes: float64 only
    if (p.theta_fixed != 0 && p.theta_fixed != 1) return 1;
    if (p.theta_fixed && (!std::isfinite(p.theta_value) || p.theta_value < 0.0)) return 1;
    double vmax = 0.0;
    for (int k = 0; k < 4; ++k) {
        if (!finite_pos(p.v[k])) return 1;
        for (int l = 0; l < k; ++l)
            if (p.v[k] == p.v[l]) return 1;  // equal speeds make Eq. (fk_eq1) singular
        vmax = std::max(vmax, p.v[k]);
    }
    // Courant numbers of Eq. (add3) must stay below one for the explicit stencil
    if (!(vmax * p.dt / p.dx < 1.0) || !(vmax * p.dt / p.dy < 1.0)) return 1;
    for (int s = 0; s < 4; ++s) {
        const fdlb_bc &b = p.bc[s];
        if (b.kind < FDLB_BC_PERIODIC || b.kind > FDLB_BC_WALL) return 1;
        if (b.kind == FDLB_BC_WALL && ((s < 2 && p.nx < 2) || (s >= 2 && p.ny < 2))) return 1;
        if (b.kind == FDLB_BC_DIRICHLET) {
            if (!finite_pos(b.rho) || !finite_pos(b.T) || !std::isfinite(b.ux) || !std::isfinite(b.uy)) return 1;
        }
        if (b.lo_kind < FDLB_BC_PERIODIC || b.lo_kind > FDLB_BC_WALL) return 1;
        if (b.lo_kind != FDLB_BC_PERIODIC) {
            if (b.kind == FDLB_BC_PERIODIC) return 1;  // a periodic side has no segments
            if (!std::isfinite(b.split) || !std::isfinite(b.split_rate)) return 1;
            if (b.lo_kind == FDLB_BC_WALL && ((s < 2 && p.nx < 2) || (s >= 2 && p.ny < 2))) return 1;
            if (b.lo_kind == FDLB_BC_DIRICHLET && (!finite_pos(b.lo_rho) || !finite_pos(b.lo_T) ||
                                                   !std::isfinite(b.lo_ux) || !std::isfinite(b.lo_uy)))
                return 1;
        }
    }
    if ((p.bc[0].kind == FDLB_BC_PERIODIC) != (p.bc[1].kind == FDLB_BC_PERIODIC)) return 1;
    if ((p.bc[2].kind == FDLB_BC_PERIODIC) != (p.bc[3].kind == FDLB_BC_PERIODIC)) return 1;
    return 0;
}

// Tile columns per dispatch group, measured on the 8192 x 2048 grid (FDLB_TILE_GROUP
// overrides).
int default_group(int prec) {
    const char *e = std::getenv("FDLB_TILE_GROUP");
    if (e && std::atoi(e) > 0) return std::atoi(e);
    return prec == FDLB_F64 ? 16 : 32;
}

// Edge tiles are cut into pieces of this shape for their launch when it divides the tile
// shape.  Measured: float64 32 x 4 pieces (0.7% off the large grid's step), whole tiles for
// float32 and deviation storage.  FDLB_EDGE_TILE (a shape id, 1-based; 0 keeps whole
// tiles) overrides.
int edge_shape_for(int shape, int prec) {
    const char *e = std::getenv("FDLB_EDGE_TILE");
    const int id = e ? std::atoi(e) : (prec == FDLB_F64 ? 7 : 0);
    if (id < 1 || id > fdlb::kNumTileShapes) return shape;
    const auto &T = fdlb::kTileShapes[shape], &E = fdlb::kTileShapes[id - 1];
    return (T.tx % E.tx == 0 && T.ty % E.ty == 0) ? id - 1 : shape;
}

// Captured steps run the smaller tile kinds as a branch beside the largest one;
// FDLB_GRAPH_FORK=0 keeps every kind on one stream.
bool default_fork() {
    const char *e = std::getenv("FDLB_GRAPH_FORK");
    return !(e && std::atoi(e) == 0);
}

// Tile shape (index into kTileShapes), measured: 64 x 8 for float64, 32 x 8 for float32
// and the deviation layout; 64 x 4 when the grid is four cells high (one tile spans a
// tube's periodic height).
int default_shape(const fdlb_params &p) {
    if (p.tblock == 2) return fdlb::kTwoStepShape;  // the two-step kernel's tiles set the grid
    if (p.tile > 0) return p.tile - 1;
    if (p.ny == 4) return 1;
    return p.precision == FDLB_F64 ? 3 : 0;
}

void fill_constants(const fdlb_params &p, Inst &I) {
    for (int k = 0; k < 4; ++k) {
        const double v = p.v[k];
        I.v[k] = v;
        I.vs[k] = v * kHalfSqrt2;
        I.eax[k] = 0.5 * (v * v);
        I.edg[k] = 0.5 * (I.vs[k] * I.vs[k] + I.vs[k] * I.vs[k]);
        I.vf[k] = (float)I.v[k];
        I.vsf[k] = (float)I.vs[k];
        const double vk2 = v * v;
        const double a = p.v[(k + 1) % 4] * p.v[(k + 1) % 4];
        const double b = p.v[(k + 2) % 4] * p.v[(k + 2) % 4];
        const double d = p.v[(k + 3) % 4] * p.v[(k + 3) % 4];
        I.FA[k] = 6.0 * (a + b + d);
        I.FB[k] = a * b + b * d + d * a;
        I.FC[k] = a * b * d / 4.0;
        I.Fden[k] = vk2 * (vk2 - a) * (vk2 - b) * (vk2 - d);
        I.Fdinv[k] = 1.0 / I.Fden[k];
    }
    // a line left out of Eq. (dis_eq1) keeps its place in the sum with a zero weight (adding
    // zero changes no value, so the float64 path still matches the oracle's sum without it)
    const int lines = p.lines == 0 ? 15 : p.lines;
    for (int al = 0; al < 2; ++al) {
        const double dr = al == 0 ? p.dx : p.dy;
        for (int kind = 0; kind < 2; ++kind)
            for (int k = 0; k < 4; ++k) {
                const double mag = kind == 0 ? I.v[k] : I.vs[k];
                const double c = mag * p.dt / dr;
                I.k1[al][kind][k] = (lines & 1) ? c / 2.0 : 0.0;
                I.k2[al][kind][k] = (lines & 2) ? c * c / 2.0 : 0.0;
                I.k3[al][kind][k] = (lines & 4) ? c * (1.0 - c * c) / 12.0 : 0.0;
                I.kk[al][kind][k] = std::fma(2.0, I.k3[al][kind][k], I.k1[al][kind][k]);
                I.kf[0][al][kind][k] = (float)I.k1[al][kind][k];
                I.kf[1][al][kind][k] = (float)I.k2[al][kind][k];
                I.kf[2][al][kind][k] = (float)I.k3[al][kind][k];
                I.kkf[al][kind][k] = (float)(I.k1[al][kind][k] + 2.0 * I.k3[al][kind][k]);
            }
    }
    I.dt = p.dt;
    I.dx = p.dx;
    I.dy = p.dy;
    I.dtau = p.dt / p.tau;
    I.cdx = p.dt / p.dx;
    I.cdy = p.dt / p.dy;
    I.lam = (lines & 8) && !p.theta_fixed ? p.lambda : 0.0;
    I.th0 = (lines & 8) && p.theta_fixed ? p.theta_value : 0.0;
    for (int s = 0; s < 4; ++s) {
        const fdlb_bc &b = p.bc[s];
        I.bc[s] = b.kind;
        I.bcstate[s][0] = b.rho;
        I.bcstate[s][1] = b.ux;
        I.bcstate[s][2] = b.uy;
        I.bcstate[s][3] = b.T;
        I.bclo[s] = b.lo_kind;
        I.bcstate[4 + s][0] = b.lo_rho;
        I.bcstate[4 + s][1] = b.lo_ux;
        I.bcstate[4 + s][2] = b.lo_uy;
        I.bcstate[4 + s][3] = b.lo_T;
        I.split0[s] = b.lo_kind != FDLB_BC_PERIODIC ? b.split : 0.0;
        I.split1[s] = b.lo_kind != FDLB_BC_PERIODIC ? b.split_rate : 0.0;
    }
    for (int s = 0; s < 8; ++s) {
        I.bcP[s] = 0.0;
        for (int q = 0; q < fdlb::NQ; ++q) I.bcf[s][q] = 0.0;
    }
}

// A side segment that moves needs the step clock advanced after every step.
bool moving_sides(const fdlb_params &p) {
    for (int s = 0; s < 4; ++s)
        if (p.bc[s].lo_kind != FDLB_BC_PERIODIC && p.bc[s].split_rate != 0.0) return true;
    return false;
}

}  // namespace

struct fdlb_ctx {
    int k = 0;
    int prec = 0;
    int shape = 0;
    int group = 1;
    int edge_shape = 0;  // shape of the edge-kind launch (edge tiles cut into pieces of it)
    std::vector<fdlb_params> params;
    std::vector<Layout> layouts;
    std::vector<Inst> h_insts;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    // side branch of a captured step: the smaller tile kinds run beside the largest one
    // (the kinds read the same half and write disjoint cells)
    hipStream_t side_stream = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool fork = true;
    Inst *d_insts = nullptr;
    Tile *d_tiles[fdlb::kNumTileKinds] = {nullptr, nullptr, nullptr, nullptr};
    int ntiles[fdlb::kNumTileKinds] = {0, 0, 0, 0};
    int tblock = 1;  // steps per pass of the two-step tiles (2) or single steps only (1)
    int32_t *d_flag = nullptr;
    int64_t *d_clock = nullptr;  // steps since the state was set (moving side segments)
    bool ticks = false;          // some instance has a moving side segment
    int wall_len = 0;            // float64 with a reflecting side: longest such side (wall pass)
    double *d_partials = nullptr;
    int nparts = 0;
    double *d_sums = nullptr;
    int half = 0;
    int64_t steps = 0;
    bool stepped = false;  // some step was enqueued since creation (a batch shares one clock)
    int device = 0;        // HIP device current at creation
    std::vector<char> is_set;
    bool state_set = false;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    std::string err;
};

namespace {

fdlb_status dev_fail(fdlb_ctx *c, hipError_t e, const char *what) {
    if (c) c->err = std::string(what) + ": " + hipGetErrorString(e);
    return FDLB_EDEVICE;
}

// The last failure of fdlb_create / fdlb_batch_create on this thread (no context exists
// to hold it); fdlb_last_error(NULL) returns it.
thread_local std::string g_create_err;

void release(fdlb_ctx *c);

// A failed step of context creation: keeps the HIP error, frees the partial context.
// hipErrorOutOfMemory is FDLB_ENOMEM, any other HIP error FDLB_EDEVICE.
fdlb_status create_fail(fdlb_ctx *c, hipError_t e, const char *what) {
    g_create_err = std::string(what) + ": " + hipGetErrorString(e);
    release(c);
    return e == hipErrorOutOfMemory ? FDLB_ENOMEM : FDLB_EDEVICE;
}

#define HIPCHK(ctx, call)                                          \
    do {                                                           \
        hipError_t e_ = (call);                                    \
        if (e_ != hipSuccess) return dev_fail((ctx), e_, #call);   \
    } while (0)

// Two timing events, destroyed on every return path.
struct EventPair {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t create() {
        hipError_t e = hipEventCreate(&e0);
        return e != hipSuccess ? e : hipEventCreate(&e1);
    }
    ~EventPair() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

// Trial launches (kernel timing, copy ceiling, autotuning) step from the current half into
// the spare one without taking the step, but their kernels still raise the sticky
// non-physical flag from values the state never holds.  The keeper reads the flag before
// the trials and writes that value back after them, on every return path (the calls using
// it synchronise the stream anyway).
struct FlagKeeper {
    fdlb_ctx *c = nullptr;
    int32_t saved = 0;
    hipError_t save(fdlb_ctx *ctx);
    ~FlagKeeper();
};

// Kind of the tile at (x0, y0): with two steps per pass, a tile of the two-step shape whose
// cells and four cells around them (the reach of two steps) lie inside the grid takes the
// two-step kernel; every other tile its single-step kind.
int host_kind(const fdlb_ctx *c, const fdlb_params &p, int shape, int x0, int y0) {
    const int TX = fdlb::kTileShapes[shape].tx, TY = fdlb::kTileShapes[shape].ty;
    if (c->tblock == 2 && shape == fdlb::kTwoStepShape && x0 >= 4 && y0 >= 4 && x0 + TX + 4 <= p.nx &&
        y0 + TY + 4 <= p.ny)
        return fdlb::kKindTwoStep;
    return fdlb::tile_kind(x0, y0, TX, TY, p.nx, p.ny, p.bc[2].kind);
}

void release(fdlb_ctx *c) {
    if (!c) return;
    for (auto &g : c->graph)
        if (g) (void)hipGraphExecDestroy(g);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->side_stream) (void)hipStreamDestroy(c->side_stream);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->d_insts) (void)hipFree(c->d_insts);
    for (auto &t : c->d_tiles)
        if (t) (void)hipFree(t);
    if (c->d_flag) (void)hipFree(c->d_flag);
    if (c->d_clock) (void)hipFree(c->d_clock);
    if (c->d_partials) (void)hipFree(c->d_partials);
    if (c->d_sums) (void)hipFree(c->d_sums);
    delete c;
}

void drop_graphs(fdlb_ctx *c) {
    for (auto &g : c->graph)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
}

// (Re)builds the tile tables for a tile shape and dispatch-group width.  Dispatch order:
// groups of `group` tile columns, row by row inside a group, so a tile's x and y neighbours
// are in flight at the same time on the same XCD and its halo rows are L2 hits (plain
// row-major order re-reads every y halo from memory).  Synchronises the stream.
fdlb_status set_tiles(fdlb_ctx *c, int shape, int group) {
    const int TX = fdlb::kTileShapes[shape].tx, TY = fdlb::kTileShapes[shape].ty;
    std::vector<Tile> tiles[fdlb::kNumTileKinds];
    for (int i = 0; i < c->k; ++i) {
        const fdlb_params &p = c->params[i];
        const int ntx = (p.nx + TX - 1) / TX, nty = (p.ny + TY - 1) / TY;
        const int g = std::max(1, std::min(group, ntx));
        std::vector<int> kind((size_t)ntx * nty);
        for (int ty = 0; ty < nty; ++ty)
            for (int tx = 0; tx < ntx; ++tx) kind[(size_t)ty * ntx + tx] = host_kind(c, p, shape, tx * TX, ty * TY);
        auto kind_at = [&](int tx, int ty) {
            return tx < 0 || ty < 0 || tx >= ntx || ty >= nty ? -1 : kind[(size_t)ty * ntx + tx];
        };
        for (int gx = 0; gx < ntx; gx += g)
            for (int ty = 0; ty < nty; ++ty)
                for (int tx = gx; tx < std::min(gx + g, ntx); ++tx) {
                    const int kd = kind_at(tx, ty);
                    int32_t flags = 0;
                    // a two-step tile whose x or y neighbour takes single steps keeps its
                    // intermediate step in slot 2 for that neighbour's second step (the
                    // stencil and the switching function reach no diagonal neighbour)
                    if (kd == fdlb::kKindTwoStep &&
                        (kind_at(tx - 1, ty) != kd || kind_at(tx + 1, ty) != kd || kind_at(tx, ty - 1) != kd ||
                         kind_at(tx, ty + 1) != kd))
                        flags = fdlb::kTileRing;
                    tiles[kd].push_back(Tile{i, tx * TX, ty * TY, flags});
                }
    }
    const int es = edge_shape_for(shape, c->prec);
    if (es != shape) {
        const int EX = fdlb::kTileShapes[es].tx, EY = fdlb::kTileShapes[es].ty;
        std::vector<Tile> pieces;
        for (const Tile &t : tiles[2]) {
            const fdlb_params &p = c->params[t.inst];
            for (int dy = 0; dy < TY; dy += EY)
                for (int dx = 0; dx < TX; dx += EX)
                    if (t.x0 + dx < p.nx && t.y0 + dy < p.ny) pieces.push_back(Tile{t.inst, t.x0 + dx, t.y0 + dy, 0});
        }
        tiles[2] = pieces;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int kd = 0; kd < fdlb::kNumTileKinds; ++kd) {
        if (c->d_tiles[kd]) (void)hipFree(c->d_tiles[kd]);
        c->d_tiles[kd] = nullptr;
        c->ntiles[kd] = (int)tiles[kd].size();
        if (tiles[kd].empty()) continue;
        const hipError_t e = hipMalloc(&c->d_tiles[kd], sizeof(Tile) * tiles[kd].size());
        if (e != hipSuccess) {
            c->d_tiles[kd] = nullptr;
            c->ntiles[kd] = 0;
            c->err = std::string("hipMalloc(tile table): ") + hipGetErrorString(e);
            return e == hipErrorOutOfMemory ? FDLB_ENOMEM : FDLB_EDEVICE;
        }
        HIPCHK(c, hipMemcpyAsync(c->d_tiles[kd], tiles[kd].data(), sizeof(Tile) * tiles[kd].size(),
                                 hipMemcpyHostToDevice, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->shape = shape;
    c->edge_shape = es;
    c->group = group;
    drop_graphs(c);
    return FDLB_OK;
}

fdlb_status build(int32_t k, const fdlb_params *p, void *stream, void *arena, size_t bytes, fdlb_ctx **out) {
    g_create_err.clear();
    if (!out) return FDLB_EINVAL;
    *out = nullptr;
    if (k < 1 || !p || !arena) return FDLB_EINVAL;
    if (reinterpret_cast<uintptr_t>(arena) % kAlign) return FDLB_EINVAL;
    size_t need = 0;
    for (int i = 0; i < k; ++i) {
        if (validate(p[i])) return FDLB_EINVAL;
        if (p[i].precision != p[0].precision || default_shape(p[i]) != default_shape(p[0]) ||
            (p[i].tblock == 2) != (p[0].tblock == 2))
            return FDLB_EINVAL;
        need += layout_of(p[i]).total;
    }
    if (bytes < need) return FDLB_EINVAL;

    fdlb_ctx *c = new (std::nothrow) fdlb_ctx();
    if (!c) return FDLB_ENOMEM;
    c->k = k;
    c->prec = p[0].precision;
    c->shape = default_shape(p[0]);
    c->tblock = p[0].tblock == 2 ? 2 : 1;
    c->stream = static_cast<hipStream_t>(stream);
    c->params.assign(p, p + k);
    c->is_set.assign(k, 0);
    c->group = default_group(c->prec);

    hipError_t e;
    if ((e = hipGetDevice(&c->device)) != hipSuccess) return create_fail(c, e, "hipGetDevice");
    if ((e = hipMalloc(&c->d_flag, sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc(&c->d_clock, sizeof(int64_t))) != hipSuccess)
        return create_fail(c, e, "hipMalloc");
    for (int i = 0; i < k; ++i) c->ticks = c->ticks || moving_sides(p[i]);
    if (FDLB_STREAM_EDGE && c->prec == FDLB_F64)
        for (int i = 0; i < k; ++i)
            for (int sd = 0; sd < 4; ++sd)
                if (p[i].bc[sd].kind == FDLB_BC_WALL || p[i].bc[sd].lo_kind == FDLB_BC_WALL)
                    c->wall_len = std::max(c->wall_len, sd < 2 ? p[i].ny : p[i].nx);
    char *base = static_cast<char *>(arena);
    size_t off = 0;
    c->h_insts.resize(k);
    for (int i = 0; i < k; ++i) {
        const Layout L = layout_of(p[i]);
        c->layouts.push_back(L);
        Inst &I = c->h_insts[i];
        std::memset(&I, 0, sizeof(I));
        I.nx = p[i].nx;
        I.ny = p[i].ny;
        I.fpitch = L.fpitch;
        I.ppitch = L.ppitch;
        I.fplane = L.fplane;
        I.wlen = L.wlen;
        I.prec = c->prec;
        const int ns = nslots(p[i]);  // slot 2 only with two steps per pass (else null)
        for (int h = 0; h < ns; ++h) {
            I.f[h] = base + off;
            off += L.f_bytes;
        }
        for (int h = 0; h < ns; ++h) {
            I.P[h] = reinterpret_cast<double *>(base + off);
            off += L.p_bytes;
        }
        for (int h = 0; h < ns; ++h) {
            I.M[h] = reinterpret_cast<double *>(base + off);
            off += L.m_bytes;
        }
        I.mplane = L.mplane;
        for (int h = 0; h < ns; ++h) {
            I.PW[h] = reinterpret_cast<double *>(base + off);
            off += L.w_bytes;
        }
        I.flag = c->d_flag;
        I.clock = c->d_clock;
        fill_constants(p[i], I);
    }
    int nparts = 0;
    for (int i = 0; i < k; ++i) nparts += fdlb::diag_blocks(p[i].nx, p[i].ny);
    c->nparts = nparts;
    if ((e = hipMalloc(&c->d_insts, sizeof(Inst) * k)) != hipSuccess ||
        (e = hipMalloc(&c->d_partials, sizeof(double) * 4 * (size_t)nparts)) != hipSuccess ||
        (e = hipMalloc(&c->d_sums, sizeof(double) * 4)) != hipSuccess)
        return create_fail(c, e, "hipMalloc");
    if ((e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&c->side_stream, hipStreamNonBlocking)) != hipSuccess)
        return create_fail(c, e, "hipStreamCreateWithFlags");
    if ((e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming)) != hipSuccess)
        return create_fail(c, e, "hipEventCreateWithFlags");
    c->fork = default_fork();
    if ((e = hipMemcpyAsync(c->d_insts, c->h_insts.data(), sizeof(Inst) * k, hipMemcpyHostToDevice, c->stream)) !=
            hipSuccess ||

        (e = hipMemsetAsync(c->d_flag, 0, sizeof(int32_t), c->stream)) != hipSuccess ||
        (e = hipMemsetAsync(c->d_clock, 0, sizeof(int64_t), c->stream)) != hipSuccess)
        return create_fail(c, e, "upload");
    for (int i = 0; i < k; ++i)
        if ((e = fdlb::launch_bc_setup(c->prec, c->d_insts, i, c->stream)) != hipSuccess)
            return create_fail(c, e, "bc_setup");
    {
        fdlb_status ts = set_tiles(c, c->shape, c->group);
        if (ts != FDLB_OK) {
            g_create_err = c->err.empty() ? "tile table: " + std::string(fdlb_strerror(ts)) : c->err;
            release(c);
            return ts;
        }
    }
    // the descriptors and tile table come from host vectors: finish before they go away
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return create_fail(c, e, "hipStreamSynchronize");
    g_create_err.clear();
    *out = c;
    return FDLB_OK;
}

hipError_t FlagKeeper::save(fdlb_ctx *ctx) {
    hipError_t e = hipMemcpyAsync(&saved, ctx->d_flag, sizeof(saved), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e == hipSuccess) c = ctx;
    return e;
}

FlagKeeper::~FlagKeeper() {
    if (!c) return;
    // `saved` lives in this object: wait for the copy before it goes away
    if (hipMemcpyAsync(c->d_flag, &saved, sizeof(saved), hipMemcpyHostToDevice, c->stream) == hipSuccess)
        (void)hipStreamSynchronize(c->stream);
}

fdlb_status check_flag(fdlb_ctx *c) {
    int32_t flag = 0;
    HIPCHK(c, hipMemcpyAsync(&flag, c->d_flag, sizeof(flag), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return flag ? FDLB_ENONPHYS : FDLB_OK;
}

// Sets instance i from device fields (4 planes) into the current half.
fdlb_status set_instance(fdlb_ctx *c, int i, const double *dfields) {
    const fdlb_params &p = c->params[i];
    HIPCHK(c, hipMemsetAsync(c->d_clock, 0, sizeof(int64_t), c->stream));
    HIPCHK(c, fdlb::launch_fill(c->prec, c->d_insts, i, p.nx, p.ny, dfields, c->half, c->stream));
    HIPCHK(c, fdlb::launch_derive(c->prec, c->d_insts, i, p.nx, p.ny, c->half, c->stream));
    c->is_set[i] = 1;
    c->state_set = std::all_of(c->is_set.begin(), c->is_set.end(), [](char s) { return s != 0; });
    c->steps = 0;
    return FDLB_OK;
}

fdlb_status set_instance_host(fdlb_ctx *c, int i, const double *rho, const double *ux, const double *uy,
                              const double *T) {
    if (!rho || !ux || !uy || !T) return FDLB_EINVAL;
    const fdlb_params &p = c->params[i];
    const size_t n = (size_t)p.nx * p.ny;
    // stage the fields in the other half's distribution planes (free until the next step)
    double *stage = static_cast<double *>(c->h_insts[i].f[1 - c->half]);
    const double *src[4] = {rho, ux, uy, T};
    for (int a = 0; a < 4; ++a)
        HIPCHK(c, hipMemcpyAsync(stage + a * n, src[a], n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemsetAsync(c->d_flag, 0, sizeof(int32_t), c->stream));
    fdlb_status s = set_instance(c, i, stage);
    if (s != FDLB_OK) return s;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return FDLB_OK;
}

fdlb_status get_instance_host(fdlb_ctx *c, int i, double *rho, double *ux, double *uy, double *T) {
    if (!rho || !ux || !uy || !T) return FDLB_EINVAL;
    if (!c->state_set) return FDLB_ESTATE;
    const fdlb_params &p = c->params[i];
    const size_t n = (size_t)p.nx * p.ny;
    double *stage = static_cast<double *>(c->h_insts[i].f[1 - c->half]);
    HIPCHK(c, fdlb::launch_moments(c->prec, c->d_insts, i, p.nx, p.ny, c->half, stage, c->stream));
    double *dst[4] = {rho, ux, uy, T};
    for (int a = 0; a < 4; ++a)
        HIPCHK(c, hipMemcpyAsync(dst[a], stage + a * n, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    return check_flag(c);
}

// The single-step tile kinds in launch order (the largest last, so it can run beside the
// others); kind 3, the two-step tiles, is launched by launch_pair.
int main_single_kind(const fdlb_ctx *c) {
    int main_kd = 0;
    for (int kd = 0; kd < fdlb::kKindTwoStep; ++kd)
        if (c->ntiles[kd] > c->ntiles[main_kd]) main_kd = kd;
    return main_kd;
}

// One single step of the single-step tile kinds from slot `in` to slot `out` on stream s
// (the smaller kinds on `side` when it is not null).  With `all`, the two-step tiles take
// the step too, as interior tiles of the single-step kernel (a lone step of a two-step
// context); without it they are left to launch_step2.
fdlb_status single_step(fdlb_ctx *c, int in, int out, hipStream_t s, hipStream_t side, bool all) {
    const int main_kd = main_single_kind(c);
    if (all && c->ntiles[fdlb::kKindTwoStep] > 0)
        HIPCHK(c, fdlb::launch_step(c->prec, c->shape, 0, c->d_insts, c->d_tiles[fdlb::kKindTwoStep],
                                    c->ntiles[fdlb::kKindTwoStep], fdlb::io_pack(in, out), side ? side : s));
    for (int kd = fdlb::kKindTwoStep - 1; kd >= 0; --kd)
        if (c->ntiles[kd] > 0)
            HIPCHK(c, fdlb::launch_step(c->prec, kd == 2 ? c->edge_shape : c->shape, kd, c->d_insts, c->d_tiles[kd],
                                        c->ntiles[kd], fdlb::io_pack(in, out), side && kd != main_kd ? side : s));
    return FDLB_OK;
}

// n steps on stream s.  branch: the tile kinds other than the largest go on the side
// stream (fork and join through events), in a graph capture a parallel branch beside the
// largest kind; without it every kind runs in turn on s.  With two steps per pass, steps
// go in pairs: the single-step tiles take slot h to slot 2 (beside the two-step kernel,
// which takes h to 1 - h and fills slot 2 on its ring tiles), then slot 2 to 1 - h.
fdlb_status launch_steps(fdlb_ctx *c, int64_t n, hipStream_t s, bool branch = false) {
    int kinds = 0;
    for (int kd = 0; kd < fdlb::kNumTileKinds; ++kd)
        if (c->ntiles[kd] > 0) ++kinds;
    branch = branch && c->fork && kinds > 1;
    auto fork = [&]() -> fdlb_status {
        HIPCHK(c, hipEventRecord(c->ev_fork, s));
        HIPCHK(c, hipStreamWaitEvent(c->side_stream, c->ev_fork, 0));
        return FDLB_OK;
    };
    auto join = [&]() -> fdlb_status {
        HIPCHK(c, hipEventRecord(c->ev_join, c->side_stream));
        HIPCHK(c, hipStreamWaitEvent(s, c->ev_join, 0));
        return FDLB_OK;
    };
    fdlb_status st;
    for (int64_t t = 0; t < n;) {
        const int h = c->half;
        if (c->tblock == 2 && n - t >= 2) {
            // first step of the single-step tiles (slot h -> 2) beside the two-step kernel
            const bool two = c->ntiles[fdlb::kKindTwoStep] > 0;
            hipStream_t sb = branch && two ? c->side_stream : s;
            if (sb != s && (st = fork()) != FDLB_OK) return st;
            if ((st = single_step(c, h, 2, sb, nullptr, false)) != FDLB_OK) return st;
            if (c->wall_len > 0) HIPCHK(c, fdlb::launch_wall_pressure(c->d_insts, c->k, c->wall_len, 2, sb));
            if (c->ticks) HIPCHK(c, fdlb::launch_tick(c->d_clock, sb));
            if (two)
                HIPCHK(c, fdlb::launch_step2(c->d_insts, c->d_tiles[fdlb::kKindTwoStep],
                                             c->ntiles[fdlb::kKindTwoStep], fdlb::io_pack(h, 1 - h), s));
            if (sb != s && (st = join()) != FDLB_OK) return st;
            // second step of the single-step tiles (slot 2 -> 1 - h)
            if ((st = single_step(c, 2, 1 - h, s, nullptr, false)) != FDLB_OK) return st;
            t += 2;
        } else {
            if (branch && (st = fork()) != FDLB_OK) return st;
            if ((st = single_step(c, h, 1 - h, s, branch ? c->side_stream : nullptr, true)) != FDLB_OK) return st;
            if (branch && (st = join()) != FDLB_OK) return st;
            t += 1;
        }
        if (c->wall_len > 0) HIPCHK(c, fdlb::launch_wall_pressure(c->d_insts, c->k, c->wall_len, 1 - h, s));
        if (c->ticks) HIPCHK(c, fdlb::launch_tick(c->d_clock, s));
        c->half ^= 1;
    }
    return FDLB_OK;
}

// One trial launch that does not advance the state (kernel timing, autotuning): kind >= 0
// launches that tile kind alone from slot h (kind 3: the two-step tiles, two steps); kind -1
// the whole step, with two steps per pass the pair of launch_steps.  The spare slots are
// overwritten; the clock is not advanced.  *steps receives the steps it stands for.
fdlb_status trial_launch(fdlb_ctx *c, int kind, int h, int *steps) {
    *steps = 1;
    if (kind == fdlb::kKindTwoStep) {
        *steps = 2;
        HIPCHK(c, fdlb::launch_step2(c->d_insts, c->d_tiles[kind], c->ntiles[kind], fdlb::io_pack(h, 1 - h), c->stream));
        return FDLB_OK;
    }
    if (kind >= 0) {
        HIPCHK(c, fdlb::launch_step(c->prec, kind == 2 ? c->edge_shape : c->shape, kind, c->d_insts, c->d_tiles[kind],
                                    c->ntiles[kind], fdlb::io_pack(h, 1 - h), c->stream));
        return FDLB_OK;
    }
    fdlb_status st;
    if (c->tblock == 2) {
        *steps = 2;
        if ((st = single_step(c, h, 2, c->stream, nullptr, false)) != FDLB_OK) return st;
        if (c->wall_len > 0) HIPCHK(c, fdlb::launch_wall_pressure(c->d_insts, c->k, c->wall_len, 2, c->stream));
        if (c->ntiles[fdlb::kKindTwoStep] > 0)
            HIPCHK(c, fdlb::launch_step2(c->d_insts, c->d_tiles[fdlb::kKindTwoStep], c->ntiles[fdlb::kKindTwoStep],
                                         fdlb::io_pack(h, 1 - h), c->stream));
        if ((st = single_step(c, 2, 1 - h, c->stream, nullptr, false)) != FDLB_OK) return st;
    } else if ((st = single_step(c, h, 1 - h, c->stream, nullptr, true)) != FDLB_OK) {
        return st;
    }
    if (c->wall_len > 0) HIPCHK(c, fdlb::launch_wall_pressure(c->d_insts, c->k, c->wall_len, 1 - h, c->stream));
    return FDLB_OK;
}

// Graph of kGraphSteps steps starting from half h (kGraphSteps is even: ends in half h).
fdlb_status ensure_graph(fdlb_ctx *c, int h) {
    if (c->graph[h]) return FDLB_OK;
    hipGraph_t g = nullptr;
    HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
    const int saved = c->half;
    c->half = h;
    fdlb_status s = launch_steps(c, kGraphSteps, c->cap_stream, true);
    c->half = saved;
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (s != FDLB_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess) return dev_fail(c, e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&c->graph[h], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        c->graph[h] = nullptr;
        return dev_fail(c, e, "hipGraphInstantiate");
    }
    return FDLB_OK;
}

}  // namespace

extern "C" {

size_t fdlb_required_bytes(const fdlb_params *p) {
    if (!p || validate(*p)) return 0;
    return layout_of(*p).total;
}

size_t fdlb_batch_required_bytes(int32_t k, const fdlb_params *p) {
    if (k < 1 || !p) return 0;
    size_t t = 0;
    for (int i = 0; i < k; ++i) {
        if (validate(p[i])) return 0;
        t += layout_of(p[i]).total;
    }
    return t;
}

fdlb_status fdlb_create(const fdlb_params *p, void *stream, void *arena, size_t arena_bytes, fdlb_ctx **out) {
    return build(1, p, stream, arena, arena_bytes, out);
}

fdlb_status fdlb_batch_create(int32_t k, const fdlb_params *p, void *stream, void *arena, size_t arena_bytes,
                              fdlb_ctx **out) {
    return build(k, p, stream, arena, arena_bytes, out);
}

fdlb_status fdlb_set_state(fdlb_ctx *c, const double *rho, const double *ux, const double *uy, const double *T) {
    if (!c || c->k != 1) return FDLB_EINVAL;
    return set_instance_host(c, 0, rho, ux, uy, T);
}

fdlb_status fdlb_set_state_device(fdlb_ctx *c, const double *fields) {
    if (!c || c->k != 1 || !fields) return FDLB_EINVAL;
    HIPCHK(c, hipMemsetAsync(c->d_flag, 0, sizeof(int32_t), c->stream));
    return set_instance(c, 0, fields);
}

fdlb_status fdlb_batch_set_state(fdlb_ctx *c, int32_t i, const double *rho, const double *ux, const double *uy,
                                 const double *T) {
    if (!c || i < 0 || i >= c->k) return FDLB_EINVAL;
    // the instances share one step clock and one non-physical flag: setting one instance
    // after the batch has stepped would restart the clock and clear the flag of all others
    if (c->k > 1 && c->stepped) return FDLB_ESTATE;
    return set_instance_host(c, i, rho, ux, uy, T);
}

fdlb_status fdlb_step(fdlb_ctx *c, int64_t nsteps) {
    if (!c || nsteps < 0) return FDLB_EINVAL;
    if (!c->state_set) return FDLB_ESTATE;
    if (nsteps > 0) c->stepped = true;
    int64_t left = nsteps;
    while (left >= kGraphSteps) {
        fdlb_status s = ensure_graph(c, c->half);
        if (s != FDLB_OK) return s;
        HIPCHK(c, hipGraphLaunch(c->graph[c->half], c->stream));
        left -= kGraphSteps;
    }
    fdlb_status s = launch_steps(c, left, c->stream);
    if (s != FDLB_OK) return s;
    c->steps += nsteps;
    return FDLB_OK;
}

fdlb_status fdlb_batch_step(fdlb_ctx *c, int64_t nsteps) { return fdlb_step(c, nsteps); }

fdlb_status fdlb_get_moments(fdlb_ctx *c, double *rho, double *ux, double *uy, double *T) {
    if (!c || c->k != 1) return FDLB_EINVAL;
    return get_instance_host(c, 0, rho, ux, uy, T);
}

fdlb_status fdlb_batch_get_moments(fdlb_ctx *c, int32_t i, double *rho, double *ux, double *uy, double *T) {
    if (!c || i < 0 || i >= c->k) return FDLB_EINVAL;
    return get_instance_host(c, i, rho, ux, uy, T);
}

fdlb_status fdlb_get_moments_device(fdlb_ctx *c, double *fields) {
    if (!c || c->k != 1 || !fields) return FDLB_EINVAL;
    if (!c->state_set) return FDLB_ESTATE;
    const fdlb_params &p = c->params[0];
    HIPCHK(c, fdlb::launch_moments(c->prec, c->d_insts, 0, p.nx, p.ny, c->half, fields, c->stream));
    return FDLB_OK;
}

size_t fdlb_f_bytes(const fdlb_ctx *c) {
    if (!c || c->k != 1) return 0;
    const fdlb_params &p = c->params[0];
    const size_t cells = (size_t)p.nx * p.ny;
    return (size_t)fdlb::NQ * cells * c->layouts[0].esize + (c->prec == FDLB_F32_DEV ? 4 * cells * 8 : 0);
}

namespace {
// The moment planes of the deviation layout, after the 33 g planes of a checkpoint.
fdlb_status copy_m(fdlb_ctx *c, char *host, const char *hsrc, bool to_host) {
    if (c->prec != FDLB_F32_DEV) return FDLB_OK;
    const fdlb_params &p = c->params[0];
    const Layout &L = c->layouts[0];
    const size_t row = (size_t)p.nx * 8;
    const size_t gbytes = (size_t)fdlb::NQ * p.nx * p.ny * L.esize;
    const Inst &I = c->h_insts[0];
    for (int a = 0; a < 4; ++a) {
        double *dev = I.M[c->half] + (size_t)a * I.mplane;
        if (to_host)
            HIPCHK(c, hipMemcpy2DAsync(host + gbytes + (size_t)a * p.ny * row, row, dev, (size_t)L.ppitch * 8, row,
                                       p.ny, hipMemcpyDeviceToHost, c->stream));
        else
            HIPCHK(c, hipMemcpy2DAsync(dev, (size_t)L.ppitch * 8, hsrc + gbytes + (size_t)a * p.ny * row, row, row,
                                       p.ny, hipMemcpyHostToDevice, c->stream));
    }
    return FDLB_OK;
}
}  // namespace

fdlb_status fdlb_get_f(fdlb_ctx *c, void *host, size_t bytes) {
    if (!c || c->k != 1 || !host || bytes != fdlb_f_bytes(c)) return FDLB_EINVAL;
    if (!c->state_set) return FDLB_ESTATE;
    const fdlb_params &p = c->params[0];
    const Layout &L = c->layouts[0];
    const char *src = static_cast<const char *>(c->h_insts[0].f[c->half]);
    char *dst = static_cast<char *>(host);
    const size_t row = (size_t)p.nx * L.esize;
    for (int q = 0; q < fdlb::NQ; ++q)
        HIPCHK(c, hipMemcpy2DAsync(dst + (size_t)q * p.ny * row, row, src + (size_t)q * L.fplane * L.esize,
                                   (size_t)L.fpitch * L.esize, row, p.ny, hipMemcpyDeviceToHost, c->stream));
    fdlb_status ms = copy_m(c, dst, nullptr, true);
    if (ms != FDLB_OK) return ms;
    return check_flag(c);
}

fdlb_status fdlb_set_f(fdlb_ctx *c, const void *host, size_t bytes) {
    if (!c || c->k != 1 || !host || bytes != fdlb_f_bytes(c)) return FDLB_EINVAL;
    const fdlb_params &p = c->params[0];
    const Layout &L = c->layouts[0];
    char *dst = static_cast<char *>(c->h_insts[0].f[c->half]);
    const char *src = static_cast<const char *>(host);
    const size_t row = (size_t)p.nx * L.esize;
    for (int q = 0; q < fdlb::NQ; ++q)
        HIPCHK(c, hipMemcpy2DAsync(dst + (size_t)q * L.fplane * L.esize, (size_t)L.fpitch * L.esize,
                                   src + (size_t)q * p.ny * row, row, row, p.ny, hipMemcpyHostToDevice, c->stream));
    fdlb_status ms = copy_m(c, nullptr, src, false);
    if (ms != FDLB_OK) return ms;
    HIPCHK(c, hipMemsetAsync(c->d_flag, 0, sizeof(int32_t), c->stream));
    HIPCHK(c, hipMemsetAsync(c->d_clock, 0, sizeof(int64_t), c->stream));
    HIPCHK(c, fdlb::launch_derive(c->prec, c->d_insts, 0, p.nx, p.ny, c->half, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->is_set[0] = 1;
    c->state_set = true;
    c->steps = 0;
    return FDLB_OK;
}

fdlb_status fdlb_diag(fdlb_ctx *c, double sums[4], int32_t *nonphys) {
    if (!c || !sums) return FDLB_EINVAL;
    if (!c->state_set) return FDLB_ESTATE;
    int off = 0;
    for (int i = 0; i < c->k; ++i) {
        const fdlb_params &p = c->params[i];
        HIPCHK(c, fdlb::launch_diag(c->prec, c->d_insts, i, p.nx, p.ny, c->half, c->d_partials, off, c->stream));
        off += fdlb::diag_blocks(p.nx, p.ny);
    }
    HIPCHK(c, fdlb::launch_diag_final(c->d_partials, c->nparts, c->d_sums, c->stream));
    HIPCHK(c, hipMemcpyAsync(sums, c->d_sums, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    fdlb_status s = check_flag(c);
    if (nonphys) *nonphys = s == FDLB_ENONPHYS ? 1 : 0;
    return s == FDLB_ENONPHYS ? FDLB_OK : s;
}

}  // extern "C"

namespace {
// Per-device address of the allocation-free diagnostics scratch, resolved once per device
// with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices] = {};

hipError_t scratch_for(int device, double **out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        double *ptr = nullptr;
        e = fdlb::diag_scratch_address(&ptr);
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        g_scratch[device] = ptr;
    }
    *out = g_scratch[device];
    return hipSuccess;
}
}  // namespace

extern "C" {

fdlb_status fdlb_diag_noalloc(fdlb_ctx *c, double sums[4], int32_t *nonphys) {
    if (!c || !sums) return FDLB_EINVAL;
    if (c->nparts > fdlb::kDiagScratchParts) {
        c->err = "fdlb_diag_noalloc: the grid needs " + std::to_string(c->nparts) +
                 " partial blocks of 256 cells; the fixed scratch holds " +
                 std::to_string(fdlb::kDiagScratchParts);
        return FDLB_EINVAL;
    }
    if (!c->state_set) return FDLB_ESTATE;
    double *scr = nullptr;
    HIPCHK(c, scratch_for(c->device, &scr));
    double *dsums = scr + 4 * (size_t)fdlb::kDiagScratchParts;
    int off = 0;
    for (int i = 0; i < c->k; ++i) {
        const fdlb_params &p = c->params[i];
        HIPCHK(c, fdlb::launch_diag(c->prec, c->d_insts, i, p.nx, p.ny, c->half, scr, off, c->stream));
        off += fdlb::diag_blocks(p.nx, p.ny);
    }
    HIPCHK(c, fdlb::launch_diag_final(scr, c->nparts, dsums, c->stream));
    HIPCHK(c, hipMemcpyAsync(sums, dsums, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    fdlb_status s = check_flag(c);
    if (nonphys) *nonphys = s == FDLB_ENONPHYS ? 1 : 0;
    return s == FDLB_ENONPHYS ? FDLB_OK : s;
}

int64_t fdlb_steps_done(const fdlb_ctx *c) { return c ? c->steps : 0; }

fdlb_status fdlb_set_clock(fdlb_ctx *c, int64_t steps) {
    if (!c || steps < 0) return FDLB_EINVAL;
    // the value is copied before the call returns (pageable source), so a local is fine
    HIPCHK(c, hipMemcpyAsync(c->d_clock, &steps, sizeof(steps), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->steps = steps;
    return FDLB_OK;
}

fdlb_status fdlb_set_tiling(fdlb_ctx *c, int32_t shape_id, int32_t group) {
    if (!c || shape_id < 1 || shape_id > fdlb::kNumTileShapes || group < 1) return FDLB_EINVAL;
    if (c->tblock == 2 && shape_id - 1 != fdlb::kTwoStepShape) return FDLB_EINVAL;
    return set_tiles(c, shape_id - 1, group);
}

fdlb_status fdlb_get_tiling(const fdlb_ctx *c, int32_t *shape_id, int32_t *group) {
    if (!c || !shape_id || !group) return FDLB_EINVAL;
    *shape_id = c->shape + 1;
    *group = c->group;
    return FDLB_OK;
}

int64_t fdlb_tile_cells(const fdlb_ctx *c, int32_t kind) {
    if (!c || kind < 0 || kind >= fdlb::kNumTileKinds) return 0;
    // cells of the tiles of this kind that lie inside the grid
    const int TX = fdlb::kTileShapes[c->shape].tx, TY = fdlb::kTileShapes[c->shape].ty;
    int64_t cells = 0;
    for (int i = 0; i < c->k; ++i) {
        const fdlb_params &p = c->params[i];
        for (int y0 = 0; y0 < p.ny; y0 += TY)
            for (int x0 = 0; x0 < p.nx; x0 += TX)
                if (host_kind(c, p, c->shape, x0, y0) == kind)
                    cells += (int64_t)std::min(TX, p.nx - x0) * std::min(TY, p.ny - y0);
    }
    return cells;
}

fdlb_status fdlb_time_kernel(fdlb_ctx *c, int32_t kind, int32_t launches, float *ms_per_launch) {
    if (!c || !ms_per_launch || launches < 1 || kind < -1 || kind >= fdlb::kNumTileKinds) return FDLB_EINVAL;
    if (!c->state_set) return FDLB_ESTATE;
    FlagKeeper keep;
    HIPCHK(c, keep.save(c));
    EventPair ev;
    HIPCHK(c, ev.create());
    const int h = c->half;
    if (kind >= 0 && c->ntiles[kind] == 0) {
        *ms_per_launch = 0.0f;
        return FDLB_OK;
    }
    // kind -1: `launches` steps (a pair counts two); a kind alone: `launches` launches
    int per = 1;
    fdlb_status st;
    for (int w = 0; w < 2; ++w)
        if ((st = trial_launch(c, kind, h, &per)) != FDLB_OK) return st;
    const int units = kind < 0 ? (launches + per - 1) / per : launches;
    HIPCHK(c, hipEventRecord(ev.e0, c->stream));
    for (int u = 0; u < units; ++u)
        if ((st = trial_launch(c, kind, h, &per)) != FDLB_OK) return st;
    HIPCHK(c, hipEventRecord(ev.e1, c->stream));
    HIPCHK(c, hipEventSynchronize(ev.e1));
    float ms = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&ms, ev.e0, ev.e1));
    *ms_per_launch = ms / (float)(kind < 0 ? units * per : units);
    return FDLB_OK;
}

fdlb_status fdlb_copy_ceiling(fdlb_ctx *c, int32_t launches, float *ms_per_launch) {
    if (!c || !ms_per_launch || launches < 1) return FDLB_EINVAL;
    if (!c->state_set) return FDLB_ESTATE;
    // the interior tiles: the single-step ones, or with two steps per pass the two-step ones
    const int kd = c->ntiles[0] > 0 ? 0 : fdlb::kKindTwoStep;
    if (c->ntiles[kd] == 0) return FDLB_EINVAL;
    EventPair ev;
    HIPCHK(c, ev.create());
    const int h = c->half;
    for (int w = 0; w < 2 + launches; ++w) {
        if (w == 2) HIPCHK(c, hipEventRecord(ev.e0, c->stream));
        HIPCHK(c, fdlb::launch_plane_copy(c->prec, c->shape, c->d_insts, c->d_tiles[kd], c->ntiles[kd], h, c->stream));
    }
    HIPCHK(c, hipEventRecord(ev.e1, c->stream));
    HIPCHK(c, hipEventSynchronize(ev.e1));
    float ms = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&ms, ev.e0, ev.e1));
    *ms_per_launch = ms / (float)launches;
    return FDLB_OK;
}

fdlb_status fdlb_autotune(fdlb_ctx *c, int32_t trial_steps, const int32_t *shape_ids, int32_t nshapes,
                          const int32_t *groups, int32_t ngroups, float *best_ms) {
    if (!c || trial_steps < 1 || nshapes < 0 || ngroups < 0) return FDLB_EINVAL;
    if (!c->state_set) return FDLB_ESTATE;
    std::vector<int> sh, gr;
    for (int i = 0; i < nshapes; ++i) {
        if (shape_ids[i] < 1 || shape_ids[i] > fdlb::kNumTileShapes) return FDLB_EINVAL;
        sh.push_back(shape_ids[i] - 1);
    }
    for (int i = 0; i < ngroups; ++i) {
        if (groups[i] < 1) return FDLB_EINVAL;
        gr.push_back(groups[i]);
    }
    if (c->tblock == 2) {
        // the two-step kernel has one tile shape: only the dispatch groups are tuned
        for (int s : sh)
            if (s != fdlb::kTwoStepShape) return FDLB_EINVAL;
        sh.assign(1, fdlb::kTwoStepShape);
    }
    if (sh.empty())
        for (int s = 0; s < fdlb::kNumTileShapes; ++s) sh.push_back(s);
    if (gr.empty()) gr = {1, 4, 8, 16, 32};
    FlagKeeper keep;
    HIPCHK(c, keep.save(c));
    EventPair ev;
    HIPCHK(c, ev.create());
    float best = -1.0f;
    int best_s = c->shape, best_g = c->group;
    const int h = c->half;
    for (int s : sh)
        for (int g : gr) {
            fdlb_status st = set_tiles(c, s, g);
            if (st != FDLB_OK) return st;
            // trial steps read the current half and write the other one without swapping:
            // the state is left exactly as it was
            int per = 1;
            fdlb_status ts;
            for (int w = 0; w < 2; ++w)
                if ((ts = trial_launch(c, -1, h, &per)) != FDLB_OK) return ts;
            const int units = (trial_steps + per - 1) / per;
            HIPCHK(c, hipEventRecord(ev.e0, c->stream));
            for (int u = 0; u < units; ++u)
                if ((ts = trial_launch(c, -1, h, &per)) != FDLB_OK) return ts;
            HIPCHK(c, hipEventRecord(ev.e1, c->stream));
            HIPCHK(c, hipEventSynchronize(ev.e1));
            float ms = 0.0f;
            HIPCHK(c, hipEventElapsedTime(&ms, ev.e0, ev.e1));
            ms /= (float)(units * per);
            if (best < 0.0f || ms < best) {
                best = ms;
                best_s = s;
                best_g = g;
            }
        }
    if (best_ms) *best_ms = best;
    return set_tiles(c, best_s, best_g);
}

void fdlb_destroy(fdlb_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    release(c);
}

const char *fdlb_strerror(fdlb_status s) {
    switch (s) {
    case FDLB_OK: return "ok";
    case FDLB_EINVAL: return "invalid argument";
    case FDLB_ENOMEM: return "out of memory";
    case FDLB_EDEVICE: return "device error";
    case FDLB_ENONPHYS: return "non-physical state (n <= 0, T <= 0, non-finite, or |u dt/dx| >= 1)";
    case FDLB_ESTATE: return "no state set";
    default: return "unknown status";
    }
}

const char *fdlb_last_error(const fdlb_ctx *c) { return c ? c->err.c_str() : g_create_err.c_str(); }

int32_t fdlb_tile_shapes(int32_t *tx_ty, int32_t cap) {
    for (int s = 0; s < fdlb::kNumTileShapes && s < cap; ++s) {
        tx_ty[2 * s] = fdlb::kTileShapes[s].tx;
        tx_ty[2 * s + 1] = fdlb::kTileShapes[s].ty;
    }
    return fdlb::kNumTileShapes;
}

}  // extern "C"
