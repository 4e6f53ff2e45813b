// Host runtime of the C interface in abft_stencil.h: validation, workspace, launch shapes,
// the online / offline / plain step sequences, graph capture, autotuning and reports.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <utility>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "abft_internal.h"

using namespace abft;

namespace {

thread_local std::string g_init_error;

constexpr int kDefaultEvents = 4096;
constexpr size_t kLdsLimit = 64 * 1024;       // check and locate kernels
constexpr size_t kSweepLdsLimit = 160 * 1024; // gfx950: 160 KB of LDS per compute unit
constexpr int kTargetTiles = 1024;     // blocks of 4 wavefronts per sweep, untuned default
constexpr int kTargetTilesWide = 256;  // blocks of 8 wavefronts: one per compute unit
constexpr int kMaxBatchClasses = 16;   // size classes (launches per sweep) of a batch

size_t esize(int dtype) { return dtype == ABFT_F32 ? 4 : 8; }

double round_to(int dtype, double v) { return dtype == ABFT_F32 ? (double)(float)v : v; }

struct CheckShape {
    int tyi = 0, tzi = 0, nyt = 0, nzt = 0, ry = 0, rz = 0;
};

}  // namespace

struct abft_ctx {
    // problem
    int nx = 0, ny = 0, nz = 0, dtype = 0, bc = 0;
    Stencil st{};
    const void* C = nullptr;
    double cs = 0.0;
    void* u[3] = {nullptr, nullptr, nullptr};
    bool own_u2 = false;
    // options
    int mode = 0, period = 1, csum = CS_F64, auto_correct = 1, input_check = 0, recompute = 0;
    int tile_x = 0;              // tile-local checksums of this many points, or 0 (rows)
    double eps = 0.0;
    std::string cache_path;
    hipStream_t stream = nullptr;
    // workspace
    std::vector<void*> allocs;
    double* B[2] = {nullptr, nullptr};
    double* W[2] = {nullptr, nullptr};  // online: index-weighted row sums beside B
    double* Et = nullptr;        // tile-local checksums: boundary terms of the input's tiles
    double* cB = nullptr;
    double* cA = nullptr;
    FlagSlot* slot[2] = {nullptr, nullptr};
    Counters* cnt = nullptr;
    abft_event* ev = nullptr;
    int ev_cap = 0;
    uint32_t* win = nullptr;     // [2 windows][first, recheck]
    uint32_t* ticket = nullptr;
    int64_t* tbase = nullptr;
    double* E = nullptr;         // [period][nz][ny] when the boundary terms do not cancel
    double* Btmp[2] = {nullptr, nullptr};  // interpolation between check chunks (long windows)
    abft_fault* faults = nullptr;
    int32_t* fault_first = nullptr;
    int64_t fault_tmax = 0;
    int nfaults = 0;
    bool mem_faults = false;     // the plan holds memory-resident flips
    // launch shapes
    SweepShape shape{};
    int nyb = 0, nzb = 0, ntiles = 0;
    CheckShape ck;
    // trajectory state
    int64_t t = 0;
    int cur = 0, bcur = 0;
    // offline state
    int ckpt = 0, wq = 1, wr = 2, bck = 0;
    int64_t win_t0 = 0, win_index = 0;
    int win_j = 0;
    bool halted = false;
    int64_t skipped = 0;
    // graphs
    std::map<std::pair<int64_t, int>, hipGraphExec_t> graphs;
    std::string err;
    // batch of grids (abft_stencil_init_batch)
    bool batch = false;
    struct Grid {
        int nx, ny, nz, tz, nyb, ntiles;
        void* u[2];
        const void* C;
        double cs;
        Stencil st;
        double* B[2];
        double* W[2];
        double* cB;
        double* cA;
        FlagSlot* slot[2];
        int sub = 0;  // which chunk count of its launch the rows take (GridDesc::sub)
    };
    std::vector<Grid> grids;
    GridDesc* d_grids = nullptr;
    // The grids of one size class share a launch of the batched sweep: its shape (lanes per
    // row, chunks, 16-byte or single-element accesses), slab depth and dispatch form.  A
    // sweep is one launch per class.
    struct Class {
        std::vector<int> grids;
        SweepShape shape{};
        int tz = 8, persistent = 1, nblocks = 0, ntiles = 0;
        size_t lds = 0;
        int2* order = nullptr;      // the class's tiles, largest first (inside d_order)
        uint32_t* queue = nullptr;  // two words of `queue`
    };
    std::vector<Class> classes;
    int2* d_order = nullptr;        // tile lists of all classes
    size_t order_cap = 0;           // entries d_order holds (the most any layout needs)
    uint32_t* queue = nullptr;      // persistent launches: two words per class
    int maxnx = 0;
    int num_cus = 0;
};

namespace {

abft_status fail(abft_ctx* c, abft_status s, const std::string& msg)
{
    if (c) c->err = msg;
    else g_init_error = msg;
    return s;
}

abft_status hip_fail(abft_ctx* c, hipError_t e, const char* what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(c, ABFT_E_HIP, m);
}

#define HIPCHK(ctx, expr)                                           \
    do {                                                            \
        hipError_t _e = (expr);                                     \
        if (_e != hipSuccess) return hip_fail((ctx), _e, #expr);    \
    } while (0)

template <typename P>
abft_status dalloc(abft_ctx* c, P** p, size_t bytes)
{
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, bytes ? bytes : 16);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, ABFT_E_NOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    c->allocs.push_back(q);
    *p = static_cast<P*>(q);
    return ABFT_OK;
}

void free_all(abft_ctx* c)
{
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    for (void* p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
}

// Star taps of radius 1 or 2 (the centre and points along one axis at distance 1 or 2) ->
// weight slots; the radius is 2 when any distance-2 tap is present.
abft_status map_taps(abft_ctx* c, const abft_problem* p)
{
    c->st = Stencil{};
    c->st.bc = p->bc;
    c->st.g = round_to(p->dtype, p->bc_value);
    c->st.rad = 1;
    // A tap off the axes (two or three offsets non-zero, each within -1..1) makes the
    // stencil a 27-point box: every tap then goes to the box weights.
    bool box = false;
    for (int k = 0; k < p->ntaps; ++k) {
        const abft_tap& t = p->taps[k];
        const int axes = (t.dx != 0) + (t.dy != 0) + (t.dz != 0);
        if (axes > 1) box = true;
    }
    if (box) {
        c->st.box = 1;
        for (int k = 0; k < p->ntaps; ++k) {
            const abft_tap& t = p->taps[k];
            if (std::abs(t.dx) > 1 || std::abs(t.dy) > 1 || std::abs(t.dz) > 1)
                return fail(c, ABFT_E_UNSUPPORTED,
                            "box stencils on the GPU take offsets within -1..1 on every axis");
            const int slot = box_slot(t.dx, t.dy, t.dz);
            if (c->st.bmask & (1u << slot)) return fail(c, ABFT_E_INVAL, "duplicate tap offset");
            if (!std::isfinite(t.w)) return fail(c, ABFT_E_INVAL, "non-finite tap weight");
            c->st.bmask |= 1u << slot;
            c->st.wb[slot] = round_to(p->dtype, t.w);
        }
        return ABFT_OK;
    }
    for (int k = 0; k < p->ntaps; ++k) {
        const abft_tap& t = p->taps[k];
        const int axes = (t.dx != 0) + (t.dy != 0) + (t.dz != 0);
        const int ad = std::abs(t.dx) + std::abs(t.dy) + std::abs(t.dz);
        if (axes > 1 || ad > 2)
            return fail(c, ABFT_E_UNSUPPORTED,
                        "GPU kernels cover star stencils of radius 1 or 2 (centre and points "
                        "along one axis)");
        int slot = W_C;
        if (t.dx != 0) slot = w_slot(0, std::abs(t.dx), t.dx);
        else if (t.dy != 0) slot = w_slot(1, std::abs(t.dy), t.dy);
        else if (t.dz != 0) slot = w_slot(2, std::abs(t.dz), t.dz);
        if (c->st.mask & (1u << slot)) return fail(c, ABFT_E_INVAL, "duplicate tap offset");
        if (!std::isfinite(t.w)) return fail(c, ABFT_E_INVAL, "non-finite tap weight");
        c->st.mask |= 1u << slot;
        c->st.w[slot] = round_to(p->dtype, t.w);
        if (ad == 2) c->st.rad = 2;
    }
    return ABFT_OK;
}

// Default launch shape: 16-byte accesses when rows are 16-byte multiples, 16 lanes per row for
// short rows (4 rows per wavefront), 64 lanes for long rows.  Grids with rows enough for one
// block of 8 wavefronts per compute unit take that (the deeper block halves the share of halo
// rows it loads and keeps more loads in flight per CU), cut into about that many z-slabs;
// smaller grids take blocks of 4 wavefronts and enough z-slabs for ~1024 blocks.
bool default_shape(int dtype, int nx, int ny, int nz, int rad, int box, SweepShape* s)
{
    const int vf = 16 / (int)esize(dtype);
    SweepShape r{};
    r.rad = rad;
    r.box = box;
    if (nx % vf == 0) {
        r.vec = vf;
        if (nx <= 16 * vf * 4) {
            r.lpr = 16;
            const int n = (nx + 16 * vf - 1) / (16 * vf);
            r.nch = n <= 1 ? 1 : n <= 2 ? 2 : 4;
        } else {
            r.lpr = 64;
            const int n = (nx + 64 * vf - 1) / (64 * vf);
            if (n > 8) return false;
            r.nch = n <= 1 ? 1 : n <= 2 ? 2 : n <= 4 ? 4 : 8;
        }
    } else {
        r.vec = 1;
        r.lpr = 64;
        if (nx <= 256) r.nch = 4;
        else if (nx <= 1024) r.nch = 16;
        else return false;
    }
    r.pf = 1;
    auto slabs = [&](int target) {
        const int ty = sweep_rows_per_block(r);
        const int64_t nyb = (ny + ty - 1) / ty;
        const int64_t nzb = std::max<int64_t>(1, std::min<int64_t>(nz, (target + nyb - 1) / nyb));
        r.tz = (int)((nz + nzb - 1) / nzb);
        return nyb * nz;  // blocks at one plane per block
    };
    r.nw = 8;
    if (slabs(kTargetTilesWide) < kTargetTilesWide || !sweep_shape_supported(dtype, r) ||
        sweep_lds_bytes(dtype, nx, r, true) > kSweepLdsLimit) {
        r.nw = 4;
        slabs(kTargetTiles);
    }
    *s = r;
    return true;
}

abft_status apply_shape(abft_ctx* c, const SweepShape& shape)
{
    SweepShape s = shape;
    s.rad = c->st.rad;  // the kernels are built per stencil radius and form
    s.box = c->st.box;
    if (!sweep_shape_supported(c->dtype, s)) return fail(c, ABFT_E_UNSUPPORTED, "launch shape");
    if ((int64_t)s.lpr * s.nch * s.vec < c->nx) return fail(c, ABFT_E_UNSUPPORTED, "row too long");
    if (s.vec > 1 && c->nx % s.vec) return fail(c, ABFT_E_UNSUPPORTED, "row not 16-byte multiple");
    if (c->tile_x && s.vec != 16 / (int)esize(c->dtype))
        return fail(c, ABFT_E_UNSUPPORTED, "tile-local checksums need 16-byte accesses");
    if (sweep_lds_bytes(c->dtype, c->nx, s, c->input_check) > kSweepLdsLimit)
        return fail(c, ABFT_E_UNSUPPORTED, "rows too long for the LDS plane buffers");
    const int ty = sweep_rows_per_block(s);
    const int64_t nyb = (c->ny + ty - 1) / ty;
    const int64_t nzb = (c->nz + s.tz - 1) / s.tz;
    if (nyb * nzb > (int64_t)1 << 30) return fail(c, ABFT_E_UNSUPPORTED, "grid too large");
    c->shape = s;
    c->nyb = (int)nyb;
    c->nzb = (int)nzb;
    c->ntiles = (int)(nyb * nzb);
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    return ABFT_OK;
}

std::string cache_key(const abft_ctx* c)
{
    std::ostringstream o;
    o << c->dtype << ' ' << c->nx << ' ' << c->ny << ' ' << c->nz << ' ' << c->mode << ' '
      << c->csum;
    if (c->st.rad != 1) o << " r" << c->st.rad;
    if (c->st.box) o << " box";
    if (c->input_check) o << " ic";
    if (c->tile_x) o << " t" << c->tile_x;
    return o.str();
}

// A tuning-cache line: six numbers and the variant's tags (words) form its key, the shape
// follows.  Returns the key and the index of the first shape token.
std::string cache_line_key(const std::vector<std::string>& tok, size_t* first)
{
    size_t i = 0;
    std::string k;
    for (; i < tok.size() && i < 6; ++i) k += (i ? " " : "") + tok[i];
    for (; i < tok.size() && !tok[i].empty() && std::isalpha((unsigned char)tok[i][0]); ++i)
        k += " " + tok[i];
    *first = i;
    return k;
}

std::vector<std::string> split_words(const std::string& line)
{
    std::istringstream in(line);
    std::vector<std::string> tok;
    for (std::string w; in >> w;) tok.push_back(w);
    return tok;
}

bool cache_lookup(const abft_ctx* c, SweepShape* s)
{
    if (c->cache_path.empty()) return false;
    std::ifstream f(c->cache_path);
    if (!f) return false;
    const std::string key = cache_key(c);
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        const std::vector<std::string> tok = split_words(line);
        size_t i = 0;
        if (cache_line_key(tok, &i) != key || tok.size() < i + 4) continue;
        SweepShape r{};
        try {
            r.lpr = std::stoi(tok[i]);
            r.nch = std::stoi(tok[i + 1]);
            r.vec = std::stoi(tok[i + 2]);
            r.tz = std::stoi(tok[i + 3]);
            r.pf = tok.size() > i + 4 ? std::stoi(tok[i + 4]) : 1;
            r.nw = tok.size() > i + 5 ? std::stoi(tok[i + 5]) : 4;
        } catch (...) {
            continue;
        }
        *s = r;
        found = true;
    }
    return found;
}

void cache_store(const abft_ctx* c)
{
    if (c->cache_path.empty()) return;
    std::vector<std::string> keep;
    {
        std::ifstream f(c->cache_path);
        std::string line;
        const std::string key = cache_key(c);
        while (f && std::getline(f, line)) {
            size_t i = 0;
            if (!line.empty() && cache_line_key(split_words(line), &i) != key)
                keep.push_back(line);
        }
    }
    std::ofstream f(c->cache_path, std::ios::trunc);
    for (auto& l : keep) f << l << '\n';
    f << cache_key(c) << ' ' << c->shape.lpr << ' ' << c->shape.nch << ' ' << c->shape.vec << ' '
      << c->shape.tz << ' ' << c->shape.pf << ' ' << c->shape.nw << '\n';
}

// Offline check tiles: an interior of tyi rows x tzi layers of the checksum plane plus a halo
// of k on each side, at most kCheckCells cells per thread, and enough tiles to spread over the
// compute units.
void check_shape(abft_ctx* c, int k)
{
    CheckShape s;
    const bool per = c->bc == ABFT_BC_PERIODIC;
    const int64_t cap = (int64_t)kCheckCells * kCheckBlock;
    auto region = [&](int tyi, int tzi, int* ry, int* rz) {
        *ry = per ? tyi + 2 * k : std::min(c->ny, tyi + 2 * k);
        *rz = per ? tzi + 2 * k : std::min(c->nz, tzi + 2 * k);
        return (int64_t)*ry * *rz;
    };
    s.tzi = std::min(c->nz, 16);
    s.tyi = std::min(c->ny, 32);
    int ry, rz;
    while (region(s.tyi, s.tzi, &ry, &rz) > cap && (s.tyi > 1 || s.tzi > 1)) {
        if (s.tyi >= s.tzi && s.tyi > 1) s.tyi = (s.tyi + 1) / 2;
        else s.tzi = (s.tzi + 1) / 2;
    }
    auto tiles = [&](int tyi, int tzi) {
        return (int64_t)((c->ny + tyi - 1) / tyi) * ((c->nz + tzi - 1) / tzi);
    };
    while (tiles(s.tyi, s.tzi) < 256 && (s.tyi > 8 || s.tzi > 4)) {
        if (s.tyi > 8) s.tyi /= 2;
        else s.tzi /= 2;
    }
    region(s.tyi, s.tzi, &s.ry, &s.rz);
    s.nyt = (c->ny + s.tyi - 1) / s.tyi;
    s.nzt = (c->nz + s.tzi - 1) / s.tzi;
    c->ck = s;
}

SweepArgs base_args(const abft_ctx* c)
{
    SweepArgs a{};
    a.C = c->C;
    a.c_scalar = c->cs;
    a.st = c->st;
    a.nx = c->nx;
    a.ny = c->ny;
    a.nz = c->nz;
    a.tz = c->shape.tz;
    a.nyb = c->nyb;
    a.ntiles = c->ntiles;
    a.cB = c->cB;
    a.eps = c->eps;
    a.cnt = c->cnt;
    a.ev = c->ev;
    a.ev_cap = c->ev_cap;
    a.faults = c->faults;
    a.fault_first = c->fault_first;
    a.fault_tmax = c->faults ? c->fault_tmax : 0;
    return a;
}

// The x-boundary terms of Theorem 1 cancel in the weighted sum (and need not be recorded for
// the offline interpolation) under the periodic rule, and under clamp for radius-1 x taps of
// equal weight; clamp with distance-2 x taps, and the constant rule, leave them.
bool boundary_terms_needed(int bc, const Stencil& st)
{
    if (bc == ABFT_BC_PERIODIC) return false;
    if (st.box) {
        // per (dy, dz) the dx = -1 and dx = +1 terms of a row cancel under clamp only with
        // equal weights
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy) {
                const int sm = box_slot(-1, dy, dz), sp = box_slot(1, dy, dz);
                const bool hm = st.bmask & (1u << sm), hp = st.bmask & (1u << sp);
                if (bc != ABFT_BC_CLAMP && (hm || hp)) return true;
                if (hm != hp || (hm && st.wb[sm] != st.wb[sp])) return true;
            }
        return false;
    }
    const uint32_t m = st.mask;
    const bool xm = m & (1u << W_XM), xp = m & (1u << W_XP);
    const bool x2 = m & ((1u << W_XM2) | (1u << W_XP2));
    if (bc == ABFT_BC_CLAMP)
        return x2 || (xm != xp) || (xm && st.w[W_XM] != st.w[W_XP]);
    return xm || xp || x2;
}

bool need_boundary_terms(const abft_ctx* c) { return boundary_terms_needed(c->bc, c->st); }

int buf_of(const abft_ctx* c, int j) { return j == 0 ? c->ckpt : ((j & 1) ? c->wq : c->wr); }

// ---- online / plain ------------------------------------------------------------------------
// Locate/correct and input repair after online sweep t, whose input is u[in] with checksums
// B[bin] and whose output is u[in ^ 1] with checksums B[bin ^ 1].
FixArgs online_fix_args(const abft_ctx* c, int in, int bin, int64_t t, const int64_t* tbase,
                        int64_t t_off)
{
    FixArgs f{};
    f.uin = c->u[in];
    f.uout = c->u[in ^ 1];
    f.Bn = c->B[bin ^ 1];
    f.cA = c->cA;
    f.Bt = c->B[bin];
    f.Wt = c->W[bin];
    f.Wn = c->W[bin ^ 1];
    f.cB = c->cB;
    f.C = c->C;
    f.c_scalar = c->cs;
    f.recompute = c->recompute;
    f.tile_x = c->tile_x;
    f.st = c->st;
    f.nx = c->nx;
    f.ny = c->ny;
    f.nz = c->nz;
    f.eps = c->eps;
    f.slot = c->slot[t & 1];
    f.cnt = c->cnt;
    f.ev = c->ev;
    f.ev_cap = c->ev_cap;
    f.t_base = tbase;
    f.t_off = t_off;
    return f;
}

abft_status enqueue_online(abft_ctx* c, int64_t n, const int64_t* tbase, int64_t t0)
{
    for (int64_t i = 0; i < n; ++i) {
        const int64_t t = c->t + i;
        SweepArgs a = base_args(c);
        a.uin = c->u[c->cur];
        a.uout = c->u[c->cur ^ 1];
        a.t_base = tbase;
        a.t_off = tbase ? t - t0 : t;
        int mode = MODE_PLAIN;
        if (c->mode == ABFT_MODE_ONLINE && c->tile_x) {
            mode = MODE_TILE;
            a.Bn = c->B[c->bcur ^ 1];
            a.Et = c->Et;
            a.zero_ptr = &c->slot[(t + 1) & 1]->count;
            a.zero_n = 2;
        } else if (c->mode == ABFT_MODE_ONLINE) {
            mode = c->input_check ? MODE_PROTM : MODE_PROT;
            a.Bt = c->B[c->bcur];
            a.Bn = c->B[c->bcur ^ 1];
            a.Wn = c->W[c->bcur ^ 1];
            a.slot = c->slot[t & 1];
            a.zero_ptr = &c->slot[(t + 1) & 1]->count;
            a.zero_n = 2;  // the next sweep's row and input-row counts
        }
        hipError_t e;
        if (c->mem_faults) {
            e = launch_mem_flip(c->dtype, c->u[c->cur], c->nx, c->ny, c->faults, c->fault_first,
                                c->fault_tmax, tbase, a.t_off, c->stream);
            if (e != hipSuccess) return hip_fail(c, e, "memory fault launch");
        }
        e = launch_sweep(c->dtype, mode, c->csum, c->shape, a, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "sweep launch");
        if (mode == MODE_TILE) {
            TileCheckArgs k{};
            k.Bt = c->B[c->bcur];
            k.Bn = c->B[c->bcur ^ 1];
            k.cB = c->cB;
            k.Et = c->Et;
            k.st = c->st;
            k.nx = c->nx;
            k.ny = c->ny;
            k.nz = c->nz;
            k.tile_x = c->tile_x;
            k.eps = c->eps;
            k.slot = c->slot[t & 1];
            k.cnt = c->cnt;
            k.ev = c->ev;
            k.ev_cap = c->ev_cap;
            k.t_base = tbase;
            k.t_off = a.t_off;
            e = launch_tile_check(k, c->stream);
            if (e != hipSuccess) return hip_fail(c, e, "tile check launch");
        }
        if (c->mode == ABFT_MODE_ONLINE && c->auto_correct) {
            const FixArgs f = online_fix_args(c, c->cur, c->bcur, t, tbase, a.t_off);
            e = launch_fixup(c->dtype, f, c->stream);
            if (e != hipSuccess) return hip_fail(c, e, "locate/correct launch");
        }
        c->cur ^= 1;
        if (c->mode == ABFT_MODE_ONLINE) c->bcur ^= 1;
    }
    c->t += n;
    return ABFT_OK;
}

// ---- offline ------------------------------------------------------------------------------
abft_status offline_sweep(abft_ctx* c, int j, int k, int attempt, const uint32_t* guard)
{
    SweepArgs a = base_args(c);
    a.uin = c->u[buf_of(c, j)];
    a.uout = c->u[buf_of(c, j + 1)];
    a.t_off = c->win_t0 + j;
    a.attempt = attempt;
    a.guard = guard;
    a.Bn = c->B[c->bck ^ 1];
    if (c->E) a.E = c->E + (size_t)j * c->nz * c->ny;
    if (j == 0 && attempt == 0) {
        a.zero_ptr = c->win + 2 * (c->win_index & 1);
        a.zero_n = 2;
    }
    const int mode = (j == k - 1) ? MODE_CSUM : MODE_PLAIN;
    // with the input check, the window's last sweep also keeps the weighted sums of the
    // checkpoint it forms
    if (mode == MODE_CSUM && c->input_check) a.Wn = c->W[c->bck ^ 1];
    hipError_t e;
    if (c->mem_faults && attempt == 0) {
        // the window's first input is the checkpoint itself
        e = launch_mem_flip(c->dtype, c->u[buf_of(c, j)], c->nx, c->ny, c->faults,
                            c->fault_first, c->fault_tmax, nullptr, a.t_off, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "memory fault launch");
    }
    e = launch_sweep(c->dtype, mode, c->csum, c->shape, a, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "offline sweep launch");
    return ABFT_OK;
}

abft_status offline_check(abft_ctx* c, int k, int attempt, const uint32_t* guard)
{
    const int chunk = std::min(k, kCheckChunk / c->st.rad);
    check_shape(c, chunk * c->st.rad);  // the dependency cone: radius x steps
    CheckArgs a{};
    a.Bdir = c->B[c->bck ^ 1];
    a.cB = c->cB;
    a.E = c->E;
    a.st = c->st;
    a.nx = c->nx;
    a.ny = c->ny;
    a.nz = c->nz;
    a.eps = c->eps;
    a.tyi = c->ck.tyi;
    a.tzi = c->ck.tzi;
    a.nyt = c->ck.nyt;
    a.nzt = c->ck.nzt;
    a.ry_max = c->ck.ry;
    a.rz_max = c->ck.rz;
    uint32_t* w = c->win + 2 * (c->win_index & 1);
    a.flag_count = attempt == 0 ? w : w + 1;
    a.guard = guard;
    a.ticket = c->ticket;
    a.cnt = c->cnt;
    a.ev = c->ev;
    a.ev_cap = c->ev_cap;
    a.attempt = attempt;
    a.auto_correct = c->auto_correct;
    a.t_first = c->win_t0;
    a.t_last = c->win_t0 + k - 1;
    const int nchunks = (k + chunk - 1) / chunk;
    for (int ch = 0; ch < nchunks; ++ch) {
        a.s0 = ch * chunk;
        a.ns = std::min(chunk, k - a.s0);
        a.Bin = ch == 0 ? c->B[c->bck] : c->Btmp[(ch - 1) & 1];
        a.Bout = ch == nchunks - 1 ? nullptr : c->Btmp[ch & 1];
        hipError_t e = launch_check(a, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "offline check launch");
    }
    return ABFT_OK;
}

void offline_rotate(abft_ctx* c, int k)
{
    const int nb = buf_of(c, k);
    int others[2], m = 0;
    for (int b = 0; b < 3; ++b)
        if (b != nb) others[m++] = b;
    c->ckpt = nb;
    c->wq = others[0];
    c->wr = others[1];
    c->bck ^= 1;
    c->win_t0 += k;
    c->win_j = 0;
    c->win_index++;
    c->cur = c->ckpt;
}

// Recompute of the window from the checkpoint (attempt 1) and its re-check.  One launch runs
// the k sweeps with grid barriers between them; where the shape's LDS leaves no room for that
// kernel's own few bytes, k guarded sweep launches do the same work.
abft_status offline_recompute(abft_ctx* c, int k, const uint32_t* guard)
{
    if (c->input_check) {
        // the checkpoint as it was written, before the window is run again from it
        hipError_t e = launch_verify_ckpt(c->dtype, c->u[buf_of(c, 0)], c->B[c->bck],
                                          c->W[c->bck], c->nx, c->ny, c->nz, c->eps, guard,
                                          c->cnt, c->ev, c->ev_cap, c->win_t0, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "checkpoint check launch");
    }
    if (c->num_cus > 0 && recover_shape_supported(c->dtype, c->shape) &&
        sweep_lds_bytes(c->dtype, c->nx, c->shape, c->input_check) + 256 <= kSweepLdsLimit) {
        RecoverArgs r{};
        r.a = base_args(c);
        r.a.attempt = 1;
        r.a.Bn = c->B[c->bck ^ 1];
        if (c->input_check) r.a.Wn = c->W[c->bck ^ 1];
        r.ckpt = c->u[buf_of(c, 0)];
        r.odd = c->u[buf_of(c, 1)];
        r.even = c->u[buf_of(c, 2)];
        r.E = c->E;
        r.k = k;
        r.t_first = c->win_t0;
        r.guard = guard;
        r.bar = c->ticket + 2;
        hipError_t e = launch_recover(c->dtype, c->csum, c->shape, r, c->num_cus, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "rollback recompute launch");
        return offline_check(c, k, 1, guard);
    }
    hipError_t e = launch_rollback_note(guard, c->cnt, c->ev, c->ev_cap, c->win_t0, k, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "rollback launch");
    for (int j = 0; j < k; ++j) {
        abft_status s = offline_sweep(c, j, k, 1, guard);
        if (s) return s;
    }
    return offline_check(c, k, 1, guard);
}

abft_status offline_close_window(abft_ctx* c, int k)
{
    abft_status s = offline_check(c, k, 0, nullptr);
    if (s) return s;
    uint32_t* w = c->win + 2 * (c->win_index & 1);
    if (c->auto_correct) {
        s = offline_recompute(c, k, w);
        if (s) return s;
        offline_rotate(c, k);
        return ABFT_OK;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    uint32_t flagged = 0;
    HIPCHK(c, hipMemcpy(&flagged, w, sizeof(flagged), hipMemcpyDeviceToHost));
    if (flagged) {
        c->halted = true;
        c->win_j = k;  // the window's sweeps are done; its result awaits correct()
        return ABFT_OK;
    }
    offline_rotate(c, k);
    return ABFT_OK;
}

abft_status enqueue_offline(abft_ctx* c, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) {
        if (c->halted) {
            c->skipped += n - i;
            return ABFT_OK;
        }
        const int j = c->win_j;
        abft_status s = offline_sweep(c, j, c->period, 0, nullptr);
        if (s) return s;
        c->win_j = j + 1;
        c->t++;
        c->cur = buf_of(c, c->win_j);
        if (c->win_j == c->period) {
            s = offline_close_window(c, c->period);
            if (s) return s;
        }
    }
    return ABFT_OK;
}

// "After completion" detection: a partial window is checked now and closed.
abft_status offline_flush(abft_ctx* c)
{
    if (c->halted || c->win_j == 0) return ABFT_OK;
    const int k = c->win_j;
    hipError_t e = launch_row_sums(c->dtype, c->u[buf_of(c, k)], 0.0, c->nx,
                                   (int64_t)c->nz * c->ny, c->B[c->bck ^ 1], c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "row checksum launch");
    return offline_close_window(c, k);
}

abft_status read_counters(abft_ctx* c, Counters* h)
{
    HIPCHK(c, hipMemcpy(h, c->cnt, sizeof(Counters), hipMemcpyDeviceToHost));
    return ABFT_OK;
}

abft_status validate_problem(const abft_problem* p)
{
    if (!p) return fail(nullptr, ABFT_E_INVAL, "problem is NULL");
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(nullptr, ABFT_E_INVAL, "extent < 1");
    if ((int64_t)p->nx * p->ny * p->nz > ((int64_t)1 << 40))
        return fail(nullptr, ABFT_E_INVAL, "grid too large");
    if (p->dtype != ABFT_F32 && p->dtype != ABFT_F64)
        return fail(nullptr, ABFT_E_INVAL, "dtype");
    if (p->bc < ABFT_BC_CLAMP || p->bc > ABFT_BC_CONSTANT)
        return fail(nullptr, ABFT_E_INVAL, "boundary rule");
    if (p->ntaps < 1 || p->ntaps > 27 || !p->taps)
        return fail(nullptr, ABFT_E_INVAL, "taps (1..27 required)");
    if (!p->u0 || !p->u1 || p->u0 == p->u1)
        return fail(nullptr, ABFT_E_INVAL, "u0 and u1 must be distinct device buffers");
    if (!std::isfinite(p->bc_value) || !std::isfinite(p->cterm_scalar))
        return fail(nullptr, ABFT_E_INVAL, "non-finite constant");
    return ABFT_OK;
}

abft_status validate_options(const abft_problem* p, const abft_options* o)
{
    if (!o) return fail(nullptr, ABFT_E_INVAL, "options is NULL");
    if (o->mode < ABFT_MODE_NONE || o->mode > ABFT_MODE_OFFLINE)
        return fail(nullptr, ABFT_E_INVAL, "mode");
    if (o->mode == ABFT_MODE_OFFLINE && o->period < 1)
        return fail(nullptr, ABFT_E_INVAL, "period must be >= 1");
    if (o->mode == ABFT_MODE_OFFLINE && o->period > kMaxPeriod)
        return fail(nullptr, ABFT_E_UNSUPPORTED, "period above 128");
    if (o->mode != ABFT_MODE_NONE && !(o->threshold > 0.0 && std::isfinite(o->threshold)))
        return fail(nullptr, ABFT_E_INVAL, "threshold must be > 0");
    if (o->csum != ABFT_CSUM_F64 && o->csum != ABFT_CSUM_F32_COMP)
        return fail(nullptr, ABFT_E_INVAL, "checksum accumulation");
    if (o->csum == ABFT_CSUM_F32_COMP && p->dtype != ABFT_F32)
        return fail(nullptr, ABFT_E_INVAL, "compensated fp32 checksums need an fp32 grid");
    if (o->max_events < 0) return fail(nullptr, ABFT_E_INVAL, "max_events");
    if (o->correction != ABFT_CORRECT_CHECKSUM && o->correction != ABFT_CORRECT_RECOMPUTE)
        return fail(nullptr, ABFT_E_INVAL, "correction");
    return ABFT_OK;
}

// Sweep variant of a batch: plain, protected, or protected with the input-side check.
int batch_mode(const abft_ctx* c)
{
    if (c->mode != ABFT_MODE_ONLINE) return MODE_PLAIN;
    return c->input_check ? MODE_PROTM : MODE_PROT;
}

// ---- batches of grids ------------------------------------------------------------------------
// Batched-sweep shapes by the longest row they hold (lpr * nch * vec points), shortest first:
// 16 lanes per row with 1, 2 or 4 chunks of 16-byte accesses, 64 lanes with 1, 2 or 4, and for
// rows that are not 16-byte multiples 64 lanes of single elements with 4 or 16 chunks.
std::vector<SweepShape> batch_shape_list(int dtype, bool vec_ok)
{
    const int vf = 16 / (int)esize(dtype);
    std::vector<SweepShape> v;
    auto add = [&](int lpr, int nch, int vec) {
        SweepShape s{};
        s.lpr = lpr;
        s.nch = nch;
        s.vec = vec;
        s.tz = 1;
        s.pf = 1;
        s.nw = kBatchWaves;
        v.push_back(s);
    };
    if (vec_ok) {
        add(16, 1, vf);
        add(16, 2, vf);
        add(16, 4, vf);
        add(64, 1, vf);
        add(64, 2, vf);
        add(64, 4, vf);
    } else {
        add(64, 4, 1);
        add(64, 16, 1);
    }
    std::stable_sort(v.begin(), v.end(), [](const SweepShape& a, const SweepShape& b) {
        return a.lpr * a.nch * a.vec < b.lpr * b.nch * b.vec;
    });
    return v;
}

int shape_width(const SweepShape& s) { return s.lpr * s.nch * s.vec; }

// The shapes that hold rows of nx points with the least width (16 lanes first), or none.
std::vector<SweepShape> batch_shapes_for(int dtype, bool vec_ok, int nx)
{
    std::vector<SweepShape> out;
    int w = 0;
    for (const SweepShape& s : batch_shape_list(dtype, vec_ok)) {
        if (shape_width(s) < nx) continue;
        if (out.empty()) w = shape_width(s);
        if (shape_width(s) != w) break;
        out.push_back(s);
    }
    return out;
}

bool grid_vec_ok(const abft_ctx* c, int g)
{
    return c->grids[g].nx % (16 / (int)esize(c->dtype)) == 0;
}

// Lays every class out: its grids' tiles for the class's slab depth (largest first, so that
// the tail of a launch is made of small tiles), its LDS size and launch size; uploads the tile
// lists and the grid descriptors.
abft_status batch_layout(abft_ctx* c)
{
    std::vector<GridDesc> desc(c->grids.size());
    std::vector<int2> order;
    std::vector<std::pair<int64_t, int2>> tiles;
    for (size_t k = 0; k < c->classes.size(); ++k) {
        auto& K = c->classes[k];
        const int ty = sweep_rows_per_block(K.shape);
        int maxtz = 1, maxnx = 1;
        tiles.clear();
        for (int g : K.grids) {
            auto& G = c->grids[g];
            G.tz = std::max(1, std::min(K.tz, G.nz));
            G.nyb = (G.ny + ty - 1) / ty;
            G.ntiles = G.nyb * ((G.nz + G.tz - 1) / G.tz);
            maxtz = std::max(maxtz, G.tz);
            maxnx = std::max(maxnx, G.nx);
            if (shape_width(K.shape) < G.nx || (K.shape.vec > 1 && G.nx % K.shape.vec))
                return fail(c, ABFT_E_UNSUPPORTED, "batch class shape does not hold its rows");
            // the fewest chunks of the launch that hold the rows
            const int cw = K.shape.lpr * K.shape.vec;
            G.sub = 0;
            if (K.shape.nchc > 0 && cw * K.shape.nchc >= G.nx) G.sub = 2;
            else if (K.shape.nchb > 0 && cw * K.shape.nchb >= G.nx) G.sub = 1;
            for (int t = 0; t < G.ntiles; ++t) {
                const int yb = t % G.nyb, zb = t / G.nyb;
                const int64_t rows = std::min(ty, G.ny - yb * ty);
                const int64_t planes = std::min(G.tz, G.nz - zb * G.tz);
                tiles.push_back({rows * planes * G.nx, int2(g, t)});
            }
        }
        std::stable_sort(tiles.begin(), tiles.end(),
                         [](const auto& a, const auto& b) { return a.first > b.first; });
        K.lds = batch_lds_bytes(c->dtype, maxnx, maxtz, K.shape, c->input_check);
        if (K.lds > kSweepLdsLimit)
            return fail(c, ABFT_E_UNSUPPORTED, "batch tiles exceed the LDS");
        K.order = c->d_order + order.size();
        K.queue = c->queue + 2 * k;
        K.ntiles = (int)tiles.size();
        for (auto& t : tiles) order.push_back(t.second);
        const int per_cu = batch_blocks_per_cu(c->dtype, batch_mode(c), c->csum, K.shape, K.lds);
        K.nblocks = K.persistent ? std::min(K.ntiles, per_cu * c->num_cus) : K.ntiles;
    }
    if (order.size() > c->order_cap || c->classes.size() > (size_t)kMaxBatchClasses)
        return fail(c, ABFT_E_UNSUPPORTED, "batch tile list");
    for (size_t g = 0; g < c->grids.size(); ++g) {
        const auto& G = c->grids[g];
        GridDesc& d = desc[g];
        d.u[0] = G.u[0];
        d.u[1] = G.u[1];
        d.C = G.C;
        d.c_scalar = G.cs;
        d.st = G.st;
        d.nx = G.nx;
        d.ny = G.ny;
        d.nz = G.nz;
        d.tz = G.tz;
        d.nyb = G.nyb;
        d.ntiles = G.ntiles;
        d.B[0] = G.B[0];
        d.B[1] = G.B[1];
        d.W[0] = G.W[0];
        d.W[1] = G.W[1];
        d.cB = G.cB;
        d.cA = G.cA;
        d.slot[0] = G.slot[0];
        d.slot[1] = G.slot[1];
        d.sub = G.sub;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(c->d_order, order.data(), order.size() * sizeof(int2),
                        hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_grids, desc.data(), desc.size() * sizeof(GridDesc),
                        hipMemcpyHostToDevice));
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    return ABFT_OK;
}

// One launch of all grids in the shape that holds the longest row (the layout before tuning);
// for radius-1 stars each grid's rows take the fewest chunks of that shape that hold them,
// where the launch form for those chunk counts exists.
abft_status batch_single_class(abft_ctx* c, int tz, int persistent)
{
    bool vec_ok = true;
    for (size_t g = 0; g < c->grids.size(); ++g) vec_ok = vec_ok && grid_vec_ok(c, (int)g);
    const std::vector<SweepShape> sh = batch_shapes_for(c->dtype, vec_ok, c->maxnx);
    if (sh.empty()) return fail(c, ABFT_E_UNSUPPORTED, "rows too long for the batched kernel");
    abft_ctx::Class K;
    for (size_t g = 0; g < c->grids.size(); ++g) K.grids.push_back((int)g);
    K.shape = sh[0];
    K.shape.rad = c->shape.rad;
    K.shape.box = c->shape.box;
    if (K.shape.rad == 1 && !K.shape.box && vec_ok) {
        const int cw = K.shape.lpr * K.shape.vec;
        std::vector<int> need;
        for (const auto& G : c->grids) {
            int n = 1;
            while (cw * n < G.nx) n *= 2;
            if (std::find(need.begin(), need.end(), n) == need.end()) need.push_back(n);
        }
        std::sort(need.rbegin(), need.rend());
        SweepShape m = K.shape;
        if (need.size() >= 2 && need.size() <= 3 && need[0] == m.nch) {
            m.nchb = need[1];
            m.nchc = need.size() > 2 ? need[2] : 0;
            if (batch_shape_supported(c->dtype, m)) K.shape = m;
        }
    }
    K.tz = tz;
    K.persistent = persistent;
    c->classes.assign(1, K);
    return batch_layout(c);
}

BatchArgs batch_args(const abft_ctx* c, int64_t t, const int64_t* tbase, int64_t t0)
{
    BatchArgs b{};
    b.grids = c->d_grids;
    b.ngrids = (int)c->grids.size();
    b.parity = (int)(t & 1);
    b.t_base = tbase;
    b.t_off = tbase ? t - t0 : t;
    b.eps = c->eps;
    b.recompute = c->recompute;
    b.cnt = c->cnt;
    b.ev = c->ev;
    b.ev_cap = c->ev_cap;
    b.faults = c->faults;
    b.fault_first = c->fault_first;
    b.fault_tmax = c->faults ? c->fault_tmax : 0;
    return b;
}

// The launch of one class in a sweep; the first class's launch clears the flag slots of the
// next sweep.
hipError_t launch_class(const abft_ctx* c, const abft_ctx::Class& K, BatchArgs b, bool first)
{
    b.ntiles = K.ntiles;
    b.order = K.order;
    b.queue = K.queue;
    b.persistent = K.persistent;
    b.zero_slots = first ? 1 : 0;
    return launch_sweep_batch(c->dtype, batch_mode(c), c->csum, K.shape, b, K.nblocks, K.lds,
                              c->stream);
}

abft_status enqueue_batch(abft_ctx* c, int64_t n, const int64_t* tbase, int64_t t0)
{
    for (int64_t i = 0; i < n; ++i) {
        const int64_t t = c->t + i;
        const BatchArgs b = batch_args(c, t, tbase, t0);
        hipError_t e;
        if (c->mem_faults) {
            e = launch_mem_flip_batch(c->dtype, c->d_grids, b.parity, c->faults, c->fault_first,
                                      c->fault_tmax, tbase, b.t_off, c->stream);
            if (e != hipSuccess) return hip_fail(c, e, "memory fault launch");
        }
        for (size_t k = 0; k < c->classes.size(); ++k) {
            e = launch_class(c, c->classes[k], b, k == 0);
            if (e != hipSuccess) return hip_fail(c, e, "batched sweep launch");
        }
        if (c->mode == ABFT_MODE_ONLINE && c->auto_correct) {
            e = launch_fixup_batch(c->dtype, b, c->maxnx, c->shape.rad, c->shape.box, c->stream);
            if (e != hipSuccess) return hip_fail(c, e, "batched locate/correct launch");
        }
    }
    c->t += n;
    c->cur = (int)(c->t & 1);
    c->bcur = c->cur;
    return ABFT_OK;
}

// Per-size-class autotuning.  The grids are grouped by the narrowest shape that holds their
// rows (classes in order of row length); every run of consecutive classes is timed as one
// launch for each shape that holds its longest row (for radius-1 stars also in a launch where
// each class's grids take the fewest chunks that hold their rows), slab depth and dispatch
// form; the split of the classes into runs whose summed launch times are least is kept.  The
// all-in-one layout (one launch in the widest shape) is one of the splits tried.
abft_status batch_autotune(abft_ctx* c)
{
    HIPCHK(c, hipStreamSynchronize(c->stream));
    Counters* scnt = nullptr;  // the timing launches count into scratch, log no events
    abft_status s = dalloc(c, &scnt, sizeof(Counters));
    if (s) return s;
    // The timing sweeps alternate each grid's two buffers as a run does, so that every sweep
    // reads what the one before it wrote (the same input swept again and again would stay in
    // the last-level cache and time faster than a run).  The current grids, checksums and
    // weighted sums are kept in a backup and restored afterwards; both buffers start from them.
    const int p0 = (int)(c->t & 1);
    const size_t es = esize(c->dtype);
    std::vector<size_t> off;
    size_t total = 0;
    for (const auto& G : c->grids) {
        off.push_back(total);
        total += ((size_t)G.nx * G.ny * G.nz * es + 255) & ~(size_t)255;
        total += (size_t)G.ny * G.nz * 8 * (G.W[p0] ? 2 : 1);
        total = (total + 255) & ~(size_t)255;
    }
    unsigned char* backup = nullptr;
    if ((s = dalloc(c, &backup, total))) return s;
    auto copy_state = [&](bool save) -> bool {
        for (size_t g = 0; g < c->grids.size(); ++g) {
            const auto& G = c->grids[g];
            const size_t nu = (size_t)G.nx * G.ny * G.nz * es, nb = (size_t)G.ny * G.nz * 8;
            unsigned char* q = backup + off[g];
            unsigned char* qb = q + ((nu + 255) & ~(size_t)255);
            struct {
                void* live;
                void* other;
                unsigned char* keep;
                size_t n;
            } parts[3] = {{G.u[p0], G.u[p0 ^ 1], q, nu},
                          {G.B[p0], G.B[p0 ^ 1], qb, nb},
                          {G.W[p0], G.W[p0 ^ 1], qb + nb, nb}};
            for (auto& P : parts) {
                if (!P.live) continue;
                if (save) {
                    if (hipMemcpyAsync(P.keep, P.live, P.n, hipMemcpyDeviceToDevice, c->stream) ||
                        hipMemcpyAsync(P.other, P.live, P.n, hipMemcpyDeviceToDevice, c->stream))
                        return false;
                } else if (hipMemcpyAsync(P.live, P.keep, P.n, hipMemcpyDeviceToDevice,
                                          c->stream)) {
                    return false;
                }
            }
        }
        return hipStreamSynchronize(c->stream) == hipSuccess;
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool saved = false;
    auto cleanup = [&]() {
        if (saved) (void)copy_state(false);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        for (void* q : {(void*)scnt, (void*)backup}) {
            auto it = std::find(c->allocs.begin(), c->allocs.end(), q);
            if (it != c->allocs.end()) c->allocs.erase(it);
            (void)hipFree(q);
        }
    };
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        return fail(c, ABFT_E_HIP, "hipEventCreate");
    }
    if (!(saved = copy_state(true))) {
        (void)hipGetLastError();
        cleanup();
        return fail(c, ABFT_E_HIP, "autotune state backup");
    }
    // base classes: (16-byte accesses, narrowest shape) per grid, in order of row length
    std::map<std::pair<int, int>, std::vector<int>> by;
    for (size_t g = 0; g < c->grids.size(); ++g) {
        const bool vo = grid_vec_ok(c, (int)g);
        const auto sh = batch_shapes_for(c->dtype, vo, c->grids[g].nx);
        if (sh.empty()) {
            cleanup();
            return fail(c, ABFT_E_UNSUPPORTED, "rows too long for the batched kernel");
        }
        by[{vo ? 0 : 1, shape_width(sh[0])}].push_back((int)g);
    }
    std::vector<std::vector<int>> base;
    std::vector<bool> base_vec;
    for (auto& kv : by) {
        base.push_back(kv.second);
        base_vec.push_back(kv.first.first == 0);
    }
    const int nb = (int)base.size();
    // each run of classes: the fastest configuration of each of its four fastest launch
    // shapes, fastest first (one entry per shape, so that the whole-sweep timings below see
    // different shapes, not one shape's slab depths)
    struct Best {
        std::vector<std::pair<float, abft_ctx::Class>> top;
        float ms() const { return top.empty() ? 1e30f : top[0].first; }
        void add(float t, const abft_ctx::Class& k)
        {
            auto same = [&](const abft_ctx::Class& o) {
                return o.shape.lpr == k.shape.lpr && o.shape.nch == k.shape.nch &&
                       o.shape.vec == k.shape.vec && o.shape.nchb == k.shape.nchb &&
                       o.shape.nchc == k.shape.nchc;
            };
            for (auto& e : top)
                if (same(e.second)) {
                    if (t < e.first) e = {t, k};
                    t = -1.f;
                    break;
                }
            if (t >= 0.f) top.push_back({t, k});
            std::stable_sort(top.begin(), top.end(),
                             [](const auto& x, const auto& y) { return x.first < y.first; });
            if (top.size() > 4) top.resize(4);
        }
    };
    std::vector<std::vector<Best>> best(nb, std::vector<Best>(nb));
    BatchArgs b = batch_args(c, c->t, nullptr, 0);
    b.faults = nullptr;
    b.fault_tmax = 0;
    b.cnt = scnt;
    b.ev = nullptr;
    b.ev_cap = 0;
    // one timing launch; every launch swaps the buffers' roles (see above)
    int flip = p0;
    auto launch_timed = [&](const abft_ctx::Class& K, bool first) {
        BatchArgs bb = b;
        bb.parity = flip;
        flip ^= 1;
        return launch_class(c, K, bb, first);
    };
    for (int i = 0; i < nb; ++i)
        for (int j = i; j < nb; ++j) {
            abft_ctx::Class K;
            bool vo = true;
            int wmax = 1;
            for (int q = i; q <= j; ++q) {
                K.grids.insert(K.grids.end(), base[q].begin(), base[q].end());
                vo = vo && base_vec[q];
                for (int g : base[q]) wmax = std::max(wmax, c->grids[g].nx);
            }
            std::vector<SweepShape> shapes = batch_shapes_for(c->dtype, vo, wmax);
            if (c->shape.rad == 1 && !c->shape.box && vo) {
                // one launch in which each class's grids take the fewest chunks that hold
                // their rows
                const size_t n1 = shapes.size();
                for (size_t q0 = 0; q0 < n1; ++q0) {
                    SweepShape sh = shapes[q0];
                    const int cw = sh.lpr * sh.vec;
                    std::vector<int> need;
                    for (int q = i; q <= j; ++q) {
                        int w = 1;
                        for (int g : base[q]) w = std::max(w, c->grids[g].nx);
                        int n = 1;
                        while (cw * n < w) n *= 2;
                        if (std::find(need.begin(), need.end(), n) == need.end()) need.push_back(n);
                    }
                    std::sort(need.rbegin(), need.rend());
                    if (need.size() < 2 || need.size() > 3 || need[0] != sh.nch) continue;
                    sh.nchb = need[1];
                    sh.nchc = need.size() > 2 ? need[2] : 0;
                    sh.rad = 1;
                    if (batch_shape_supported(c->dtype, sh)) shapes.push_back(sh);
                }
            }
            for (SweepShape sh : shapes)
                for (int tz : {2, 4, 8, 16, 32, 1 << 20})
                    for (int p : {1, 0}) {
                        sh.rad = c->shape.rad;
                        sh.box = c->shape.box;
                        K.shape = sh;
                        K.tz = tz;
                        K.persistent = p;
                        c->classes.assign(1, K);
                        if (batch_layout(c)) continue;  // e.g. tiles beyond the LDS
                        const abft_ctx::Class& L = c->classes[0];
                        float ms = 1e30f;
                        bool ok = launch_timed(L, true) == hipSuccess &&
                                  launch_timed(L, true) == hipSuccess;
                        for (int grp = 0; ok && grp < 3; ++grp) {
                            ok = hipEventRecord(e0, c->stream) == hipSuccess;
                            for (int r = 0; ok && r < 5; ++r)
                                ok = launch_timed(L, true) == hipSuccess;
                            float gms = 0.f;
                            ok = ok && hipEventRecord(e1, c->stream) == hipSuccess &&
                                 hipEventSynchronize(e1) == hipSuccess &&
                                 hipEventElapsedTime(&gms, e0, e1) == hipSuccess;
                            if (ok) ms = std::min(ms, gms / 5);
                        }
                        if (!ok) {
                            (void)hipGetLastError();
                            (void)hipStreamSynchronize(c->stream);
                            continue;
                        }
                        best[i][j].add(ms, L);
                    }
        }
    // least summed time over the splits into runs of consecutive classes
    std::vector<float> f(nb + 1, 1e30f);
    std::vector<int> from(nb + 1, -1);
    f[0] = 0.f;
    for (int j = 0; j < nb; ++j)
        for (int i = 0; i <= j; ++i)
            if (f[i] + best[i][j].ms() < f[j + 1]) {
                f[j + 1] = f[i] + best[i][j].ms();
                from[j + 1] = i;
            }
    std::vector<std::pair<int, int>> runs;
    for (int j = nb; j > 0 && from[j] >= 0; j = from[j]) runs.push_back({from[j], j - 1});
    if (runs.empty() || f[nb] >= 1e29f) {
        cleanup();
        (void)batch_single_class(c, 8, 1);
        return fail(c, ABFT_E_UNSUPPORTED, "no batched launch shape ran");
    }
    std::reverse(runs.begin(), runs.end());
    // Launch times of one run alone only approximate a whole sweep (the runs' launches follow
    // one another, and configurations within a few percent trade places between timings): the
    // split found above, the same split with one run in its runner-up shape, and the one-launch
    // layouts of the four best shapes are timed again as whole sweeps, in alternation, and the
    // fastest is kept.
    std::vector<std::vector<abft_ctx::Class>> finalists;
    {
        std::vector<abft_ctx::Class> opt;
        for (auto& r : runs) opt.push_back(best[r.first][r.second].top[0].second);
        finalists.push_back(opt);
        for (size_t q = 0; q < runs.size(); ++q) {
            const Best& bb = best[runs[q].first][runs[q].second];
            if (bb.top.size() < 2) continue;
            std::vector<abft_ctx::Class> alt = opt;
            alt[q] = bb.top[1].second;
            finalists.push_back(alt);
        }
        // the one-launch layouts: the best of each of the four fastest shapes
        const Best& all = best[0][nb - 1];
        for (size_t q = runs.size() > 1 ? 0 : 1; q < all.top.size(); ++q)
            finalists.push_back({all.top[q].second});
    }
    auto time_sweeps = [&](const std::vector<abft_ctx::Class>& layout, int reps) -> float {
        c->classes = layout;
        if (batch_layout(c)) return -1.f;
        // a sweep's class launches share its parity
        auto sweep = [&]() {
            bool ok = true;
            const int f = flip;
            for (size_t k = 0; ok && k < c->classes.size(); ++k) {
                flip = f;
                ok = launch_timed(c->classes[k], k == 0) == hipSuccess;
            }
            return ok;
        };
        bool ok = sweep();
        ok = ok && hipEventRecord(e0, c->stream) == hipSuccess;
        for (int r = 0; ok && r < reps; ++r) ok = sweep();
        float ms = 0.f;
        ok = ok && hipEventRecord(e1, c->stream) == hipSuccess &&
             hipEventSynchronize(e1) == hipSuccess &&
             hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        if (!ok) {
            (void)hipGetLastError();
            (void)hipStreamSynchronize(c->stream);
            return -1.f;
        }
        return ms / reps;
    };
    std::vector<float> fin(finalists.size(), 1e30f);
    for (int round = 0; round < 5; ++round)
        for (size_t q = 0; q < finalists.size(); ++q) {
            const float ms = time_sweeps(finalists[q], 10);
            if (ms > 0.f) fin[q] = std::min(fin[q], ms);
        }
    size_t pick = 0;
    for (size_t q = 1; q < finalists.size(); ++q)
        if (fin[q] < fin[pick]) pick = q;
    cleanup();
    c->classes = finalists[pick];
    s = batch_layout(c);
    if (s) return s;
    // the timing sweeps used both flag slots of every grid: both start empty again
    for (auto& G : c->grids)
        for (int q = 0; q < 2; ++q) {
            hipError_t e = launch_fill_u32(&G.slot[q]->count, 0u, 2, c->stream);
            if (e != hipSuccess) return hip_fail(c, e, "reset");
        }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return ABFT_OK;
}

}  // namespace

namespace {

// Everything init does before it allocates: the context's fields from the problem and options,
// the device's compute units, the stencil's weight slots, the checks of what the kernels cover
// and the launch shape (from the tuning cache when use_cache is set, else the default).
abft_status configure(abft_ctx* c, const abft_problem* p, const abft_options* o, void* hip_stream,
                      bool use_cache)
{
    c->nx = p->nx;
    c->ny = p->ny;
    c->nz = p->nz;
    c->dtype = p->dtype;
    c->bc = p->bc;
    c->C = p->cterm;
    c->cs = round_to(p->dtype, p->cterm_scalar);
    c->u[0] = p->u0;
    c->u[1] = p->u1;
    c->mode = o->mode;
    c->period = o->mode == ABFT_MODE_OFFLINE ? o->period : 1;
    c->eps = o->threshold;
    c->csum = o->csum == ABFT_CSUM_F32_COMP ? CS_F32C : CS_F64;
    c->auto_correct = o->auto_correct ? 1 : 0;
    c->recompute = o->correction == ABFT_CORRECT_RECOMPUTE ? 1 : 0;
    c->input_check = (o->input_check && o->mode != ABFT_MODE_NONE) ? 1 : 0;
    c->tile_x = o->tile_x;
    c->ev_cap = o->max_events ? o->max_events : kDefaultEvents;
    if (use_cache && o->tuning_cache) c->cache_path = o->tuning_cache;
    c->stream = static_cast<hipStream_t>(hip_stream);
    {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
            return fail(c, ABFT_E_HIP, "device query failed");
        c->num_cus = prop.multiProcessorCount;
    }
    abft_status s = map_taps(c, p);
    if (s) return s;
    c->st.xterms = need_boundary_terms(c) ? 1 : 0;
    if (c->tile_x != 0) {
        // tiles are the 16 lanes x 16 bytes one lane group of the sweep holds of a row
        const int tt = 16 * (16 / (int)esize(c->dtype));
        if (c->tile_x != tt || c->nx % tt || c->st.box || c->input_check ||
            c->mode == ABFT_MODE_OFFLINE || c->csum != CS_F64)
            return fail(c, ABFT_E_UNSUPPORTED, "tile-local checksums: online star stencils, "
                                               "T = 64 (fp32) or 32 (fp64), T dividing nx, "
                                               "fp64 accumulation");
    }
    SweepShape shape{};
    if (c->st.rad == 2) {
        // the shifted-line sums of Theorem 1 (and the periodic wrap) need every axis that
        // carries a distance-2 tap to be at least 2 long
        for (int ax = 0; ax < 3; ++ax) {
            const int n = ax == 0 ? c->nx : ax == 1 ? c->ny : c->nz;
            const uint32_t m2 = (1u << w_slot(ax, 2, -1)) | (1u << w_slot(ax, 2, 1));
            if ((c->st.mask & m2) && n < 2)
                return fail(c, ABFT_E_UNSUPPORTED, "distance-2 taps along an axis of length 1");
        }
    }
    const bool cached = use_cache && cache_lookup(c, &shape);
    shape.rad = c->st.rad;
    shape.box = c->st.box;
    if (!cached || !sweep_shape_supported(c->dtype, shape)) {
        if (!default_shape(c->dtype, c->nx, c->ny, c->nz, c->st.rad, c->st.box, &shape))
            return fail(c, ABFT_E_UNSUPPORTED, "row length beyond the GPU kernels");
    }
    s = apply_shape(c, shape);
    if (s) return s;
    if (fixup_lds_bytes(c->nx, c->st.box) > (c->st.box ? kSweepLdsLimit : kLdsLimit) ||
        c->nx > 4 * kFixBlock)
        return fail(c, ABFT_E_UNSUPPORTED, "rows too long for the locate kernel");
    if (c->mode == ABFT_MODE_OFFLINE) {
        check_shape(c, std::min(c->period, kCheckChunk / c->st.rad) * c->st.rad);
        if ((int64_t)c->ck.ry * c->ck.rz > (int64_t)kCheckCells * kCheckBlock)
            return fail(c, ABFT_E_UNSUPPORTED, "offline period too long for this grid");
    }
    return ABFT_OK;
}

abft_status init_impl(const abft_problem* p, const abft_options* o, void* hip_stream,
                      abft_ctx** out)
{
    g_init_error.clear();
    if (!out) return fail(nullptr, ABFT_E_INVAL, "out is NULL");
    *out = nullptr;
    abft_status s = validate_problem(p);
    if (s) return s;
    s = validate_options(p, o);
    if (s) return s;

    abft_ctx* c = new abft_ctx();
    try {
        auto bail = [&](abft_status st) {
            g_init_error = c->err;
            free_all(c);
            delete c;
            return st;
        };
        s = configure(c, p, o, hip_stream, true);
        if (s) return bail(s);

        // checksum entries: one per row, or one per tile of each row
        const size_t nrows = (size_t)c->nz * c->ny * (c->tile_x ? c->nx / c->tile_x : 1),
                     ncols = (size_t)c->nz * c->nx;
        const size_t gbytes = (size_t)c->nx * c->ny * c->nz * esize(c->dtype);
        if ((s = dalloc(c, &c->B[0], nrows * 8)) || (s = dalloc(c, &c->B[1], nrows * 8)) ||
            (s = dalloc(c, &c->cB, nrows * 8)) || (s = dalloc(c, &c->cA, ncols * 8)) ||
            (s = dalloc(c, &c->slot[0], sizeof(FlagSlot))) ||
            (s = dalloc(c, &c->slot[1], sizeof(FlagSlot))) ||
            (s = dalloc(c, &c->cnt, sizeof(Counters))) ||
            (s = dalloc(c, &c->ev, (size_t)c->ev_cap * sizeof(abft_event))) ||
            (s = dalloc(c, &c->win, 4 * sizeof(uint32_t))) ||
            (s = dalloc(c, &c->ticket, 4 * sizeof(uint32_t))) ||
            (s = dalloc(c, &c->tbase, sizeof(int64_t))))
            return bail(s);
        if (c->input_check &&
            ((s = dalloc(c, &c->W[0], nrows * 8)) || (s = dalloc(c, &c->W[1], nrows * 8))))
            return bail(s);
        if (c->tile_x && (s = dalloc(c, &c->Et, nrows * 8))) return bail(s);
        if (c->mode == ABFT_MODE_OFFLINE) {
            if (p->u2 != nullptr) {
                if (p->u2 == p->u0 || p->u2 == p->u1)
                    return bail(fail(c, ABFT_E_INVAL, "u2 must differ from u0 and u1"));
                c->u[2] = p->u2;
            } else {
                if ((s = dalloc(c, &c->u[2], gbytes))) return bail(s);
                c->own_u2 = true;
            }
            if (need_boundary_terms(c) && (s = dalloc(c, &c->E, (size_t)c->period * nrows * 8)))
                return bail(s);
            if (c->period > kCheckChunk / c->st.rad &&
                ((s = dalloc(c, &c->Btmp[0], nrows * 8)) || (s = dalloc(c, &c->Btmp[1], nrows * 8))))
                return bail(s);
        }

        hipError_t e;
#define INIT_CHK(expr)                                      \
        if ((e = (expr)) != hipSuccess) {                       \
            hip_fail(c, e, #expr);                              \
            return bail(ABFT_E_HIP);                            \
        }
        INIT_CHK(launch_fill_u32(reinterpret_cast<uint32_t*>(c->cnt), 0u,
                                 sizeof(Counters) / 4, c->stream));
        INIT_CHK(launch_fill_u32(&c->slot[0]->count, 0u, 2, c->stream));
        INIT_CHK(launch_fill_u32(&c->slot[1]->count, 0u, 2, c->stream));
        INIT_CHK(launch_fill_u32(c->win, 0u, 4, c->stream));
        INIT_CHK(launch_fill_u32(c->ticket, 0u, 4, c->stream));
        INIT_CHK(launch_set_i64(c->tbase, 0, c->stream));
        // Theorem 1's constant-term checksums and the checksums of u^0
        // a tile is a contiguous run of tile_x points, so tile sums are row sums of that length
        const int line = c->tile_x ? c->tile_x : c->nx;
        INIT_CHK(launch_row_sums(c->dtype, c->C, c->cs, line, (int64_t)nrows, c->cB, c->stream));
        INIT_CHK(launch_col_sums(c->dtype, c->C, c->cs, c->nx, c->ny, c->nz, c->cA, c->stream));
        INIT_CHK(launch_row_sums(c->dtype, c->u[0], 0.0, line, (int64_t)nrows, c->B[0], c->stream));
        if (c->W[0] != nullptr)
            INIT_CHK(launch_weighted_row_sums(c->dtype, c->u[0], c->nx, (int64_t)nrows, c->W[0],
                                              c->stream));
        INIT_CHK(hipStreamSynchronize(c->stream));
#undef INIT_CHK
        *out = c;
        return ABFT_OK;
    } catch (...) {
        // a host exception (allocation) after the context was made: nothing leaks
        free_all(c);
        delete c;
        throw;
    }
}

abft_status step_impl(abft_ctx* c, int64_t nsweeps)
{
    if (!c) return ABFT_E_INVAL;
    if (nsweeps < 0) return fail(c, ABFT_E_INVAL, "nsweeps < 0");
    if (c->halted) return fail(c, ABFT_E_STATE, "offline window awaits abft_stencil_correct");
    if (c->batch) return enqueue_batch(c, nsweeps, nullptr, 0);
    if (c->mode == ABFT_MODE_OFFLINE) return enqueue_offline(c, nsweeps);
    return enqueue_online(c, nsweeps, nullptr, 0);
}

abft_status step_graph_impl(abft_ctx* c, int64_t nsweeps)
{
    if (!c) return ABFT_E_INVAL;
    if (nsweeps < 0) return fail(c, ABFT_E_INVAL, "nsweeps < 0");
    if (nsweeps == 0) return ABFT_OK;
    if (c->mode == ABFT_MODE_OFFLINE)
        return fail(c, ABFT_E_UNSUPPORTED, "graph steps cover the online and plain modes");
    if (c->stream == nullptr)
        return fail(c, ABFT_E_UNSUPPORTED, "graph capture needs a non-null stream");
    hipError_t e = launch_set_i64(c->tbase, c->t, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "sweep base");
    const auto key = std::make_pair(nsweeps, c->cur);
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
        const int64_t t_save = c->t;
        const int cur_save = c->cur, bcur_save = c->bcur;
        HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
        abft_status s = c->batch ? enqueue_batch(c, nsweeps, c->tbase, t_save)
                                 : enqueue_online(c, nsweeps, c->tbase, t_save);
        hipGraph_t g = nullptr;
        hipError_t ce = hipStreamEndCapture(c->stream, &g);
        c->t = t_save;
        c->cur = cur_save;
        c->bcur = bcur_save;
        if (s) {
            if (g) (void)hipGraphDestroy(g);
            return s;
        }
        if (ce != hipSuccess) return hip_fail(c, ce, "hipStreamEndCapture");
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
        it = c->graphs.emplace(key, ex).first;
    }
    HIPCHK(c, hipGraphLaunch(it->second, c->stream));
    c->t += nsweeps;
    if (nsweeps & 1) {
        c->cur ^= 1;
        if (c->mode == ABFT_MODE_ONLINE) c->bcur ^= 1;
    }
    return ABFT_OK;
}

abft_status check_impl(abft_ctx* c, abft_report* out)
{
    if (!c) return ABFT_E_INVAL;
    if (c->mode == ABFT_MODE_OFFLINE) {
        abft_status s = offline_flush(c);
        if (s) return s;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    Counters h{};
    abft_status s = read_counters(c, &h);
    if (s) return s;
    if (h.barrier_timeouts > 0) {
        // a recompute gave up waiting for its grid: its result and the barrier are not to be
        // trusted; the barrier words are cleared so that the next recompute can run
        uint32_t* bt = reinterpret_cast<uint32_t*>(&c->cnt->barrier_timeouts);
        hipError_t e = launch_fill_u32(c->ticket + 2, 0u, 2, c->stream);
        if (e == hipSuccess) e = launch_fill_u32(bt, 0u, 2, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "barrier reset");
        return fail(c, ABFT_E_HIP, "offline recompute: a grid barrier timed out");
    }
    int64_t pending = 0;
    if (c->batch && c->mode == ABFT_MODE_ONLINE && !c->auto_correct && c->t > 0) {
        for (auto& G : c->grids) {
            uint32_t n[2] = {0, 0};
            HIPCHK(c, hipMemcpy(n, &G.slot[(c->t - 1) & 1]->count, 8, hipMemcpyDeviceToHost));
            pending += (int64_t)n[0] + n[1];
        }
    } else if (c->mode == ABFT_MODE_ONLINE && !c->auto_correct && c->t > 0) {
        uint32_t n[2] = {0, 0};  // flagged output rows, flagged input rows
        HIPCHK(c, hipMemcpy(n, &c->slot[(c->t - 1) & 1]->count, 8, hipMemcpyDeviceToHost));
        pending = (int64_t)n[0] + n[1];
    } else if (c->halted) {
        uint32_t n = 0;
        HIPCHK(c, hipMemcpy(&n, c->win + 2 * (c->win_index & 1), 4, hipMemcpyDeviceToHost));
        pending = n;
    }
    if (out) {
        out->sweeps_done = c->mode == ABFT_MODE_OFFLINE ? c->win_t0 + c->win_j : c->t;
        out->rows_flagged = (int64_t)h.rows_flagged;
        out->cols_flagged = (int64_t)h.cols_flagged;
        out->corrected = (int64_t)h.corrected;
        out->checksum_faults = (int64_t)h.checksum_faults;
        out->uncorrectable = (int64_t)h.uncorrectable;
        out->windows_checked = (int64_t)h.windows_checked;
        out->windows_flagged = (int64_t)h.windows_flagged;
        out->rollbacks = (int64_t)h.rollbacks;
        out->persistent = (int64_t)h.persistent;
        out->events_total = (int64_t)h.events_total;
        out->pending = pending;
        out->sweeps_skipped = c->skipped;
        out->mem_flagged = (int64_t)h.mem_flagged;
        out->mem_corrected = (int64_t)h.mem_corrected;
        out->mem_unlocated = (int64_t)h.mem_unlocated;
        double nm = 0.0;
        std::memcpy(&nm, &h.noise_bits, sizeof(nm));
        out->max_noise = nm;
        out->nevents = 0;
        if (out->events && out->events_cap > 0) {
            const int64_t n =
                std::min<int64_t>({(int64_t)h.events_total, (int64_t)c->ev_cap,
                                   (int64_t)out->events_cap});
            if (n > 0)
                HIPCHK(c, hipMemcpy(out->events, c->ev, (size_t)n * sizeof(abft_event),
                                    hipMemcpyDeviceToHost));
            out->nevents = (int32_t)n;
        }
    }
    return ABFT_OK;
}

abft_status correct_impl(abft_ctx* c, abft_report* inout)
{
    if (!c) return ABFT_E_INVAL;
    Counters before{};
    abft_status s = read_counters(c, &before);
    if (s) return s;
    if (c->batch && c->mode == ABFT_MODE_ONLINE && !c->auto_correct && c->t > 0) {
        const BatchArgs b = batch_args(c, c->t - 1, nullptr, 0);
        hipError_t e = launch_fixup_batch(c->dtype, b, c->maxnx, c->shape.rad, c->shape.box,
                                          c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "batched locate/correct launch");
    } else if (c->mode == ABFT_MODE_ONLINE && !c->auto_correct && c->t > 0) {
        const int64_t t = c->t - 1;
        const FixArgs f = online_fix_args(c, c->cur ^ 1, c->bcur ^ 1, t, nullptr, t);
        hipError_t e = launch_fixup(c->dtype, f, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "locate/correct launch");
    } else if (c->mode == ABFT_MODE_OFFLINE && c->halted) {
        const int k = c->win_j;
        s = offline_recompute(c, k, nullptr);
        if (s) return s;
        c->halted = false;
        offline_rotate(c, k);
    }
    s = check_impl(c, inout);
    if (s) return s;
    Counters after{};
    s = read_counters(c, &after);
    if (s) return s;
    if (after.uncorrectable > before.uncorrectable || after.persistent > before.persistent)
        return fail(c, ABFT_E_UNCORRECTABLE, "detection could not be corrected");
    return ABFT_OK;
}

abft_status current_impl(abft_ctx* c, int32_t grid, void** dev_ptr, int64_t* sweep)
{
    if (!c) return ABFT_E_INVAL;
    if (c->batch) {
        if (grid < 0 || grid >= (int)c->grids.size()) return fail(c, ABFT_E_INVAL, "grid index");
        if (dev_ptr) *dev_ptr = c->grids[grid].u[c->t & 1];
        if (sweep) *sweep = c->t;
        return ABFT_OK;
    }
    if (grid != 0) return fail(c, ABFT_E_INVAL, "grid index");
    if (dev_ptr) *dev_ptr = c->u[c->cur];
    if (sweep) *sweep = c->mode == ABFT_MODE_OFFLINE ? c->win_t0 + c->win_j : c->t;
    return ABFT_OK;
}

abft_status checksums_impl(abft_ctx* c, int32_t grid, double** dev_ptr)
{
    if (!c || !dev_ptr) return ABFT_E_INVAL;
    if (c->batch) {
        if (grid < 0 || grid >= (int)c->grids.size()) return fail(c, ABFT_E_INVAL, "grid index");
        *dev_ptr = c->grids[grid].B[c->t & 1];
        return ABFT_OK;
    }
    if (grid != 0) return fail(c, ABFT_E_INVAL, "grid index");
    *dev_ptr = c->mode == ABFT_MODE_OFFLINE ? c->B[c->bck] : c->B[c->bcur];
    return ABFT_OK;
}

abft_status inject_impl(abft_ctx* c, const abft_fault* f, int32_t n)
{
    if (!c || n < 0 || (n > 0 && !f)) return c ? fail(c, ABFT_E_INVAL, "fault plan") : ABFT_E_INVAL;
    const int bits = c->dtype == ABFT_F32 ? 32 : 64;
    std::vector<abft_fault> v(f, f + n);
    for (const auto& x : v) {
        int nx = c->nx, ny = c->ny, nz = c->nz;
        if (c->batch) {
            if (x.grid < 0 || x.grid >= (int)c->grids.size())
                return fail(c, ABFT_E_INVAL, "fault grid index");
            nx = c->grids[x.grid].nx;
            ny = c->grids[x.grid].ny;
            nz = c->grids[x.grid].nz;
        } else if (x.grid != 0) {
            return fail(c, ABFT_E_INVAL, "fault grid index");
        }
        if (x.sweep < 0 || x.z < 0 || x.z >= nz || x.y < 0 || x.y >= ny || x.x < 0 ||
            x.x >= nx || x.bit < 0 || x.bit >= bits || x.attempt < 0 || x.attempt > 1 ||
            (x.kind != ABFT_FAULT_STORE && x.kind != ABFT_FAULT_MEMORY))
            return fail(c, ABFT_E_INVAL, "fault outside the grid or word");
        if (x.kind == ABFT_FAULT_MEMORY && x.attempt != 0)
            return fail(c, ABFT_E_UNSUPPORTED, "memory faults fire on the first attempt");
    }
    std::stable_sort(v.begin(), v.end(),
                     [](const abft_fault& a, const abft_fault& b) { return a.sweep < b.sweep; });
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // drop the old plan
    for (void* p : {static_cast<void*>(c->faults), static_cast<void*>(c->fault_first)}) {
        if (!p) continue;
        auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
        if (it != c->allocs.end()) c->allocs.erase(it);
        (void)hipFree(p);
    }
    c->faults = nullptr;
    c->fault_first = nullptr;
    c->fault_tmax = 0;
    c->nfaults = 0;
    c->mem_faults = false;
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    if (n == 0) return ABFT_OK;
    const int64_t tmax = v.back().sweep + 1;
    if (tmax > (int64_t)1 << 26) return fail(c, ABFT_E_INVAL, "fault sweep index too large");
    std::vector<int32_t> first((size_t)tmax + 1);
    size_t i = 0;
    for (int64_t t = 0; t <= tmax; ++t) {
        while (i < v.size() && v[i].sweep < t) ++i;
        first[(size_t)t] = (int32_t)i;
    }
    abft_status s;
    if ((s = dalloc(c, &c->faults, v.size() * sizeof(abft_fault))) ||
        (s = dalloc(c, &c->fault_first, first.size() * sizeof(int32_t))))
        return s;
    HIPCHK(c, hipMemcpy(c->faults, v.data(), v.size() * sizeof(abft_fault),
                        hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->fault_first, first.data(), first.size() * sizeof(int32_t),
                        hipMemcpyHostToDevice));
    c->fault_tmax = tmax;
    c->nfaults = n;
    c->mem_faults = std::any_of(v.begin(), v.end(),
                                [](const abft_fault& x) { return x.kind == ABFT_FAULT_MEMORY; });
    return ABFT_OK;
}

abft_status autotune_impl(abft_ctx* c)
{
    if (!c) return ABFT_E_INVAL;
    if (c->batch) return batch_autotune(c);
    if (c->mode == ABFT_MODE_OFFLINE && (c->win_j != 0 || c->halted))
        return fail(c, ABFT_E_STATE, "autotune in offline mode needs a closed window");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // scratch control structures so that timing runs leave the context's state untouched
    FlagSlot* sslot = nullptr;
    Counters* scnt = nullptr;
    double* sB = nullptr;
    double* sW = nullptr;
    double* sB2 = nullptr;
    double* sW2 = nullptr;
    void* su = nullptr;
    abft_status s;
    const size_t nrows = (size_t)c->nz * c->ny * (c->tile_x ? c->nx / c->tile_x : 1);
    const bool offline = c->mode == ABFT_MODE_OFFLINE;
    if ((s = dalloc(c, &sslot, sizeof(FlagSlot))) || (s = dalloc(c, &scnt, sizeof(Counters))) ||
        (s = dalloc(c, &sB, nrows * 8)) || (s = dalloc(c, &sW, nrows * 8)) ||
        (s = dalloc(c, &sB2, nrows * 8)) || (s = dalloc(c, &sW2, nrows * 8)))
        return s;
    if (!offline && (s = dalloc(c, &su, (size_t)c->nx * c->ny * c->nz * esize(c->dtype))))
        return s;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    const int vf = 16 / (int)esize(c->dtype);
    std::vector<SweepShape> cands;
    for (int vec : {vf, 1}) {
        if (vec > 1 && c->nx % vec) continue;
        if (c->tile_x && vec != vf) continue;  // tiles are 16 lanes of 16-byte accesses
        for (int lpr : {16, 64})
            for (int nch : {1, 2, 4, 8, 16}) {
                for (int pf : {1, 2})
                    for (int nw : {4, 8}) {
                        SweepShape sh{lpr, nch, vec, 1, pf, nw, c->st.rad, c->st.box};
                        if (!sweep_shape_supported(c->dtype, sh)) continue;
                        if ((int64_t)lpr * nch * vec < c->nx) continue;
                        if ((int64_t)lpr * (nch / 2) * vec >= c->nx && nch > 1) continue;  // minimal
                        if (sweep_lds_bytes(c->dtype, c->nx, sh, c->input_check) > kSweepLdsLimit)
                            continue;
                        for (int tz : {2, 4, 8, 16, 32, 64, 128}) {
                            if (tz > c->nz && tz != 2) continue;
                            sh.tz = std::min(tz, c->nz);
                            cands.push_back(sh);
                        }
                    }
            }
        if (!cands.empty()) break;  // prefer 16-byte accesses when they apply
    }
    const SweepShape keep = c->shape;
    SweepShape best = keep;
    float best_ms = 1e30f;
    const int mode = c->mode != ABFT_MODE_ONLINE ? MODE_PLAIN
                     : (c->tile_x ? MODE_TILE : (c->input_check ? MODE_PROTM : MODE_PROT));
    // The timing launches form one run, each reading what the one before wrote (the same
    // input swept again and again would stay in the last-level cache and time faster than a
    // run does): the first reads the current grid, the rest alternate between two scratch
    // grids (the other buffer and a scratch allocation; in offline mode the window's two
    // free buffers), with the checksums alternating in the same way.
    void* const ua = offline ? c->u[buf_of(c, 1)] : c->u[c->cur ^ 1];
    void* const ub = offline ? c->u[buf_of(c, 2)] : su;
    int64_t nt = 0;  // timing launches so far
    // one candidate: `groups` timed groups of `reps` launches, the best group's mean; a
    // negative value when the shape does not launch
    auto time_shape = [&](const SweepShape& sh, int groups, int reps) -> float {
        if (apply_shape(c, sh)) return -1.f;
        SweepArgs a = base_args(c);
        a.faults = nullptr;
        a.cnt = scnt;
        a.ev = nullptr;
        a.ev_cap = 0;
        a.slot = sslot;
        if (mode == MODE_TILE) a.Et = sW;  // the sweep's tile boundary terms (scratch)
        a.t_off = c->t;
        // the launch after `nt` others (see `nt`)
        auto sweep = [&]() {
            const bool odd = nt & 1;
            a.uin = nt == 0 ? c->u[c->cur] : (odd ? ua : ub);
            a.uout = odd ? ub : ua;
            a.Bt = nt == 0 ? (offline ? c->B[c->bck] : c->B[c->bcur]) : (odd ? sB : sB2);
            a.Bn = odd ? sB2 : sB;
            if (mode == MODE_PROTM) a.Wn = odd ? sW2 : sW;
            ++nt;
            return launch_sweep(c->dtype, mode, c->csum, c->shape, a, c->stream);
        };
        for (int w = 0; w < 2; ++w)
            if (sweep() != hipSuccess) {
                (void)hipGetLastError();
                return -1.f;
            }
        float ms = 1e30f;
        for (int g = 0; g < groups; ++g) {
            if (hipEventRecord(e0, c->stream) != hipSuccess) return -1.f;
            for (int r = 0; r < reps; ++r) (void)sweep();
            float gms = 0.f;
            if (hipEventRecord(e1, c->stream) != hipSuccess ||
                hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&gms, e0, e1) != hipSuccess)
                return -1.f;
            ms = std::min(ms, gms / reps);
        }
        return ms;
    };
    // every candidate briefly (best of three groups of five launches), then the three fastest
    // again in alternation (five rounds of ten launches each), so that a shape is not chosen
    // on one lucky group
    std::vector<std::pair<float, SweepShape>> timed;
    for (const SweepShape& sh : cands) {
        const float ms = time_shape(sh, 3, 5);
        if (ms > 0.f) timed.push_back({ms, sh});
    }
    std::stable_sort(timed.begin(), timed.end(),
                     [](const auto& x, const auto& y) { return x.first < y.first; });
    if (timed.size() > 3) timed.resize(3);
    std::vector<float> fine(timed.size(), 1e30f);
    for (int round = 0; round < 5; ++round)
        for (size_t q = 0; q < timed.size(); ++q) {
            const float ms = time_shape(timed[q].second, 1, 10);
            if (ms > 0.f) fine[q] = std::min(fine[q], ms);
        }
    for (size_t q = 0; q < timed.size(); ++q)
        if (fine[q] < best_ms) {
            best_ms = fine[q];
            best = timed[q].second;
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (void* p : {static_cast<void*>(sslot), static_cast<void*>(scnt), static_cast<void*>(sB),
                    static_cast<void*>(sW), static_cast<void*>(sB2), static_cast<void*>(sW2), su}) {
        auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
        if (it != c->allocs.end()) c->allocs.erase(it);
        (void)hipFree(p);
    }
    s = apply_shape(c, best);
    if (s) return s;
    cache_store(c);
    return ABFT_OK;
}

abft_status launch_shape_impl(const abft_ctx* c, int32_t* rows_per_block,
                              int32_t* planes_per_block, int32_t* lanes_per_row)
{
    if (!c) return ABFT_E_INVAL;
    SweepShape sh = c->shape;
    if (c->batch && !c->classes.empty()) {
        // the launch of the size class holding the most points
        int64_t most = -1;
        for (const auto& K : c->classes) {
            int64_t pts = 0;
            for (int g : K.grids) pts += (int64_t)c->grids[g].nx * c->grids[g].ny * c->grids[g].nz;
            if (pts > most) {
                most = pts;
                sh = K.shape;
                sh.tz = K.tz;
            }
        }
    }
    if (rows_per_block) *rows_per_block = sweep_rows_per_block(sh);
    if (planes_per_block) *planes_per_block = sh.tz;
    if (lanes_per_row) *lanes_per_row = sh.lpr;
    return ABFT_OK;
}

void destroy_impl(abft_ctx* c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    free_all(c);
    delete c;
}

abft_status init_batch_impl(const abft_problem* p, int32_t n, const abft_options* o,
                            void* hip_stream, abft_ctx** out)
{
    g_init_error.clear();
    if (!out) return fail(nullptr, ABFT_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!p || n < 1) return fail(nullptr, ABFT_E_INVAL, "batch needs n >= 1 problems");
    abft_status s;
    for (int i = 0; i < n; ++i) {
        if ((s = validate_problem(&p[i]))) return s;
        if ((s = validate_options(&p[i], o))) return s;
        if (p[i].dtype != p[0].dtype) return fail(nullptr, ABFT_E_INVAL, "mixed dtypes in a batch");
    }
    if (o->mode == ABFT_MODE_OFFLINE)
        return fail(nullptr, ABFT_E_UNSUPPORTED, "batches run the online and plain modes");

    abft_ctx* c = new abft_ctx();
    try {
        c->batch = true;
        c->dtype = p[0].dtype;
        c->mode = o->mode;
        c->eps = o->threshold;
        c->csum = o->csum == ABFT_CSUM_F32_COMP ? CS_F32C : CS_F64;
        c->auto_correct = o->auto_correct ? 1 : 0;
        c->recompute = o->correction == ABFT_CORRECT_RECOMPUTE ? 1 : 0;
        c->input_check = (o->input_check && o->mode == ABFT_MODE_ONLINE) ? 1 : 0;
        c->ev_cap = o->max_events ? o->max_events : kDefaultEvents;
        c->stream = static_cast<hipStream_t>(hip_stream);
        if (o->tile_x != 0)
            return fail(nullptr, ABFT_E_UNSUPPORTED, "batches keep whole-row checksums");
        auto bail = [&](abft_status st) {
            g_init_error = c->err;
            free_all(c);
            delete c;
            return st;
        };
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
            return bail(fail(c, ABFT_E_HIP, "device query failed"));
        c->num_cus = prop.multiProcessorCount;

        // the worst-case tile list: one plane per tile, 4 rows per block (64 lanes per row)
        size_t order_cap = 0;
        for (int i = 0; i < n; ++i) {
            c->maxnx = std::max(c->maxnx, p[i].nx);
            order_cap += (size_t)((p[i].ny + 3) / 4) * p[i].nz;
        }
        if (c->maxnx > 64 * 16)
            return bail(fail(c, ABFT_E_UNSUPPORTED, "rows too long for the batched kernel"));
        c->shape = SweepShape{};
        c->shape.nw = kBatchWaves;
        c->grids.resize(n);
        for (int i = 0; i < n; ++i) {
            auto& G = c->grids[i];
            // per-grid stencil: reuse the single-grid tap mapping on a scratch context
            abft_ctx tmp;
            if ((s = map_taps(&tmp, &p[i]))) return bail(fail(c, s, tmp.err));
            tmp.st.xterms = boundary_terms_needed(p[i].bc, tmp.st) ? 1 : 0;
            // one kernel form per batch: every grid has the first grid's radius and form
            if (i == 0) {
                c->shape.rad = tmp.st.rad;
                c->shape.box = tmp.st.box;
            } else if (tmp.st.rad != c->shape.rad || tmp.st.box != c->shape.box) {
                return bail(fail(c, ABFT_E_UNSUPPORTED, "batched grids share the stencil form"));
            }
            if (tmp.st.rad == 2)
                for (int ax = 0; ax < 3; ++ax) {
                    const int len = ax == 0 ? p[i].nx : ax == 1 ? p[i].ny : p[i].nz;
                    const uint32_t m2 = (1u << w_slot(ax, 2, -1)) | (1u << w_slot(ax, 2, 1));
                    if ((tmp.st.mask & m2) && len < 2)
                        return bail(fail(c, ABFT_E_UNSUPPORTED, "distance-2 taps along an axis of "
                                                                "length 1"));
                }
            G.st = tmp.st;
            G.nx = p[i].nx;
            G.ny = p[i].ny;
            G.nz = p[i].nz;
            G.u[0] = p[i].u0;
            G.u[1] = p[i].u1;
            G.C = p[i].cterm;
            G.cs = round_to(c->dtype, p[i].cterm_scalar);
            const size_t nrows = (size_t)G.nz * G.ny, ncols = (size_t)G.nz * G.nx;
            if ((s = dalloc(c, &G.B[0], nrows * 8)) || (s = dalloc(c, &G.B[1], nrows * 8)) ||
                (s = dalloc(c, &G.cB, nrows * 8)) || (s = dalloc(c, &G.cA, ncols * 8)) ||
                (s = dalloc(c, &G.slot[0], sizeof(FlagSlot))) ||
                (s = dalloc(c, &G.slot[1], sizeof(FlagSlot))))
                return bail(s);
            G.W[0] = G.W[1] = nullptr;
            if (i == n - 1 &&
                (fixup_lds_bytes(c->maxnx, c->shape.box) > (c->shape.box ? kSweepLdsLimit : kLdsLimit) ||
                 c->maxnx > 4 * kFixBlock))
                return bail(fail(c, ABFT_E_UNSUPPORTED, "rows too long for the locate kernel"));
            if (c->input_check &&
                ((s = dalloc(c, &G.W[0], nrows * 8)) || (s = dalloc(c, &G.W[1], nrows * 8))))
                return bail(s);
        }
        if ((s = dalloc(c, &c->cnt, sizeof(Counters))) ||
            (s = dalloc(c, &c->ev, (size_t)c->ev_cap * sizeof(abft_event))) ||
            (s = dalloc(c, &c->queue, 2 * kMaxBatchClasses * sizeof(uint32_t))) ||
            (s = dalloc(c, &c->d_order, order_cap * sizeof(int2))) ||
            (s = dalloc(c, &c->tbase, sizeof(int64_t))) ||
            (s = dalloc(c, &c->d_grids, (size_t)n * sizeof(GridDesc))))
            return bail(s);

        hipError_t e;
#define INIT_CHK(expr)                                      \
        if ((e = (expr)) != hipSuccess) {                       \
            hip_fail(c, e, #expr);                              \
            return bail(ABFT_E_HIP);                            \
        }
        INIT_CHK(launch_fill_u32(reinterpret_cast<uint32_t*>(c->cnt), 0u,
                                 sizeof(Counters) / 4, c->stream));
        INIT_CHK(launch_fill_u32(c->queue, 0u, 2 * kMaxBatchClasses, c->stream));
        INIT_CHK(launch_set_i64(c->tbase, 0, c->stream));
        for (auto& G : c->grids) {
            const int64_t nrows = (int64_t)G.nz * G.ny;
            INIT_CHK(launch_fill_u32(&G.slot[0]->count, 0u, 2, c->stream));
            INIT_CHK(launch_fill_u32(&G.slot[1]->count, 0u, 2, c->stream));
            INIT_CHK(launch_row_sums(c->dtype, G.C, G.cs, G.nx, nrows, G.cB, c->stream));
            INIT_CHK(launch_col_sums(c->dtype, G.C, G.cs, G.nx, G.ny, G.nz, G.cA, c->stream));
            INIT_CHK(launch_row_sums(c->dtype, G.u[0], 0.0, G.nx, nrows, G.B[0], c->stream));
            if (G.W[0] != nullptr)
                INIT_CHK(launch_weighted_row_sums(c->dtype, G.u[0], G.nx, nrows, G.W[0], c->stream));
        }
        INIT_CHK(hipStreamSynchronize(c->stream));
#undef INIT_CHK
        c->order_cap = order_cap;
        if ((s = batch_single_class(c, 8, 1))) return bail(s);
        *out = c;
        return ABFT_OK;
    } catch (...) {
        // a host exception (allocation) after the context was made: nothing leaks
        free_all(c);
        delete c;
        throw;
    }
}

// Every entry point is a named roctx range, so that a profiler's trace shows the library's
// calls around the kernels they enqueue (free when no profiler listens).
struct TraceRange {
    explicit TraceRange(const char* name) noexcept { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
};

// Host exceptions (an allocation failing inside the standard library) never cross the C
// boundary: every entry point turns them into ABFT_E_NOMEM.
template <typename F>
abft_status no_throw(abft_ctx* c, const char* name, F&& f) noexcept
{
    const TraceRange range(name);
    try {
        return f();
    } catch (...) {
        try {
            fail(c, ABFT_E_NOMEM, "host allocation failed");
        } catch (...) {
        }
        return ABFT_E_NOMEM;
    }
}

}  // namespace

// ---- the allocation-free run (abft_stencil_run_noalloc, abft_noalloc.hip) ------------------
namespace abft {

abft_status run_error(abft_status s, const char* msg) noexcept
{
    try {
        g_init_error = msg;
    } catch (...) {
    }
    return s;
}

abft_status noalloc_layout(const abft_problem* p, const abft_options* o, const abft_fault* f,
                           int32_t nf, size_t limit, NoAllocLayout* L)
{
    g_init_error.clear();
    abft_status s = validate_problem(p);
    if (s) return s;
    if ((s = validate_options(p, o))) return s;
    if (o->mode == ABFT_MODE_OFFLINE)
        return fail(nullptr, ABFT_E_UNSUPPORTED,
                    "the allocation-free run covers the online and plain modes");
    if (o->tile_x != 0)
        return fail(nullptr, ABFT_E_UNSUPPORTED, "the allocation-free run keeps row checksums");
    if (nf < 0 || (nf > 0 && !f)) return fail(nullptr, ABFT_E_INVAL, "fault plan");
    const int bits = p->dtype == ABFT_F32 ? 32 : 64;
    for (int32_t i = 0; i < nf; ++i) {
        const abft_fault& x = f[i];
        if (x.grid != 0 || x.sweep < 0 || x.z < 0 || x.z >= p->nz || x.y < 0 || x.y >= p->ny ||
            x.x < 0 || x.x >= p->nx || x.bit < 0 || x.bit >= bits || x.attempt != 0 ||
            (x.kind != ABFT_FAULT_STORE && x.kind != ABFT_FAULT_MEMORY))
            return fail(nullptr, ABFT_E_INVAL, "fault outside the grid or word");
        if (i > 0 && x.sweep < f[i - 1].sweep)
            return fail(nullptr, ABFT_E_INVAL, "the fault plan must be sorted by sweep");
    }
    L->tmax = nf > 0 ? f[nf - 1].sweep + 1 : 0;
    if (L->tmax > (int64_t)1 << 26)
        return fail(nullptr, ABFT_E_INVAL, "fault sweep index too large");
    L->ev_cap = o->max_events ? o->max_events : kDefaultEvents;
    const size_t nrows = (size_t)p->nz * p->ny, ncols = (size_t)p->nz * p->nx;
    const bool wsums = o->input_check && o->mode == ABFT_MODE_ONLINE;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) & ~(size_t)255;
        return at;
    };
    L->B[0] = take(nrows * 8);
    L->B[1] = take(nrows * 8);
    L->W[0] = wsums ? take(nrows * 8) : 0;
    L->W[1] = wsums ? take(nrows * 8) : 0;
    L->wsums = wsums;
    L->cB = take(nrows * 8);
    L->cA = take(ncols * 8);
    L->slot[0] = take(sizeof(FlagSlot));
    L->slot[1] = take(sizeof(FlagSlot));
    L->cnt = take(sizeof(Counters));
    L->ev = take((size_t)L->ev_cap * sizeof(abft_event));
    L->faults = take((size_t)nf * sizeof(abft_fault));
    L->first = take((size_t)(L->tmax + 1) * sizeof(int32_t));
    L->total = off;
    if (L->total > limit) {
        char m[160];
        std::snprintf(m, sizeof(m), "the run needs %zu bytes of workspace; the static scratch "
                                    "holds %zu", L->total, limit);
        return fail(nullptr, ABFT_E_UNSUPPORTED, m);
    }
    return ABFT_OK;
}

abft_status run_in_workspace(const abft_problem* p, const abft_options* o, const abft_fault* f,
                             int32_t nf, int64_t nsweeps, void* hip_stream, unsigned char* ws,
                             const NoAllocLayout& L, abft_report* out)
{
    if (nsweeps < 0) return fail(nullptr, ABFT_E_INVAL, "nsweeps < 0");
    abft_ctx c;  // on the stack: its containers stay empty, every buffer lies in ws
    auto done = [&](abft_status st) {
        if (st) g_init_error = c.err;
        return st;
    };
    abft_status s = configure(&c, p, o, hip_stream, false);
    if (s) return done(s);
    auto at = [&](size_t off) { return static_cast<void*>(ws + off); };
    c.B[0] = static_cast<double*>(at(L.B[0]));
    c.B[1] = static_cast<double*>(at(L.B[1]));
    if (L.wsums) {
        c.W[0] = static_cast<double*>(at(L.W[0]));
        c.W[1] = static_cast<double*>(at(L.W[1]));
    }
    c.cB = static_cast<double*>(at(L.cB));
    c.cA = static_cast<double*>(at(L.cA));
    c.slot[0] = static_cast<FlagSlot*>(at(L.slot[0]));
    c.slot[1] = static_cast<FlagSlot*>(at(L.slot[1]));
    c.cnt = static_cast<Counters*>(at(L.cnt));
    c.ev = static_cast<abft_event*>(at(L.ev));
    c.ev_cap = L.ev_cap;
    if (nf > 0) {
        c.faults = static_cast<abft_fault*>(at(L.faults));
        c.fault_first = static_cast<int32_t*>(at(L.first));
        c.fault_tmax = L.tmax;
        c.nfaults = nf;
        for (int32_t i = 0; i < nf; ++i)
            c.mem_faults = c.mem_faults || f[i].kind == ABFT_FAULT_MEMORY;
    }
    // the scratch keeps the last run's contents: everything that must start at zero is cleared
    // by fill kernels, the rest is written before it is read
    hipError_t e;
#define RUN_CHK(expr)                        \
    if ((e = (expr)) != hipSuccess) {        \
        hip_fail(&c, e, #expr);              \
        return done(ABFT_E_HIP);             \
    }
    RUN_CHK(launch_fill_u32(reinterpret_cast<uint32_t*>(c.cnt), 0u, sizeof(Counters) / 4,
                            c.stream));
    RUN_CHK(launch_fill_u32(&c.slot[0]->count, 0u, 2, c.stream));
    RUN_CHK(launch_fill_u32(&c.slot[1]->count, 0u, 2, c.stream));
    if (nf > 0) {
        RUN_CHK(hipMemcpyAsync(c.faults, f, (size_t)nf * sizeof(abft_fault),
                               hipMemcpyHostToDevice, c.stream));
        RUN_CHK(launch_fault_index(c.faults, nf, c.fault_first, c.fault_tmax, c.stream));
    }
    RUN_CHK(launch_row_sums(c.dtype, c.C, c.cs, c.nx, (int64_t)c.nz * c.ny, c.cB, c.stream));
    RUN_CHK(launch_col_sums(c.dtype, c.C, c.cs, c.nx, c.ny, c.nz, c.cA, c.stream));
    RUN_CHK(launch_row_sums(c.dtype, c.u[0], 0.0, c.nx, (int64_t)c.nz * c.ny, c.B[0], c.stream));
    if (c.W[0] != nullptr)
        RUN_CHK(launch_weighted_row_sums(c.dtype, c.u[0], c.nx, (int64_t)c.nz * c.ny, c.W[0],
                                         c.stream));
#undef RUN_CHK
    if ((s = enqueue_online(&c, nsweeps, nullptr, 0))) return done(s);
    return done(check_impl(&c, out));
}

}  // namespace abft

// ==========================================================================================
extern "C" {

const char* abft_strerror(abft_status s)
{
    switch (s) {
    case ABFT_OK: return "ok";
    case ABFT_E_INVAL: return "invalid argument";
    case ABFT_E_UNSUPPORTED: return "not supported by the GPU kernels";
    case ABFT_E_NOMEM: return "out of memory";
    case ABFT_E_HIP: return "HIP runtime error";
    case ABFT_E_STATE: return "call not allowed in the current state";
    case ABFT_E_UNCORRECTABLE: return "detected corruption could not be corrected";
    }
    return "unknown status";
}

const char* abft_last_error(const abft_ctx* ctx)
{
    return ctx ? ctx->err.c_str() : g_init_error.c_str();
}

abft_status abft_stencil_init(const abft_problem* p, const abft_options* o, void* hip_stream,
                              abft_ctx** out)
{
    if (out) *out = nullptr;
    return no_throw(nullptr, "abft_stencil_init",
                    [&] { return init_impl(p, o, hip_stream, out); });
}

abft_status abft_stencil_init_batch(const abft_problem* p, int32_t n, const abft_options* o,
                                    void* hip_stream, abft_ctx** out)
{
    if (out) *out = nullptr;
    return no_throw(nullptr, "abft_stencil_init_batch", [&] {
        return init_batch_impl(p, n, o, hip_stream, out);
    });
}

abft_status abft_stencil_step(abft_ctx* c, int64_t nsweeps)
{
    return no_throw(c, "abft_stencil_step", [&] { return step_impl(c, nsweeps); });
}

abft_status abft_stencil_step_graph(abft_ctx* c, int64_t nsweeps)
{
    return no_throw(c, "abft_stencil_step_graph", [&] { return step_graph_impl(c, nsweeps); });
}

abft_status abft_stencil_check(abft_ctx* c, abft_report* out)
{
    return no_throw(c, "abft_stencil_check", [&] { return check_impl(c, out); });
}

abft_status abft_stencil_correct(abft_ctx* c, abft_report* inout)
{
    return no_throw(c, "abft_stencil_correct", [&] { return correct_impl(c, inout); });
}

abft_status abft_stencil_current(abft_ctx* c, int32_t grid, void** dev_ptr, int64_t* sweep)
{
    return no_throw(c, "abft_stencil_current", [&] {
        return current_impl(c, grid, dev_ptr, sweep);
    });
}

abft_status abft_stencil_checksums(abft_ctx* c, int32_t grid, double** dev_ptr)
{
    return no_throw(c, "abft_stencil_checksums", [&] { return checksums_impl(c, grid, dev_ptr); });
}

abft_status abft_stencil_inject(abft_ctx* c, const abft_fault* f, int32_t n)
{
    return no_throw(c, "abft_stencil_inject", [&] { return inject_impl(c, f, n); });
}

abft_status abft_stencil_autotune(abft_ctx* c)
{
    return no_throw(c, "abft_stencil_autotune", [&] { return autotune_impl(c); });
}

abft_status abft_stencil_launch_shape(const abft_ctx* c, int32_t* rows_per_block,
                                      int32_t* planes_per_block, int32_t* lanes_per_row)
{
    return no_throw(nullptr, "abft_stencil_launch_shape", [&] {
        return launch_shape_impl(c, rows_per_block, planes_per_block, lanes_per_row);
    });
}

void abft_stencil_destroy(abft_ctx* c)
{
    const TraceRange range("abft_stencil_destroy");
    try {
        destroy_impl(c);
    } catch (...) {
    }
}

}  // extern "C"
