// Host side of the C ABI (include/rt.h): argument validation, scene storage,
// Morton ordering of blocks, and the launch sequence of build and trace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "scene_impl.h"

using namespace rt;

namespace rt {
// build.hip: counts negative or non-finite input values (scene creation)
hipError_t launch_validate(const Inputs& in, int model, int n_lam, int n_lines, int dim, unsigned long long* count,
                           hipStream_t s);
}  // namespace rt

namespace {

thread_local std::string g_err;

rt_status fail(rt_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define RT_HIP(call)                                                                                  \
    do {                                                                                              \
        hipError_t e_ = (call);                                                                       \
        if (e_ != hipSuccess) return fail(RT_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_));    \
    } while (0)

int ilog2(int v)
{
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}

}  // namespace

rt_status rt::set_error(rt_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define RT_TRY(call)                        \
    do {                                    \
        rt_status s_ = (call);              \
        if (s_ != RT_OK) return s_;         \
    } while (0)

extern "C" {

const char* rt_last_error(void) { return g_err.c_str(); }

const char* rt_version(void) { return "rt 0.1 (gfx950)"; }

}  // extern "C"

// Descriptor checks shared by rt_scene_create and rt_scene_workspace_bytes (inp may be null: no input checks).
static rt_status check_desc(const rt_scene_desc* d, const rt_scene_inputs* inp)
{
    if (d->dim != 2 && d->dim != 3) return fail(RT_E_ARG, "dim must be 2 or 3 (got %d)", d->dim);
    if (d->brick != 8 && d->brick != 16) return fail(RT_E_ARG, "brick must be 8 or 16 (got %d)", d->brick);
    const int log2B = ilog2(d->brick);
    if (d->n_levels < 1 || d->n_levels > log2B + 1 || d->n_levels > RT_MAX_LEVELS)
        return fail(RT_E_ARG, "n_levels must be in [1, log2(brick)+1] (got %d)", d->n_levels);
    if (d->dim == 3 && d->brick == 16) return fail(RT_E_UNSUPPORTED, "3D scenes use 8^3 bricks");
    for (int a = 0; a < 3; ++a) {
        int na = d->n[a];
        if (a < d->dim) {
            if (na <= 0 || na % d->brick != 0 || na > 8192)
                return fail(RT_E_ARG, "n[%d] = %d must be a positive multiple of brick, at most 8192", a, na);
        } else if (na != 1) {
            return fail(RT_E_ARG, "n[%d] must be 1 for a %dD scene", a, d->dim);
        }
    }
    if (!(d->ds0 > 0.0)) return fail(RT_E_ARG, "ds0 must be positive");
    if (d->n_lam < 1) return fail(RT_E_ARG, "n_lam must be >= 1");
    if (d->model == RT_MODEL_STATIC) {
        if (d->emission != RT_EMIS_STATIC && d->emission != RT_EMIS_PREFILTER)
            return fail(RT_E_ARG, "static model supports RT_EMIS_STATIC and RT_EMIS_PREFILTER only");
        if (inp && (!inp->d_eta || !inp->d_chi)) return fail(RT_E_ARG, "static model needs d_eta and d_chi");
    } else if (d->model == RT_MODEL_LINES) {
        if (d->n_lines < 1 || d->n_lines > RT_MAX_LINES) return fail(RT_E_ARG, "n_lines must be in [1, %d]", RT_MAX_LINES);
        if (d->profile != RT_PROFILE_GAUSS && d->profile != RT_PROFILE_VOIGT) return fail(RT_E_ARG, "bad profile");
        if (d->emission < RT_EMIS_STATIC || d->emission > RT_EMIS_PREFILTER) return fail(RT_E_ARG, "bad emission");
        if (d->emission == RT_EMIS_VELINTERP && d->n_v < 2) return fail(RT_E_ARG, "n_v must be >= 2");
        if (d->vgrid != RT_VGRID_FULL && d->vgrid != RT_VGRID_ORTHANT) return fail(RT_E_ARG, "bad vgrid %d", d->vgrid);
        if (!d->h_lam || !d->h_lam0) return fail(RT_E_ARG, "lines model needs h_lam and h_lam0");
        if (inp && (!inp->d_eta_star || !inp->d_chi_star || !inp->d_damp || !inp->d_inv_dld || !inp->d_eta_bg ||
                    !inp->d_chi_bg || !inp->d_vel))
            return fail(RT_E_ARG, "lines model needs every line input");
        for (int l = 0; l < d->n_lam; ++l)
            if (!(d->h_lam[l] > 0.0)) return fail(RT_E_ARG, "wavelengths must be positive");
        for (int l = 0; l < d->n_lines; ++l)
            if (!(d->h_lam0[l] > 0.0)) return fail(RT_E_ARG, "rest wavelengths must be positive");
    } else {
        return fail(RT_E_ARG, "bad model %d", d->model);
    }
    return RT_OK;
}

// LDS a trace workgroup stages: the packed block states, and the slot table on grids of <= kSlotLdsMax blocks.
static long long trace_lds_bytes(const Geo& g)
{
    // state words, the slot table on small grids, the level_dist table, and the angle-integrated
    // kernel's J and psi sums (2 x kLam floats per lane of a 256-lane workgroup)
    return 8ll * g.n_state_words + (g.nblocks <= kSlotLdsMax ? 4ll * g.nblocks : 0ll) + 4ll * kMaxLevels +
           2ll * kLam * 256 * 4;
}

static void make_geo(const rt_scene_desc* d, Geo& g)
{
    const int log2B = ilog2(d->brick);
    std::memset(&g, 0, sizeof(g));
    g.dim = d->dim;
    g.B = d->brick;
    g.log2B = log2B;
    g.n_levels = d->n_levels;
    g.nblocks = 1;
    for (int a = 0; a < 3; ++a) {
        g.n[a] = d->n[a];
        g.nb[a] = a < d->dim ? d->n[a] / d->brick : 1;
        g.nblocks *= g.nb[a];
    }
    g.bvox = 1 << (d->dim * log2B);
    int off = 0;
    for (int m = 0; m <= RT_MAX_LEVELS; ++m) {
        g.lvl_off[m] = off;
        if (m < d->n_levels) off += 1 << (d->dim * (log2B - m));
    }
    g.cells = off;
    g.lvl_pack = 0;
    for (int m = 0; m < kMaxLevels; ++m) g.lvl_pack |= (unsigned long long)g.lvl_off[m] << (11 * m);
    g.n_state_words = (int)((g.nblocks + kStatesPerWord - 1) / kStatesPerWord);
    g.feat_level = std::min(2, d->n_levels - 1);
}

// Direction classes of the velocity-interpolation grids.
static int vclasses(const rt_scene_desc* d) { return d->vgrid == RT_VGRID_ORTHANT ? 1 << d->dim : 1; }

// The scene's workspace in the order it is carved.  First the pieces sized by
// the block count: Morton order, occupancy, slot table, active list and count,
// levels, packed states, device error counters and the input-check counter.
static bool carve_fixed(const Geo& g, Carver& c, SceneBufs& B, unsigned long long** d_bad)
{
    const size_t nb = (size_t)g.nblocks;
    return c.take(&B.morton, nb) && c.take(&B.active, nb) && c.take(&B.slot, nb) && c.take(&B.active_list, nb) &&
           c.take(&B.n_active, 1) && c.take(&B.levels, nb) && c.take(&B.states, (size_t)g.n_state_words) &&
           c.take(&B.err, 4) && c.take(d_bad, 1);
}

// Then the pieces sized by the active-block count: level statistics of the
// cache features, and the stored values of the emission mode (static values,
// velocity grids and node values, or the Core-and-Voigt chain and its
// reduced-precision copy).
static bool carve_active(const rt_scene_desc* d, const Geo& g, long long na, Carver& c, SceneBufs& B)
{
    const size_t cells = (size_t)na * g.cells;
    if (!c.take(&B.fstats, ((size_t)na << (d->dim * (g.log2B - g.feat_level))) * kLam)) return false;
    if (d->emission == RT_EMIS_STATIC || d->emission == RT_EMIS_PREFILTER)
        if (!c.take((float**)&B.vals, cells * kLam * 2)) return false;
    if (d->emission == RT_EMIS_PREFILTER)  // one record per signed axis of every cell (level 0 unused)
        if (!c.take((float**)&B.pf, cells * (size_t)(2 * d->dim) * kLam * 2)) return false;
    if (d->model == RT_MODEL_LINES && d->emission == RT_EMIS_VELINTERP) {
        const size_t nq = (size_t)vclasses(d);
        if (!c.take(&B.vgrid, nq * cells) || !c.take(&B.vrange, nq * cells) ||
            !c.take(&B.vnodes, nq * cells * (size_t)d->n_v * kLam * 2))
            return false;
    }
    if (d->model == RT_MODEL_LINES && d->emission == RT_EMIS_CAV) {
        const size_t rec = (size_t)cav_rec_floats(d->n_lines);
        if (!c.take(&B.cav, cells * rec) || !c.take((uint16_t**)&B.cav_lp, cells * rec)) return false;
    }
    return true;
}

// Workspace bytes of a scene with na active blocks (the carving above, dry run).
static size_t scene_bytes(const rt_scene_desc* d, const Geo& g, long long na)
{
    Carver c;
    SceneBufs B;
    unsigned long long* bad = nullptr;
    carve_fixed(g, c, B, &bad);
    carve_active(d, g, na, c, B);
    return c.used;
}

// Bytes of the block-count part alone (what rt_scene_count_active needs).
static size_t fixed_bytes(const Geo& g)
{
    Carver c;
    SceneBufs B;
    unsigned long long* bad = nullptr;
    carve_fixed(g, c, B, &bad);
    return c.used;
}

static void bind_inputs(const rt_scene_inputs* inp, const Geo& g, Inputs& in)
{
    in.eta = inp->d_eta;
    in.chi = inp->d_chi;
    in.eta_star = inp->d_eta_star;
    in.chi_star = inp->d_chi_star;
    in.damp = inp->d_damp;
    in.inv_dld = inp->d_inv_dld;
    in.eta_bg = inp->d_eta_bg;
    in.chi_bg = inp->d_chi_bg;
    in.vel = inp->d_vel;
    in.mask = inp->d_block_mask;
    in.nvox = (long long)g.n[0] * g.n[1] * g.n[2];
}

// Input check, block classification, Morton order and slots (Sect. 2.3.1) into
// the block-count pieces of B; reads the active count back (synchronises s).
static rt_status classify_blocks(const rt_scene_desc* d, const Geo& g, const Inputs& in, SceneBufs& B,
                                 unsigned long long* d_bad, hipStream_t s, int32_t* h_na)
{
    // Morton order of all blocks (geometry only)
    std::vector<std::pair<uint64_t, int32_t>> mo((size_t)g.nblocks);
    for (long long b = 0; b < g.nblocks; ++b) {
        uint32_t bc[3] = {(uint32_t)(b % g.nb[0]), (uint32_t)((b / g.nb[0]) % g.nb[1]),
                          (uint32_t)(b / ((long long)g.nb[0] * g.nb[1]))};
        uint64_t code = 0;
        for (int bit = 0; bit < 21; ++bit)
            for (int a = 0; a < g.dim; ++a) code |= (uint64_t)((bc[a] >> bit) & 1u) << (bit * g.dim + a);
        mo[(size_t)b] = {code, (int32_t)b};
    }
    std::sort(mo.begin(), mo.end());
    std::vector<int32_t> morton((size_t)g.nblocks);
    for (size_t i = 0; i < mo.size(); ++i) morton[i] = mo[i].second;
    hipError_t e;
    if ((e = hipMemcpyAsync(B.morton, morton.data(), morton.size() * sizeof(int32_t), hipMemcpyHostToDevice, s)) !=
        hipSuccess)
        return fail(RT_E_HIP, "upload: %s", hipGetErrorString(e));
    // step-cap hits, first ray that hit the cap, probe indices outside the grid, unused; input-check count
    unsigned long long err0[5] = {0ull, ~0ull, 0ull, 0ull, 0ull};
    if ((e = hipMemcpyAsync(B.err, err0, 4 * sizeof(unsigned long long), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(d_bad, err0 + 4, sizeof(unsigned long long), hipMemcpyHostToDevice, s)) != hipSuccess)
        return fail(RT_E_HIP, "upload: %s", hipGetErrorString(e));
    if ((e = launch_validate(in, d->model, d->n_lam, d->n_lines, d->dim, d_bad, s)) != hipSuccess)
        return fail(RT_E_HIP, "validate: %s", hipGetErrorString(e));
    if ((e = launch_classify(g, in, d->model, d->n_lam, d->n_lines, d->dense, B.active, s)) != hipSuccess)
        return fail(RT_E_HIP, "classify: %s", hipGetErrorString(e));
    if ((e = launch_slots(g, B.morton, B.active, B.slot, B.active_list, B.n_active, s)) != hipSuccess)
        return fail(RT_E_HIP, "slots: %s", hipGetErrorString(e));
    if ((e = launch_fill_levels(g, B.levels, s)) != hipSuccess) return fail(RT_E_HIP, "levels: %s", hipGetErrorString(e));
    int32_t na = 0;
    unsigned long long n_bad = 0;
    if ((e = hipMemcpyAsync(&na, B.n_active, sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipMemcpyAsync(&n_bad, d_bad, sizeof(n_bad), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return fail(RT_E_HIP, "readback: %s", hipGetErrorString(e));
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(RT_E_HIP, "synchronize: %s", hipGetErrorString(e));
    if (n_bad) return fail(RT_E_ARG, "inputs hold %llu negative or non-finite values", n_bad);
    *h_na = na;
    return RT_OK;
}

// Device-to-host copy ordered on the caller's stream, then that stream synchronised.
static rt_status copy_back(void* h, const void* d, size_t bytes, hipStream_t s)
{
    hipError_t e = hipMemcpyAsync(h, d, bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(RT_E_HIP, "device-to-host copy: %s", hipGetErrorString(e));
    return RT_OK;
}

static rt_status check_ws(const void* d_ws, size_t ws_bytes, size_t need, const char* who)
{
    if (!d_ws) return fail(RT_E_ARG, "%s: null workspace", who);
    if ((uintptr_t)d_ws % 256 != 0) return fail(RT_E_ARG, "%s: workspace must be 256-byte aligned", who);
    if (ws_bytes < need) return fail(RT_E_ARG, "%s: workspace of %zu bytes, %zu needed", who, ws_bytes, need);
    return RT_OK;
}

extern "C" {

rt_status rt_scene_workspace_bytes(const rt_scene_desc* d, int64_t n_active, size_t* h_bytes)
{
    g_err.clear();
    if (!d || !h_bytes) return fail(RT_E_ARG, "null argument");
    RT_TRY(check_desc(d, nullptr));
    Geo g;
    make_geo(d, g);
    if (n_active < 0 || n_active > g.nblocks) return fail(RT_E_ARG, "n_active must be in [0, %lld]", g.nblocks);
    if (trace_lds_bytes(g) > kLdsPerCuBytes)
        return fail(RT_E_UNSUPPORTED, "%lld blocks: their packed states need %lld bytes of LDS per trace workgroup, more "
                    "than a compute unit holds (%lld)", g.nblocks, trace_lds_bytes(g), kLdsPerCuBytes);
    *h_bytes = scene_bytes(d, g, n_active);
    return RT_OK;
}

rt_status rt_scene_count_active(const rt_scene_desc* d, const rt_scene_inputs* inp, void* d_ws, size_t ws_bytes,
                                void* stream, int64_t* h_n_active)
{
    g_err.clear();
    if (!d || !inp || !h_n_active) return fail(RT_E_ARG, "null argument");
    RT_TRY(check_desc(d, inp));
    Geo g;
    make_geo(d, g);
    RT_TRY(check_ws(d_ws, ws_bytes, fixed_bytes(g), "rt_scene_count_active"));
    Inputs in;
    std::memset(&in, 0, sizeof(in));
    bind_inputs(inp, g, in);
    Carver c;
    c.base = (char*)d_ws;
    c.cap = ws_bytes;
    SceneBufs B;
    std::memset(&B, 0, sizeof(B));
    unsigned long long* d_bad = nullptr;
    carve_fixed(g, c, B, &d_bad);
    int32_t na = 0;
    RT_TRY(classify_blocks(d, g, in, B, d_bad, (hipStream_t)stream, &na));
    *h_n_active = na;
    return RT_OK;
}

rt_status rt_scene_create(const rt_scene_desc* d, const rt_scene_inputs* inp, void* d_ws, size_t ws_bytes,
                          void* stream, rt_scene** out)
{
    g_err.clear();
    if (!d || !inp || !out) return fail(RT_E_ARG, "null argument");
    *out = nullptr;
    hipStream_t s = (hipStream_t)stream;
    RT_TRY(check_desc(d, inp));
    Geo g0;
    make_geo(d, g0);
    RT_TRY(check_ws(d_ws, ws_bytes, fixed_bytes(g0), "rt_scene_create"));
    {
        // the trace kernels stage the packed block states (and small grids' slot tables) in LDS
        int dev = 0, max_lds = 0;
        RT_HIP(hipGetDevice(&dev));
        RT_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        const long long need = trace_lds_bytes(g0);
        if (need > (long long)max_lds)
            return fail(RT_E_UNSUPPORTED, "%lld blocks: their packed states need %lld bytes of LDS per trace "
                        "workgroup, the device allows %d", g0.nblocks, need, max_lds);
    }

    rt_scene* sc = new (std::nothrow) rt_scene();
    if (!sc) return fail(RT_E_ARG, "out of host memory");
    auto cleanup = [&](rt_status st) {
        delete sc;
        return st;
    };
    sc->desc = *d;
    sc->desc.h_lam = nullptr;  // the handle keeps its own copies
    sc->desc.h_lam0 = nullptr;
    Geo& g = sc->g;
    g = g0;
    if (d->model == RT_MODEL_LINES) {
        sc->lam.assign(d->h_lam, d->h_lam + d->n_lam);
        sc->lam0.assign(d->h_lam0, d->h_lam0 + d->n_lines);
    }
    Inputs& in = sc->in;
    std::memset(&in, 0, sizeof(in));
    bind_inputs(inp, g, in);
    SceneBufs& B = sc->b;
    std::memset(&B, 0, sizeof(B));
    Carver c;
    c.base = (char*)d_ws;
    c.cap = ws_bytes;
    unsigned long long* d_bad = nullptr;
    carve_fixed(g, c, B, &d_bad);
    int32_t na = 0;
    rt_status st;
    if ((st = classify_blocks(d, g, in, B, d_bad, s, &na)) != RT_OK) return cleanup(st);
    sc->n_active = na;
    const size_t cells = (size_t)na * g.cells;
    if (d->model == RT_MODEL_LINES && d->emission == RT_EMIS_VELINTERP &&
        cells * (size_t)d->n_v * kLam * 2 >= (size_t)1 << 31)  // per class, node offsets in the trace are 32-bit
        return cleanup(fail(RT_E_UNSUPPORTED, "velocity-node storage of one direction class exceeds 2^31 floats"));
    if (d->model == RT_MODEL_LINES && d->emission == RT_EMIS_CAV &&
        sizeof(double) * (size_t)(4 * d->n_lines + 2 + d->dim) * g.cells > 160 * 1024)
        return cleanup(fail(RT_E_UNSUPPORTED, "too many lines for the LDS chain"));
    const size_t need = scene_bytes(d, g, na);
    if (ws_bytes < need)
        return cleanup(fail(RT_E_ARG, "rt_scene_create: %d active blocks need a workspace of %zu bytes (got %zu)", na,
                            need, ws_bytes));
    carve_active(d, g, na, c, B);
    sc->bytes = c.used;
    hipError_t e;
    if (d->model == RT_MODEL_LINES && d->emission == RT_EMIS_VELINTERP) {
        if ((e = launch_vgrid(g, in, B, na, d->n_v, vclasses(d), s)) != hipSuccess)
            return cleanup(fail(RT_E_HIP, "velocity grid: %s", hipGetErrorString(e)));
    }
    if (d->model == RT_MODEL_LINES && d->emission == RT_EMIS_CAV) {
        sc->cav_rec = cav_rec_floats(d->n_lines);
        if ((e = launch_cav_chain(g, in, B, na, d->n_lines, d->ds0, RT_AVG_LINEAR, s)) != hipSuccess)
            return cleanup(fail(RT_E_HIP, "core-and-voigt chain: %s", hipGetErrorString(e)));
        sc->cav_mode = RT_AVG_LINEAR;
    }
    *out = sc;
    return RT_OK;
}


static LamBatch make_batch(const rt_scene* sc, int lam_begin, int lam_end)
{
    LamBatch lb;
    std::memset(&lb, 0, sizeof(lb));
    lb.nl = lam_end - lam_begin;
    lb.n_lines = sc->desc.model == RT_MODEL_LINES ? sc->desc.n_lines : 0;
    lb.profile = sc->desc.profile;
    for (int l = 0; l < kLam; ++l) {
        int il = lam_begin + std::min(l, lb.nl - 1);
        lb.lam[l] = sc->lam.empty() ? 0.0 : sc->lam[(size_t)il];
    }
    for (int k = 0; k < kMaxLines; ++k) lb.lam0[k] = k < lb.n_lines ? sc->lam0[(size_t)k] : 1.0;
    for (int k = 0; k < kMaxLines; ++k) {
        lb.k0[k] = (float)(lb.lam0[k] / kCkms);
        for (int l = 0; l < kLam; ++l) {
            lb.dl[l][k] = (float)(lb.lam[l] - lb.lam0[k]);
            lb.rr[l][k] = (float)(lb.lam[l] / lb.lam0[k]);
            lb.sr[l][k] = (float)(0.56418958354775628 * lb.lam0[k] / lb.lam[l]);
        }
    }
    return lb;
}

rt_status rt_scene_build(rt_scene* sc, const rt_build_params* p, int32_t lam_begin, int32_t lam_end, void* stream)
{
    g_err.clear();
    if (!sc || !p) return fail(RT_E_ARG, "null argument");
    hipStream_t s = (hipStream_t)stream;
    const rt_scene_desc& d = sc->desc;
    if (lam_begin < 0 || lam_end > d.n_lam || lam_end <= lam_begin || lam_end - lam_begin > kLam)
        return fail(RT_E_ARG, "wavelength batch [%d, %d) invalid (n_lam %d, at most %d per batch)", lam_begin,
                    lam_end, d.n_lam, kLam);
    if (!(p->iod_threshold >= 0.0)) return fail(RT_E_ARG, "iod_threshold must be >= 0");
    if (!(p->tau_thin >= 0.0)) return fail(RT_E_ARG, "tau_thin must be >= 0");
    if (p->avg_mode != RT_AVG_LOG && p->avg_mode != RT_AVG_LINEAR) return fail(RT_E_ARG, "bad avg_mode");
    if (p->storage < RT_F32 || p->storage > RT_F16) return fail(RT_E_ARG, "bad storage dtype");
    const bool static_emis = d.emission == RT_EMIS_STATIC || d.emission == RT_EMIS_PREFILTER;
    LamBatch lb = make_batch(sc, lam_begin, lam_end);
    const Geo& g = sc->g;
    int cap = p->max_level < 0 ? -1 : p->max_level;
    RT_HIP(launch_fill_levels(g, sc->b.levels, s));
    if (p->iod_frame != RT_IOD_REST && p->iod_frame != RT_IOD_CORE) return fail(RT_E_ARG, "bad iod_frame");
    const int vrule = (d.model == RT_MODEL_LINES && (d.emission == RT_EMIS_CAV || p->iod_frame == RT_IOD_CORE)) ? 1 : 0;
    RT_HIP(launch_build_static(g, sc->in, sc->b, sc->n_active, d.model, vrule, lb, lam_begin, d.ds0, p->iod_threshold,
                               p->tau_thin, cap, p->avg_mode, p->storage, static_emis ? 1 : 0, s));
    if (d.model == RT_MODEL_LINES && d.emission == RT_EMIS_VELINTERP)
        RT_HIP(launch_velinterp_nodes(g, sc->in, sc->b, sc->n_active, lb, d.n_v, vclasses(&d), d.ds0, p->avg_mode,
                                      p->storage, s));
    if (d.emission == RT_EMIS_PREFILTER)
        RT_HIP(launch_build_prefilter(g, sc->in, sc->b, sc->n_active, d.model, lb, lam_begin, d.ds0, p->storage, s));
    RT_HIP(launch_pack_states(g, sc->b.levels, sc->b.states, s));
    if (d.model == RT_MODEL_LINES && d.emission == RT_EMIS_CAV && p->avg_mode != sc->cav_mode) {
        // the wavelength-independent chain follows the stored-value mode of the build
        RT_HIP(launch_cav_chain(g, sc->in, sc->b, sc->n_active, d.n_lines, d.ds0, p->avg_mode, s));
        sc->cav_mode = p->avg_mode;
        sc->cav_lp_dtype = -1;
    }
    if (d.emission == RT_EMIS_CAV && p->storage != RT_F32 && sc->cav_lp_dtype != p->storage) {
        // the chain does not depend on the wavelength: encode it once per dtype
        RT_HIP(launch_cav_encode(sc->b.cav, sc->b.cav_lp, (long long)sc->n_active * g.cells * sc->cav_rec, p->storage, s));
        sc->cav_lp_dtype = p->storage;
    }
    sc->batch_begin = lam_begin;
    sc->batch_end = lam_end;
    sc->storage = p->storage;
    return RT_OK;
}

}  // extern "C"

TraceLaunch rt::make_trace(const rt_scene* sc, const rt_trace_params* p)
{
    TraceLaunch t;
    std::memset(&t, 0, sizeof(t));
    const Geo& g = sc->g;
    t.g = g;
    t.states = sc->b.states;
    t.slot = sc->b.slot;
    t.vals = sc->b.vals;
    t.pf = sc->b.pf;
    t.vgrid = sc->b.vgrid;
    t.vnodes = sc->b.vnodes;
    t.cav = sc->b.cav;
    t.cav_lp = sc->b.cav_lp;
    t.mode = p->mode;
    t.max_level = p->max_level < 0 ? 127 : p->max_level;
    t.graded = 0;
    for (int m = 0; m < kMaxLevels; ++m) {
        t.level_dist[m] = m == 0 ? 0.f : p->level_dist[m];
        if (m > 0 && p->level_dist[m] != 0.f) t.graded = p->grade_mode == RT_GRADE_PATH ? 2 : 1;
    }
    int cap = 16;
    for (int a = 0; a < g.dim; ++a) cap += 2 * g.n[a];
    t.step_cap = p->step_cap > 0 ? p->step_cap : cap;
    t.active_list = sc->b.active_list;
    t.I0 = p->I0;
    t.ds0 = (float)sc->desc.ds0;
    t.emission = sc->desc.emission;
    t.storage = sc->storage;
    t.n_v = sc->desc.n_v;
    t.n_vclass = vclasses(&sc->desc);
    t.n_active = sc->n_active;
    t.cav_rec = sc->cav_rec;
    t.lb = make_batch(sc, sc->batch_begin, sc->batch_end);
    t.stats = p->d_stats;
    t.err = sc->b.err;
    t.fstats = sc->b.fstats;
    return t;
}

// Checks shared by the per-direction trace entry points (pointers checked by the caller).
static rt_status check_trace(const rt_scene* sc, const rt_trace_params* p, int32_t n_dir, const int32_t* d_probes,
                             int64_t n_probes, const char* who)
{
    if (sc->batch_begin < 0) return fail(RT_E_STATE, "%s before rt_scene_build", who);
    if (p->mode != RT_TRACE_LEVEL0 && p->mode != RT_TRACE_VLM) return fail(RT_E_ARG, "bad trace mode");
    if (n_dir < 1) return fail(RT_E_ARG, "n_dir must be >= 1");
    for (int m = 1; m < RT_MAX_LEVELS; ++m)
        if (!(p->level_dist[m] >= 0.f)) return fail(RT_E_ARG, "level_dist[%d] must be >= 0", m);
    if (p->grade_mode != RT_GRADE_BLOCK_ENTRY && p->grade_mode != RT_GRADE_PATH)
        return fail(RT_E_ARG, "bad grade_mode %d", (int)p->grade_mode);
    if (n_probes < 0) return fail(RT_E_ARG, "n_probes must be >= 0");
    if (n_probes == 0) return RT_OK;  // nothing to trace (probe and output pointers may be null)
    const long long all = (long long)sc->n_active * sc->g.bvox;
    if (!d_probes && n_probes != all)
        return fail(RT_E_ARG, "all-probes trace needs n_probes = %lld (got %lld)", all, (long long)n_probes);
    // waves: n_dir x 64-probe tiles, padded to eight equal chunks in 3D
    if ((long long)n_dir * ((n_probes + 63) / 64 + 7) > (long long)0x7fffffff * 4)
        return fail(RT_E_ARG, "launch too large");
    return RT_OK;
}

extern "C" {

rt_status rt_trace(const rt_scene* sc, const rt_trace_params* p, const float* d_dirs, int32_t n_dir,
                   const int32_t* d_probes, int64_t n_probes, float* d_I, void* stream)
{
    g_err.clear();
    if (!sc || !p || !d_dirs || (!d_I && n_probes != 0)) return fail(RT_E_ARG, "null argument");
    rt_status st = check_trace(sc, p, n_dir, d_probes, n_probes, "rt_trace");
    if (st != RT_OK || n_probes == 0) return st;
    TraceLaunch t = make_trace(sc, p);
    t.dirs = d_dirs;
    t.n_dir = n_dir;
    t.probes = d_probes;
    t.n_probes = n_probes;
    t.I = d_I;
    RT_HIP(launch_trace(t, (hipStream_t)stream));
    return RT_OK;
}

rt_status rt_trace_interval(const rt_scene* sc, const rt_trace_params* p, const float* d_dirs, int32_t n_dir,
                            const int32_t* d_probes, int64_t n_probes, double t1, double t2, float* d_I, float* d_T,
                            void* stream)
{
    g_err.clear();
    if (!sc || !p || !d_dirs || (!d_I && n_probes != 0)) return fail(RT_E_ARG, "null argument");
    if (!(t1 >= 0.0) || !(t1 < INFINITY)) return fail(RT_E_ARG, "t1 must be finite and >= 0 (got %g)", t1);
    if (!(t2 >= t1)) return fail(RT_E_ARG, "t2 must be >= t1 (got t1 = %g, t2 = %g)", t1, t2);
    rt_status st = check_trace(sc, p, n_dir, d_probes, n_probes, "rt_trace_interval");
    if (st != RT_OK || n_probes == 0) return st;
    TraceLaunch t = make_trace(sc, p);
    t.dirs = d_dirs;
    t.n_dir = n_dir;
    t.probes = d_probes;
    t.n_probes = n_probes;
    t.I = d_I;
    t.interval = 1;
    t.t_lo = t1;
    t.t_hi = t2;
    t.T_out = d_T;
    RT_HIP(launch_trace(t, (hipStream_t)stream));
    return RT_OK;
}

}  // extern "C"

// Direction chunks of an angle-integrated trace: ~2^18 waves, as many as a
// per-direction trace of a mid-size scene launches (latency hiding needs them),
// never more chunks than directions.
static long long j_target_chunks(int n_dir, long long n_probes)
{
    const long long tiles = (n_probes + 63) / 64;
    if (tiles <= 0) return 1;
    long long c = ((1ll << 18) + tiles - 1) / tiles;
    if (c < 1) c = 1;
    if (c > n_dir) c = n_dir;
    return c;
}

extern "C" {

rt_status rt_trace_j_workspace_bytes(const rt_scene* sc, int32_t n_dir, int64_t n_probes, int32_t with_psi,
                                     size_t* h_bytes)
{
    g_err.clear();
    if (!sc || !h_bytes) return fail(RT_E_ARG, "null argument");
    if (n_dir < 1 || n_probes < 0) return fail(RT_E_ARG, "n_dir must be >= 1 and n_probes >= 0");
    const long long c = j_target_chunks(n_dir, n_probes);
    *h_bytes = c <= 1 ? 0 : (size_t)c * kLam * (size_t)n_probes * sizeof(float) * (with_psi ? 2 : 1);
    return RT_OK;
}

}  // extern "C"

// rt_trace_j with the chunk partials in d_work (nullable: one chunk).
static rt_status trace_j_impl(const rt_scene* sc, const rt_trace_params* p, const float* d_dirs, const float* d_weights,
                              int32_t n_dir, const int32_t* d_probes, int64_t n_probes, float* d_J, float* d_psi,
                              float* d_work, size_t work_bytes, hipStream_t s)
{
    const int nl = sc->batch_end - sc->batch_begin;
    const long long per_chunk = (long long)nl * n_probes * (d_psi ? 2 : 1);
    long long chunks = j_target_chunks(n_dir, n_probes);
    if (d_work) {
        const long long fit = (long long)(work_bytes / sizeof(float)) / per_chunk;
        if (chunks > fit) chunks = fit;
    } else {
        chunks = 1;
    }
    if (chunks < 1) chunks = 1;
    const int dpc = (int)((n_dir + chunks - 1) / chunks);
    chunks = (n_dir + dpc - 1) / dpc;
    if (((n_probes + 63) / 64) * chunks > (long long)0x7fffffff * 4) return fail(RT_E_ARG, "launch too large");
    TraceLaunch t = make_trace(sc, p);
    t.dirs = d_dirs;
    t.n_dir = n_dir;
    t.probes = d_probes;
    t.n_probes = n_probes;
    t.jmode = 1;
    t.dirs_per_chunk = dpc;
    t.weights = d_weights;
    if (chunks == 1) {
        t.part_J = d_J;
        t.part_psi = d_psi;
        RT_HIP(launch_trace(t, s));
        return RT_OK;
    }
    const long long n = (long long)nl * n_probes;
    t.part_J = d_work;
    t.part_psi = d_psi ? d_work + chunks * n : nullptr;
    RT_HIP(launch_trace(t, s));
    RT_HIP(launch_reduce_chunks(t.part_J, (int)chunks, n, d_J, s));
    if (d_psi) RT_HIP(launch_reduce_chunks(t.part_psi, (int)chunks, n, d_psi, s));
    return RT_OK;
}

// Device scratch of rt_trace_j_noalloc: the direction-chunk partials of J and
// psi.  One copy per device, held until the process ends; host code uses only
// the address hipGetSymbolAddress returns for the current device.
static constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) float scratch[kNoAllocScratchBytes / sizeof(float)];

static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static float* g_scratch_ptr[kMaxDevices];

// Address of the current device's scratch, looked up once per device.
static rt_status scratch_address(float** out)
{
    int dev = -1;
    RT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(RT_E_UNSUPPORTED, "device ordinal %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return fail(RT_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = (float*)ptr;
    }
    *out = g_scratch_ptr[dev];
    return RT_OK;
}

extern "C" {

rt_status rt_trace_j(const rt_scene* sc, const rt_trace_params* p, const float* d_dirs, const float* d_weights,
                     int32_t n_dir, const int32_t* d_probes, int64_t n_probes, float* d_J, float* d_psi, float* d_work,
                     size_t work_bytes, void* stream)
{
    g_err.clear();
    if (!sc || !p || !d_dirs || !d_weights || (!d_J && n_probes != 0)) return fail(RT_E_ARG, "null argument");
    rt_status st = check_trace(sc, p, n_dir, d_probes, n_probes, "rt_trace_j");
    if (st != RT_OK || n_probes == 0) return st;
    return trace_j_impl(sc, p, d_dirs, d_weights, n_dir, d_probes, n_probes, d_J, d_psi, d_work, work_bytes,
                        (hipStream_t)stream);
}

rt_status rt_trace_j_noalloc(const rt_scene* sc, const rt_trace_params* p, const float* d_dirs,
                             const float* d_weights, int32_t n_dir, const int32_t* d_probes, int64_t n_probes,
                             float* d_J, float* d_psi, void* stream)
{
    g_err.clear();
    if (!sc || !p || !d_dirs || !d_weights || (!d_J && n_probes != 0)) return fail(RT_E_ARG, "null argument");
    rt_status st = check_trace(sc, p, n_dir, d_probes, n_probes, "rt_trace_j_noalloc");
    if (st != RT_OK || n_probes == 0) return st;
    // the chunking rt_trace_j takes with a workspace of rt_trace_j_workspace_bytes
    const long long chunks = j_target_chunks(n_dir, n_probes);
    const size_t nl = (size_t)(sc->batch_end - sc->batch_begin);
    const size_t need = chunks <= 1 ? 0 : (size_t)chunks * nl * (size_t)n_probes * sizeof(float) * (d_psi ? 2 : 1);
    if (need > kNoAllocScratchBytes)
        return fail(RT_E_ARG,
                    "rt_trace_j_noalloc: %lld probes x %d directions need %zu bytes of chunk partials, more than "
                    "its %zu-byte device scratch (use rt_trace_j with a workspace)",
                    (long long)n_probes, n_dir, need, kNoAllocScratchBytes);
    float* work = nullptr;
    if (need > 0) RT_TRY(scratch_address(&work));
    return trace_j_impl(sc, p, d_dirs, d_weights, n_dir, d_probes, n_probes, d_J, d_psi, work,
                        work ? kNoAllocScratchBytes : 0, (hipStream_t)stream);
}

rt_status rt_trace_truncated(const rt_scene* sc, const rt_trace_params* p, float t_trunc, int32_t gen,
                             const uint8_t* d_fallback, const float* d_dirs, int32_t n_dir, const int32_t* d_probes,
                             int64_t n_probes, float* d_I_near, float* d_T_near, float* d_I_far, float* d_feat,
                             float* d_fstat, void* stream)
{
    g_err.clear();
    if (!sc || !p || !d_dirs || !d_I_near || !d_T_near || !d_feat || !d_fstat) return fail(RT_E_ARG, "null argument");
    if (gen && !d_I_far) return fail(RT_E_ARG, "generation mode needs d_I_far");
    if (!(t_trunc > 0.f)) return fail(RT_E_ARG, "t_trunc must be positive");
    if (sc->batch_begin < 0) return fail(RT_E_STATE, "rt_trace_truncated before rt_scene_build");
    if (p->mode != RT_TRACE_LEVEL0 && p->mode != RT_TRACE_VLM) return fail(RT_E_ARG, "bad trace mode");
    if (n_dir < 1) return fail(RT_E_ARG, "n_dir must be >= 1");
    if (p->grade_mode != RT_GRADE_BLOCK_ENTRY && p->grade_mode != RT_GRADE_PATH)
        return fail(RT_E_ARG, "bad grade_mode %d", (int)p->grade_mode);
    if (sc->g.nblocks >= (1ll << 24)) return fail(RT_E_UNSUPPORTED, "truncated march needs fewer than 2^24 blocks");
    const long long all = (long long)sc->n_active * sc->g.bvox;
    if (!d_probes && n_probes != all) return fail(RT_E_ARG, "all-probes trace needs n_probes = %lld", all);
    if (n_probes <= 0) return n_probes == 0 ? RT_OK : fail(RT_E_ARG, "n_probes must be >= 0");
    TraceLaunch t = make_trace(sc, p);
    t.dirs = d_dirs;
    t.n_dir = n_dir;
    t.probes = d_probes;
    t.n_probes = n_probes;
    t.trunc = 1;
    t.gen = gen ? 1 : 0;
    t.t_trunc = (double)t_trunc;
    t.fallback = gen ? nullptr : d_fallback;
    t.I_near = d_I_near;
    t.T_near = d_T_near;
    t.I_far = d_I_far;
    t.feat = (float4*)d_feat;
    t.fstat_out = (float4*)d_fstat;
    RT_HIP(launch_trace(t, (hipStream_t)stream));
    return RT_OK;
}

rt_status rt_scene_get_info(const rt_scene* sc, rt_scene_info* h)
{
    if (!sc || !h) return fail(RT_E_ARG, "null argument");
    h->n_blocks = sc->g.nblocks;
    h->n_active = sc->n_active;
    h->n_probes = (int64_t)sc->n_active * sc->g.bvox;
    h->cells_per_brick = sc->g.cells;
    h->storage_bytes = (int64_t)sc->bytes;
    h->batch_begin = sc->batch_begin;
    h->batch_end = sc->batch_end;
    h->n_state_words = sc->g.n_state_words;
    h->reserved_ = 0;
    return RT_OK;
}

rt_status rt_scene_active_blocks(const rt_scene* sc, int32_t* h, void* stream)
{
    if (!sc || !h) return fail(RT_E_ARG, "null argument");
    if (sc->n_active == 0) return RT_OK;
    return copy_back(h, sc->b.active_list, sizeof(int32_t) * (size_t)sc->n_active, (hipStream_t)stream);
}

rt_status rt_scene_levels(const rt_scene* sc, int8_t* h, void* stream)
{
    if (!sc || !h) return fail(RT_E_ARG, "null argument");
    if (sc->batch_begin < 0) return fail(RT_E_STATE, "no batch built");
    return copy_back(h, sc->b.levels, (size_t)sc->g.nblocks, (hipStream_t)stream);
}

rt_status rt_scene_states(const rt_scene* sc, uint64_t* h, void* stream)
{
    if (!sc || !h) return fail(RT_E_ARG, "null argument");
    if (sc->batch_begin < 0) return fail(RT_E_STATE, "no batch built");
    return copy_back(h, sc->b.states, sizeof(uint64_t) * (size_t)sc->g.n_state_words, (hipStream_t)stream);
}

rt_status rt_scene_cell_values(const rt_scene* sc, int32_t n, const int32_t* h_cells, float* h_out, void* stream)
{
    if (!sc || !h_cells || !h_out || n < 0) return fail(RT_E_ARG, "bad argument");
    if (sc->batch_begin < 0) return fail(RT_E_STATE, "no batch built");
    if (!sc->b.vals) return fail(RT_E_UNSUPPORTED, "cell values exist for static emission only");
    if (n == 0) return RT_OK;
    for (int i = 0; i < n; ++i) {
        const int32_t* c = h_cells + 4 * i;
        for (int a = 0; a < 3; ++a)
            if (c[a] < 0 || c[a] >= sc->g.n[a]) return fail(RT_E_ARG, "cell %d outside the grid", i);
        if (c[3] < 0 || c[3] >= sc->g.n_levels) return fail(RT_E_ARG, "cell %d level out of range", i);
    }
    int32_t* dc = nullptr;
    float* dout = nullptr;
    RT_HIP(hipMalloc(&dc, sizeof(int32_t) * 4 * (size_t)n));
    hipError_t e = hipMalloc(&dout, sizeof(float) * 2 * kLam * (size_t)n);
    if (e != hipSuccess) {
        (void)hipFree(dc);
        return fail(RT_E_HIP, "hipMalloc: %s", hipGetErrorString(e));
    }
    hipStream_t s = (hipStream_t)stream;
    e = hipMemcpyAsync(dc, h_cells, sizeof(int32_t) * 4 * (size_t)n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_read_cells(sc->g, sc->b, sc->storage, n, dc, dout, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h_out, dout, sizeof(float) * 2 * kLam * (size_t)n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(dc);
    (void)hipFree(dout);
    if (e != hipSuccess) return fail(RT_E_HIP, "cell values: %s", hipGetErrorString(e));
    return RT_OK;
}

rt_status rt_debug_visited(const rt_scene* sc, const rt_trace_params* p, int32_t probe_vox, const float* h_dir,
                           int32_t cap, int32_t* h_cells, double* h_t, int32_t* h_count, void* stream)
{
    if (!sc || !p || !h_dir || !h_cells || !h_t || !h_count || cap < 1) return fail(RT_E_ARG, "bad argument");
    if (sc->batch_begin < 0) return fail(RT_E_STATE, "no batch built");
    if (probe_vox < 0 || probe_vox >= sc->in.nvox) return fail(RT_E_ARG, "probe outside the grid");
    if (p->grade_mode != RT_GRADE_BLOCK_ENTRY && p->grade_mode != RT_GRADE_PATH)
        return fail(RT_E_ARG, "bad grade_mode %d", (int)p->grade_mode);
    hipStream_t s = (hipStream_t)stream;
    TraceLaunch t = make_trace(sc, p);
    int32_t* dc = nullptr;
    double* dt = nullptr;
    int32_t* dn = nullptr;
    hipError_t e = hipMalloc(&dc, sizeof(int32_t) * 4 * (size_t)cap);
    if (e == hipSuccess) e = hipMalloc(&dt, sizeof(double) * 2 * (size_t)cap);
    if (e == hipSuccess) e = hipMalloc(&dn, sizeof(int32_t));
    float w[3] = {h_dir[0], sc->g.dim > 1 ? h_dir[1] : 0.f, sc->g.dim > 2 ? h_dir[2] : 0.f};
    if (e == hipSuccess) e = launch_debug_visited(t, probe_vox, w[0], w[1], w[2], cap, dc, dt, dn, s);
    int32_t n = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&n, dn, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    int ncp = std::min(std::max(n, 0), cap);
    if (e == hipSuccess && ncp > 0)
        e = hipMemcpyAsync(h_cells, dc, sizeof(int32_t) * 4 * (size_t)ncp, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && ncp > 0) e = hipMemcpyAsync(h_t, dt, sizeof(double) * 2 * (size_t)ncp, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (dc) (void)hipFree(dc);
    if (dt) (void)hipFree(dt);
    if (dn) (void)hipFree(dn);
    if (e != hipSuccess) return fail(RT_E_HIP, "debug visited: %s", hipGetErrorString(e));
    *h_count = n;
    if (n < 0) return fail(RT_E_DEVICE, "step cap reached");
    if (n > cap) return fail(RT_E_ARG, "cap %d too small for %d cells", cap, n);
    return RT_OK;
}

rt_status rt_scene_device_error(const rt_scene* sc, rt_device_err* h, void* stream)
{
    if (!sc || !h) return fail(RT_E_ARG, "null argument");
    unsigned long long v[4];
    RT_TRY(copy_back(v, sc->b.err, sizeof(v), (hipStream_t)stream));
    h->step_cap_hits = v[0];
    h->first_ray = v[0] ? (long long)v[1] : -1;
    h->bad_probes = v[2];
    return RT_OK;
}

rt_status rt_scene_reset_device_error(rt_scene* sc, void* stream)
{
    if (!sc) return fail(RT_E_ARG, "null argument");
    unsigned long long err0[4] = {0ull, ~0ull, 0ull, 0ull};
    RT_HIP(hipMemcpyAsync(sc->b.err, err0, sizeof(err0), hipMemcpyHostToDevice, (hipStream_t)stream));
    RT_HIP(hipStreamSynchronize((hipStream_t)stream));
    return RT_OK;
}

void rt_scene_destroy(rt_scene* sc) { delete sc; }  // the device memory is the caller's workspace

}  // extern "C"

// ------------------------------------------------------------------ batching
struct rt_batch {
    std::vector<BatchJob> jobs;
    BatchJob* d_jobs = nullptr;
    unsigned* counter = nullptr;
    unsigned long long* err = nullptr;
    unsigned* claims = nullptr;
    unsigned total_tiles = 0;
    int wg_waves = 4, n_wgs = 0, tiles_per_pop = 1;
    std::vector<BatchSeg> segs;  // one persistent launch per dimension present
};

// The batch's workspace: the job table, the queue counters (one per launch),
// the error counters.
static bool carve_batch(size_t n_jobs, Carver& c, BatchJob** jobs, unsigned** counter, unsigned long long** err)
{
    return c.take(jobs, n_jobs) && c.take(counter, 64) && c.take(err, 4);
}

struct rt_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static int device_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
    return cus;
}

extern "C" {

rt_status rt_batch_workspace_bytes(int32_t n_jobs, size_t* h_bytes)
{
    g_err.clear();
    if (!h_bytes || n_jobs < 1) return fail(RT_E_ARG, "need at least one job");
    Carver c;
    BatchJob* j;
    unsigned* q;
    unsigned long long* e;
    carve_batch((size_t)n_jobs, c, &j, &q, &e);
    *h_bytes = c.used;
    return RT_OK;
}

rt_status rt_batch_create(const rt_batch_job* jobs, int32_t n_jobs, const rt_batch_params* p, void* d_ws,
                          size_t ws_bytes, void* stream, rt_batch** out)
{
    g_err.clear();
    if (!jobs || !out || n_jobs < 1) return fail(RT_E_ARG, "need at least one job");
    *out = nullptr;
    size_t need = 0;
    RT_TRY(rt_batch_workspace_bytes(n_jobs, &need));
    RT_TRY(check_ws(d_ws, ws_bytes, need, "rt_batch_create"));
    rt_batch_params bp = p ? *p : rt_batch_params{0, 0, 0, 0, nullptr, 0, 0};
    int wg_waves = bp.wg_waves ? bp.wg_waves : 4;
    int wgs_per_cu = bp.wgs_per_cu ? bp.wgs_per_cu : 2;
    int tpp = bp.tiles_per_pop ? bp.tiles_per_pop : 1;
    if (wg_waves != 1 && wg_waves != 2 && wg_waves != 4 && wg_waves != 8) return fail(RT_E_ARG, "wg_waves must be 1, 2, 4 or 8");
    if (wgs_per_cu < 1 || wgs_per_cu > 16) return fail(RT_E_ARG, "wgs_per_cu must be in [1, 16]");
    if (tpp < 1 || tpp > 64) return fail(RT_E_ARG, "tiles_per_pop must be in [1, 64]");
    if (bp.tile_shape != RT_TILE_ROWS && bp.tile_shape != RT_TILE_CUBES)
        return fail(RT_E_ARG, "tile_shape must be RT_TILE_ROWS or RT_TILE_CUBES");
    std::vector<BatchJob> bj((size_t)n_jobs);
    std::vector<double> cost((size_t)n_jobs);
    for (int j = 0; j < n_jobs; ++j) {
        const rt_batch_job& J = jobs[j];
        const rt_scene* sc = J.scene;
        if (!sc || !J.d_dirs || !J.d_I) return fail(RT_E_ARG, "job %d: null scene, directions or output", j);
        if (sc->batch_begin < 0) return fail(RT_E_STATE, "job %d: scene has no built batch", j);
        if (sc->desc.emission != RT_EMIS_STATIC)
            return fail(RT_E_UNSUPPORTED, "job %d: batched trace supports static emission (not prefiltered)", j);
        if (J.n_dir < 1) return fail(RT_E_ARG, "job %d: n_dir must be >= 1", j);
        const rt_trace_params& tp = J.params;
        if (tp.mode != RT_TRACE_LEVEL0 && tp.mode != RT_TRACE_VLM) return fail(RT_E_ARG, "job %d: bad mode", j);
        if (tp.grade_mode != RT_GRADE_BLOCK_ENTRY && tp.grade_mode != RT_GRADE_PATH)
            return fail(RT_E_ARG, "job %d: bad grade_mode", j);
        TraceLaunch t = make_trace(sc, &tp);
        BatchJob& b = bj[(size_t)j];
        std::memset(&b, 0, sizeof(b));
        b.g = t.g;
        b.states = t.states;
        b.slot = t.slot;
        b.vals = t.vals;
        b.active_list = t.active_list;
        b.dirs = J.d_dirs;
        b.I = J.d_I;
        b.n_probes = (long long)sc->n_active * sc->g.bvox;
        b.tiles = (int)((b.n_probes + 63) / 64);
        b.n_dir = J.n_dir;
        b.nl = sc->batch_end - sc->batch_begin;
        b.mode = t.mode;
        b.max_level = t.max_level;
        b.graded = t.graded;
        b.step_cap = t.step_cap;
        b.storage = t.storage;
        b.tile_shape = bp.tile_shape;
        b.I0 = t.I0;
        b.ds0 = t.ds0;
        for (int m = 0; m < kMaxLevels; ++m) b.level_dist[m] = t.level_dist[m];
        double diam = 0;
        for (int a = 0; a < sc->g.dim; ++a) diam += sc->g.n[a];
        cost[(size_t)j] = (double)J.n_dir * (double)b.n_probes * diam;
    }
    std::vector<int> order((size_t)n_jobs);
    for (int j = 0; j < n_jobs; ++j) order[(size_t)j] = j;
    // 2D jobs first, then 3D (one launch each); within a dimension costliest first unless order = 1
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (bj[(size_t)a].g.dim != bj[(size_t)b].g.dim) return bj[(size_t)a].g.dim < bj[(size_t)b].g.dim;
        return bp.order == 0 && cost[(size_t)a] > cost[(size_t)b];
    });
    rt_batch* bt = new (std::nothrow) rt_batch();
    if (!bt) return fail(RT_E_ARG, "out of host memory");
    unsigned long long tile = 0;
    for (int j : order) {
        BatchJob b = bj[(size_t)j];
        b.tile0 = (unsigned)tile;
        tile += (unsigned long long)b.tiles * b.n_dir;
        bt->jobs.push_back(b);
    }
    if (tile >= (1ull << 31)) {
        delete bt;
        return fail(RT_E_ARG, "too many tiles in one batch (%llu)", tile);
    }
    bt->total_tiles = (unsigned)tile;
    for (int j = 0; j < (int)bt->jobs.size(); ++j) {
        const BatchJob& b = bt->jobs[(size_t)j];
        if (bt->segs.empty() || bt->segs.back().dim != b.g.dim)
            bt->segs.push_back(BatchSeg{b.g.dim, b.storage, j, j, b.tile0, b.tile0});
        BatchSeg& g = bt->segs.back();
        if (g.storage != b.storage) g.storage = -1;
        g.j1 = j + 1;
        g.tile_end = b.tile0 + (unsigned)b.tiles * (unsigned)b.n_dir;
    }
    bt->wg_waves = wg_waves;
    bt->tiles_per_pop = tpp;
    bt->n_wgs = device_cus() * wgs_per_cu;
    bt->claims = bp.d_claims;
    hipStream_t s = (hipStream_t)stream;
    Carver c;
    c.base = (char*)d_ws;
    c.cap = ws_bytes;
    carve_batch(bt->jobs.size(), c, &bt->d_jobs, &bt->counter, &bt->err);
    unsigned long long err0[2] = {0ull, ~0ull};
    hipError_t e = hipMemcpyAsync(bt->d_jobs, bt->jobs.data(), sizeof(BatchJob) * bt->jobs.size(),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(bt->err, err0, sizeof(err0), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        delete bt;
        return fail(RT_E_HIP, "batch setup: %s", hipGetErrorString(e));
    }
    *out = bt;
    return RT_OK;
}

rt_status rt_batch_run(const rt_batch* bt, void* stream)
{
    if (!bt) return fail(RT_E_ARG, "null batch");
    RT_HIP(launch_batched(bt->d_jobs, bt->segs.data(), (int)bt->segs.size(), bt->wg_waves, bt->n_wgs,
                          bt->tiles_per_pop, bt->counter, bt->claims, bt->err, (hipStream_t)stream));
    return RT_OK;
}

rt_status rt_batch_tiles(const rt_batch* bt, int64_t* h)
{
    if (!bt || !h) return fail(RT_E_ARG, "null argument");
    *h = bt->total_tiles;
    return RT_OK;
}

rt_status rt_batch_device_error(const rt_batch* bt, rt_device_err* h, void* stream)
{
    if (!bt || !h) return fail(RT_E_ARG, "null argument");
    unsigned long long v[2];
    RT_TRY(copy_back(v, bt->err, sizeof(v), (hipStream_t)stream));
    h->step_cap_hits = v[0];
    h->first_ray = v[0] ? (long long)v[1] : -1;
    h->bad_probes = 0;  // batched jobs trace every probe of their scenes
    return RT_OK;
}

void rt_batch_destroy(rt_batch* bt) { delete bt; }  // the device memory is the caller's workspace

rt_status rt_batch_autotune(const rt_batch_job* jobs, int32_t n_jobs, int32_t reps, void* d_ws, size_t ws_bytes,
                            void* stream, rt_batch_params* best, float* best_ms)
{
    if (!jobs || !best || !best_ms || reps < 1) return fail(RT_E_ARG, "bad argument");
    hipStream_t s = (hipStream_t)stream;
    const int waves[] = {2, 4, 8};
    const int per_cu[] = {1, 2, 4};
    const int pops[] = {1, 4};
    const int shapes[] = {RT_TILE_ROWS, RT_TILE_CUBES};
    hipEvent_t e0, e1;
    RT_HIP(hipEventCreate(&e0));
    RT_HIP(hipEventCreate(&e1));
    float best_t = 3.0e38f;
    rt_batch_params bestp = {4, 2, 1, 0, nullptr, RT_TILE_ROWS, 0};
    rt_status st = RT_OK;
    for (int w : waves)
        for (int c : per_cu)
            for (int q : pops)
                for (int sh : shapes) {
                    rt_batch_params p = {w, c, q, 0, nullptr, sh, 0};
                    rt_batch* bt = nullptr;
                    if ((st = rt_batch_create(jobs, n_jobs, &p, d_ws, ws_bytes, stream, &bt)) != RT_OK) goto done;
                    if ((st = rt_batch_run(bt, stream)) != RT_OK) {
                        rt_batch_destroy(bt);
                        goto done;
                    }
                    {
                        hipError_t e = hipEventRecord(e0, s);
                        for (int r = 0; r < reps && e == hipSuccess; ++r) {
                            if (rt_batch_run(bt, stream) != RT_OK) e = hipErrorUnknown;
                        }
                        if (e == hipSuccess) e = hipEventRecord(e1, s);
                        if (e == hipSuccess) e = hipEventSynchronize(e1);
                        float ms = 0.f;
                        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                        rt_batch_destroy(bt);
                        if (e != hipSuccess) {
                            st = fail(RT_E_HIP, "autotune timing: %s", hipGetErrorString(e));
                            goto done;
                        }
                        ms /= (float)reps;
                        if (ms < best_t) {
                            best_t = ms;
                            bestp = p;
                        }
                    }
                }
done:
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != RT_OK) return st;
    *best = bestp;
    *best_ms = best_t;
    return RT_OK;
}

rt_status rt_graph_begin(void* stream)
{
    RT_HIP(hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeRelaxed));
    return RT_OK;
}

rt_status rt_graph_end(void* stream, rt_graph** out)
{
    if (!out) return fail(RT_E_ARG, "null argument");
    rt_graph* g = new (std::nothrow) rt_graph();
    if (!g) return fail(RT_E_ARG, "out of host memory");
    hipError_t e = hipStreamEndCapture((hipStream_t)stream, &g->graph);
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        if (g->graph) (void)hipGraphDestroy(g->graph);
        delete g;
        return fail(RT_E_HIP, "graph capture: %s", hipGetErrorString(e));
    }
    *out = g;
    return RT_OK;
}

rt_status rt_graph_launch(const rt_graph* g, void* stream)
{
    if (!g) return fail(RT_E_ARG, "null graph");
    RT_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return RT_OK;
}

void rt_graph_destroy(rt_graph* g)
{
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

}  // extern "C"
