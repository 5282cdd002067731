// Formal-solution march: hierarchical DDA over the adapted brick grid
// (Sect. 2.3, Alg. 1) with the piecewise-constant update of Eq. RteIntegral
// applied front-to-back for a batch of 8 wavelengths held in registers.
//
// Traversal decisions are exact.  The ray is x(t) = p - t w with p a voxel
// centre, so 2 |p_a - k| is an odd integer for every integer plane k.  The
// crossing time of axis a is d_a / |w_a| (d_a = |p_a - k_a|); "axis a before
// axis b" is decided by comparing d_a |w_b| with d_b |w_a| in FP64, where both
// products are exact (14-bit integer x 24-bit mantissa).  t itself is only
// used for segment lengths.  Ties (the ray through a cell corner) step every
// tied axis at once and emit no zero-length segment; at a change of MIP level
// the non-crossing axes are re-located with the same exact predicate, and a
// position exactly on a plane belongs to the cell the ray moves into.  This
// replaces the two floating-point nudges of Sect. 2.3.1: t is recomputed
// from integer plane indices every step, so it never drifts.
//
// Block states (3 bits, 21 per 64-bit word, Sect. 2.3.1) are staged in LDS
// for the whole grid; the storage slot of a block is read once per block
// visit and kept in a register (the "cached block index" of Sect. 2.3.1).
#include "common.h"
#include "profile.h"

namespace rt {

// Scenes have at most 8192 voxels per axis (checked at creation): block
// coordinates stay below 2^10 and block indices below 2^30, so block
// arithmetic is exact in 32 bits and its products in 24 bits.
__device__ __forceinline__ int block_level(const uint64_t* sts, long long b, int mode, int maxl)
{
    const unsigned bb = (unsigned)b;
    const unsigned w = bb / (unsigned)kStatesPerWord;
    const unsigned sh = 3u * (bb - w * (unsigned)kStatesPerWord);
    int s = (int)((sts[w] >> sh) & 7ull);
    if (s == 0) return -1;
    int l = mode == RT_TRACE_LEVEL0 ? 0 : s - 1;
    return l < maxl ? l : maxl;
}

// Block index of an in-grid cell.
template <int D>
__device__ __forceinline__ long long block_of(const Geo& g, const int* c)
{
    const unsigned l = (unsigned)g.log2B;
    unsigned r = (unsigned)c[1] >> l;
    if (D > 2) r += __umul24((unsigned)g.nb[1], (unsigned)c[2] >> l);
    return (long long)(((unsigned)c[0] >> l) + __umul24((unsigned)g.nb[0], r));
}

// Fine cell (multiple of nvs inside [c0, c0 + vs)) containing x_a(t*) with
// t* = d2s / (2 |w_s|); on a plane, the cell the ray moves into.
__device__ __noinline__ int fine_cell(int p2a, double wa, double aws, double d2s, int c0, int vs, int nvs, int sta)
{
    const double rhs = d2s * wa;  // exact
    double xa = 0.5 * (double)p2a - (d2s * 0.5 / aws) * wa;
    int j = ((int)floor(xa)) & ~(nvs - 1);
    if (j < c0) j = c0;
    if (j > c0 + vs - nvs) j = c0 + vs - nvs;
    // x_a(t*) >= j  <=>  (p2a - 2 j) |w_s| >= d2s w_a   (exact products)
    while (j + nvs <= c0 + vs - nvs && (double)(p2a - 2 * (j + nvs)) * aws >= rhs) j += nvs;
    while (j > c0 && !((double)(p2a - 2 * j) * aws >= rhs)) j -= nvs;
    if (sta < 0 && j > c0 && (double)(p2a - 2 * j) * aws == rhs) j -= nvs;
    return j;
}

struct Counters {
    unsigned segs, empty, lvlchg;
};

// The level_dist table of a traversal, held in registers (the traversal reads it at
// every block change; a memory read there would wait for every load in flight).
struct LevelDist {
    float v[kMaxLevels];
    __device__ __forceinline__ explicit LevelDist(const float* ld)
    {
#pragma unroll
        for (int m = 0; m < kMaxLevels; ++m) v[m] = ld[m];
    }
    // v[k] for 0 <= k < nlev, else +inf (a select chain: no indexed register access)
    __device__ __forceinline__ float at(int k, int nlev) const
    {
        float r = INFINITY;
#pragma unroll
        for (int m = 0; m < kMaxLevels; ++m) r = (k == m && m < nlev) ? v[m] : r;
        return r;
    }
};

// Distance-graded cap at a block entered at t = d2 / (2 |w_s|): the largest m
// with level_dist[1..m] <= t, decided exactly as d2/2 >= level_dist[m] |w_s|.
__device__ __forceinline__ int graded_cap(const LevelDist& ld, int nlev, double d2, double aws)
{
    int cap = 0;
    bool go = true;
#pragma unroll
    for (int m = 1; m < kMaxLevels; ++m) {
        go = go && m < nlev && d2 * 0.5 >= (double)ld.v[m] * aws;
        cap = go ? m : cap;
    }
    return cap;
}

// Path-graded cap at path length t: the largest m with ld[1..m] <= t.
__device__ __forceinline__ int path_cap(const LevelDist& ld, int nlev, double t)
{
    int cap = 0;
    bool go = true;
#pragma unroll
    for (int m = 1; m < kMaxLevels; ++m) {
        go = go && m < nlev && (double)ld.v[m] <= t;
        cap = go ? m : cap;
    }
    return cap;
}

// MIP-0 coordinate on axis a (step sign st, |w_a| = aw) of the point x(t) of the
// ray from the voxel centre pv, in the cell the ray moves into when x(t) lies on
// a face.  Plane j >= 1 lies at doubled distance 2j - 1 from the centre and is
// crossed by t iff 2j - 1 <= 2 t |w_a|; an fma rounds once, so its sign is that
// of the exact difference, and floor(t |w_a| + 1/2) is at most one too high.
// Returns false when the point is past the grid on this axis.
__device__ __forceinline__ bool mip0_coord(int pva, int st, double aw, double t, int na, int& ca)
{
    if (st == 0) {
        ca = pva;
        return true;
    }
    const double e = floor(fma(t, aw, 0.5));
    if (!(e <= (double)na + 2.0)) return false;
    int nj = (int)e;
    if (nj > 0 && fma(-2.0 * t, aw, (double)(2 * nj - 1)) > 0.0) --nj;
    ca = pva + st * nj;
    return (unsigned)ca < (unsigned)na;
}

// Traverses the adapted grid from voxel centre pv upwind along -w.  Calls
// vis.seg(c, level, block, t0, t1) for every non-empty cell in order of
// increasing t.  Returns 0 when the ray left the grid, 1 at the step cap and
// 2 when the visitor asked to stop (truncated march).
// graded = 1: a block's level is also capped by the path length at which the
// ray enters it (ld: level_dist); graded = 2: capped by the path length of each
// point, so the cap rises at t = ld[m] inside a cell, where the cell is split
// and the ray re-located at the new level.
// With Iv, only the path interval [t_lo, t_hi] is traversed (a radiance
// interval): the start cell is the one holding x(t_lo) (on a plane, the one the
// ray moves into), the last segment ends at t_hi, and a plane crossed exactly
// at t_hi belongs to this interval.  Returns 3 when t_hi was reached inside the
// grid and 4 when the ray had left the grid by t_lo (no segment).
// LdDemand: ldp is the workgroup's LDS copy of level_dist, read where it is needed (start, cap rises,
// block changes) rather than held in registers for the whole traversal.
template <int D, bool Iv = false, bool LdDemand = false, class Vis>
__device__ __forceinline__ int hdda(const Geo& g, const uint64_t* sts, int mode, int maxl, int graded,
                                    const float* ldp, const int* pv, const float* wf, int step_cap, Vis& vis,
                                    Counters& cnt, double t_lo = 0.0, double t_hi = 0.0)
{
    const float kZeroLd[kMaxLevels] = {};
    const LevelDist ldr(LdDemand ? kZeroLd : ldp);
    auto LD = [&]() -> LevelDist {
        if constexpr (LdDemand) return LevelDist(ldp);
        else return ldr;
    };
    // Per axis: the doubled centre p2 = 2 p (odd), the step sign st, the cell c at the current
    // level (size vs); the next plane is k = c + (st > 0 ? vs : 0), and dd = |p2 - 2 k| (twice the
    // distance to it) is kept exactly.  |w_a| is kept in FP32 (exact when widened to FP64).
    int p2[3], st[3], c[3];
    float af[3];
    double iw[3], dd[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        p2[a] = 1;
        st[a] = 0;
        c[a] = 0;
        af[a] = 0.f;
        iw[a] = 0.0;
        dd[a] = 1.0;
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
        p2[a] = 2 * pv[a] + 1;
        af[a] = fabsf(wf[a]);
        iw[a] = af[a] > 0.f ? 0.5 / (double)af[a] : 0.0;  // half the reciprocal: t = dd iw
        st[a] = wf[a] > 0.f ? -1 : (wf[a] < 0.f ? 1 : 0);
    }
    int c0[3] = {pv[0], pv[1], pv[2]};
    double t = 0.0;
    if constexpr (Iv) {
        // MIP-0 cell at t_lo
        bool in = true;
#pragma unroll
        for (int a = 0; a < D; ++a) in = mip0_coord(pv[a], st[a], (double)af[a], t_lo, g.n[a], c0[a]) && in;
        if (!in) return 4;
        t = t_lo;
    }
    // path-graded cap and the path length at which it next rises
    int capp = 127;
    float tb = INFINITY;  // a level_dist value (FP32, exact in FP64)
    if (graded == 2) {
        capp = path_cap(LD(), g.n_levels, t);
        tb = LD().at(capp + 1, g.n_levels);
    }
    long long blk = block_of<D>(g, c0);
    int cap0 = maxl;
    if (graded == 2) {
        cap0 = capp < maxl ? capp : maxl;
    } else if (graded) {
        int cg = 0;
        if constexpr (Iv) {
            // the start block was entered when the ray crossed the last of its entry faces
            // (time dn / (2 an); 0 in the probe's own block)
            double dn = 0.0, an = 1.0;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const int ba = c0[a] >> g.log2B;
                if (st[a] == 0 || ba == (pv[a] >> g.log2B)) continue;
                const int kf = (st[a] > 0 ? ba : ba + 1) << g.log2B;
                const double df = (double)abs(p2[a] - 2 * kf);
                if (df * an > dn * (double)af[a]) {
                    dn = df;
                    an = (double)af[a];
                }
            }
            cg = graded_cap(LD(), g.n_levels, dn, an);
        } else {
            cg = path_cap(LD(), g.n_levels, 0.0);
        }
        cap0 = cg < maxl ? cg : maxl;
    }
    // path grading: lraw is the block's level before the path cap; the cap binds only where
    // lraw > capp, and only there can its rise at tb change the level
    int lraw = graded == 2 ? block_level(sts, blk, mode, maxl) : 0;
    int lvl = graded == 2 ? (lraw < capp ? lraw : capp) : block_level(sts, blk, mode, cap0);
    int vs = lvl < 0 ? g.B : (1 << lvl);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        c[a] = c0[a] & ~(vs - 1);
        dd[a] = (double)abs(p2[a] - 2 * (c[a] + (st[a] > 0 ? vs : 0)));
    }
    for (int step = 0; step < step_cap; ++step) {
        int s0;
        unsigned tie;
        double tn;
        if constexpr (D == 2) {
            // axis a crosses first iff dd_a |w_b| < dd_b |w_a|; an axis with w_a = 0 has a zero
            // product on the right and never wins, so no special case is needed
            const double lhs = dd[0] * (double)af[1], rhs = dd[1] * (double)af[0];
            const bool x0 = lhs <= rhs, x1 = rhs <= lhs;
            tie = (x0 ? 1u : 0u) | (x1 ? 2u : 0u);
            s0 = x0 ? 0 : 1;
            tn = x0 ? dd[0] * iw[0] : dd[1] * iw[1];
        } else {
            s0 = -1;
            tie = 0;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                if (st[a] == 0) continue;
                if (s0 < 0) {
                    s0 = a;
                    tie = 1u << a;
                } else {
                    double lhs = dd[a] * (double)af[s0];
                    double rhs = dd[s0] * (double)af[a];
                    if (lhs < rhs) {
                        s0 = a;
                        tie = 1u << a;
                    } else if (lhs == rhs) {
                        tie |= 1u << a;
                    }
                }
            }
            tn = dd[s0] * iw[s0];
        }
        const double d2s0 = dd[s0];
        const double aws = (double)af[s0];
        // the segment ends at the next crossing, unless the path-graded cap rises first (ev 1:
        // the cell is split at tb) or the interval ends first (ev 2); both tests are exact in sign
        int ev = 0;
        double te = tn;
        if (graded == 2 && lraw > capp && (!Iv || (double)tb < t_hi) && fma(-2.0 * (double)tb, aws, d2s0) > 0.0) {
            ev = 1;
            te = (double)tb;
        } else if (Iv && fma(-2.0 * t_hi, aws, d2s0) > 0.0) {
            ev = 2;
            te = t_hi;
        }
        if (lvl >= 0) {
            if (ev == 0 || te > t) {
                if (vis.seg(c, lvl, blk, t, te)) return 2;
                ++cnt.segs;
            }
        } else {
            ++cnt.empty;
        }
        if (ev != 0) {
            if (ev == 2) return 3;
            // the cap rises at t = tb and binds here, so the level rises: re-locate from x(t),
            // which lies in the current cell
            t = te;
            capp = path_cap(LD(), g.n_levels, t);
            tb = LD().at(capp + 1, g.n_levels);
            const int nl = lraw < capp ? lraw : capp;
            ++cnt.lvlchg;
            const int nvs = 1 << nl;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                int ca = c[a];
                mip0_coord(pv[a], st[a], (double)af[a], t, g.n[a], ca);
                c[a] = ca & ~(nvs - 1);
                dd[a] = (double)abs(p2[a] - 2 * (c[a] + (st[a] > 0 ? nvs : 0)));
            }
            lvl = nl;
            vs = nvs;
            continue;
        }
        t = tn;
        // advance the crossing axes (branch-free: the other axes add 0 and keep their block)
        bool out = false, bchg = false;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const bool sa = (tie >> a) & 1u;
            const int sv = sa ? st[a] * vs : 0;
            const int cold = c[a];
            c[a] += sv;
            dd[a] += sa ? (double)(2 * vs) : 0.0;
            out = out || (unsigned)c[a] >= (unsigned)g.n[a];
            bchg = bchg || (c[a] >> g.log2B) != (cold >> g.log2B);
        }
        if (out) return 0;
        if (bchg) {
            blk = block_of<D>(g, c);
            int nl;
            if (graded == 2) {
                // the path cap at the crossing (exact), and the new block's level under it
                capp = graded_cap(LD(), g.n_levels, d2s0, aws);
                tb = LD().at(capp + 1, g.n_levels);
                lraw = block_level(sts, blk, mode, maxl);
                nl = lraw < capp ? lraw : capp;
            } else {
                int capb = maxl;
                if (graded) {
                    int cg = graded_cap(LD(), g.n_levels, d2s0, aws);
                    capb = cg < maxl ? cg : maxl;
                }
                nl = block_level(sts, blk, mode, capb);
            }
            if (nl != lvl) {
                ++cnt.lvlchg;
                int nvs = nl < 0 ? g.B : (1 << nl);
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    // a crossing axis re-locates from the voxel next to the plane just crossed
                    if ((tie >> a) & 1u) c[a] = (st[a] > 0 ? c[a] : c[a] + vs - 1) & ~(nvs - 1);
                    else if (st[a] == 0) c[a] = pv[a] & ~(nvs - 1);
                    else if (nvs >= vs) c[a] &= ~(nvs - 1);
                    else c[a] = fine_cell(p2[a], (double)wf[a], aws, d2s0, c[a], vs, nvs, st[a]);
                    dd[a] = (double)abs(p2[a] - 2 * (c[a] + (st[a] > 0 ? nvs : 0)));
                }
                lvl = nl;
                vs = nvs;
            }
        }
    }
    return 1;
}

// ------------------------------------------------------------ RTE update
// One segment, one wavelength, front to back:
//   I += T eta dt g(tau),  T *= exp(-tau),  g(tau) = (1 - exp(-tau)) / tau,
// which is S (1 - exp(-tau)) with S = eta/chi and stays finite at chi = 0.
// The exponent is taken in base 2, a = chi dt log2(e) (exp(-tau) = 2^-a), and
// h = dt g(tau) is (1 - 2^-a) / chi above tau = 1/32 (cancellation < 2e-6
// relative) and the series dt (1 - tau/2 + tau^2/6) = dt + q1 a + q2 a^2 below
// (truncation < tau^3/24 < 1.3e-6 relative).  dt, dt log2(e), q1 = -dt ln2/2
// and q2 = dt ln2^2/6 are per-segment constants shared by the wavelength batch.
struct SegK {
    float dt, dtl, q1, q2;
    __device__ __forceinline__ explicit SegK(float d)
        : dt(d), dtl(d * 1.4426950408889634f), q1(d * -0.34657359027997264f), q2(d * 0.08007550231970024f)
    {
    }
};

// returns the segment's transmission exp(-tau)
__device__ __forceinline__ float rte_step(float& I, float& Tr, float eta, float chi, const SegK& k)
{
    const float a = chi * k.dtl;
    const float e = __builtin_amdgcn_exp2f(-a);
    const float hs = fmaf(a, fmaf(a, k.q2, k.q1), k.dt);
    const float r = __builtin_amdgcn_rcpf(chi);
    const float hd = fmaf(-e, r, r);  // (1 - e) / chi in one rounding
    const float h = a < 0.045084220027780106f ? hs : hd;  // tau < 1/32
    I = fmaf(Tr * eta, h, I);
    Tr *= e;
    return e;
}

// A node record as loaded (kLam (eta, chi) pairs: 64 B in FP32, 32 B in BF16 / FP16), decoded to
// FP32 separately so a pipelined visitor can keep the raw words in flight.
template <typename T>
struct RawRec {
    uint4 q[kLam * 2 * sizeof(T) / 16];
};

template <typename T>
__device__ __forceinline__ RawRec<T> fetch_rec(const T* r)
{
    RawRec<T> o;
    const uint4* r4 = (const uint4*)r;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(o.q) / sizeof(uint4)); ++i) o.q[i] = r4[i];
    return o;
}

template <typename T>
__device__ __forceinline__ void decode_rec(const RawRec<T>& raw, float* e, float* c);

template <>
__device__ __forceinline__ void decode_rec<float>(const RawRec<float>& raw, float* e, float* c)
{
#pragma unroll
    for (int q = 0; q < kLam / 2; ++q) {
        const uint4 v = raw.q[q];
        e[2 * q] = __uint_as_float(v.x);
        c[2 * q] = __uint_as_float(v.y);
        e[2 * q + 1] = __uint_as_float(v.z);
        c[2 * q + 1] = __uint_as_float(v.w);
    }
}

__device__ __forceinline__ float bf16_lo(unsigned u) { return __uint_as_float(u << 16); }
__device__ __forceinline__ float bf16_hi(unsigned u) { return __uint_as_float(u & 0xffff0000u); }

template <>
__device__ __forceinline__ void decode_rec<__hip_bfloat16>(const RawRec<__hip_bfloat16>& raw, float* e, float* c)
{
#pragma unroll
    for (int q = 0; q < kLam / 4; ++q) {
        const uint4 v = raw.q[q];
        const unsigned u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            e[4 * q + j] = bf16_lo(u[j]);
            c[4 * q + j] = bf16_hi(u[j]);
        }
    }
}

template <>
__device__ __forceinline__ void decode_rec<__half>(const RawRec<__half>& raw, float* e, float* c)
{
#pragma unroll
    for (int q = 0; q < kLam / 4; ++q) {
        const uint4 v = raw.q[q];
        unsigned u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            __half2 h = *reinterpret_cast<__half2*>(&u[j]);
            float2 f = __half22float2(h);
            e[4 * q + j] = f.x;
            c[4 * q + j] = f.y;
        }
    }
}

template <typename T>
__device__ __forceinline__ void load_rec(const T* r, float* e, float* c)
{
    decode_rec<T>(fetch_rec<T>(r), e, c);
}

// First cell of level lvl inside a block record, unpacked from the launch's
// 11-bit level offsets (a block holds at most 585 cells): a per-lane indexed
// load here would sit in front of every cell fetch.
__device__ __forceinline__ int level_offset(const Geo& g, int lvl)
{
    return (int)((g.lvl_pack >> (11 * lvl)) & 2047ull);
}

// Storage slot of block blk: from the trace workgroup's LDS copy of the slot
// table (placed after the state words) on small grids, else from global memory.
__device__ __forceinline__ long long block_slot(const Geo& g, const int32_t* slot, int lds, long long blk)
{
    // Each branch completes its own read (the empty asm takes the value as an operand), so the LDS
    // branch never waits on vector-memory loads in flight (the node records a pipelined visitor has
    // issued); the explicit LDS pointer keeps the two reads from merging into one generic read.
    int32_t v;
    if (lds) {
        extern __shared__ uint64_t lds_words[];
        typedef __attribute__((address_space(3))) const int32_t LdsI32;
        v = ((const LdsI32*)(lds_words + g.n_state_words))[blk];
        asm volatile("; slot from LDS" : "+v"(v));
    } else {
        v = slot[blk];
        asm volatile("; slot from global memory" : "+v"(v));
    }
    return v;
}

// LDS copy of the launch's level_dist table, after the state words and (on small grids) the slot table.
__device__ __forceinline__ float* lds_level_dist(const TraceLaunch& t, uint64_t* sts)
{
    return (float*)((int32_t*)(sts + t.g.n_state_words) + (t.slot_lds ? t.g.nblocks : 0));
}

// Copies the block-state words, on small grids the slot table, and the level_dist table to LDS.
__device__ __forceinline__ void stage_blocks(const TraceLaunch& t, uint64_t* sts)
{
    for (int i = threadIdx.x; i < t.g.n_state_words; i += blockDim.x) sts[i] = t.states[i];
    if (t.slot_lds) {
        int32_t* ls = (int32_t*)(sts + t.g.n_state_words);
        for (long long i = threadIdx.x; i < t.g.nblocks; i += blockDim.x) ls[i] = t.slot[i];
    }
    if (threadIdx.x < kMaxLevels) lds_level_dist(t, sts)[threadIdx.x] = t.level_dist[threadIdx.x];
    __syncthreads();
}

__device__ __forceinline__ int local_index(const Geo& g, const int* c, int lvl, int D)
{
    int sl = g.log2B - lvl;
    int lx = (c[0] & (g.B - 1)) >> lvl, ly = (c[1] & (g.B - 1)) >> lvl;
    int li = lx + (ly << sl);
    if (D > 2) li += ((c[2] & (g.B - 1)) >> lvl) << (2 * sl);
    return li;
}

// Four consecutive values of a record, decoded to FP32 (index i counts groups of 4).
template <typename T>
__device__ __forceinline__ float4 load4(const T* r, int i);

template <>
__device__ __forceinline__ float4 load4<float>(const float* r, int i)
{
    return ((const float4*)r)[i];
}

template <>
__device__ __forceinline__ float4 load4<__hip_bfloat16>(const __hip_bfloat16* r, int i)
{
    const uint2 v = ((const uint2*)r)[i];
    return make_float4(bf16_lo(v.x), bf16_hi(v.x), bf16_lo(v.y), bf16_hi(v.y));
}

template <>
__device__ __forceinline__ float4 load4<__half>(const __half* r, int i)
{
    uint2 v = ((const uint2*)r)[i];
    const float2 a = __half22float2(*reinterpret_cast<__half2*>(&v.x));
    const float2 b = __half22float2(*reinterpret_cast<__half2*>(&v.y));
    return make_float4(a.x, a.y, b.x, b.y);
}

// --------------------------------------------------------- accumulators
// Plain: the whole ray, front to back.
struct AccPlain {
    static constexpr bool kTrunc = false;
    static constexpr bool kJ = false;
    static constexpr bool kIv = false;
    float I[kLam], Tr[kLam];
    __device__ void init(const TraceLaunch*)
    {
#pragma unroll
        for (int l = 0; l < kLam; ++l) {
            I[l] = 0.f;
            Tr[l] = 1.f;
        }
    }
    __device__ __forceinline__ bool add(const float* e, const float* x, const int*, int, long long, double t0,
                                        double t1, float dsf)
    {
        add_dt(e, x, (float)(t1 - t0) * dsf);
        return false;
    }
    // the same update for a segment of length dt (in units of ds0 already applied)
    __device__ __forceinline__ void add_dt(const float* e, const float* x, float dt)
    {
        const SegK k(dt);
#pragma unroll
        for (int l = 0; l < kLam; ++l) rte_step(I[l], Tr[l], e[l], x[l], k);
    }
};

// Radiance interval [t_lo, t_hi]: the plain accumulator over the interval's
// segments; the caller also receives the interval's transmittance.
struct AccIv : AccPlain {
    static constexpr bool kIv = true;
};

// Truncated: the near field t < t_trunc and the far field t >= t_trunc are
// accumulated separately (the cell that straddles t_trunc is split there,
// exactly, since eta and chi are constant in it).  Generation mode keeps
// marching to record the far field; inference mode stops at t_trunc, unless
// the block reached there is flagged in the fallback map, in which case the
// ray continues as a full march.  t* = max(t_trunc, entry of the first
// non-empty cell beyond it): the far field from t* equals the one from t_trunc.
template <bool Gen>
struct AccTrunc {
    static constexpr bool kTrunc = true;
    static constexpr bool kJ = false;
    static constexpr bool kIv = false;
    static constexpr bool kGen = Gen;  // generation mode: also accumulate the far field
    float In[kLam], Tn[kLam];
    float If[Gen ? kLam : 1], Tf[Gen ? kLam : 1];
    double tt;
    const uint8_t* fallback;  // inference only
    int reached, fb, tlvl;
    int tc[3];
    long long tblk;
    double tstar;
    __device__ void init(const TraceLaunch* t)
    {
#pragma unroll
        for (int l = 0; l < kLam; ++l) {
            In[l] = 0.f;
            Tn[l] = 1.f;
        }
        if constexpr (Gen) {
#pragma unroll
            for (int l = 0; l < kLam; ++l) {
                If[l] = 0.f;
                Tf[l] = 1.f;
            }
        }
        tt = t->t_trunc;
        fallback = Gen ? nullptr : t->fallback;
        reached = fb = 0;
        tlvl = 0;
        tc[0] = tc[1] = tc[2] = 0;
        tblk = 0;
        tstar = 0.0;
    }
    __device__ __forceinline__ void near(const float* e, const float* x, double t0, double t1, float dsf)
    {
        const SegK k((float)(t1 - t0) * dsf);
#pragma unroll
        for (int l = 0; l < kLam; ++l) rte_step(In[l], Tn[l], e[l], x[l], k);
    }
    __device__ __forceinline__ void far(const float* e, const float* x, double t0, double t1, float dsf)
    {
        if constexpr (Gen) {
            const SegK k((float)(t1 - t0) * dsf);
#pragma unroll
            for (int l = 0; l < kLam; ++l) rte_step(If[l], Tf[l], e[l], x[l], k);
        }
    }
    __device__ __forceinline__ bool add(const float* e, const float* x, const int* c, int lvl, long long blk,
                                        double t0, double t1, float dsf)
    {
        if (reached) {
            // generation: the far field; inference continues past the point only after a fallback
            if constexpr (Gen) far(e, x, t0, t1, dsf);
            else near(e, x, t0, t1, dsf);
            return false;
        }
        if (t1 <= tt) {
            near(e, x, t0, t1, dsf);
            return false;
        }
        reached = 1;
        tstar = t0 > tt ? t0 : tt;
        tc[0] = c[0];
        tc[1] = c[1];
        tc[2] = c[2];
        tlvl = lvl;
        tblk = blk;
        if constexpr (!Gen) {
            if (fallback && fallback[blk]) {
                // full march from here on, without splitting this cell: the result is
                // bit-identical to the plain march
                fb = 1;
                near(e, x, t0, t1, dsf);
                return false;
            }
            if (t0 < tt) near(e, x, t0, tt, dsf);
            return true;
        } else {
            if (t0 < tt) near(e, x, t0, tt, dsf);
            far(e, x, tstar, t1, dsf);
            return false;
        }
    }
};

// Lanes of an angle-integrated workgroup: its J and psi accumulators live in LDS, lane-major.
constexpr int kJStride = 256;

// Angle integration: the plain march, plus 1 - exp(-tau) of the first segment
// (the probe's own cell up to its boundary), whose weighted sum over directions
// is the diagonal of the approximate operator.
struct AccJ {
    static constexpr bool kTrunc = false;
    static constexpr bool kJ = true;
    static constexpr bool kIv = false;
    float I[kLam], Tr[kLam];
    int first;
    float* pacc;  // the lane's psi accumulators in LDS (wavelength l at pacc[l * kJStride])
    float wdir;   // the direction's quadrature weight
    __device__ void init(const TraceLaunch*)
    {
#pragma unroll
        for (int l = 0; l < kLam; ++l) {
            I[l] = 0.f;
            Tr[l] = 1.f;
        }
        first = 1;
    }
    __device__ __forceinline__ bool add(const float* e, const float* x, const int*, int, long long, double t0,
                                        double t1, float dsf)
    {
        add_dt(e, x, (float)(t1 - t0) * dsf);
        return false;
    }
    // The first segment's 1 - exp(-tau) enters the weighted psi sum at once (psi += w (1 - exp(-tau_1))).
    // A traversed segment always has dt > 0 (t1 > t0, and the difference of two crossing times is far
    // above FP32's smallest subnormal), so the zero-length segment a pipelined visitor starts with leaves
    // "first" set (it adds w x 0, which leaves the sum unchanged).
    __device__ __forceinline__ void add_dt(const float* e, const float* x, float dt)
    {
        const SegK k(dt);
#pragma unroll
        for (int l = 0; l < kLam; ++l) {
            const float tr = rte_step(I[l], Tr[l], e[l], x[l], k);
            if (first) pacc[l * kJStride] = fmaf(wdir, 1.0f - tr, pacc[l * kJStride]);
        }
        if (dt > 0.f) first = 0;
    }
};

// Whether an accumulator is the inference-mode truncated one (no far-field accumulation).
template <class A>
constexpr bool trunc_inference()
{
    if constexpr (A::kTrunc) return !A::kGen;
    else return false;
}

// ------------------------------------------------------------- visitors
template <int D, typename T, class Acc = AccPlain>
struct VisStatic {
    using AccT = Acc;
    static constexpr int kMinWaves = (!Acc::kTrunc && !Acc::kJ) ? 4 : 1;
    // the same one-segment software pipeline as the velocity-interpolation visitor (every accumulator but
    // the truncated ones; the angle-integrated one in 2D only, where its registers allow it): a cell's
    // record is loaded at its visit and applied at the next one or in finish()
    static constexpr bool kPipe = !Acc::kTrunc && (!Acc::kJ || D == 2);
    const Geo* g;
    const int32_t* slot;
    const T* vals;
    long long cur_blk;
    long long base;
    float dsf;
    int slot_lds;
    RawRec<T> pr;  // pending segment's record, as loaded
    float pdt;     // its length
    Acc acc;
    __device__ void init_src(const Geo* geo, const int32_t* sl, const void* v, float ds0)
    {
        g = geo;
        slot = sl;
        vals = (const T*)v;
        cur_blk = -1;
        base = 0;
        dsf = ds0;
        slot_lds = 0;
#pragma unroll
        for (int i = 0; i < (int)(sizeof(pr.q) / sizeof(uint4)); ++i) pr.q[i] = make_uint4(0u, 0u, 0u, 0u);
        pdt = 0.f;
    }
    __device__ void init(const TraceLaunch* t, const float*)
    {
        init_src(&t->g, t->slot, t->vals, t->ds0);
        slot_lds = t->slot_lds;
        acc.init(t);
    }
    __device__ __forceinline__ void apply_pending()
    {
        float e[kLam], x[kLam];
        decode_rec<T>(pr, e, x);
        acc.add_dt(e, x, pdt);
    }
    __device__ __forceinline__ void finish()
    {
        if constexpr (kPipe) apply_pending();
    }
    __device__ __forceinline__ bool seg(const int* c, int lvl, long long blk, double t0, double t1)
    {
        if (blk != cur_blk) {
            cur_blk = blk;
            base = block_slot(*g, slot, slot_lds, blk) * g->cells;
        }
        const T* r = vals + (base + level_offset(*g, lvl) + local_index(*g, c, lvl, D)) * (kLam * 2);
        if constexpr (kPipe) {
            apply_pending();
            pr = fetch_rec<T>(r);
            pdt = (float)(t1 - t0) * dsf;
            return false;
        } else {
            float e[kLam], x[kLam];
            load_rec<T>(r, e, x);
            return acc.add(e, x, c, lvl, blk, t0, t1, dsf);
        }
    }
};

// Prefiltered cells (Sect. 5.1): level 0 reads the stored MIP-0 values, a
// merged cell the records of the signed axes the ray propagates along
// (k = 2a + (w_a < 0)), blended with weights w_a^2 / sum w^2 fixed per ray.
template <int D, typename T, class Acc = AccPlain>
struct VisPrefilter {
    using AccT = Acc;
    static constexpr int kMinWaves = (D == 2 && !Acc::kTrunc && !Acc::kJ) ? 4 : 1;
    const TraceLaunch* tl;
    const T* vals;
    const T* pf;
    long long cur_blk;
    long long base;
    float dsf;
    float wgt[D];
    int kax[D];
    Acc acc;
    __device__ void init(const TraceLaunch* t, const float* wf)
    {
        tl = t;
        vals = (const T*)t->vals;
        pf = (const T*)t->pf;
        cur_blk = -1;
        base = 0;
        dsf = t->ds0;
        float s = 0.f;
#pragma unroll
        for (int a = 0; a < D; ++a) s = fmaf(wf[a], wf[a], s);
#pragma unroll
        for (int a = 0; a < D; ++a) {
            wgt[a] = wf[a] * wf[a] / s;
            kax[a] = 2 * a + (wf[a] < 0.f ? 1 : 0);
        }
        acc.init(t);
    }
    __device__ __forceinline__ bool seg(const int* c, int lvl, long long blk, double t0, double t1)
    {
        if (blk != cur_blk) {
            cur_blk = blk;
            base = block_slot(tl->g, tl->slot, tl->slot_lds, blk) * tl->g.cells;
        }
        const long long cell = base + level_offset(tl->g, lvl) + local_index(tl->g, c, lvl, D);
        float e[kLam], x[kLam];
        if (lvl == 0) {
            load_rec<T>(vals + cell * (kLam * 2), e, x);
        } else {
#pragma unroll
            for (int l = 0; l < kLam; ++l) e[l] = x[l] = 0.f;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                float ea[kLam], xa[kLam];
                load_rec<T>(pf + (cell * (2 * D) + kax[a]) * (kLam * 2), ea, xa);
#pragma unroll
                for (int l = 0; l < kLam; ++l) {
                    e[l] = fmaf(wgt[a], ea[l], e[l]);
                    x[l] = fmaf(wgt[a], xa[l], x[l]);
                }
            }
        }
        return acc.add(e, x, c, lvl, blk, t0, t1, dsf);
    }
};

// T: storage of the node records (FP32, or BF16 / FP16 at half the record size).
// The direction class (full grid, or the orthant of w) is fixed per ray, so the
// class's grid records and node values are selected once at initialisation.
template <int D, typename T = float, class Acc = AccPlain>
struct VisVelinterp {
    using AccT = Acc;
    static constexpr int kMinWaves = (D == 2 && !Acc::kTrunc && !Acc::kJ) ? 4 : 1;
    // All accumulators but the truncated ones (and the angle-integrated one in 3D, whose registers would
    // drop a wave per SIMD) take a one-segment software pipeline: a segment's node records
    // are loaded when it is visited and applied at the next visit (or in finish()), so their latency
    // overlaps the traversal step in between, and the next cell's node coordinate is read before the
    // pending update, which overlaps that read.  Segments are applied in order with the same
    // arithmetic; the pipeline starts with a zero-length, zero-valued segment, which leaves I and T
    // unchanged bit for bit (tau = 0 takes the series branch: h = 0, exp(-0) = 1).
    static constexpr bool kPipe = !Acc::kTrunc && (!Acc::kJ || D == 2);
    const TraceLaunch* tl;
    const float4* vgrid;
    const T* vnodes;
    long long cur_blk;
    long long base;
    float dsf;
    float w[3];
    RawRec<T> pr0, pr1;  // pending segment's two node records, as loaded
    float pwt, pdt;      // its interpolation weight and length
    Acc acc;
    __device__ void init(const TraceLaunch* t, const float* wf)
    {
        tl = t;
        cur_blk = -1;
        base = 0;
        dsf = t->ds0;
        w[0] = wf[0];
        w[1] = wf[1];
        w[2] = D > 2 ? wf[2] : 0.f;
        int q = 0;
        if (t->n_vclass > 1) q = (w[0] < 0.f ? 1 : 0) | (w[1] < 0.f ? 2 : 0) | (D > 2 && w[2] < 0.f ? 4 : 0);
        const long long ncell_all = (long long)t->n_active * t->g.cells;
        vgrid = t->vgrid + q * ncell_all;
        vnodes = (const T*)t->vnodes + q * ncell_all * t->n_v * (kLam * 2);
#pragma unroll
        for (int i = 0; i < (int)(sizeof(pr0.q) / sizeof(uint4)); ++i) pr0.q[i] = pr1.q[i] = make_uint4(0u, 0u, 0u, 0u);
        pwt = pdt = 0.f;
        acc.init(t);
    }
    __device__ __forceinline__ void apply_pending()
    {
        float e0[kLam], x0[kLam], e1[kLam], x1[kLam], ee[kLam], xx[kLam];
        decode_rec<T>(pr0, e0, x0);
        decode_rec<T>(pr1, e1, x1);
#pragma unroll
        for (int l = 0; l < kLam; ++l) {
            ee[l] = fmaf(pwt, e1[l] - e0[l], e0[l]);
            xx[l] = fmaf(pwt, x1[l] - x0[l], x0[l]);
        }
        acc.add_dt(ee, xx, pdt);
    }
    // applies the last pending segment (called once the traversal has ended)
    __device__ __forceinline__ void finish()
    {
        if constexpr (kPipe) apply_pending();
    }
    __device__ __forceinline__ bool seg(const int* c, int lvl, long long blk, double t0, double t1)
    {
        if (blk != cur_blk) {
            cur_blk = blk;
            base = block_slot(tl->g, tl->slot, tl->slot_lds, blk) * tl->g.cells;
        }
        const unsigned cellin = (unsigned)(level_offset(tl->g, lvl) + local_index(tl->g, c, lvl, D));
        const unsigned cell = (unsigned)base + cellin;
        // node coordinate f = g . w + off = (vbar . w - lo) (n_v - 1) / (hi - lo) over the cell's range
        // [lo, hi] of projected velocities (g = off = 0 for an empty range: node 0 is used)
        float4 vg = vgrid[cell];
        if constexpr (kPipe) apply_pending();
        float f = fmaf(vg.x, w[0], fmaf(vg.y, w[1], vg.w));
        if (D > 2) f = fmaf(vg.z, w[2], f);
        const int nv = tl->n_v;
        int kn = (int)floorf(f);
        kn = kn < 0 ? 0 : (kn > nv - 2 ? nv - 2 : kn);
        float wt = f - (float)kn;
        // node planes of the brick: [node][cell], one record 64 B in FP32 (32 B in BF16 / FP16); the two nodes
        // around u are one plane apart
        const unsigned cells = (unsigned)tl->g.cells;
        const T* r0 = vnodes + ((unsigned)base * (unsigned)nv + (unsigned)kn * cells + cellin) * (unsigned)(kLam * 2);
        if constexpr (kPipe) {
            pr0 = fetch_rec<T>(r0);
            pr1 = fetch_rec<T>(r0 + cells * (unsigned)(kLam * 2));
            pwt = wt;
            pdt = (float)(t1 - t0) * dsf;
            return false;
        } else {
            float e0[kLam], x0[kLam], e1[kLam], x1[kLam];
            load_rec<T>(r0, e0, x0);
            load_rec<T>(r0 + cells * (unsigned)(kLam * 2), e1, x1);
            float ee[kLam], xx[kLam];
#pragma unroll
            for (int l = 0; l < kLam; ++l) {
                ee[l] = fmaf(wt, e1[l] - e0[l], e0[l]);
                xx[l] = fmaf(wt, x1[l] - x0[l], x0[l]);
            }
            return acc.add(ee, xx, c, lvl, blk, t0, t1, dsf);
        }
    }
};

// Whether a visitor is software-pipelined.  The pipelined ones traverse with the level_dist table read
// from LDS where it is needed (nothing in their traversal may wait on vector-memory loads, and holding
// the table in registers spilled scalar registers); the others keep it in scalar registers, read once
// from the launch's arguments, which costs the VALU-bound Core-and-Voigt march fewer instructions.
template <class V, class = void>
struct Pipelined {
    static constexpr bool v = false;
};
template <class V>
struct Pipelined<V, std::void_t<decltype(V::kPipe)>> {
    static constexpr bool v = V::kPipe;
};

// Ends a traversal: visitors with a pending (software-pipelined) segment apply it.
template <class V>
__device__ __forceinline__ auto finish_visit(V& v, int) -> decltype(v.finish(), void())
{
    v.finish();
}
template <class V>
__device__ __forceinline__ void finish_visit(V&, long)
{
}

// NL: lines the kernel is compiled for (2 or kMaxLines); scenes with up to two
// lines use NL = 2, which halves the per-segment line state and code.
template <int D, typename T = float, class Acc = AccPlain, int NL = kMaxLines>
struct VisCav {
    using AccT = Acc;
    // the plain 3D march needs a few registers more than three waves per SIMD allow; the
    // inference-mode truncated march (the cache path, mostly full-length fallback rays) is held
    // to three waves in 3D with two lines as well
    static constexpr int kMinWaves = Acc::kJ ? 1
                                     : Acc::kTrunc ? ((D == 3 && NL == 2 && trunc_inference<Acc>()) ? 3 : 1)
                                     : (D == 2 && NL == 2) ? 4 : (D == 3 ? 3 : 1);
    const TraceLaunch* tl;
    long long cur_blk;
    long long base;
    float dsf;
    float w[3];
    Acc acc;
    __device__ void init(const TraceLaunch* t, const float* wf)
    {
        tl = t;
        cur_blk = -1;
        base = 0;
        dsf = t->ds0;
        w[0] = wf[0];
        w[1] = wf[1];
        w[2] = D > 2 ? wf[2] : 0.f;
        acc.init(t);
    }
    __device__ __forceinline__ bool seg(const int* c, int lvl, long long blk, double t0, double t1)
    {
        if (blk != cur_blk) {
            cur_blk = blk;
            base = block_slot(tl->g, tl->slot, tl->slot_lds, blk) * tl->g.cells;
        }
        long long cell = base + level_offset(tl->g, lvl) + local_index(tl->g, c, lvl, D);
        const T* r = (const T*)(sizeof(T) == 4 ? (const void*)tl->cav : tl->cav_lp) + cell * tl->cav_rec;
        const int nln = tl->lb.n_lines;
        float ls[NL][4];
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            if (k < nln) {
                float4 q = load4<T>(r, k);
                ls[k][0] = q.x;
                ls[k][1] = q.y;
                ls[k][2] = q.z;
                ls[k][3] = q.w;
            }
        }
        float4 bgv = load4<T>(r, nln);  // eta_bg, chi_bg, vx, vy
        float vz = 0.f;
        if (D > 2) vz = load4<T>(r, nln + 1).x;
        float u = bgv.z * w[0] + bgv.w * w[1] + vz * w[2];
        const bool voigt = tl->lb.profile == RT_PROFILE_VOIGT;
        float eo[kLam], xo[kLam];
#pragma unroll
        for (int l = 0; l < kLam; ++l) {
            float ee = bgv.x, xx = bgv.y;
#pragma unroll
            for (int k = 0; k < NL; ++k) {
                if (k < nln) {
                    // per-batch constants lam - lam0, lam / lam0, lam0 / c: scalar kernel arguments
                    float x = fmaf(tl->lb.k0[k], u, tl->lb.dl[l][k]) * ls[k][3];
                    float phi;
                    if (!voigt) {
                        phi = __expf(-x * x);
                    } else {
                        float r2 = tl->lb.rr[l][k];
                        phi = voigt_h(ls[k][2] * r2 * r2, x) * ls[k][3] * tl->lb.sr[l][k];
                    }
                    ee = fmaf(ls[k][0], phi, ee);
                    xx = fmaf(ls[k][1], phi, xx);
                }
            }
            eo[l] = ee;
            xo[l] = xx;
        }
        return acc.add(eo, xo, c, lvl, blk, t0, t1, dsf);
    }
};

// ------------------------------------------------------------ trace kernel
// A caller's probe index outside the grid's voxels: the ray is not traced, its
// outputs are NaN, and the first direction's ray counts it in err[2].
__device__ __forceinline__ bool bad_probe(const TraceLaunch& t, long long v)
{
    return v < 0 || v >= (long long)t.g.n[0] * t.g.n[1] * t.g.n[2];
}

template <class Acc>
__device__ __forceinline__ void write_bad_probe(const TraceLaunch& t, long long dir, long long probe)
{
    const float nan = __builtin_nanf("");
    const int nl = t.lb.nl;
    if (dir == 0) atomicAdd(&t.err[2], 1ull);
    for (int l = 0; l < nl; ++l) {
        const long long q = ((long long)dir * nl + l) * t.n_probes + probe;
        if constexpr (Acc::kTrunc) {
            t.I_near[q] = nan;
            t.T_near[q] = nan;
            if constexpr (Acc::kGen) t.I_far[q] = nan;
            t.fstat_out[q] = make_float4(0.f, 0.f, 0.f, 0.f);
        } else {
            t.I[q] = nan;
            if (Acc::kIv && t.T_out) t.T_out[q] = nan;
        }
    }
    if constexpr (Acc::kTrunc) t.feat[dir * t.n_probes + probe] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// One ray (direction dir, probe index probe) of a trace launch.
// Voxel (lx, ly, lz) of a brick that brick-local probe `local` stands for, in wave-tile order: x-consecutive
// rows (64 lanes: a 16 x 4 strip of a 16^2 brick, an 8 x 8 x 1 slab of an 8^3 one) or cube tiles of side
// ts = 8 (2D) or 4 (3D), x-fastest inside a tile and tiles x-fastest inside the brick (bricks smaller than
// a tile: the whole brick).  Either way a bijection of the brick's voxels.
template <int D>
__device__ __forceinline__ void tile_voxel(int local, int log2B, bool cubes, int& lx, int& ly, int& lz)
{
    if (cubes) {
        const int lts = min(log2B, D == 2 ? 3 : 2), ts = 1 << lts, ltn = log2B - lts;
        const int r = local & ((1 << (D * lts)) - 1), t = local >> (D * lts);
        lx = ((t & ((1 << ltn) - 1)) << lts) | (r & (ts - 1));
        ly = (((t >> ltn) & ((1 << ltn) - 1)) << lts) | ((r >> lts) & (ts - 1));
        lz = D > 2 ? (((t >> (2 * ltn)) << lts) | (r >> (2 * lts))) : 0;
    } else {
        const int B = 1 << log2B;
        lx = local & (B - 1);
        ly = (local >> log2B) & (B - 1);
        lz = D > 2 ? local >> (2 * log2B) : 0;
    }
}

// rt_trace's probe index (x-fastest inside the brick) of the voxel that wave-tile position p takes.  In
// 3D the march's waves take 4 x 4 x 4 cube tiles (their 64 parallel rays start in a compact block of
// voxels; 2.6 % faster than 8 x 8 x 1 slabs on the 3D Core-and-Voigt march); in 2D x-consecutive rows
// (a 16 x 4 strip measured 4 % faster than an 8 x 8 square on the 2D velocity-interpolation march).
template <int D>
__device__ __forceinline__ long long cube_tile_probe(long long p, int log2B)
{
    if constexpr (D == 2) return p;
    const int bits = D * log2B;
    int lx, ly, lz;
    tile_voxel<D>((int)(p & ((1ll << bits) - 1)), log2B, true, lx, ly, lz);
    return ((p >> bits) << bits) + lx + (ly << log2B) + (lz << (2 * log2B));
}

template <int D, class Vis>
__device__ __forceinline__ void trace_ray(const TraceLaunch& t, const uint64_t* sts, long long dir, long long probe,
                                          Counters& cnt)
{
    int pv[3] = {0, 0, 0};
    if (t.probes) {
        long long v = t.probes[probe];
        if (bad_probe(t, v)) {
            write_bad_probe<typename Vis::AccT>(t, dir, probe);
            return;
        }
        pv[0] = (int)(v % t.g.n[0]);
        pv[1] = (int)((v / t.g.n[0]) % t.g.n[1]);
        pv[2] = (int)(v / ((long long)t.g.n[0] * t.g.n[1]));
    } else {
        long long slot = probe >> (D * t.g.log2B);
        int local = (int)(probe & (t.g.bvox - 1));
        int blk = t.active_list[slot];
        int bcx = blk % t.g.nb[0], bcy = (blk / t.g.nb[0]) % t.g.nb[1], bcz = blk / (t.g.nb[0] * t.g.nb[1]);
        pv[0] = bcx * t.g.B + (local & (t.g.B - 1));
        pv[1] = bcy * t.g.B + ((local >> t.g.log2B) & (t.g.B - 1));
        if (D > 2) pv[2] = bcz * t.g.B + (local >> (2 * t.g.log2B));
    }
    float wf[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < D; ++a) wf[a] = t.dirs[dir * D + a];

    Vis vis;
    vis.init(&t, wf);
    constexpr bool kIv = Vis::AccT::kIv;
    extern __shared__ uint64_t lds_words[];
    constexpr bool kLdsLd = Pipelined<Vis>::v;
    int rc = hdda<D, kIv, kLdsLd>(t.g, sts, t.mode, t.max_level, t.graded,
                                  kLdsLd ? lds_level_dist(t, lds_words) : t.level_dist, pv, wf, t.step_cap, vis, cnt,
                                  t.t_lo, t.t_hi);
    finish_visit(vis, 0);
    int capped = rc == 1;
    const int nl = t.lb.nl;
    if constexpr (kIv) {
        // I0 enters only through the interval in which the ray leaves the grid
        const float I0 = rc == 0 ? t.I0 : 0.f;
#pragma unroll
        for (int l = 0; l < kLam; ++l) {
            if (l >= nl) continue;
            const long long q = ((long long)dir * nl + l) * t.n_probes + probe;
            t.I[q] = fmaf(vis.acc.Tr[l], I0, vis.acc.I[l]);
            if (t.T_out) t.T_out[q] = vis.acc.Tr[l];
        }
    } else if constexpr (!Vis::AccT::kTrunc) {
#pragma unroll
        for (int l = 0; l < kLam; ++l) {
            if (l < nl) t.I[((long long)dir * nl + l) * t.n_probes + probe] = fmaf(vis.acc.Tr[l], t.I0, vis.acc.I[l]);
        }
    } else {
        const auto& A = vis.acc;
        const bool query = A.reached && !A.fb;
        const long long pidx = dir * t.n_probes + probe;
#pragma unroll
        for (int l = 0; l < kLam; ++l) {
            if (l >= nl) continue;
            const long long q = ((long long)dir * nl + l) * t.n_probes + probe;
            t.I_near[q] = query ? A.In[l] : fmaf(A.Tn[l], t.I0, A.In[l]);
            t.T_near[q] = query ? A.Tn[l] : 0.f;
            if constexpr (Vis::AccT::kGen) t.I_far[q] = query ? fmaf(A.Tf[l], t.I0, A.If[l]) : t.I0;
        }
        float px = 0.f, py = 0.f, pz = 0.f;
        if (query) {
            px = (float)((double)pv[0] + 0.5 - A.tstar * (double)wf[0]);
            py = (float)((double)pv[1] + 0.5 - A.tstar * (double)wf[1]);
            if (D > 2) pz = (float)((double)pv[2] + 0.5 - A.tstar * (double)wf[2]);
            else pz = 0.5f;
        }
        // w: 0 without a query, else 1 + the block whose cell holds the truncation point
        // (exact in FP32 up to 2^24 blocks; the held-out check flags this block)
        t.feat[pidx] = make_float4(px, py, pz, query ? (float)(A.tblk + 1) : 0.f);
        // level statistics of the feature-level cell at the truncation point
        const int fl = t.g.feat_level;
        const int sl = t.g.log2B - fl;
        int lx = (A.tc[0] & (t.g.B - 1)) >> fl, ly = (A.tc[1] & (t.g.B - 1)) >> fl;
        int lz = D > 2 ? ((A.tc[2] & (t.g.B - 1)) >> fl) : 0;
        long long fcell = query ? (long long)t.slot[A.tblk] * (1ll << (D * sl)) + lx + (ly << sl) + (lz << (2 * sl)) : 0;
#pragma unroll
        for (int l = 0; l < kLam; ++l) {
            if (l >= nl) continue;
            float4 st = query ? t.fstats[fcell * kLam + l] : make_float4(0.f, 0.f, 0.f, 0.f);
            t.fstat_out[((long long)dir * nl + l) * t.n_probes + probe] = st;
        }
    }
    if (capped) {
        atomicAdd(&t.err[0], 1ull);
        atomicMin(&t.err[1], (unsigned long long)(dir * t.n_probes + probe));
    }
}

template <int D, class Vis>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Vis::kMinWaves)))
k_trace(TraceLaunch t)
{
    extern __shared__ uint64_t sts[];
    stage_blocks(t, sts);
    // XCD-aware order: workgroups are dealt round-robin over the 8 XCDs; give
    // each XCD a contiguous range of (direction, probe tile) work.
    const unsigned G = gridDim.x, wg = blockIdx.x;
    const unsigned q = G / 8u, r = G % 8u, xcd = wg % 8u, i = wg / 8u;
    const unsigned lwg = xcd < r ? xcd * (q + 1u) + i : r * (q + 1u) + (xcd - r) * q + i;
    const long long tiles = (t.n_probes + 63) / 64;
    // one direction per wave: keep the wave index (and with it the direction, its
    // step signs and reciprocals) in scalar registers
    const long long wave = (long long)lwg * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    // 2D: direction-major over all tiles, so the waves in flight march parallel rays through
    // the same volume and share its cells in L2.  3D (a much larger volume per direction):
    // each XCD takes one eighth of the probe tiles, a compact region in Morton order, for
    // every direction (direction-major inside it), so its own L2 holds that region's cells.
    const long long per = D == 3 ? (tiles + 7) / 8 : tiles;
    const long long xc = D == 3 ? wave / (per * t.n_dir) : 0;
    const long long rem = wave - xc * per * t.n_dir;
    const long long dir = rem / per;
    const long long tile = xc * per + (rem - dir * per);
    const long long pos = tile * 64 + lane;
    const bool in_grid = xc < 8 && dir < t.n_dir && tile < tiles;
    // implicit probes (every active voxel) in the dimension's wave-tile order; a caller's probe list in its own order
    const long long probe = t.probes ? pos : cube_tile_probe<D>(pos, t.g.log2B);
    Counters cnt = {0, 0, 0};
    if (in_grid && pos < t.n_probes) trace_ray<D, Vis>(t, sts, dir, probe, cnt);
    if (t.stats) {
        // the whole wave is active again here; [4] sums the longest ray of each wave
        // (in traversal steps), so ([0] + [2]) / (64 [4]) is the lane utilisation
        const bool live = in_grid && pos < t.n_probes;
        unsigned steps = cnt.segs + cnt.empty, wmax = steps;
        for (int o = 32; o > 0; o >>= 1) wmax = max(wmax, (unsigned)__shfl_xor((int)wmax, o, 64));
        if (live) {
            atomicAdd(&t.stats[0], (unsigned long long)cnt.segs);
            atomicAdd(&t.stats[1], 1ull);
            atomicAdd(&t.stats[2], (unsigned long long)cnt.empty);
            atomicAdd(&t.stats[3], (unsigned long long)cnt.lvlchg);
        }
        if (lane == 0 && in_grid) atomicAdd(&t.stats[4], (unsigned long long)wmax);
    }
}

// Angle-integrated trace: a wave takes 64 probes and a chunk of directions,
// marches them one direction after another (the direction stays uniform across
// the wave) and accumulates J = sum_d w_d I_d and psi = sum_d w_d (1 - exp(-tau_1,d))
// in registers; one partial per chunk is written (the caller's chunks are summed
// in a fixed order afterwards).
// Waves per SIMD the angle-integrated kernel is held to: 4 for the software-pipelined visitors (with
// its J and psi sums in LDS their march fits the plain march's registers; a few per-direction values
// spill outside the segment loop), else the compiler's choice.
template <class V>
struct MinWavesJ {
    static constexpr int v = Pipelined<V>::v ? 4 : 1;
};

template <int D, class Vis>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MinWavesJ<Vis>::v))) k_trace_j(TraceLaunch t)
{
    extern __shared__ uint64_t sts[];
    stage_blocks(t, sts);
    const unsigned G = gridDim.x, wg = blockIdx.x;
    const unsigned q = G / 8u, r = G % 8u, xcd = wg % 8u, i = wg / 8u;
    const unsigned lwg = xcd < r ? xcd * (q + 1u) + i : r * (q + 1u) + (xcd - r) * q + i;
    const long long tiles = (t.n_probes + 63) / 64;
    const long long wave = (long long)lwg * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const long long chunk = wave / tiles;
    const long long pos = (wave - chunk * tiles) * 64 + lane;
    const long long probe = t.probes ? pos : cube_tile_probe<D>(pos, t.g.log2B);
    const long long d0 = chunk * t.dirs_per_chunk;
    if (d0 >= t.n_dir) return;  // whole wave
    const long long d1 = d0 + t.dirs_per_chunk < t.n_dir ? d0 + t.dirs_per_chunk : t.n_dir;
    bool live = pos < t.n_probes;
    int pv[3] = {0, 0, 0};
    if (live) {
        if (t.probes) {
            long long v = t.probes[probe];
            if (bad_probe(t, v)) {
                // not traced: NaN partials make the probe's J and psi NaN
                if (chunk == 0) atomicAdd(&t.err[2], 1ull);
                const int nl = t.lb.nl;
                for (int l = 0; l < nl; ++l) {
                    const long long o = (chunk * nl + l) * t.n_probes + probe;
                    t.part_J[o] = __builtin_nanf("");
                    if (t.part_psi) t.part_psi[o] = __builtin_nanf("");
                }
                return;
            }
            pv[0] = (int)(v % t.g.n[0]);
            pv[1] = (int)((v / t.g.n[0]) % t.g.n[1]);
            pv[2] = (int)(v / ((long long)t.g.n[0] * t.g.n[1]));
        } else {
            long long slot = probe >> (D * t.g.log2B);
            int local = (int)(probe & (t.g.bvox - 1));
            int blk = t.active_list[slot];
            int bcx = blk % t.g.nb[0], bcy = (blk / t.g.nb[0]) % t.g.nb[1], bcz = blk / (t.g.nb[0] * t.g.nb[1]);
            pv[0] = bcx * t.g.B + (local & (t.g.B - 1));
            pv[1] = bcy * t.g.B + ((local >> t.g.log2B) & (t.g.B - 1));
            if (D > 2) pv[2] = bcz * t.g.B + (local >> (2 * t.g.log2B));
        }
    }
    // J and psi sums of the lane, in LDS (lane-major: column threadIdx.x), which keeps the march's
    // registers at the plain march's count
    __shared__ float jsum[kLam * kJStride], psum[kLam * kJStride];
    float* const jl = jsum + threadIdx.x;
    float* const pl = psum + threadIdx.x;
#pragma unroll
    for (int l = 0; l < kLam; ++l) jl[l * kJStride] = pl[l * kJStride] = 0.f;
    for (long long dir = d0; dir < d1; ++dir) {
        if (!live) continue;
        float wf[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int a = 0; a < D; ++a) wf[a] = t.dirs[dir * D + a];
        const float w = t.weights[dir];
        Vis vis;
        vis.init(&t, wf);
        vis.acc.pacc = pl;
        vis.acc.wdir = w;
        Counters cnt = {0, 0, 0};
        constexpr bool kLdsLd = Pipelined<Vis>::v;
        const int rc = hdda<D, false, kLdsLd>(t.g, sts, t.mode, t.max_level, t.graded,
                                              kLdsLd ? lds_level_dist(t, sts) : t.level_dist, pv, wf, t.step_cap, vis,
                                              cnt);
        finish_visit(vis, 0);
        if (rc == 1) {
            atomicAdd(&t.err[0], 1ull);
            atomicMin(&t.err[1], (unsigned long long)(dir * t.n_probes + probe));
        }
#pragma unroll
        for (int l = 0; l < kLam; ++l) jl[l * kJStride] = fmaf(w, fmaf(vis.acc.Tr[l], t.I0, vis.acc.I[l]), jl[l * kJStride]);
    }
    if (!live) return;
    const int nl = t.lb.nl;
#pragma unroll
    for (int l = 0; l < kLam; ++l) {
        if (l >= nl) continue;
        const long long o = (chunk * nl + l) * t.n_probes + probe;
        t.part_J[o] = jl[l * kJStride];
        if (t.part_psi) t.part_psi[o] = pl[l * kJStride];
    }
}

// out[i] = sum over chunks c (in order) of part[c n + i]
__global__ void k_reduce_chunks(const float* part, int n_chunks, long long n, float* out)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
    for (int c = 0; c < n_chunks; ++c) s += part[(long long)c * n + i];
    out[i] = s;
}

hipError_t launch_reduce_chunks(const float* part, int n_chunks, long long n, float* out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_chunks, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part, n_chunks, n, out);
    return hipGetLastError();
}

template <int D, class Vis>
static hipError_t launch_one(const TraceLaunch& t0, hipStream_t s)
{
    TraceLaunch t = t0;
    long long tiles = (t.n_probes + 63) / 64;
    size_t shm = sizeof(uint64_t) * (size_t)t.g.n_state_words + sizeof(float) * kMaxLevels;
    // small grids: the slot table joins the state words in LDS (at most 32 KiB more per workgroup)
    t.slot_lds = t.g.nblocks <= kSlotLdsMax ? 1 : 0;
    if (t.slot_lds) shm += sizeof(int32_t) * (size_t)t.g.nblocks;
    if constexpr (Vis::AccT::kJ) {
        const long long n_chunks = (t.n_dir + t.dirs_per_chunk - 1) / t.dirs_per_chunk;
        const long long wgs = (tiles * n_chunks + 3) / 4;
        if (wgs <= 0) return hipSuccess;
        hipLaunchKernelGGL((k_trace_j<D, Vis>), dim3((unsigned)wgs), dim3(256), shm, s, t);
    } else {
        // 3D: eight equal tile chunks (one per XCD), the last padded
        const long long waves = (D == 3 ? 8 * ((tiles + 7) / 8) : tiles) * t.n_dir;
        const long long wgs = (waves + 3) / 4;
        if (wgs <= 0) return hipSuccess;
        hipLaunchKernelGGL((k_trace<D, Vis>), dim3((unsigned)wgs), dim3(256), shm, s, t);
    }
    return hipGetLastError();
}

template <int D, class Acc, int NL>
static hipError_t launch_cav_nl(const TraceLaunch& t, hipStream_t s)
{
    if (t.storage == RT_F32) return launch_one<D, VisCav<D, float, Acc, NL>>(t, s);
    if (t.storage == RT_BF16) return launch_one<D, VisCav<D, __hip_bfloat16, Acc, NL>>(t, s);
    return launch_one<D, VisCav<D, __half, Acc, NL>>(t, s);
}

template <int D, class Acc>
static hipError_t launch_cav(const TraceLaunch& t, hipStream_t s)
{
    if (t.lb.n_lines <= 2) return launch_cav_nl<D, Acc, 2>(t, s);
    return launch_cav_nl<D, Acc, kMaxLines>(t, s);
}

template <class Acc>
static hipError_t launch_trace_acc(const TraceLaunch& t, hipStream_t s)
{
    if (t.emission == RT_EMIS_STATIC) {
        if (t.g.dim == 2) {
            if (t.storage == RT_F32) return launch_one<2, VisStatic<2, float, Acc>>(t, s);
            if (t.storage == RT_BF16) return launch_one<2, VisStatic<2, __hip_bfloat16, Acc>>(t, s);
            return launch_one<2, VisStatic<2, __half, Acc>>(t, s);
        }
        if (t.storage == RT_F32) return launch_one<3, VisStatic<3, float, Acc>>(t, s);
        if (t.storage == RT_BF16) return launch_one<3, VisStatic<3, __hip_bfloat16, Acc>>(t, s);
        return launch_one<3, VisStatic<3, __half, Acc>>(t, s);
    }
    if (t.emission == RT_EMIS_PREFILTER) {
        if (t.g.dim == 2) {
            if (t.storage == RT_F32) return launch_one<2, VisPrefilter<2, float, Acc>>(t, s);
            if (t.storage == RT_BF16) return launch_one<2, VisPrefilter<2, __hip_bfloat16, Acc>>(t, s);
            return launch_one<2, VisPrefilter<2, __half, Acc>>(t, s);
        }
        if (t.storage == RT_F32) return launch_one<3, VisPrefilter<3, float, Acc>>(t, s);
        if (t.storage == RT_BF16) return launch_one<3, VisPrefilter<3, __hip_bfloat16, Acc>>(t, s);
        return launch_one<3, VisPrefilter<3, __half, Acc>>(t, s);
    }
    if (t.emission == RT_EMIS_VELINTERP) {
        if (t.g.dim == 2) {
            if (t.storage == RT_F32) return launch_one<2, VisVelinterp<2, float, Acc>>(t, s);
            if (t.storage == RT_BF16) return launch_one<2, VisVelinterp<2, __hip_bfloat16, Acc>>(t, s);
            return launch_one<2, VisVelinterp<2, __half, Acc>>(t, s);
        }
        if (t.storage == RT_F32) return launch_one<3, VisVelinterp<3, float, Acc>>(t, s);
        if (t.storage == RT_BF16) return launch_one<3, VisVelinterp<3, __hip_bfloat16, Acc>>(t, s);
        return launch_one<3, VisVelinterp<3, __half, Acc>>(t, s);
    }
    if (t.g.dim == 2) {
        return launch_cav<2, Acc>(t, s);
    }
    return launch_cav<3, Acc>(t, s);
}

hipError_t launch_trace(const TraceLaunch& t, hipStream_t s)
{
    if (t.jmode) return launch_trace_acc<AccJ>(t, s);
    if (t.interval) return launch_trace_acc<AccIv>(t, s);
    if (t.trunc) return t.gen ? launch_trace_acc<AccTrunc<true>>(t, s) : launch_trace_acc<AccTrunc<false>>(t, s);
    return launch_trace_acc<AccPlain>(t, s);
}

// --------------------------------------------------- debug: visited cells
struct VisRecord {
    int32_t* cells;
    double* tt;
    int cap;
    int n;
    __device__ bool seg(const int* c, int lvl, long long, double t0, double t1)
    {
        if (n < cap) {
            cells[4 * n] = c[0];
            cells[4 * n + 1] = c[1];
            cells[4 * n + 2] = c[2];
            cells[4 * n + 3] = lvl;
            tt[2 * n] = t0;
            tt[2 * n + 1] = t1;
        }
        ++n;
        return false;
    }
};

template <int D>
__global__ void k_debug_visited(TraceLaunch t, int probe_vox, float wx, float wy, float wz, int cap,
                                int32_t* cells, double* tt, int32_t* count)
{
    extern __shared__ uint64_t sts[];
    for (int i = threadIdx.x; i < t.g.n_state_words; i += blockDim.x) sts[i] = t.states[i];
    __syncthreads();
    if (threadIdx.x != 0) return;
    int pv[3] = {(int)(probe_vox % t.g.n[0]), (int)((probe_vox / t.g.n[0]) % t.g.n[1]),
                 (int)(probe_vox / (t.g.n[0] * t.g.n[1]))};
    float wf[3] = {wx, wy, wz};
    VisRecord vis{cells, tt, cap, 0};
    Counters cnt = {0, 0, 0};
    int capped = hdda<D>(t.g, sts, t.mode, t.max_level, t.graded, t.level_dist, pv, wf, t.step_cap, vis, cnt);
    *count = capped ? -1 : vis.n;
}

hipError_t launch_debug_visited(const TraceLaunch& t, int probe_vox, float wx, float wy, float wz, int cap,
                                int32_t* cells, double* tt, int32_t* count, hipStream_t s)
{
    size_t shm = sizeof(uint64_t) * (size_t)t.g.n_state_words;
    if (t.g.dim == 2)
        hipLaunchKernelGGL(k_debug_visited<2>, dim3(1), dim3(64), shm, s, t, probe_vox, wx, wy, wz, cap, cells, tt,
                           count);
    else
        hipLaunchKernelGGL(k_debug_visited<3>, dim3(1), dim3(64), shm, s, t, probe_vox, wx, wy, wz, cap, cells, tt,
                           count);
    return hipGetLastError();
}

// ------------------------------------------------------ batched persistent
// One queue of 64-probe tiles over all jobs (scenes).  Each wave pops tiles
// with one atomic per `tiles_per_pop` tiles and traces them until the queue is
// empty, so uneven scenes and uneven ray lengths balance dynamically.  Every
// wave exits once the counter has passed the last tile.
template <int D, typename T>
__device__ __forceinline__ void batched_ray(const BatchJob& J, long long dir, long long probe, unsigned long long* err)
{
    const long long slot = probe >> (D * J.g.log2B);
    const int local = (int)(probe & (J.g.bvox - 1));
    int lx, ly, lz;
    tile_voxel<D>(local, J.g.log2B, J.tile_shape == RT_TILE_CUBES, lx, ly, lz);
    // the output keeps rt_trace's probe order (x-fastest inside the brick) whatever the tile shape
    const long long out_probe = (slot << (D * J.g.log2B)) + lx + (ly << J.g.log2B) + (lz << (2 * J.g.log2B));
    const int blk = J.active_list[slot];
    int pv[3] = {0, 0, 0};
    pv[0] = (blk % J.g.nb[0]) * J.g.B + lx;
    pv[1] = ((blk / J.g.nb[0]) % J.g.nb[1]) * J.g.B + ly;
    if (D > 2) pv[2] = (blk / (J.g.nb[0] * J.g.nb[1])) * J.g.B + lz;
    float wf[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < D; ++a) wf[a] = J.dirs[dir * D + a];
    VisStatic<D, T> vis;
    vis.init_src(&J.g, J.slot, J.vals, J.ds0);
    vis.acc.init(nullptr);
    Counters cnt = {0, 0, 0};
    int capped = hdda<D>(J.g, J.states, J.mode, J.max_level, J.graded, J.level_dist, pv, wf, J.step_cap, vis, cnt) == 1;
    finish_visit(vis, 0);
#pragma unroll
    for (int l = 0; l < kLam; ++l)
        if (l < J.nl) J.I[((long long)dir * J.nl + l) * J.n_probes + out_probe] = fmaf(vis.acc.Tr[l], J.I0, vis.acc.I[l]);
    if (capped) {
        atomicAdd(&err[0], 1ull);
        atomicMin(&err[1], (unsigned long long)(J.tile0 * 64ull + (unsigned long long)(dir * J.tiles * 64 + out_probe)));
    }
}

// Queue counters of the launch segments start at their first tile.
__global__ void k_reset_queue(unsigned* counter, unsigned t0, unsigned t1)
{
    counter[0] = t0;
    counter[1] = t1;
}

// Tiles of one job of the queue: binary search over the jobs' first tiles
// (uniform across the wave).
__device__ __forceinline__ int job_of_tile(const BatchJob* __restrict__ jobs, int j0, int j1, unsigned tile)
{
    int lo = j0, hi = j1 - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].tile0 <= tile) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// One persistent launch over the jobs [j0, j1) of one dimension, whose tiles are
// [tile_begin, tile_end).  AnyT: the storage dtype is dispatched per job (a mix);
// otherwise every job stores T.
template <int D, typename T, bool AnyT>
__global__ void __launch_bounds__(512) k_batched(const BatchJob* __restrict__ jobs, int j0, int j1, unsigned tile_end,
                                                 int tiles_per_pop, unsigned* counter, unsigned* claims,
                                                 unsigned long long* err)
{
    const int lane = threadIdx.x & 63;
    for (;;) {
        unsigned base = 0;
        if (lane == 0) base = atomicAdd(counter, (unsigned)tiles_per_pop);
        // wave-uniform from here: the job lookup and its fields stay in scalar registers
        base = (unsigned)__builtin_amdgcn_readfirstlane((int)base);
        if (base >= tile_end) break;
        for (int q = 0; q < tiles_per_pop; ++q) {
            const unsigned tile = base + (unsigned)q;
            if (tile >= tile_end) break;
            const BatchJob& J = jobs[job_of_tile(jobs, j0, j1, tile)];
            const long long lt = (long long)(tile - J.tile0);
            const long long dir = lt / J.tiles;
            const long long probe = (lt - dir * J.tiles) * 64 + lane;
            if (claims && lane == 0) atomicAdd(&claims[tile], 1u);
            if (probe >= J.n_probes) continue;
            if constexpr (!AnyT) {
                batched_ray<D, T>(J, dir, probe, err);
            } else {
                if (J.storage == RT_F32) batched_ray<D, float>(J, dir, probe, err);
                else if (J.storage == RT_BF16) batched_ray<D, __hip_bfloat16>(J, dir, probe, err);
                else batched_ray<D, __half>(J, dir, probe, err);
            }
        }
    }
}

template <int D>
static void launch_batched_dim(const BatchSeg& g, const BatchJob* d_jobs, int wg_waves, int n_wgs, int tiles_per_pop,
                               unsigned* counter, unsigned* claims, unsigned long long* err, hipStream_t s)
{
    const dim3 grid((unsigned)n_wgs), block((unsigned)(64 * wg_waves));
    if (g.storage == RT_F32)
        hipLaunchKernelGGL((k_batched<D, float, false>), grid, block, 0, s, d_jobs, g.j0, g.j1, g.tile_end,
                           tiles_per_pop, counter, claims, err);
    else if (g.storage == RT_BF16)
        hipLaunchKernelGGL((k_batched<D, __hip_bfloat16, false>), grid, block, 0, s, d_jobs, g.j0, g.j1, g.tile_end,
                           tiles_per_pop, counter, claims, err);
    else if (g.storage == RT_F16)
        hipLaunchKernelGGL((k_batched<D, __half, false>), grid, block, 0, s, d_jobs, g.j0, g.j1, g.tile_end,
                           tiles_per_pop, counter, claims, err);
    else
        hipLaunchKernelGGL((k_batched<D, float, true>), grid, block, 0, s, d_jobs, g.j0, g.j1, g.tile_end,
                           tiles_per_pop, counter, claims, err);
}

hipError_t launch_batched(const BatchJob* d_jobs, const BatchSeg* segs, int n_segs, int wg_waves, int n_wgs,
                          int tiles_per_pop, unsigned* counter, unsigned* claims, unsigned long long* err,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(1), 0, s, counter, n_segs > 0 ? segs[0].tile_begin : 0u,
                       n_segs > 1 ? segs[1].tile_begin : 0u);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int i = 0; i < n_segs; ++i) {
        if (segs[i].dim == 2)
            launch_batched_dim<2>(segs[i], d_jobs, wg_waves, n_wgs, tiles_per_pop, counter + i, claims, err, s);
        else
            launch_batched_dim<3>(segs[i], d_jobs, wg_waves, n_wgs, tiles_per_pop, counter + i, claims, err, s);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace rt
