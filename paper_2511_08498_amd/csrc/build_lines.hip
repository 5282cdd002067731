// Level chains of the moving-medium line model.
//
//  * Velocity interpolation (Sect. 3.1): every cell of every level gets a
//    velocity grid of n_v nodes uniform in [-V, V], V = max |v| over its MIP-0
//    voxels, plus the mean velocity vbar used to project the ray direction.
//    The node value of a level-m cell is the average (log or linear mode) over
//    its MIP-0 voxels of eta, chi evaluated as if each voxel's projected
//    velocity were the node velocity.
//  * Core and Voigt (Sect. 3.2): eta*, chi* and the background averaged in
//    the stored-value mode, damping, 1/Doppler width and velocity linearly.
//
// Averages over a cell's voxels follow the fixed pairwise order of the level
// statistics (x pairs, then y, then z, level by level).
#include "common.h"
#include "profile.h"

namespace rt {

__device__ __forceinline__ void voxel_of(const Geo& g, int blk, int tid, int D, long long& v)
{
    int bc0 = blk % g.nb[0], bc1 = (blk / g.nb[0]) % g.nb[1], bc2 = blk / (g.nb[0] * g.nb[1]);
    int lx = tid & (g.B - 1), ly = (tid >> g.log2B) & (g.B - 1), lz = D > 2 ? (tid >> (2 * g.log2B)) : 0;
    v = (long long)(bc0 * g.B + lx) + (long long)g.n[0] * ((long long)(bc1 * g.B + ly) + (long long)g.n[1] * (bc2 * g.B + lz));
}

template <int D>
__device__ __forceinline__ void children(int tid, int side, int* idx)
{
    const int sidec = 2 * side;
    int cx = tid % side, cy = (tid / side) % side, cz = D > 2 ? tid / (side * side) : 0;
    int k = 0;
    for (int dz = 0; dz < (D > 2 ? 2 : 1); ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) idx[k++] = (2 * cx + dx) + sidec * ((2 * cy + dy) + sidec * (2 * cz + dz));
}

template <int D, typename F>
__device__ __forceinline__ F tsum(const F* q)
{
    if (D == 2) return (q[0] + q[1]) + (q[2] + q[3]);
    return ((q[0] + q[1]) + (q[2] + q[3])) + ((q[4] + q[5]) + (q[6] + q[7]));
}

// ------------------------------------------------------ velocity grid (V, vbar)
template <int D>
__global__ void k_vgrid(Geo g, Inputs in, SceneBufs bufs)
{
    extern __shared__ double lds[];  // per cell: V, vx, vy, vz
    const int slot = blockIdx.x, tid = threadIdx.x;
    const int blk = bufs.active_list[slot];
    long long v;
    voxel_of(g, blk, tid, D, v);
    double vv[3] = {0, 0, 0}, q = 0.0;
    for (int a = 0; a < D; ++a) {
        vv[a] = in.vel[(long long)a * in.nvox + v];
        q += vv[a] * vv[a];
    }
    double* s0 = lds + 4 * tid;
    s0[0] = sqrt(q);
    s0[1] = vv[0];
    s0[2] = vv[1];
    s0[3] = vv[2];
    const long long rec = (long long)slot * g.cells;
    bufs.vgrid[rec + tid] = make_float4((float)s0[0], (float)vv[0], (float)vv[1], (float)vv[2]);
    __syncthreads();
    for (int m = 1; m < g.n_levels; ++m) {
        const int side = g.B >> m;
        const int ncell = D == 2 ? side * side : side * side * side;
        if (tid < ncell) {
            int idx[8];
            children<D>(tid, side, idx);
            const double* sc = lds + 4 * g.lvl_off[m - 1];
            double* so = lds + 4 * (g.lvl_off[m] + tid);
            double qq[8];
            double V = 0.0;
            for (int j = 0; j < (1 << D); ++j) V = fmax(V, sc[4 * idx[j]]);
            so[0] = V;
            for (int f = 1; f < 4; ++f) {
                for (int j = 0; j < (1 << D); ++j) qq[j] = sc[4 * idx[j] + f];
                so[f] = tsum<D>(qq) / (1 << D);
            }
            bufs.vgrid[rec + g.lvl_off[m] + tid] = make_float4((float)so[0], (float)so[1], (float)so[2], (float)so[3]);
        }
        __syncthreads();
    }
}

hipError_t launch_vgrid(const Geo& g, const Inputs& in, const SceneBufs& b, int n_active, hipStream_t s)
{
    if (n_active == 0) return hipSuccess;
    size_t shm = sizeof(double) * 4 * (size_t)g.cells;
    if (g.dim == 2) hipLaunchKernelGGL(k_vgrid<2>, dim3(n_active), dim3(g.bvox), shm, s, g, in, b);
    else hipLaunchKernelGGL(k_vgrid<3>, dim3(n_active), dim3(g.bvox), shm, s, g, in, b);
    return hipGetLastError();
}

// ------------------------------------------------------ velocity node values
// Block (slot, level m); thread = MIP-0 voxel of the brick.  For every batch
// wavelength and node, each voxel evaluates eta, chi at the node velocity of
// its level-m cell; the brick is then reduced m times in the pairwise order.
template <int D>
__global__ void k_velinterp_nodes(Geo g, Inputs in, SceneBufs bufs, LamBatch lb, int n_v, double ds0, int avg_mode)
{
    extern __shared__ float fl[];  // [2][bvox] working values, then reduced in place
    const int slot = blockIdx.x, m = blockIdx.y, tid = threadIdx.x;
    const int blk = bufs.active_list[slot];
    const int B = g.B, bvox = g.bvox;
    long long v;
    voxel_of(g, blk, tid, D, v);
    // level-m cell of this voxel
    int lx = tid & (B - 1), ly = (tid >> g.log2B) & (B - 1), lz = D > 2 ? (tid >> (2 * g.log2B)) : 0;
    const int side = B >> m;
    int cell = (lx >> m) + side * ((ly >> m) + side * (lz >> m));
    const long long rec = (long long)slot * g.cells + g.lvl_off[m];
    const float Vc = bufs.vgrid[rec + cell].x;
    const int ncell = D == 2 ? side * side : side * side * side;
    const bool logm = avg_mode == RT_AVG_LOG;
    float* fe = fl;
    float* fc = fl + bvox;
    for (int l = 0; l < lb.nl; ++l) {
        for (int kn = 0; kn < n_v; ++kn) {
            float uk = Vc > 0.f ? -Vc + 2.0f * Vc * (float)kn / (float)(n_v - 1) : 0.f;
            float ee = in.eta_bg[v], cc = in.chi_bg[v];
            for (int k = 0; k < lb.n_lines; ++k) {
                long long o = (long long)k * in.nvox + v;
                float idl = in.inv_dld[o];
                float x = ((float)(lb.lam[l] - lb.lam0[k]) + (float)(lb.lam0[k] / kCkms) * uk) * idl;
                float phi = line_shape(lb.profile, x, in.damp[o], lb.lam[l], lb.lam0[k], idl);
                ee += in.eta_star[o] * phi;
                cc += in.chi_star[o] * phi;
            }
            if (m > 0 && logm) {
                float se = ee * (float)ds0, sc = cc * (float)ds0;
                ee = __logf(se > 1e-37f ? se : 1e-37f);
                cc = __logf(sc > 1e-37f ? sc : 1e-37f);
            }
            // pairwise reduction of the brick into level-m cells, level by level
            // (sub-level s holds (B >> s)^D values at the front of the array).
            fe[tid] = ee;
            fc[tid] = cc;
            __syncthreads();
            for (int s = 1; s <= m; ++s) {
                const int sd = B >> s;
                const int nc = D == 2 ? sd * sd : sd * sd * sd;
                float re = 0.f, rc = 0.f;
                if (tid < nc) {
                    int idx[8];
                    children<D>(tid, sd, idx);
                    float q[8];
                    for (int j = 0; j < (1 << D); ++j) q[j] = fe[idx[j]];
                    re = tsum<D>(q) / (float)(1 << D);
                    for (int j = 0; j < (1 << D); ++j) q[j] = fc[idx[j]];
                    rc = tsum<D>(q) / (float)(1 << D);
                }
                __syncthreads();
                if (tid < nc) {
                    fe[tid] = re;
                    fc[tid] = rc;
                }
                __syncthreads();
            }
            if (tid < ncell) {
                float oe = fe[tid], oc = fc[tid];
                if (m > 0 && logm) {
                    oe = __expf(oe) / (float)ds0;
                    oc = __expf(oc) / (float)ds0;
                }
                float* r = bufs.vnodes + (((rec + tid) * n_v + kn) * kLam + l) * 2;
                r[0] = oe;
                r[1] = oc;
            }
            __syncthreads();
        }
    }
}

hipError_t launch_velinterp_nodes(const Geo& g, const Inputs& in, const SceneBufs& b, int n_active,
                                  const LamBatch& lb, int n_v, double ds0, int avg_mode, hipStream_t s)
{
    if (n_active == 0) return hipSuccess;
    size_t shm = sizeof(float) * 2 * (size_t)g.bvox;
    dim3 grid((unsigned)n_active, (unsigned)g.n_levels);
    if (g.dim == 2) hipLaunchKernelGGL(k_velinterp_nodes<2>, grid, dim3(g.bvox), shm, s, g, in, b, lb, n_v, ds0, avg_mode);
    else hipLaunchKernelGGL(k_velinterp_nodes<3>, grid, dim3(g.bvox), shm, s, g, in, b, lb, n_v, ds0, avg_mode);
    return hipGetLastError();
}

// ------------------------------------------------------ Core-and-Voigt chain
// Per cell record: [line k: eta*, chi*, a, 1/dlD] ... [eta_bg, chi_bg, vx, vy] [vz, 0, 0, 0].
// LDS holds the FP64 averages of every field at every level.
template <int D>
__global__ void k_cav_chain(Geo g, Inputs in, SceneBufs bufs, int n_lines, double ds0, int avg_mode)
{
    extern __shared__ double lds[];
    const int nf = 4 * n_lines + 2 + D;   // fields per cell
    const int slot = blockIdx.x, tid = threadIdx.x;
    const int blk = bufs.active_list[slot];
    const int rec_f = cav_rec_floats(n_lines);
    long long v;
    voxel_of(g, blk, tid, D, v);
    const bool logm = avg_mode == RT_AVG_LOG;
    // field f is "log-averaged" when it is eta*, chi* or a background and the mode is LOG
    auto is_logf = [&](int f) { return logm && (f < 4 * n_lines ? (f & 3) < 2 : f < 4 * n_lines + 2); };
    double* s0 = lds + (size_t)nf * tid;
    for (int k = 0; k < n_lines; ++k) {
        long long o = (long long)k * in.nvox + v;
        s0[4 * k] = in.eta_star[o];
        s0[4 * k + 1] = in.chi_star[o];
        s0[4 * k + 2] = in.damp[o];
        s0[4 * k + 3] = in.inv_dld[o];
    }
    s0[4 * n_lines] = in.eta_bg[v];
    s0[4 * n_lines + 1] = in.chi_bg[v];
    for (int a = 0; a < D; ++a) s0[4 * n_lines + 2 + a] = in.vel[(long long)a * in.nvox + v];
    const long long rec = (long long)slot * g.cells;
    {
        float* o = bufs.cav + (rec + tid) * rec_f;
        for (int f = 0; f < rec_f; ++f) o[f] = 0.f;
        for (int f = 0; f < nf; ++f) o[f] = (float)s0[f];
    }
    // convert log-averaged fields to ln(q ds0) for the chain
    for (int f = 0; f < nf; ++f)
        if (is_logf(f)) {
            double q = s0[f] * ds0;
            s0[f] = log(q > 1e-300 ? q : 1e-300);
        }
    __syncthreads();
    for (int m = 1; m < g.n_levels; ++m) {
        const int side = g.B >> m;
        const int ncell = D == 2 ? side * side : side * side * side;
        if (tid < ncell) {
            int idx[8];
            children<D>(tid, side, idx);
            const double* sc = lds + (size_t)nf * g.lvl_off[m - 1];
            double* so = lds + (size_t)nf * (g.lvl_off[m] + tid);
            float* o = bufs.cav + (rec + g.lvl_off[m] + tid) * rec_f;
            for (int f = 0; f < rec_f; ++f) o[f] = 0.f;
            double q[8];
            for (int f = 0; f < nf; ++f) {
                for (int j = 0; j < (1 << D); ++j) q[j] = sc[(size_t)nf * idx[j] + f];
                double mval = tsum<D>(q) / (1 << D);
                so[f] = mval;
                o[f] = (float)(is_logf(f) ? exp(mval) / ds0 : mval);
            }
        }
        __syncthreads();
    }
}

hipError_t launch_cav_chain(const Geo& g, const Inputs& in, const SceneBufs& b, int n_active, int n_lines,
                            double ds0, int avg_mode, hipStream_t s)
{
    if (n_active == 0) return hipSuccess;
    const int nf = 4 * n_lines + 2 + g.dim;
    size_t shm = sizeof(double) * (size_t)nf * g.cells;
    if (g.dim == 2) hipLaunchKernelGGL(k_cav_chain<2>, dim3(n_active), dim3(g.bvox), shm, s, g, in, b, n_lines, ds0, avg_mode);
    else hipLaunchKernelGGL(k_cav_chain<3>, dim3(n_active), dim3(g.bvox), shm, s, g, in, b, n_lines, ds0, avg_mode);
    return hipGetLastError();
}

}  // namespace rt
