// Level chains of the moving-medium line model.
//
//  * Velocity interpolation (Sect. 3.1): every cell of every level gets, per
//    direction class (one full grid, or one per orthant of directions as in
//    the quadrant-by-quadrant solution of Sect. 4.1), a velocity grid of n_v
//    nodes uniform over the projected velocities its MIP-0 voxels reach from
//    that class ([-V, V], V = max |v|, for the full grid), plus the mean
//    velocity vbar used to project the ray direction.  The node value of a
//    level-m cell is the average (log or linear mode) over its MIP-0 voxels of
//    eta, chi evaluated as if each voxel's projected velocity were the node
//    velocity.
//  * Core and Voigt (Sect. 3.2): eta*, chi* and the background averaged in
//    the stored-value mode, damping, 1/Doppler width and velocity linearly.
//
// The vbar and Core-and-Voigt chains average children level by level in
// the fixed pairwise order of the level statistics (x pairs, then y, then z).
// Velocity-node values are FP32 sums over the cell's voxels (values only).
#include "common.h"
#include "profile.h"

#include <type_traits>

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

// ------------------------------------------------------ velocity grids
// Projected-velocity range of one voxel over the directions of class q.  Full
// grid (n_vclass = 1): [-|v|, |v|].  Orthant q (bit a set <=> w_a < 0): with
// b_a = +-v_a signed by the orthant, u = sum_a b_a |w_a| over non-negative unit
// vectors, whose maximum is the length of the positive part of b (or, with no
// positive component, the largest b_a, on an axis) and whose minimum is minus
// the length of the negative part (or the smallest b_a).
template <int D>
__device__ __forceinline__ void voxel_vrange(const double* v, int q, int n_vclass, double& lo, double& hi)
{
    if (n_vclass == 1) {
        double s2 = 0.0;
        for (int a = 0; a < D; ++a) s2 += v[a] * v[a];
        hi = sqrt(s2);
        lo = -hi;
        return;
    }
    double pos = 0.0, neg = 0.0, bmax = -1e300, bmin = 1e300;
    bool any_pos = false, any_neg = false;
    for (int a = 0; a < D; ++a) {
        const double b = ((q >> a) & 1) ? -v[a] : v[a];
        if (b > 0.0) {
            pos += b * b;
            any_pos = true;
        }
        if (b < 0.0) {
            neg += b * b;
            any_neg = true;
        }
        bmax = fmax(bmax, b);
        bmin = fmin(bmin, b);
    }
    hi = any_pos ? sqrt(pos) : bmax;
    lo = any_neg ? -sqrt(neg) : bmin;
}

// Trace record of a cell for one class: node coordinate f = g . w + off.
template <int D>
__device__ __forceinline__ float4 vgrid_rec(const double* vb, double lo, double hi, int n_v)
{
    if (!(hi > lo)) return make_float4(0.f, 0.f, 0.f, 0.f);
    const double s = (double)(n_v - 1) / (hi - lo);
    return make_float4((float)(vb[0] * s), (float)(vb[1] * s), D > 2 ? (float)(vb[2] * s) : 0.f, (float)(-lo * s));
}

// One workgroup per active brick, one thread per MIP-0 voxel; the classes are
// taken one after the other.  LDS per cell: vbar[D] (FP64 means of the
// children in the pairwise order), then the class's (lo, hi) (min / max over
// the children).
template <int D>
__global__ void k_vgrid(Geo g, Inputs in, SceneBufs bufs, int n_v, int n_vclass)
{
    extern __shared__ double lds[];
    constexpr int stride = D + 2;
    const int slot = blockIdx.x, tid = threadIdx.x;
    const int blk = bufs.active_list[slot];
    const long long ncell_all = (long long)gridDim.x * g.cells;  // = n_active cells: one class's record count
    const long long rec = (long long)slot * g.cells;
    long long v;
    voxel_of(g, blk, tid, D, v);
    for (int q = 0; q < n_vclass; ++q) {
        double* s0 = lds + (size_t)stride * tid;
        for (int a = 0; a < D; ++a) s0[a] = in.vel[(long long)a * in.nvox + v];
        double lo, hi;
        voxel_vrange<D>(s0, q, n_vclass, lo, hi);
        s0[D] = lo;
        s0[D + 1] = hi;
        bufs.vgrid[q * ncell_all + rec + tid] = vgrid_rec<D>(s0, lo, hi, n_v);
        bufs.vrange[q * ncell_all + rec + tid] = make_float2((float)lo, (float)hi);
        __syncthreads();
        for (int m = 1; m < g.n_levels; ++m) {
            const int side = g.B >> m;
            const int ncell = D == 2 ? side * side : side * side * side;
            if (tid < ncell) {
                int idx[8];
                children<D>(tid, side, idx);
                const double* sc = lds + (size_t)stride * g.lvl_off[m - 1];
                double* so = lds + (size_t)stride * (g.lvl_off[m] + tid);
                double qq[8];
                for (int a = 0; a < D; ++a) {
                    for (int j = 0; j < (1 << D); ++j) qq[j] = sc[stride * idx[j] + a];
                    so[a] = tsum<D>(qq) / (1 << D);
                }
                double clo = 1e300, chi = -1e300;
                for (int j = 0; j < (1 << D); ++j) {
                    clo = fmin(clo, sc[stride * idx[j] + D]);
                    chi = fmax(chi, sc[stride * idx[j] + D + 1]);
                }
                so[D] = clo;
                so[D + 1] = chi;
                const long long o = q * ncell_all + rec + g.lvl_off[m] + tid;
                bufs.vgrid[o] = vgrid_rec<D>(so, clo, chi, n_v);
                bufs.vrange[o] = make_float2((float)clo, (float)chi);
            }
            __syncthreads();
        }
    }
}

hipError_t launch_vgrid(const Geo& g, const Inputs& in, const SceneBufs& b, int n_active, int n_v, int n_vclass,
                        hipStream_t s)
{
    if (n_active == 0) return hipSuccess;
    size_t shm = sizeof(double) * (size_t)(g.dim + 2) * (size_t)g.cells;
    if (g.dim == 2) hipLaunchKernelGGL(k_vgrid<2>, dim3(n_active), dim3(g.bvox), shm, s, g, in, b, n_v, n_vclass);
    else hipLaunchKernelGGL(k_vgrid<3>, dim3(n_active), dim3(g.bvox), shm, s, g, in, b, n_v, n_vclass);
    return hipGetLastError();
}

// ------------------------------------------------------ velocity node values
// One workgroup per (active brick, direction class); one thread per (level
// cell, node) item.  The workgroup first stages the brick's voxel inputs in
// LDS ([voxel][eta_bg, chi_bg, then eta*, chi*, a, 1/dlD per line]); each
// thread then walks its cell's MIP-0 voxels, evaluates eta, chi at the node
// velocity for all 8 batch wavelengths and accumulates them (ln values in log
// mode) in registers, and writes the item's record: 64 bytes in FP32, or 32
// bytes rounded to nearest even in BF16 / FP16 (packed at half the stride in
// the same buffer).  Values, not decisions: FP32 sums.  (The 41 node items of
// a cell read the same voxels, so the LDS reads broadcast; read from global
// memory, every voxel step waited on a dependent load.)
__device__ __forceinline__ unsigned enc_bits(__hip_bfloat16, float v)
{
    return __bfloat16_as_ushort(Codec<__hip_bfloat16>::enc(v));
}
__device__ __forceinline__ unsigned enc_bits(__half, float v) { return __half_as_ushort(Codec<__half>::enc(v)); }

// PROF: the line profile (Gaussian or Voigt) and NL: the lines the loops are unrolled for (2, or kMaxLines),
// both fixed per launch, so the per-voxel loop has no branch on either.
template <int D, typename T, int PROF, int NL>
__global__ void __launch_bounds__(256) k_velinterp_nodes2(Geo g, Inputs in, SceneBufs bufs, LamBatch lb, int n_v,
                                                          float ds0, int avg_mode)
{
    const int slot = blockIdx.x, q_cls = blockIdx.y;
    const long long ncell_all = (long long)gridDim.x * g.cells;
    const int blk = bufs.active_list[slot];
    const int B = g.B;
    const int bc0 = blk % g.nb[0], bc1 = (blk / g.nb[0]) % g.nb[1], bc2 = blk / (g.nb[0] * g.nb[1]);
    const bool logm = avg_mode == RT_AVG_LOG;
    const int total = g.cells * n_v;
    float lam_dl[kLam][kMaxLines];
    float k0[kMaxLines];
    for (int k = 0; k < kMaxLines; ++k) {
        k0[k] = (float)(lb.lam0[k] / kCkms);
        for (int l = 0; l < kLam; ++l) lam_dl[l][k] = (float)(lb.lam[l] - lb.lam0[k]);
    }
    extern __shared__ float sv[];
    const int nper = 2 + 4 * lb.n_lines;
    for (int i = threadIdx.x; i < g.bvox; i += blockDim.x) {
        const int ix = i % B, iy = (i / B) % B, iz = D > 2 ? i / (B * B) : 0;
        const long long v = (long long)(bc0 * B + ix) +
                            (long long)g.n[0] * ((long long)(bc1 * B + iy) + (long long)g.n[1] * (bc2 * B + iz));
        float* o = sv + i * nper;
        o[0] = in.eta_bg[v];
        o[1] = in.chi_bg[v];
        for (int k = 0; k < lb.n_lines; ++k) {
            const long long ok = (long long)k * in.nvox + v;
            o[2 + 4 * k] = in.eta_star[ok];
            o[3 + 4 * k] = in.chi_star[ok];
            o[4 + 4 * k] = in.damp[ok];
            o[5 + 4 * k] = in.inv_dld[ok];
        }
    }
    __syncthreads();
    for (int item = threadIdx.x; item < total; item += blockDim.x) {
        // items ordered coarse level first so the long ones start early
        int rem = item, m = g.n_levels - 1;
        for (; m > 0; --m) {
            int nc = g.lvl_off[m + 1] - g.lvl_off[m];
            if (rem < nc * n_v) break;
            rem -= nc * n_v;
        }
        // inside a level, cells fastest: the lanes of a wave write adjacent records of one node plane
        const int ncm = g.lvl_off[m + 1] - g.lvl_off[m];
        const int kn = rem / ncm, cell = rem - kn * ncm;
        const int side = B >> m, size = 1 << m;
        const int cx = cell % side, cy = (cell / side) % side, cz = D > 2 ? cell / (side * side) : 0;
        const long long rec = q_cls * ncell_all + (long long)slot * g.cells + g.lvl_off[m] + cell;
        const float2 vr = bufs.vrange[rec];
        const float uk = vr.y > vr.x ? vr.x + (vr.y - vr.x) * (float)kn / (float)(n_v - 1) : vr.x;
        float ae[kLam], ac[kLam];
#pragma unroll
        for (int l = 0; l < kLam; ++l) ae[l] = ac[l] = 0.f;
        const int nvx = D > 2 ? size * size * size : size * size;
        for (int q = 0; q < nvx; ++q) {
            int qx = q & (size - 1), qy = (q >> m) & (size - 1), qz = D > 2 ? q >> (2 * m) : 0;
            const float* pv = sv + ((cx * size + qx) + B * ((cy * size + qy) + B * (cz * size + qz))) * nper;
            float eb = pv[0], cb = pv[1];
            float es[NL], cs[NL], a0[NL], idl[NL];
#pragma unroll
            for (int k = 0; k < NL; ++k) {
                const bool on = k < lb.n_lines;
                es[k] = on ? pv[2 + 4 * k] : 0.f;
                cs[k] = on ? pv[3 + 4 * k] : 0.f;
                a0[k] = on ? pv[4 + 4 * k] : 0.f;
                idl[k] = on ? pv[5 + 4 * k] : 0.f;
            }
#pragma unroll
            for (int l = 0; l < kLam; ++l) {
                float ee = eb, cc = cb;
#pragma unroll
                for (int k = 0; k < NL; ++k) {
                    if (k >= lb.n_lines) break;
                    float x = fmaf(k0[k], uk, lam_dl[l][k]) * idl[k];
                    float phi = line_shape(PROF, x, a0[k], lb.lam[l], lb.lam0[k], idl[k]);
                    ee = fmaf(es[k], phi, ee);
                    cc = fmaf(cs[k], phi, cc);
                }
                if (m > 0 && logm) {
                    float se = ee * ds0, sc = cc * ds0;
                    ee = __logf(se > 1e-37f ? se : 1e-37f);
                    cc = __logf(sc > 1e-37f ? sc : 1e-37f);
                }
                ae[l] += ee;
                ac[l] += cc;
            }
        }
        const float inv = 1.0f / (float)nvx;
        float r[2 * kLam];
#pragma unroll
        for (int l = 0; l < kLam; ++l) {
            float oe = ae[l] * inv, oc = ac[l] * inv;
            if (m > 0 && logm) {
                oe = __expf(oe) / ds0;
                oc = __expf(oc) / ds0;
            }
            r[2 * l] = oe;
            r[2 * l + 1] = oc;
        }
        // node-major inside a brick: [class][slot][node][cell], so that neighbouring cells' records at one node
        // are adjacent (rays of a wave and consecutive cells of a ray mostly take the same node)
        const long long o = (((long long)q_cls * gridDim.x + slot) * n_v * g.cells + (long long)kn * g.cells +
                             g.lvl_off[m] + cell) * (kLam * 2);  // in elements of T
        if constexpr (std::is_same<T, float>::value) {
            float4* out = (float4*)(bufs.vnodes + o);
#pragma unroll
            for (int q = 0; q < kLam / 2; ++q) out[q] = make_float4(r[4 * q], r[4 * q + 1], r[4 * q + 2], r[4 * q + 3]);
        } else {
            uint4* out = (uint4*)((T*)bufs.vnodes + o);
            unsigned wd[kLam];
#pragma unroll
            for (int q = 0; q < kLam; ++q) wd[q] = enc_bits(T(), r[2 * q]) | (enc_bits(T(), r[2 * q + 1]) << 16);
#pragma unroll
            for (int q = 0; q < kLam / 4; ++q) out[q] = make_uint4(wd[4 * q], wd[4 * q + 1], wd[4 * q + 2], wd[4 * q + 3]);
        }
    }
}

template <int D, int PROF, int NL>
static void launch_nodes_typed(dim3 grid, size_t shm, const Geo& g, const Inputs& in, const SceneBufs& b,
                               const LamBatch& lb, int n_v, float ds0, int avg_mode, int storage, hipStream_t s)
{
    if (storage == RT_F32)
        hipLaunchKernelGGL((k_velinterp_nodes2<D, float, PROF, NL>), grid, dim3(256), shm, s, g, in, b, lb, n_v, ds0,
                           avg_mode);
    else if (storage == RT_BF16)
        hipLaunchKernelGGL((k_velinterp_nodes2<D, __hip_bfloat16, PROF, NL>), grid, dim3(256), shm, s, g, in, b, lb,
                           n_v, ds0, avg_mode);
    else
        hipLaunchKernelGGL((k_velinterp_nodes2<D, __half, PROF, NL>), grid, dim3(256), shm, s, g, in, b, lb, n_v, ds0,
                           avg_mode);
}

template <int D>
static void launch_nodes_dim(const Geo& g, const Inputs& in, const SceneBufs& b, int n_active, const LamBatch& lb,
                             int n_v, int n_vclass, float ds0, int avg_mode, int storage, hipStream_t s)
{
    const dim3 grid(n_active, n_vclass);
    const size_t shm = sizeof(float) * (size_t)g.bvox * (size_t)(2 + 4 * lb.n_lines);  // <= 512 x 18 floats
    const bool two = lb.n_lines <= 2;
    if (lb.profile == RT_PROFILE_GAUSS) {
        if (two) launch_nodes_typed<D, RT_PROFILE_GAUSS, 2>(grid, shm, g, in, b, lb, n_v, ds0, avg_mode, storage, s);
        else launch_nodes_typed<D, RT_PROFILE_GAUSS, kMaxLines>(grid, shm, g, in, b, lb, n_v, ds0, avg_mode, storage, s);
    } else {
        if (two) launch_nodes_typed<D, RT_PROFILE_VOIGT, 2>(grid, shm, g, in, b, lb, n_v, ds0, avg_mode, storage, s);
        else launch_nodes_typed<D, RT_PROFILE_VOIGT, kMaxLines>(grid, shm, g, in, b, lb, n_v, ds0, avg_mode, storage, s);
    }
}

hipError_t launch_velinterp_nodes(const Geo& g, const Inputs& in, const SceneBufs& b, int n_active,
                                  const LamBatch& lb, int n_v, int n_vclass, double ds0, int avg_mode, int storage,
                                  hipStream_t s)
{
    if (n_active == 0) return hipSuccess;
    if (g.dim == 2) launch_nodes_dim<2>(g, in, b, n_active, lb, n_v, n_vclass, (float)ds0, avg_mode, storage, s);
    else launch_nodes_dim<3>(g, in, b, n_active, lb, n_v, n_vclass, (float)ds0, avg_mode, storage, s);
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

namespace rt {

// Reduced-precision copy of the Core-and-Voigt chain (round to nearest even).
template <typename T>
__global__ void k_cav_encode(const float* cav, T* out, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = Codec<T>::enc(cav[i]);
}

hipError_t launch_cav_encode(const float* cav, void* out, long long n, int storage, hipStream_t s)
{
    if (n <= 0) return hipSuccess;  // no active block
    const unsigned nb = (unsigned)((n + 255) / 256);
    if (storage == RT_BF16)
        hipLaunchKernelGGL(k_cav_encode<__hip_bfloat16>, dim3(nb), dim3(256), 0, s, cav, (__hip_bfloat16*)out, n);
    else
        hipLaunchKernelGGL(k_cav_encode<__half>, dim3(nb), dim3(256), 0, s, cav, (__half*)out, n);
    return hipGetLastError();
}

}  // namespace rt
