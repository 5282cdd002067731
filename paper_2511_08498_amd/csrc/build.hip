// Scene construction kernels: block classification, Morton-ordered slots
// (Sect. 2.3.1 offset table), the per-batch mip chain with the index of
// dispersion and VLM level selection (Sect. 2.1-2.2), state packing.
//
// This translation unit is compiled with -ffp-contract=off: the level
// statistics are FP64 sums in a fixed pairwise order (x pairs, then y, then z)
// so that block levels are reproducible to the last bit.
#include "common.h"
#include "profile.h"

namespace rt {

// ------------------------------------------------------------------ classify
__global__ void k_classify(Geo g, Inputs in, int model, int n_lam, int n_lines, int dense, uint8_t* active)
{
    const long long b = blockIdx.x;
    int bc[3] = {(int)(b % g.nb[0]), (int)((b / g.nb[0]) % g.nb[1]), (int)(b / ((long long)g.nb[0] * g.nb[1]))};
    int any = 0;
    if (dense) {
        any = 1;
    } else if (in.mask) {
        any = in.mask[b] != 0;
    } else {
        for (int i = threadIdx.x; i < g.bvox && !any; i += blockDim.x) {
            int lx = i & (g.B - 1), ly = (i >> g.log2B) & (g.B - 1), lz = g.dim > 2 ? (i >> (2 * g.log2B)) : 0;
            long long v = (long long)(bc[0] * g.B + lx) +
                          (long long)g.n[0] * ((long long)(bc[1] * g.B + ly) + (long long)g.n[1] * (bc[2] * g.B + lz));
            if (model == RT_MODEL_STATIC) {
                for (int l = 0; l < n_lam; ++l)
                    if (in.eta[(long long)l * in.nvox + v] != 0.f || in.chi[(long long)l * in.nvox + v] != 0.f) {
                        any = 1;
                        break;
                    }
            } else {
                if (in.eta_bg[v] != 0.f || in.chi_bg[v] != 0.f) any = 1;
                for (int l = 0; l < n_lines; ++l)
                    if (in.eta_star[(long long)l * in.nvox + v] != 0.f || in.chi_star[(long long)l * in.nvox + v] != 0.f)
                        any = 1;
            }
        }
    }
    any = __syncthreads_or(any);
    if (threadIdx.x == 0) active[b] = (uint8_t)(any ? 1 : 0);
}

hipError_t launch_classify(const Geo& g, const Inputs& in, int model, int n_lam, int n_lines, int dense,
                           uint8_t* active, hipStream_t s)
{
    hipLaunchKernelGGL(k_classify, dim3((unsigned)g.nblocks), dim3(256), 0, s, g, in, model, n_lam, n_lines, dense,
                       active);
    return hipGetLastError();
}

// ---------------------------------------------------------------- validate
// Counts input values that are negative or not finite (eta, chi, line
// strengths, damping, Doppler widths, background) or not finite (velocity).
__device__ __forceinline__ int bad_nonneg(float x) { return !(x >= 0.f && x <= 3.402823466e38f); }
__device__ __forceinline__ int bad_finite(float x) { return !(x >= -3.402823466e38f && x <= 3.402823466e38f); }

__global__ void k_validate(Inputs in, int model, int n_lam, int n_lines, int dim, unsigned long long* count)
{
    unsigned long long c = 0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < in.nvox; v += stride) {
        if (model == RT_MODEL_STATIC) {
            for (int l = 0; l < n_lam; ++l)
                c += bad_nonneg(in.eta[(long long)l * in.nvox + v]) + bad_nonneg(in.chi[(long long)l * in.nvox + v]);
        } else {
            for (int l = 0; l < n_lines; ++l) {
                const long long o = (long long)l * in.nvox + v;
                c += bad_nonneg(in.eta_star[o]) + bad_nonneg(in.chi_star[o]) + bad_nonneg(in.damp[o]) +
                     bad_nonneg(in.inv_dld[o]);
            }
            c += bad_nonneg(in.eta_bg[v]) + bad_nonneg(in.chi_bg[v]);
            for (int a = 0; a < dim; ++a) c += bad_finite(in.vel[(long long)a * in.nvox + v]);
        }
    }
    for (int o = 32; o > 0; o >>= 1) c += (unsigned long long)__shfl_xor((long long)c, o, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, c);
}

hipError_t launch_validate(const Inputs& in, int model, int n_lam, int n_lines, int dim, unsigned long long* count,
                           hipStream_t s)
{
    if (in.nvox <= 0) return hipSuccess;
    long long blocks = (in.nvox + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_validate, dim3((unsigned)blocks), dim3(256), 0, s, in, model, n_lam, n_lines, dim, count);
    return hipGetLastError();
}

// ------------------------------------------------------------------- slots
// One workgroup walks the Morton order in chunks of 1024 blocks and assigns
// each active block the next storage slot (exclusive prefix sum).
__global__ void __launch_bounds__(1024) k_slots(long long nb, const int32_t* morton, const uint8_t* active,
                                                int32_t* slot, int32_t* active_list, int32_t* n_active)
{
    __shared__ int wsum[16];
    __shared__ int base_s;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (tid == 0) base_s = 0;
    __syncthreads();
    for (long long c0 = 0; c0 < nb; c0 += 1024) {
        long long i = c0 + tid;
        int b = i < nb ? morton[i] : -1;
        int f = (b >= 0 && active[b]) ? 1 : 0;
        // inclusive scan inside the wave
        int x = f;
        for (int o = 1; o < 64; o <<= 1) {
            int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[wid] = x;
        __syncthreads();
        int off = 0;
        for (int w = 0; w < wid; ++w) off += wsum[w];
        int base = base_s;
        int excl = base + off + x - f;
        if (b >= 0) {
            slot[b] = f ? excl : -1;
            if (f) active_list[excl] = b;
        }
        __syncthreads();
        if (tid == 0) {
            int tot = 0;
            for (int w = 0; w < 16; ++w) tot += wsum[w];
            base_s = base + tot;
        }
        __syncthreads();
    }
    if (tid == 0) *n_active = base_s;
}

hipError_t launch_slots(const Geo& g, const int32_t* morton, const uint8_t* active, int32_t* slot,
                        int32_t* active_list, int32_t* n_active, hipStream_t s)
{
    hipLaunchKernelGGL(k_slots, dim3(1), dim3(1024), 0, s, g.nblocks, morton, active, slot, active_list, n_active);
    return hipGetLastError();
}

__global__ void k_fill_levels(long long nb, int8_t* levels)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nb) levels[i] = -1;
}

hipError_t launch_fill_levels(const Geo& g, int8_t* levels, hipStream_t s)
{
    unsigned blocks = (unsigned)((g.nblocks + 255) / 256);
    hipLaunchKernelGGL(k_fill_levels, dim3(blocks), dim3(256), 0, s, g.nblocks, levels);
    return hipGetLastError();
}

// ------------------------------------------------------------- mip chain
// Level statistics of one level-m cell from its 2^D children at level m-1
// (LDS, FP64): mean and population variance (two-pass) in the pairwise order.
__device__ inline double pair4(double a, double b, double c, double d) { return (a + b) + (c + d); }

template <int D>
__device__ inline double tree_sum(const double* q)
{
    if (D == 2) return pair4(q[0], q[1], q[2], q[3]);
    return pair4(q[0], q[1], q[2], q[3]) + pair4(q[4], q[5], q[6], q[7]);
}

struct Lvl0 {
    double xe, xc, le, lc;  // ln(eta ds0), ln(chi ds0), eta, chi
};

// MIP-0 value of voxel v for batch wavelength l: given (static model), or
// the line model with each line at projected velocity u = 0 (vrule 0: the rest
// frame used by velocity interpolation, Sect. 3.1) or at the shift within
// [-|v|, |v|] closest to the line core, u* = clamp(c (1 - lam/lam0)) (vrule 1:
// Core and Voigt, Sect. 3.2).  Evaluated in FP64 in the order of the defining
// expressions, x = (lam - lam0 (1 - u/c)) / dlD and eta = bg + sum (s eta*) phi
// (s = lam0/lam for Voigt lines, 1 for Gaussian ones), because these values
// decide the levels: a Gaussian line is exp(-x^2) in FP64, so a level test
// moves only where an index of dispersion lies within rounding of the
// threshold; a Voigt line takes the single-precision profile of the march
// (relative error below 1e-4), promoted.
__device__ inline void mip0_value(const Inputs& in, int model, int vrule, int dim, const LamBatch& lb,
                                  int lam_global, int l, long long v, double& e, double& c)
{
    if (model == RT_MODEL_STATIC) {
        e = in.eta[(long long)lam_global * in.nvox + v];
        c = in.chi[(long long)lam_global * in.nvox + v];
        return;
    }
    double ee = in.eta_bg[v], cc = in.chi_bg[v];
    double sp = 0.0;
    if (vrule == 1) {
        double q = 0.0;
        for (int a = 0; a < dim; ++a) {
            const double va = in.vel[(long long)a * in.nvox + v];
            q += va * va;
        }
        sp = sqrt(q);
    }
    const double lam = lb.lam[l];
    for (int k = 0; k < lb.n_lines; ++k) {
        const long long o = (long long)k * in.nvox + v;
        const double lam0 = lb.lam0[k];
        const double idl = in.inv_dld[o];
        double u = 0.0;
        if (vrule == 1) {
            u = kCkms * (1.0 - lam / lam0);
            if (u > sp) u = sp;
            if (u < -sp) u = -sp;
        }
        const double x = (lam - lam0 * (1.0 - u / kCkms)) * idl;
        double phi, sc;
        if (lb.profile == RT_PROFILE_GAUSS) {
            phi = exp(-x * x);
            sc = 1.0;
        } else {
            const double r = lam / lam0;
            phi = (double)voigt_h((float)(in.damp[o] * r * r), (float)x) * idl / 1.7724538509055160273;
            sc = lam0 / lam;
        }
        ee += sc * (double)in.eta_star[o] * phi;
        cc += sc * (double)in.chi_star[o] * phi;
    }
    e = ee;
    c = cc;
}

template <int D, typename T>
__global__ void k_build_static(Geo g, Inputs in, SceneBufs bufs, int model, int vrule, LamBatch lb, int lam_begin,
                               double ds0, double T_iod, double tau_thin, int cap, int avg_mode,
                               int write_values)
{
    extern __shared__ double lds[];
    __shared__ int pass_all[kMaxLevels];
    const int slot = blockIdx.x;
    const int blk = bufs.active_list[slot];
    const int tid = threadIdx.x;
    const int B = g.B, L = g.n_levels;
    int bc[3] = {blk % g.nb[0], (blk / g.nb[0]) % g.nb[1], blk / (g.nb[0] * g.nb[1])};
    int lx = tid & (B - 1), ly = (tid >> g.log2B) & (B - 1), lz = D > 2 ? (tid >> (2 * g.log2B)) : 0;
    long long v = (long long)(bc[0] * B + lx) +
                  (long long)g.n[0] * ((long long)(bc[1] * B + ly) + (long long)g.n[1] * (bc[2] * B + lz));
    T* vals = (T*)bufs.vals;
    const long long rec0 = (long long)slot * g.cells;
    int Lmax = L - 1;
    if (cap >= 0 && cap < Lmax) Lmax = cap;
    int lv_batch = 127;
    // LDS: level m occupies cells_m * 4 doubles starting at lvl_off[m] * 4.
    for (int l = 0; l < lb.nl; ++l) {
        double e, c;
        mip0_value(in, model, vrule, D, lb, lam_begin + l, l, v, e, c);
        if (write_values) {
            T* r = vals + ((rec0 + tid) * kLam + l) * 2;
            r[0] = Codec<T>::enc((float)e);
            r[1] = Codec<T>::enc((float)c);
        }
        double qe = e * ds0, qc = c * ds0;
        double* s0 = lds + 4 * tid;
        s0[0] = log(qe > 1e-300 ? qe : 1e-300);
        s0[1] = log(qc > 1e-300 ? qc : 1e-300);
        s0[2] = e;
        s0[3] = c;
        if (bufs.fstats && g.feat_level == 0)
            bufs.fstats[((long long)slot * g.bvox + tid) * kLam + l] =
                make_float4((float)s0[1], 0.f, (float)s0[0], 0.f);
        if (tid < kMaxLevels) pass_all[tid] = 1;
        __syncthreads();
        for (int m = 1; m < L; ++m) {
            const int side = B >> m, sidec = B >> (m - 1);
            const int ncell = D == 2 ? side * side : side * side * side;
            if (tid < ncell) {
                int cx = tid % side, cy = (tid / side) % side, cz = D > 2 ? tid / (side * side) : 0;
                const double* sc = lds + 4 * g.lvl_off[m - 1];
                int idx[8];
                int k = 0;
                for (int dz = 0; dz < (D > 2 ? 2 : 1); ++dz)
                    for (int dy = 0; dy < 2; ++dy)
                        for (int dx = 0; dx < 2; ++dx)
                            idx[k++] = (2 * cx + dx) + sidec * ((2 * cy + dy) + sidec * (2 * cz + dz));
                constexpr int nch = 1 << D;
                double q[8];
                double st[4];  // mean_e, mean_c, lin_e, lin_c
                double var[2];
                for (int f = 0; f < 2; ++f) {
                    for (int j = 0; j < nch; ++j) q[j] = sc[4 * idx[j] + f];
                    double mean = tree_sum<D>(q) / nch;
                    for (int j = 0; j < nch; ++j) {
                        double d = sc[4 * idx[j] + f] - mean;
                        q[j] = d * d;
                    }
                    var[f] = tree_sum<D>(q) / nch;
                    st[f] = mean;
                }
                for (int f = 2; f < 4; ++f) {
                    for (int j = 0; j < nch; ++j) q[j] = sc[4 * idx[j] + f];
                    st[f] = tree_sum<D>(q) / nch;
                }
                // stored values: geometric (LOG) or arithmetic (LINEAR) mean; slots 2 and 3
                // always carry the arithmetic means of the MIP-0 values the cell covers
                double le, lc;
                if (avg_mode == RT_AVG_LOG) {
                    le = exp(st[0]) / ds0;
                    lc = exp(st[1]) / ds0;
                } else {
                    le = st[2];
                    lc = st[3];
                }
                double* so = lds + 4 * (g.lvl_off[m] + tid);
                so[0] = st[0];
                so[1] = st[1];
                so[2] = st[2];
                so[3] = st[3];
                double iod_e = var[0] == 0.0 ? 0.0 : (st[0] == 0.0 ? __builtin_inf() : fabs(var[0] / st[0]));
                double iod_c = var[1] == 0.0 ? 0.0 : (st[1] == 0.0 ? __builtin_inf() : fabs(var[1] / st[1]));
                // thin bypass on the cell's optical side with the box-filtered chi
                int thin = st[3] * (double)(1 << m) * ds0 < tau_thin;
                int pass = thin || (iod_e <= T_iod && iod_c <= T_iod);
                if (!pass) pass_all[m] = 0;
                if (bufs.fstats && m == g.feat_level)
                    bufs.fstats[((long long)slot * ncell + tid) * kLam + l] =
                        make_float4((float)st[1], (float)var[1], (float)st[0], (float)var[0]);
                if (write_values) {
                    T* r = vals + ((rec0 + g.lvl_off[m] + tid) * kLam + l) * 2;
                    r[0] = Codec<T>::enc((float)le);
                    r[1] = Codec<T>::enc((float)lc);
                }
            }
            __syncthreads();
        }
        int lv = 0;
        for (int m = 1; m <= Lmax; ++m) {
            if (!pass_all[m]) break;
            lv = m;
        }
        lv_batch = lv < lv_batch ? lv : lv_batch;
        __syncthreads();
    }
    if (tid == 0) bufs.levels[blk] = (int8_t)(lb.nl > 0 ? lv_batch : 0);
}

hipError_t launch_build_static(const Geo& g, const Inputs& in, const SceneBufs& b, int n_active, int model,
                               int vrule, const LamBatch& lb, int lam_begin, double ds0, double T, double tau_thin,
                               int cap, int avg_mode, int storage, int write_values, hipStream_t s)
{
    if (n_active == 0) return hipSuccess;
    size_t shm = sizeof(double) * 4 * (size_t)g.cells;
    dim3 grid((unsigned)n_active), block((unsigned)g.bvox);
#define RT_LAUNCH_BS(DD, TT)                                                                              \
    hipLaunchKernelGGL((k_build_static<DD, TT>), grid, block, shm, s, g, in, b, model, vrule, lb, lam_begin, ds0, \
                       T, tau_thin, cap, avg_mode, write_values)
    if (g.dim == 2) {
        if (storage == RT_F32) RT_LAUNCH_BS(2, float);
        else if (storage == RT_BF16) RT_LAUNCH_BS(2, __hip_bfloat16);
        else RT_LAUNCH_BS(2, __half);
    } else {
        if (storage == RT_F32) RT_LAUNCH_BS(3, float);
        else if (storage == RT_BF16) RT_LAUNCH_BS(3, __hip_bfloat16);
        else RT_LAUNCH_BS(3, __half);
    }
#undef RT_LAUNCH_BS
    return hipGetLastError();
}

// ---------------------------------------------------------- prefiltering
// Prefiltered merged cells (Sect. 5.1): for a level-m cell and a signed axis
// k = 2a + (propagation towards -a), every row of MIP-0 voxels parallel to a is
// solved exactly from I = 0 at its entry face, voxel by voxel in the direction
// of propagation; the cell keeps the homogeneous cell of its side with the
// same row-averaged transfer (Ibar, Tbar = mean T_row, 1 - Tbar = mean(1 - T_row),
// each summed on its own): chi = -ln(Tbar) / side (from 1 - Tbar below 1/2, from
// Tbar above, the mean row optical depth when every row's T underflows),
// eta = Ibar chi / (1 - Tbar) (Ibar / side when Tbar = 1).  FP64 from the
// MIP-0 values (the same values as the level test),
// rows summed in a fixed order (lowest cross axis fastest).  One workgroup per
// active block, one thread per MIP-0 voxel; the (cell, axis) pairs of a level
// are shared out over the threads.
template <int D, typename T>
__global__ void k_build_prefilter(Geo g, Inputs in, SceneBufs bufs, int model, LamBatch lb, int lam_begin, double ds0)
{
    extern __shared__ double lds[];
    constexpr int K = 2 * D;
    const int slot = blockIdx.x;
    const int blk = bufs.active_list[slot];
    const int tid = threadIdx.x;
    const int B = g.B, L = g.n_levels;
    const int bc[3] = {blk % g.nb[0], (blk / g.nb[0]) % g.nb[1], blk / (g.nb[0] * g.nb[1])};
    const int lx = tid & (B - 1), ly = (tid >> g.log2B) & (B - 1), lz = D > 2 ? (tid >> (2 * g.log2B)) : 0;
    const long long v = (long long)(bc[0] * B + lx) +
                        (long long)g.n[0] * ((long long)(bc[1] * B + ly) + (long long)g.n[1] * (bc[2] * B + lz));
    double* le = lds;
    double* lc = lds + g.bvox;
    T* pf = (T*)bufs.pf;
    const long long rec0 = (long long)slot * g.cells;
    for (int l = 0; l < lb.nl; ++l) {
        double e, c;
        mip0_value(in, model, 0, D, lb, lam_begin + l, l, v, e, c);
        le[tid] = e;
        lc[tid] = c;
        __syncthreads();
        for (int m = 1; m < L; ++m) {
            const int side = 1 << m, ncs = B >> m;
            const int ncell = D == 2 ? ncs * ncs : ncs * ncs * ncs;
            for (int task = tid; task < ncell * K; task += blockDim.x) {
                const int ci = task / K, k = task - ci * K;
                const int a = k >> 1, neg = k & 1;
                const int b0 = a == 0 ? 1 : 0;                    // cross axes, lowest first
                const int b1 = D > 2 ? (a == 2 ? 1 : 2) : -1;
                const int corner[3] = {(ci % ncs) * side, ((ci / ncs) % ncs) * side, D > 2 ? (ci / (ncs * ncs)) * side : 0};
                const int e1 = b1 >= 0 ? side : 1;
                double sumI = 0.0, sumA = 0.0, sumT = 0.0, sumTau = 0.0;
                for (int r1 = 0; r1 < e1; ++r1)
                    for (int r0 = 0; r0 < side; ++r0) {
                        double I = 0.0, tau_row = 0.0;
                        for (int j = 0; j < side; ++j) {
                            int p[3] = {corner[0], corner[1], corner[2]};
                            p[b0] += r0;
                            if (b1 >= 0) p[b1] += r1;
                            p[a] += neg ? side - 1 - j : j;  // entry face first
                            const int q = p[0] + B * (p[1] + B * p[2]);
                            const double tau = lc[q] * ds0;
                            if (tau == 0.0) I += le[q] * ds0;
                            else I = I * exp(-tau) + (le[q] / lc[q]) * (-expm1(-tau));
                            tau_row += tau;
                        }
                        sumI += I;
                        sumA += -expm1(-tau_row);
                        sumT += exp(-tau_row);
                        sumTau += tau_row;
                    }
                const double rows = (double)side * (double)e1;
                const double Ibar = sumI / rows, absorbed = sumA / rows, Tbar = sumT / rows, Lside = side * ds0;
                double ce = 0.0, ee;
                if (absorbed > 0.0) {
                    const double tau_eff = absorbed < 0.5 ? -log1p(-absorbed) : (Tbar > 0.0 ? -log(Tbar) : sumTau / rows);
                    ce = tau_eff / Lside;
                    ee = Ibar * tau_eff / (absorbed * Lside);
                } else {
                    ee = Ibar / Lside;
                }
                T* r = pf + (((rec0 + g.lvl_off[m] + ci) * K + k) * kLam + l) * 2;
                r[0] = Codec<T>::enc((float)ee);
                r[1] = Codec<T>::enc((float)ce);
            }
        }
        __syncthreads();
    }
}

hipError_t launch_build_prefilter(const Geo& g, const Inputs& in, const SceneBufs& b, int n_active, int model,
                                  const LamBatch& lb, int lam_begin, double ds0, int storage, hipStream_t s)
{
    if (n_active == 0 || g.n_levels < 2) return hipSuccess;
    const size_t shm = sizeof(double) * 2 * (size_t)g.bvox;
    const dim3 grid((unsigned)n_active), block((unsigned)g.bvox);
#define RT_LAUNCH_PF(DD, TT) \
    hipLaunchKernelGGL((k_build_prefilter<DD, TT>), grid, block, shm, s, g, in, b, model, lb, lam_begin, ds0)
    if (g.dim == 2) {
        if (storage == RT_F32) RT_LAUNCH_PF(2, float);
        else if (storage == RT_BF16) RT_LAUNCH_PF(2, __hip_bfloat16);
        else RT_LAUNCH_PF(2, __half);
    } else {
        if (storage == RT_F32) RT_LAUNCH_PF(3, float);
        else if (storage == RT_BF16) RT_LAUNCH_PF(3, __hip_bfloat16);
        else RT_LAUNCH_PF(3, __half);
    }
#undef RT_LAUNCH_PF
    return hipGetLastError();
}

// ------------------------------------------------------------------ states
__global__ void k_pack_states(long long nb, int nw, const int8_t* levels, uint64_t* states)
{
    int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nw) return;
    uint64_t word = 0;
    for (int j = 0; j < kStatesPerWord; ++j) {
        long long b = (long long)w * kStatesPerWord + j;
        if (b >= nb) break;
        uint64_t st = (uint64_t)(levels[b] + 1) & 7ull;
        word |= st << (3 * j);
    }
    states[w] = word;
}

hipError_t launch_pack_states(const Geo& g, const int8_t* levels, uint64_t* states, hipStream_t s)
{
    unsigned blocks = (unsigned)((g.n_state_words + 255) / 256);
    hipLaunchKernelGGL(k_pack_states, dim3(blocks), dim3(256), 0, s, g.nblocks, g.n_state_words, levels, states);
    return hipGetLastError();
}

// ---------------------------------------------------------- cell readback
template <typename T>
__global__ void k_read_cells(Geo g, SceneBufs bufs, int n, const int32_t* cells, float* out)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int x = cells[4 * i], y = cells[4 * i + 1], z = cells[4 * i + 2], m = cells[4 * i + 3];
    int bx = x >> g.log2B, by = y >> g.log2B, bz = z >> g.log2B;
    long long blk = bx + (long long)g.nb[0] * (by + (long long)g.nb[1] * bz);
    int slot = bufs.slot[blk];
    float* o = out + (long long)i * kLam * 2;
    if (slot < 0) {
        for (int j = 0; j < 2 * kLam; ++j) o[j] = __builtin_nanf("");
        return;
    }
    int side = g.B >> m;
    int cx = (x & (g.B - 1)) >> m, cy = (y & (g.B - 1)) >> m, cz = (z & (g.B - 1)) >> m;
    int local = cx + side * (cy + side * cz);
    const T* r = (const T*)bufs.vals + (((long long)slot * g.cells + g.lvl_off[m] + local) * kLam) * 2;
    for (int j = 0; j < 2 * kLam; ++j) o[j] = Codec<T>::dec(r[j]);
}

hipError_t launch_read_cells(const Geo& g, const SceneBufs& b, int storage, int n, const int32_t* cells,
                             float* out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    unsigned blocks = (unsigned)((n + 127) / 128);
    if (storage == RT_F32) hipLaunchKernelGGL(k_read_cells<float>, dim3(blocks), dim3(128), 0, s, g, b, n, cells, out);
    else if (storage == RT_BF16)
        hipLaunchKernelGGL(k_read_cells<__hip_bfloat16>, dim3(blocks), dim3(128), 0, s, g, b, n, cells, out);
    else hipLaunchKernelGGL(k_read_cells<__half>, dim3(blocks), dim3(128), 0, s, g, b, n, cells, out);
    return hipGetLastError();
}

}  // namespace rt
