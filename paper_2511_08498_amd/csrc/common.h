// Internal structures shared by the host API and the HIP kernels of the
// formal-solution library.  Not part of the C ABI (see include/rt.h).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "../../include/rt.h"

namespace rt {

constexpr int kLam = RT_LAM_BATCH;   // wavelengths per batch, kept in registers by the march
constexpr int kMaxLines = RT_MAX_LINES;
constexpr int kMaxLevels = RT_MAX_LEVELS;
constexpr long long kSlotLdsMax = 8192;  // blocks whose slot table a trace workgroup keeps in LDS (32 KiB)
constexpr long long kLdsPerCuBytes = 160 * 1024;  // LDS of one gfx950 compute unit: a workgroup never gets more
constexpr int kStatesPerWord = 21;   // 3-bit block states per 64-bit word
constexpr double kCkms = 299792.458; // speed of light, km/s

// Grid geometry of a scene.
struct Geo {
    int dim;
    int n[3];
    int B;            // block side
    int log2B;
    int nb[3];        // blocks per axis (1 beyond dim)
    int n_levels;
    int bvox;         // B^dim voxels per block
    int cells;        // cells per block over all levels
    int lvl_off[kMaxLevels + 1];  // first cell of each level inside a block record
    unsigned long long lvl_pack;  // lvl_off[m] in bits 11m .. 11m + 10, m < kMaxLevels (cells < 2^11)
    long long nblocks;
    int n_state_words;
    int feat_level;   // level whose statistics are kept as neural-cache features (min(2, n_levels - 1))
};

// Wavelength constants of one batch (line model).  Doubles: the kernels form
// lam - lam0 in FP64 before narrowing, which keeps the profile argument accurate.
struct LamBatch {
    int nl;        // wavelengths in this batch (<= kLam)
    int n_lines;
    int profile;   // rt_profile
    int pad_;
    double lam[kLam];
    double lam0[kMaxLines];
    // FP32 per-batch constants of the line evaluation (read as kernel arguments):
    float dl[kLam][kMaxLines];  // lam - lam0
    float rr[kLam][kMaxLines];  // lam / lam0
    float sr[kLam][kMaxLines];  // lam0 / (sqrt(pi) lam): the Voigt profile's normalisation and wavelength scaling
    float k0[kMaxLines];        // lam0 / c
};

// Device buffers owned by a scene.
struct SceneBufs {
    int32_t* morton;        // [nblocks] block ids in Morton order (all blocks)
    uint8_t* active;        // [nblocks]
    int32_t* slot;          // [nblocks] storage slot, -1 empty
    int32_t* active_list;   // [nblocks] first n_active: block ids in Morton order
    int32_t* n_active;      // [1]
    int8_t* levels;         // [nblocks] current batch
    uint64_t* states;       // [n_state_words]
    void* vals;             // [n_active][cells][kLam][2] static emission values (storage dtype)
    void* pf;               // [n_active][cells][2 dim][kLam][2] prefiltered cells, signed axis k = 2a + (w_a < 0)
    // velocity interpolation, per direction class q (1 class for the full grid, 2^dim orthants):
    float4* vgrid;          // [n_vclass][n_active][cells] (gx, gy, gz, off): node coordinate of direction w
                            // f = g . w + off = (vbar . w - lo) (n_v - 1) / (hi - lo); g = 0, off = 0 if hi = lo
    float2* vrange;         // [n_vclass][n_active][cells] (lo, hi) node range of projected velocities
    float* vnodes;          // [n_vclass][n_active][n_v][cells][kLam][2] node values (node-major in a brick)
    float* cav;             // [n_active][cells][cav_rec] line parameters (Core and Voigt)
    void* cav_lp;           // the same in BF16 or FP16 (reduced-precision storage), 2 bytes per value
    float4* fstats;         // [n_active][cells at feat_level][kLam]: mean, var of ln(chi ds0), mean, var of ln(eta ds0)
    unsigned long long* err;  // [2]: step-cap hits, first ray id (min)
};

// Inputs (caller-owned device pointers).
struct Inputs {
    const float* eta;
    const float* chi;
    const float* eta_star;
    const float* chi_star;
    const float* damp;
    const float* inv_dld;
    const float* eta_bg;
    const float* chi_bg;
    const float* vel;
    const uint8_t* mask;
    long long nvox;
};

// Record of Core-and-Voigt parameters per cell: per line eta*, chi*, a, 1/dlD;
// then eta_bg, chi_bg; then vbar[3]; padded to a multiple of 4 floats.
__host__ __device__ inline int cav_rec_floats(int n_lines)
{
    int r = 4 * n_lines + 2 + 3;
    return (r + 3) & ~3;
}

// ---------------------------------------------------------------- dtype codecs
template <typename T>
struct Codec;
template <>
struct Codec<float> {
    __device__ static float dec(float v) { return v; }
    __device__ static float enc(float v) { return v; }
};
template <>
struct Codec<__hip_bfloat16> {
    __device__ static float dec(__hip_bfloat16 v) { return __bfloat162float(v); }
    __device__ static __hip_bfloat16 enc(float v) { return __float2bfloat16(v); }  // round to nearest even
};
template <>
struct Codec<__half> {
    __device__ static float dec(__half v) { return __half2float(v); }
    __device__ static __half enc(float v) { return __float2half_rn(v); }
};

inline size_t dtype_bytes(int dt) { return dt == RT_F32 ? 4 : 2; }

// ------------------------------------------------------------------ launchers
// build.hip
hipError_t launch_classify(const Geo& g, const Inputs& in, int model, int n_lam, int n_lines, int dense,
                           uint8_t* active, hipStream_t s);
hipError_t launch_slots(const Geo& g, const int32_t* morton, const uint8_t* active, int32_t* slot,
                        int32_t* active_list, int32_t* n_active, hipStream_t s);
hipError_t launch_fill_levels(const Geo& g, int8_t* levels, hipStream_t s);
hipError_t launch_build_static(const Geo& g, const Inputs& in, const SceneBufs& b, int n_active, int model,
                               int vrule, const LamBatch& lb, int lam_begin, double ds0, double T, double tau_thin,
                               int cap, int avg_mode, int storage, int write_values, hipStream_t s);
hipError_t launch_pack_states(const Geo& g, const int8_t* levels, uint64_t* states, hipStream_t s);
hipError_t launch_build_prefilter(const Geo& g, const Inputs& in, const SceneBufs& b, int n_active, int model,
                                  const LamBatch& lb, int lam_begin, double ds0, int storage, hipStream_t s);
hipError_t launch_vgrid(const Geo& g, const Inputs& in, const SceneBufs& b, int n_active, int n_v, int n_vclass,
                        hipStream_t s);
hipError_t launch_velinterp_nodes(const Geo& g, const Inputs& in, const SceneBufs& b, int n_active,
                                  const LamBatch& lb, int n_v, int n_vclass, double ds0, int avg_mode, int storage,
                                  hipStream_t s);
hipError_t launch_cav_chain(const Geo& g, const Inputs& in, const SceneBufs& b, int n_active, int n_lines,
                            double ds0, int avg_mode, hipStream_t s);
hipError_t launch_read_cells(const Geo& g, const SceneBufs& b, int storage, int n, const int32_t* cells,
                             float* out, hipStream_t s);
hipError_t launch_cav_encode(const float* cav, void* out, long long n, int storage, hipStream_t s);

// march.hip
struct TraceLaunch {
    Geo g;
    const uint64_t* states;
    const int32_t* slot;
    int slot_lds;  // the trace kernels copy slot[] to LDS after the state words (grids of <= kSlotLdsMax blocks)
    const void* vals;
    const void* pf;            // prefiltered cells (RT_EMIS_PREFILTER)
    const float4* vgrid;
    const float* vnodes;
    int n_vclass;              // velocity-grid direction classes: 1 (full grid) or 2^dim (orthants)
    int n_active;              // active blocks (records per class = n_active * cells)
    const float* cav;
    const void* cav_lp;  // BF16/FP16 copy of cav, used when storage != RT_F32
    const float* dirs;
    int n_dir;
    int mode;
    int max_level;
    int step_cap;
    int graded;                      // nonzero when level_dist has a nonzero entry
    float level_dist[kMaxLevels];    // distance-graded level cap
    const int32_t* probes;   // nullable
    const int32_t* active_list;
    long long n_probes;
    float* I;
    float I0;
    float ds0;
    int emission;
    int storage;
    int n_v;
    int cav_rec;
    LamBatch lb;
    unsigned long long* stats;
    unsigned long long* err;
    // truncated march (neural radiance cache)
    int trunc;
    int gen;
    double t_trunc;
    const uint8_t* fallback;   // [nblocks] 1 = march on past t_trunc
    const float4* fstats;
    float* I_near;
    float* T_near;
    float* I_far;
    float4* feat;              // [n_dir][n_probes]
    float4* fstat_out;         // [n_dir][nl][n_probes]
    // angle-integrated output (mean intensity J and the diagonal operator)
    int jmode;
    int dirs_per_chunk;
    const float* weights;      // [n_dir] quadrature weights
    float* part_J;             // [n_chunks][nl][n_probes]
    float* part_psi;           // [n_chunks][nl][n_probes], nullable
    // radiance interval [t_lo, t_hi] of each ray
    int interval;
    double t_lo;
    double t_hi;
    float* T_out;              // [n_dir][nl][n_probes] interval transmittance, nullable
};
hipError_t launch_trace(const TraceLaunch& t, hipStream_t s);
hipError_t launch_reduce_chunks(const float* part, int n_chunks, long long n, float* out, hipStream_t s);

// One job of the batched persistent trace (static emission).
struct BatchJob {
    Geo g;
    const uint64_t* states;
    const int32_t* slot;
    const void* vals;
    const int32_t* active_list;
    const float* dirs;
    float* I;
    long long n_probes;
    unsigned tile0;     // first queue tile of this job
    int tiles;          // 64-probe tiles per direction
    int n_dir;
    int nl;
    int mode;
    int max_level;
    int graded;
    int step_cap;
    int storage;
    int tile_shape;     // rt_batch_params.tile_shape
    float I0;
    float ds0;
    float level_dist[kMaxLevels];
};
// A run of jobs of one dimension: one persistent launch each (at most 2: 2D, 3D).
struct BatchSeg {
    int dim;
    int storage;        // dtype shared by the segment's jobs, -1 for a mix
    int j0, j1;         // jobs [j0, j1)
    unsigned tile_begin, tile_end;
};
hipError_t launch_batched(const BatchJob* d_jobs, const BatchSeg* segs, int n_segs, int wg_waves, int n_wgs,
                          int tiles_per_pop, unsigned* counter, unsigned* claims, unsigned long long* err,
                          hipStream_t s);
hipError_t launch_debug_visited(const TraceLaunch& t, int probe_vox, float wx, float wy, float wz, int cap,
                                int32_t* cells, double* tt, int32_t* count, hipStream_t s);

}  // namespace rt
