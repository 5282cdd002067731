/*
 * FP64 CPU oracle for the formal solution with variance-limited mipmaps.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant generator with the HIP library and includes
 * nothing from it.  Plain, slow and written to be checked by eye against
 * the paper (Osborne 2025, "A Simple Ray Acceleration Structure for Non-LTE
 * Radiative Transfer"):
 *
 *   orc_ray_cells     dense MIP-0 voxel list of a long characteristic
 *                     (Sect. 2.3: exact path length per voxel, AW87 on a
 *                     single-resolution grid): every crossing time of an
 *                     integer plane, sorted, zero-length pieces dropped,
 *                     each piece's voxel = floor(x(t_mid)).
 *   orc_ray_segments  cells of the adapted grid (Sect. 2.3, Alg. 1 output):
 *                     the dense list mapped to each block's MIP level
 *                     (FloorToStep), empty blocks dropped, consecutive equal
 *                     cells merged.
 *   orc_levels        mip chain (Sect. 2.1, box filter over 2^D children) in
 *                     log space, index of dispersion (Eq. IoD) and the VLM
 *                     level per block (Sect. 2.2; thin-cell bypass at
 *                     chi ds < 0.25).
 *   orc_lines_mip0    per-voxel emissivity/opacity of the line model
 *                     (Eqs. EtaTot/ChiTot, EtaTotDir/ChiTotDir) at rest or at
 *                     the Doppler shift closest to the line core (Sect. 3.2).
 *   orc_march         piecewise-constant formal solution (Eq. RteIntegral
 *                     with constant eta, chi per cell), iterated from the
 *                     upwind boundary to the probe:
 *                         I <- I exp(-tau) + (eta/chi) (1 - exp(-tau)),
 *                     with emissivity/opacity per cell from stored values
 *                     (static), the exact line model (Classic), velocity
 *                     interpolation (Sect. 3.1) or Core and Voigt (Sect. 3.2).
 *   orc_march_interval  the same over a radiance interval t in [t1, t2]
 *                     (Sect. 2.3, Eq. Ray and the HDDA procedure of Alg. 1
 *                     take [t1, t2]; Sect. 4.1 radiance cascades): the
 *                     ray's pieces clipped to the interval, the recurrence
 *                     started from 0 (or from I0 when the ray leaves the
 *                     grid inside the interval), plus the interval's
 *                     transmittance T = prod exp(-tau).
 *   orc_prefilter     prefiltered level cells (Sect. 5.1: the transfer
 *                     equation precomputed along the +-x, y, z axes and
 *                     interpolated between these): for every merged cell and
 *                     signed axis, the exact transfer (I, T) of each MIP-0 row
 *                     of the cell along that axis, averaged over the rows, and
 *                     the homogeneous cell with the same (I, T) over the
 *                     cell's side; the march blends the axes of a ray's
 *                     direction with weights w_a^2.
 *   orc_voigt_h       H(a,x) = Re w(x + i a) by Weideman's rational series
 *                     with N = 64 terms in FP64 (an independent method from
 *                     the single-precision profile of the GPU path).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_C_KMS 299792.458

/* ------------------------------------------------------------------ */
/* scene description                                                   */
/* ------------------------------------------------------------------ */
enum { ORC_STATIC = 0, ORC_CLASSIC = 1, ORC_VELINTERP = 2, ORC_CAV = 3, ORC_PREFILTER = 4 };
enum { ORC_GAUSS = 0, ORC_VOIGT = 1 };
enum { ORC_AVG_LOG = 0, ORC_AVG_LINEAR = 1 };
enum { ORC_GRADE_ENTRY = 0, ORC_GRADE_PATH = 1 };
enum { ORC_VGRID_FULL = 0, ORC_VGRID_ORTHANT = 1 };

typedef struct orc_scene {
    int32_t dim;
    int32_t n[3];       /* voxels per axis; n[2] = 1 in 2D */
    int32_t brick;      /* block side B */
    int32_t n_levels;   /* MIP levels 0 .. n_levels-1 */
    int32_t n_lam;      /* wavelengths handled by one march call */
    int32_t profile;    /* ORC_GAUSS / ORC_VOIGT */
    int32_t n_lines;
    int32_t n_v;        /* velocity nodes (velocity interpolation) */
    int32_t avg_mode;   /* ORC_AVG_LOG / ORC_AVG_LINEAR for stored level values */
    int32_t grade_mode; /* ORC_GRADE_ENTRY / ORC_GRADE_PATH (distance-graded level cap) */
    double ds0;         /* physical side of a MIP-0 voxel */
    double I0;          /* intensity entering at the upwind boundary */
    /* static: [n_lam][level_total] FP64 values of every level (level 0 first) */
    const double* st_eta;
    const double* st_chi;
    /* line model (MIP-0 inputs) */
    const double* lam;      /* [n_lam] nm */
    const double* lam0;     /* [n_lines] nm */
    const float* eta_star;  /* [n_lines][nvox] */
    const float* chi_star;  /* [n_lines][nvox] */
    const float* damp;      /* [n_lines][nvox] Voigt damping at lam0 */
    const float* inv_dld;   /* [n_lines][nvox] 1 / Doppler width, 1/nm */
    const float* eta_bg;    /* [nvox] */
    const float* chi_bg;    /* [nvox] */
    const float* vel;       /* [dim][nvox] km/s */
    /* distance-graded level cap: level m only in blocks entered at path length
     * >= level_dist[m] (m = 1 .. n_levels-1); NULL = no grading */
    const double* level_dist;
    /* velocity-interpolation node grid: ORC_VGRID_FULL (one grid over [-V, V]
     * for every direction) or ORC_VGRID_ORTHANT (one grid per orthant of
     * directions, over the projections reachable from it) */
    int32_t vgrid_mode;
    /* prefiltered cells: [n_lam][level_total][2 dim] equivalent eta, chi per
     * signed axis k = 2 a + (propagation towards -a); levels >= 1 are read */
    const double* pf_eta;
    const double* pf_chi;
} orc_scene;

static int64_t nvox_of(const orc_scene* s) { return (int64_t)s->n[0] * s->n[1] * s->n[2]; }

static int64_t vox_index(const orc_scene* s, const int32_t c[3])
{
    return c[0] + (int64_t)s->n[0] * (c[1] + (int64_t)s->n[1] * c[2]);
}

/* total length of the concatenated level grids (level m has n_a >> m cells per axis) */
int64_t orc_level_total(int32_t dim, const int32_t n[3], int32_t n_levels)
{
    int64_t tot = 0;
    for (int m = 0; m < n_levels; ++m) {
        int64_t c = 1;
        for (int a = 0; a < dim; ++a) c *= (n[a] >> m);
        tot += c;
    }
    return tot;
}

static int64_t level_offset(const orc_scene* s, int m)
{
    return orc_level_total(s->dim, s->n, m);
}

static int64_t level_index(const orc_scene* s, int m, const int32_t c[3])
{
    int64_t nx = s->n[0] >> m, ny = s->dim > 1 ? (s->n[1] >> m) : 1;
    int64_t i = (c[0] >> m);
    if (s->dim > 1) i += nx * (c[1] >> m);
    if (s->dim > 2) i += nx * ny * (c[2] >> m);
    return i;
}

/* ------------------------------------------------------------------ */
/* dense cell list (MIP 0)                                             */
/* ------------------------------------------------------------------ */
/*
 * Ray x(t) = p - t w, p the centre of voxel pv, t in [0, t_exit], x(t_exit)
 * on the bounding box.  Cells are listed from the probe (t = 0) upwind.
 * Returns the number of cells, or -1 if cap is too small.
 */
int orc_ray_cells(int32_t dim, const int32_t n[3], const int32_t pv[3], const float w[3], int cap,
                  int32_t* cell, double* tin, double* tout)
{
    double p[3] = {0, 0, 0}, wd[3] = {0, 0, 0};
    int32_t k[3] = {0, 0, 0}, st[3] = {0, 0, 0};
    double texit = INFINITY;
    for (int a = 0; a < dim; ++a) {
        p[a] = pv[a] + 0.5;
        wd[a] = (double)w[a];
        if (wd[a] > 0) {
            st[a] = -1;
            k[a] = pv[a];
            double te = p[a] / wd[a];
            if (te < texit) texit = te;
        } else if (wd[a] < 0) {
            st[a] = +1;
            k[a] = pv[a] + 1;
            double te = (p[a] - n[a]) / wd[a];
            if (te < texit) texit = te;
        }
    }
    int cnt = 0;
    double t0 = 0.0;
    for (;;) {
        double tn = texit;
        for (int a = 0; a < dim; ++a) {
            if (!st[a]) continue;
            double ta = (p[a] - k[a]) / wd[a];
            if (ta < tn) tn = ta;
        }
        if (tn > t0) {
            if (cnt >= cap) return -1;
            double tm = 0.5 * (t0 + tn);
            for (int a = 0; a < 3; ++a) cell[3 * cnt + a] = 0;
            for (int a = 0; a < dim; ++a) cell[3 * cnt + a] = (int32_t)floor(p[a] - tm * wd[a]);
            tin[cnt] = t0;
            tout[cnt] = tn;
            ++cnt;
        }
        for (int a = 0; a < dim; ++a) {
            if (!st[a]) continue;
            if ((p[a] - k[a]) / wd[a] == tn) k[a] += st[a];
        }
        t0 = tn;
        if (t0 >= texit) break;
    }
    return cnt;
}

/*
 * Cells of the adapted grid along the ray.  levels[b] is the MIP level of
 * block b (-1 = empty); levels == NULL means every cell at level 0,
 * including empty blocks (the dense march).  Output cells are the level's
 * coarse coordinates (multiples of 2^level).  Returns count or -1.
 */
/*
 * Distance-graded level cap (near field at full resolution): level_dist[m]
 * (m = 1 .. n_levels-1, nullable) is the path length from the probe beyond
 * which level m may be used, following the per-cascade MIP caps of Sect. 4.1
 * (full resolution near the probe, coarser proxies further out).  The cap is
 * the largest m with level_dist[1..m] <= t, taken
 *   ORC_GRADE_ENTRY: at t = t_entry, the path length at which the ray enters
 *                    the block (0 for the probe's own block), for the whole
 *                    block;
 *   ORC_GRADE_PATH:  at every point of the ray, so the cap rises exactly at
 *                    t = level_dist[m] (the cascade intervals of Sect. 4.1,
 *                    whose caps hold along the interval's path length); a
 *                    voxel piece that straddles level_dist[m] is split there.
 */
static int graded_cap(const orc_scene* s, const double* level_dist, double t_entry)
{
    int cap = 0;
    if (!level_dist) return 127;
    for (int m = 1; m < s->n_levels; ++m) {
        if (!(level_dist[m] <= t_entry)) break;
        cap = m;
    }
    return cap;
}

int orc_ray_segments_graded(const orc_scene* s, const int8_t* levels, const double* level_dist, const int32_t pv[3],
                            const float w[3], int cap, int32_t* cell, int32_t* lvl, double* tin, double* tout,
                            int32_t* scratch_cell, double* scratch_tin, double* scratch_tout, int scratch_cap)
{
    int nd = orc_ray_cells(s->dim, s->n, pv, w, scratch_cap, scratch_cell, scratch_tin, scratch_tout);
    if (nd < 0) return -1;
    int B = s->brick;
    int32_t nb[3] = {1, 1, 1};
    for (int a = 0; a < s->dim; ++a) nb[a] = s->n[a] / B;
    const int by_path = levels && level_dist && s->grade_mode == ORC_GRADE_PATH;
    int cnt = 0;
    int64_t cur_b = -1;
    int cur_cap = 127;
    for (int i = 0; i < nd; ++i) {
        const int32_t* c = scratch_cell + 3 * i;
        int Lb = 0;
        if (levels) {
            int64_t b = c[0] / B + (int64_t)nb[0] * (c[1] / B + (int64_t)nb[1] * (c[2] / B));
            if (b != cur_b) {
                cur_b = b;
                cur_cap = graded_cap(s, level_dist, scratch_tin[i]);
            }
            Lb = levels[b];
            if (Lb < 0) continue;
        }
        /* sub-pieces: the voxel piece, split at the path-graded boundaries inside it */
        double cut[8];
        int nc = 0;
        cut[nc++] = scratch_tin[i];
        if (by_path)
            for (int m = 1; m < s->n_levels && nc < 7; ++m)
                if (level_dist[m] > scratch_tin[i] && level_dist[m] < scratch_tout[i]) cut[nc++] = level_dist[m];
        for (int x = 1; x < nc; ++x) /* sort the cuts (level_dist need not increase) */
            for (int y = x; y > 1 && cut[y] < cut[y - 1]; --y) {
                double tmp = cut[y];
                cut[y] = cut[y - 1];
                cut[y - 1] = tmp;
            }
        cut[nc] = scratch_tout[i];
        for (int q = 0; q < nc; ++q) {
            if (!(cut[q + 1] > cut[q])) continue;
            int L = Lb;
            if (levels) {
                const int cp = by_path ? graded_cap(s, level_dist, cut[q]) : cur_cap;
                if (L > cp) L = cp;
            }
            int32_t cc[3];
            for (int a = 0; a < 3; ++a) cc[a] = c[a] & ~((1 << L) - 1);
            if (cnt > 0 && lvl[cnt - 1] == L && cell[3 * (cnt - 1)] == cc[0] && cell[3 * (cnt - 1) + 1] == cc[1] &&
                cell[3 * (cnt - 1) + 2] == cc[2]) {
                tout[cnt - 1] = cut[q + 1];
                continue;
            }
            if (cnt >= cap) return -1;
            for (int a = 0; a < 3; ++a) cell[3 * cnt + a] = cc[a];
            lvl[cnt] = L;
            tin[cnt] = cut[q];
            tout[cnt] = cut[q + 1];
            ++cnt;
        }
    }
    return cnt;
}

int orc_ray_segments(const orc_scene* s, const int8_t* levels, const int32_t pv[3], const float w[3], int cap,
                     int32_t* cell, int32_t* lvl, double* tin, double* tout, int32_t* scratch_cell,
                     double* scratch_tin, double* scratch_tout, int scratch_cap)
{
    return orc_ray_segments_graded(s, levels, s->level_dist, pv, w, cap, cell, lvl, tin, tout, scratch_cell,
                                   scratch_tin, scratch_tout, scratch_cap);
}

/* ------------------------------------------------------------------ */
/* Voigt function, Weideman (1994) rational series, N = 64, FP64       */
/* ------------------------------------------------------------------ */
#define WEID_N 64
static double weid_coef[WEID_N + 1];
static double weid_L;
static int weid_ready = 0;

static void weid_init(void)
{
    if (weid_ready) return;
    const int N = WEID_N, M = 2 * N;
    double L = sqrt(N / sqrt(2.0));
    for (int nn = 1; nn <= N; ++nn) {
        double acc = 0.0;
        for (int j = -M + 1; j <= M - 1; ++j) {
            double th = j * M_PI / M;
            double t = L * tan(0.5 * th);
            double g = exp(-t * t) * (L * L + t * t);
            acc += g * cos(nn * th);
        }
        weid_coef[nn] = acc / (2.0 * M);
    }
    weid_L = L;
    weid_ready = 1;
}

/* H(a, x) = Re w(x + i a).  w(z) ~ pi^-1/2/(L - iz) + 2/(L - iz)^2 sum_n c_n Z^(n-1),
 * Z = (L + iz)/(L - iz). */
double orc_voigt_h(double a, double x)
{
    weid_init();
    double L = weid_L;
    /* iz = i x - a */
    double dr = L + a, di = -x;      /* L - i z = (L + a) - i x */
    double nr = L - a, ni = x;       /* L + i z = (L - a) + i x */
    double den = dr * dr + di * di;
    double Zr = (nr * dr + ni * di) / den;
    double Zi = (ni * dr - nr * di) / den;
    /* Horner: p = c_N Z^(N-1) + ... + c_1 */
    double pr = weid_coef[WEID_N], pi = 0.0;
    for (int nn = WEID_N - 1; nn >= 1; --nn) {
        double tr = pr * Zr - pi * Zi;
        double ti = pr * Zi + pi * Zr;
        pr = tr + weid_coef[nn];
        pi = ti;
    }
    /* 1/(L - iz) */
    double ir = dr / den, ii = -di / den;
    /* 1/(L - iz)^2 */
    double i2r = ir * ir - ii * ii, i2i = 2.0 * ir * ii;
    double wr = 2.0 * (pr * i2r - pi * i2i) + ir / sqrt(M_PI);
    return wr;
}

/* ------------------------------------------------------------------ */
/* line model                                                          */
/* ------------------------------------------------------------------ */
/*
 * One line's (eta, chi) contribution at wavelength lam for projected
 * velocity u (km/s), with the line's parameters at the cell.
 *   Gaussian (peak-normalised): phi = exp(-x^2).
 *   Voigt (Sect. 3.2): phi = H(a(lam), x) / (sqrt(pi) dlD), eta*, chi* scaled
 *   by lam0/lam and a(lam) = (lam/lam0)^2 a(lam0).
 * x = (lam - lam0 (1 - u/c)) / dlD: the line centre seen along the ray is
 * at lam0 (1 - u/c) (profile argument lam + (v.w/c) lam0).
 */
static void line_eval(int profile, double lam, double lam0, double eta_s, double chi_s, double a0,
                      double inv_dld, double u, double* eta, double* chi)
{
    double x = (lam - lam0 * (1.0 - u / ORC_C_KMS)) * inv_dld;
    double phi, sc;
    if (profile == ORC_GAUSS) {
        phi = exp(-x * x);
        sc = 1.0;
    } else {
        double r = lam / lam0;
        phi = orc_voigt_h(a0 * r * r, x) * inv_dld / sqrt(M_PI);
        sc = lam0 / lam;
    }
    *eta = sc * eta_s * phi;
    *chi = sc * chi_s * phi;
}

/* eta, chi of MIP-0 voxel v at wavelength index il for projected velocity u */
static void voxel_emis(const orc_scene* s, int64_t v, int il, double u, double* eta, double* chi)
{
    int64_t nv = nvox_of(s);
    double e = s->eta_bg[v], c = s->chi_bg[v];
    for (int l = 0; l < s->n_lines; ++l) {
        double el, cl;
        line_eval(s->profile, s->lam[il], s->lam0[l], s->eta_star[l * nv + v], s->chi_star[l * nv + v],
                  s->damp[l * nv + v], s->inv_dld[l * nv + v], u, &el, &cl);
        e += el;
        c += cl;
    }
    *eta = e;
    *chi = c;
}

static double voxel_speed(const orc_scene* s, int64_t v)
{
    int64_t nv = nvox_of(s);
    double q = 0.0;
    for (int a = 0; a < s->dim; ++a) {
        double va = s->vel[a * nv + v];
        q += va * va;
    }
    return sqrt(q);
}

/*
 * MIP-0 eta, chi of the line model at wavelength lam[il] for every voxel.
 * rule 0: at rest (u = 0) -- the frame used for the IoD of velocity
 *         interpolation (Sect. 3.1).
 * rule 1: each line at the Doppler shift in [-|v|, |v|] that brings it
 *         closest to the line core, u* = clamp(c (1 - lam/lam0)) (Sect. 3.2).
 */
void orc_lines_mip0(const orc_scene* s, int il, int rule, double* eta, double* chi)
{
    int64_t nv = nvox_of(s);
    for (int64_t v = 0; v < nv; ++v) {
        double e = s->eta_bg[v], c = s->chi_bg[v];
        double sp = voxel_speed(s, v);
        for (int l = 0; l < s->n_lines; ++l) {
            double u = 0.0;
            if (rule == 1) {
                u = ORC_C_KMS * (1.0 - s->lam[il] / s->lam0[l]);
                if (u > sp) u = sp;
                if (u < -sp) u = -sp;
            }
            double el, cl;
            line_eval(s->profile, s->lam[il], s->lam0[l], s->eta_star[l * nv + v], s->chi_star[l * nv + v],
                      s->damp[l * nv + v], s->inv_dld[l * nv + v], u, &el, &cl);
            e += el;
            c += cl;
        }
        eta[v] = e;
        chi[v] = c;
    }
}

/* ------------------------------------------------------------------ */
/* mip chain and VLM levels                                            */
/* ------------------------------------------------------------------ */
/* children of level-m cell (cx,cy,cz in level-m units) at level m-1, in the
 * fixed pairwise order: x pairs, then y, then z. */
static void child_idx(int dim, int64_t nxc, int64_t nyc, int64_t cx, int64_t cy, int64_t cz, int64_t* idx)
{
    int k = 0;
    for (int dz = 0; dz < (dim > 2 ? 2 : 1); ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                int64_t x = 2 * cx + dx, y = 2 * cy + dy, z = 2 * cz + dz;
                idx[k++] = x + nxc * (y + nyc * z);
            }
}

static double pair_sum(int dim, const double* q)
{
    if (dim == 2) return (q[0] + q[1]) + (q[2] + q[3]);
    return ((q[0] + q[1]) + (q[2] + q[3])) + ((q[4] + q[5]) + (q[6] + q[7]));
}

/*
 * One wavelength: MIP-0 eta, chi (FP64, full grid) -> VLM level per block.
 *   x = ln(max(q ds0, 1e-300)) for q in {eta, chi} at level 0;
 *   level m >= 1: xbar = mean of the 2^D children's xbar (pairwise order),
 *   Var = mean of (child - xbar)^2 (two-pass), IoD = |Var / xbar| (+inf if
 *   xbar = 0 < Var, 0 if Var = 0);
 *   a cell passes if chi_a 2^m ds0 < tau_thin (its optical side is thin),
 *   chi_a being the arithmetic mean of the MIP-0 chi it covers (the box
 *   filter of Sect. 2.1, whatever the stored-value mode), or
 *   IoD(eta) <= T and IoD(chi) <= T;
 *   block level = largest m <= min(n_levels - 1, cap) with every cell of
 *   levels 1..m inside the block passing; -1 for an inactive block.
 * Stored level values (out_eta/out_chi, nullable, concatenated level grids):
 *   LOG mode exp(xbar)/ds0, LINEAR mode pairwise mean of the linear values.
 * Returns the number of active voxels whose value had to be clamped.
 */
int64_t orc_levels(const orc_scene* s, const double* eta0, const double* chi0, const uint8_t* block_active,
                   double T, double tau_thin, int32_t cap, int8_t* levels_out, double* out_eta, double* out_chi)
{
    const int D = s->dim, B = s->brick, L = s->n_levels;
    const int64_t tot = orc_level_total(D, s->n, L);
    double* xe = (double*)malloc(sizeof(double) * tot);
    double* xc = (double*)malloc(sizeof(double) * tot);
    double* le = (double*)malloc(sizeof(double) * tot);
    double* lc = (double*)malloc(sizeof(double) * tot);
    double* ac = (double*)malloc(sizeof(double) * tot); /* arithmetic mean of MIP-0 chi over the cell */
    uint8_t* pass = (uint8_t*)malloc(tot);
    int64_t nv = nvox_of(s), clamped = 0;
    int32_t nb[3] = {1, 1, 1};
    for (int a = 0; a < D; ++a) nb[a] = s->n[a] / B;
    /* level 0 */
    for (int64_t v = 0; v < nv; ++v) {
        int32_t c[3] = {(int32_t)(v % s->n[0]), (int32_t)((v / s->n[0]) % s->n[1]),
                        (int32_t)(v / ((int64_t)s->n[0] * s->n[1]))};
        int64_t b = c[0] / B + (int64_t)nb[0] * (c[1] / B + (int64_t)nb[1] * (c[2] / B));
        double qe = eta0[v] * s->ds0, qc = chi0[v] * s->ds0;
        if (block_active[b] && (qe <= 1e-300 || qc <= 1e-300)) ++clamped;
        xe[v] = log(qe > 1e-300 ? qe : 1e-300);
        xc[v] = log(qc > 1e-300 ? qc : 1e-300);
        le[v] = eta0[v];
        lc[v] = chi0[v];
        ac[v] = chi0[v];
        pass[v] = 1;
    }
    /* levels 1..L-1 */
    for (int m = 1; m < L; ++m) {
        int64_t off_c = level_offset(s, m - 1), off = level_offset(s, m);
        int64_t nxc = s->n[0] >> (m - 1), nyc = D > 1 ? s->n[1] >> (m - 1) : 1;
        int64_t nx = s->n[0] >> m, ny = D > 1 ? s->n[1] >> m : 1, nz = D > 2 ? s->n[2] >> m : 1;
        int nch = 1 << D;
        for (int64_t cz = 0; cz < nz; ++cz)
            for (int64_t cy = 0; cy < ny; ++cy)
                for (int64_t cx = 0; cx < nx; ++cx) {
                    int64_t idx[8];
                    child_idx(D, nxc, nyc, cx, cy, cz, idx);
                    double q[8];
                    int64_t o = off + cx + nx * (cy + ny * cz);
                    double mean_e, mean_c, var_e, var_c;
                    for (int k = 0; k < nch; ++k) q[k] = xe[off_c + idx[k]];
                    mean_e = pair_sum(D, q) / nch;
                    for (int k = 0; k < nch; ++k) q[k] = (xe[off_c + idx[k]] - mean_e) * (xe[off_c + idx[k]] - mean_e);
                    var_e = pair_sum(D, q) / nch;
                    for (int k = 0; k < nch; ++k) q[k] = xc[off_c + idx[k]];
                    mean_c = pair_sum(D, q) / nch;
                    for (int k = 0; k < nch; ++k) q[k] = (xc[off_c + idx[k]] - mean_c) * (xc[off_c + idx[k]] - mean_c);
                    var_c = pair_sum(D, q) / nch;
                    xe[o] = mean_e;
                    xc[o] = mean_c;
                    for (int k = 0; k < nch; ++k) q[k] = le[off_c + idx[k]];
                    double lin_e = pair_sum(D, q) / nch;
                    for (int k = 0; k < nch; ++k) q[k] = lc[off_c + idx[k]];
                    double lin_c = pair_sum(D, q) / nch;
                    for (int k = 0; k < nch; ++k) q[k] = ac[off_c + idx[k]];
                    ac[o] = pair_sum(D, q) / nch;
                    if (s->avg_mode == ORC_AVG_LOG) {
                        le[o] = exp(mean_e) / s->ds0;
                        lc[o] = exp(mean_c) / s->ds0;
                    } else {
                        le[o] = lin_e;
                        lc[o] = lin_c;
                    }
                    double iod_e = var_e == 0.0 ? 0.0 : (mean_e == 0.0 ? INFINITY : fabs(var_e / mean_e));
                    double iod_c = var_c == 0.0 ? 0.0 : (mean_c == 0.0 ? INFINITY : fabs(var_c / mean_c));
                    int thin = ac[o] * (double)(1 << m) * s->ds0 < tau_thin;
                    pass[o] = (uint8_t)(thin || (iod_e <= T && iod_c <= T));
                }
    }
    /* block levels */
    int64_t nbt = (int64_t)nb[0] * nb[1] * nb[2];
    int Lmax = L - 1;
    if (cap >= 0 && cap < Lmax) Lmax = cap;
    for (int64_t b = 0; b < nbt; ++b) {
        if (!block_active[b]) {
            levels_out[b] = -1;
            continue;
        }
        int32_t bc[3] = {(int32_t)(b % nb[0]), (int32_t)((b / nb[0]) % nb[1]), (int32_t)(b / ((int64_t)nb[0] * nb[1]))};
        int lv = 0;
        for (int m = 1; m <= Lmax; ++m) {
            int side = B >> m, ok = 1;
            int64_t off = level_offset(s, m);
            int64_t nx = s->n[0] >> m, ny = D > 1 ? s->n[1] >> m : 1;
            for (int z = 0; z < (D > 2 ? side : 1) && ok; ++z)
                for (int y = 0; y < side && ok; ++y)
                    for (int x = 0; x < side; ++x) {
                        int64_t cx = (int64_t)bc[0] * side + x, cy = (int64_t)bc[1] * side + y;
                        int64_t cz = (int64_t)bc[2] * side + z;
                        if (!pass[off + cx + nx * (cy + ny * cz)]) {
                            ok = 0;
                            break;
                        }
                    }
            if (!ok) break;
            lv = m;
        }
        levels_out[b] = (int8_t)lv;
    }
    if (out_eta) memcpy(out_eta, le, sizeof(double) * tot);
    if (out_chi) memcpy(out_chi, lc, sizeof(double) * tot);
    free(xe);
    free(xc);
    free(le);
    free(lc);
    free(ac);
    free(pass);
    return clamped;
}

/* ------------------------------------------------------------------ */
/* cell parameters at a MIP level (recursive pairwise means)           */
/* ------------------------------------------------------------------ */
typedef double (*vox_fn)(const orc_scene* s, int64_t v, const void* ctx);

/* mean of f over the voxels of the cube [c, c + size) in the pairwise tree order */
static double cube_mean(const orc_scene* s, vox_fn f, const void* ctx, const int32_t c[3], int size)
{
    if (size == 1) return f(s, vox_index(s, c), ctx);
    int h = size / 2, D = s->dim;
    double q[8];
    int k = 0;
    for (int dz = 0; dz < (D > 2 ? 2 : 1); ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                int32_t cc[3] = {c[0] + dx * h, c[1] + dy * h, c[2] + dz * h};
                q[k++] = cube_mean(s, f, ctx, cc, h);
            }
    return pair_sum(D, q) / (1 << D);
}

static double cube_max(const orc_scene* s, vox_fn f, const void* ctx, const int32_t c[3], int size)
{
    double best = -INFINITY;
    for (int z = 0; z < (s->dim > 2 ? size : 1); ++z)
        for (int y = 0; y < size; ++y)
            for (int x = 0; x < size; ++x) {
                int32_t cc[3] = {c[0] + x, c[1] + y, c[2] + z};
                double q = f(s, vox_index(s, cc), ctx);
                if (q > best) best = q;
            }
    return best;
}

typedef struct { int which; int line; } field_ctx;
/* which: 0 eta*, 1 chi*, 2 damp, 3 inv_dld, 4 eta_bg, 5 chi_bg, 6.. vel[a] */
static double field_raw(const orc_scene* s, int64_t v, const void* vctx)
{
    const field_ctx* c = (const field_ctx*)vctx;
    int64_t nv = nvox_of(s);
    switch (c->which) {
    case 0: return s->eta_star[c->line * nv + v];
    case 1: return s->chi_star[c->line * nv + v];
    case 2: return s->damp[c->line * nv + v];
    case 3: return s->inv_dld[c->line * nv + v];
    case 4: return s->eta_bg[v];
    case 5: return s->chi_bg[v];
    default: return s->vel[(c->which - 6) * nv + v];
    }
}
static double field_log(const orc_scene* s, int64_t v, const void* ctx)
{
    double q = field_raw(s, v, ctx) * s->ds0;
    return log(q > 1e-300 ? q : 1e-300);
}
static double field_speed(const orc_scene* s, int64_t v, const void* ctx)
{
    (void)ctx;
    return voxel_speed(s, v);
}

/* averaged quantity stored for eta/chi-like fields: LOG or LINEAR mode */
static double cell_avg_q(const orc_scene* s, int which, int line, const int32_t c[3], int size)
{
    field_ctx fc = {which, line};
    if (size == 1) return field_raw(s, vox_index(s, c), &fc);
    if (s->avg_mode == ORC_AVG_LOG) return exp(cube_mean(s, field_log, &fc, c, size)) / s->ds0;
    return cube_mean(s, field_raw, &fc, c, size);
}
static double cell_lin(const orc_scene* s, int which, int line, const int32_t c[3], int size)
{
    field_ctx fc = {which, line};
    return cube_mean(s, field_raw, &fc, c, size);
}

typedef struct { int il; double u; int q; } node_ctx; /* q: 0 eta, 1 chi */
static double node_val(const orc_scene* s, int64_t v, const void* vctx)
{
    const node_ctx* c = (const node_ctx*)vctx;
    double e, x;
    voxel_emis(s, v, c->il, c->u, &e, &x);
    return c->q ? x : e;
}
static double node_log(const orc_scene* s, int64_t v, const void* ctx)
{
    double q = node_val(s, v, ctx) * s->ds0;
    return log(q > 1e-300 ? q : 1e-300);
}

/*
 * Range of projected velocities u = v . w of MIP-0 voxel v over the unit
 * directions w of one orthant (class q: bit a set <=> w_a < 0).  With
 * b_a = v_a for a positive axis and -v_a for a negative one, u = sum_a b_a |w_a|
 * over the non-negative part of the unit sphere.  Its largest value is the
 * length of the positive part of b when some b_a > 0 (the direction along that
 * part lies in the orthant), otherwise the largest b_a (on an axis); the
 * smallest value likewise with the negative part.
 */
static void voxel_orthant_range(const orc_scene* s, int64_t v, int q, double* lo, double* hi)
{
    int64_t nv = nvox_of(s);
    double pos = 0.0, neg = 0.0, bmax = -INFINITY, bmin = INFINITY;
    int any_pos = 0, any_neg = 0;
    for (int a = 0; a < s->dim; ++a) {
        double b = s->vel[a * nv + v];
        if ((q >> a) & 1) b = -b;
        if (b > 0.0) {
            pos += b * b;
            any_pos = 1;
        }
        if (b < 0.0) {
            neg += b * b;
            any_neg = 1;
        }
        if (b > bmax) bmax = b;
        if (b < bmin) bmin = b;
    }
    *hi = any_pos ? sqrt(pos) : bmax;
    *lo = any_neg ? -sqrt(neg) : bmin;
}

typedef struct { int q; int want_hi; } orth_ctx;
/* hi, or -lo, of a voxel's orthant range (so that both bounds are maxima) */
static double field_orth(const orc_scene* s, int64_t v, const void* vctx)
{
    const orth_ctx* c = (const orth_ctx*)vctx;
    double lo, hi;
    voxel_orthant_range(s, v, c->q, &lo, &hi);
    return c->want_hi ? hi : -lo;
}

/*
 * Node range [lo, hi] of a level cell for the ray direction w (Sect. 3.1: the
 * grid spans the projections of velocity reachable in the cell, from the
 * MIP-0 voxels it contains).  Full grid: [-V, V], V = max |v|.  Orthant grid
 * (the quadrant-by-quadrant solution of Sect. 4.1): the union of the cell's
 * voxel ranges over the orthant holding w.
 */
static void cell_vrange(const orc_scene* s, const int32_t c[3], int size, const double* wd, double* lo, double* hi)
{
    if (s->vgrid_mode == ORC_VGRID_ORTHANT) {
        int q = 0;
        for (int a = 0; a < s->dim; ++a)
            if (wd[a] < 0.0) q |= 1 << a;
        orth_ctx ch = {q, 1}, cl = {q, 0};
        *hi = cube_max(s, field_orth, &ch, c, size);
        *lo = -cube_max(s, field_orth, &cl, c, size);
    } else {
        double V = cube_max(s, field_speed, NULL, c, size);
        *lo = -V;
        *hi = V;
    }
}

/*
 * Velocity interpolation (Sect. 3.1): a level cell carries n_v nodes u_k
 * uniform in its range [lo, hi] (above); a node value is the average over the
 * cell's MIP-0 voxels of eta, chi evaluated at projected velocity u_k; the
 * ray's projected velocity u = vbar . w (vbar = mean velocity of the cell) is
 * interpolated linearly between the two bracketing nodes.  An empty range
 * (lo = hi, e.g. V = 0) uses its single value.
 */
static void cell_velinterp(const orc_scene* s, const int32_t c[3], int size, const double* wd, int il,
                           double* eta, double* chi)
{
    double lo, hi;
    cell_vrange(s, c, size, wd, &lo, &hi);
    double u = 0.0;
    for (int a = 0; a < s->dim; ++a) u += cell_lin(s, 6 + a, 0, c, size) * wd[a];
    int nvn = s->n_v;
    int k = 0;
    double wgt = 0.0;
    if (hi > lo) {
        double f = (u - lo) / (hi - lo) * (nvn - 1);
        k = (int)floor(f);
        if (k < 0) k = 0;
        if (k > nvn - 2) k = nvn - 2;
        wgt = f - k;
    }
    double nodes_e[2], nodes_c[2];
    for (int j = 0; j < 2; ++j) {
        double uk = (hi > lo) ? (lo + (hi - lo) * (double)(k + j) / (double)(nvn - 1)) : lo;
        for (int q = 0; q < 2; ++q) {
            node_ctx nc = {il, uk, q};
            double val;
            if (size == 1)
                val = node_val(s, vox_index(s, c), &nc);
            else if (s->avg_mode == ORC_AVG_LOG)
                val = exp(cube_mean(s, node_log, &nc, c, size)) / s->ds0;
            else
                val = cube_mean(s, node_val, &nc, c, size);
            if (q == 0) nodes_e[j] = val;
            else nodes_c[j] = val;
        }
    }
    *eta = (1.0 - wgt) * nodes_e[0] + wgt * nodes_e[1];
    *chi = (1.0 - wgt) * nodes_c[0] + wgt * nodes_c[1];
}

/*
 * Core and Voigt (Sect. 3.2): the cell's eta*, chi* (and background) are
 * averaged in the stored-value mode, damping, 1/Doppler width and velocity
 * linearly; the line profile is evaluated with these averaged parameters at
 * the ray's projected velocity u = vbar . w.  At level 0 this is exactly the
 * Classic per-voxel evaluation.
 */
static void cell_cav(const orc_scene* s, const int32_t c[3], int size, const double* wd, int il, double* eta,
                     double* chi)
{
    double u = 0.0;
    for (int a = 0; a < s->dim; ++a) u += cell_lin(s, 6 + a, 0, c, size) * wd[a];
    double e = cell_avg_q(s, 4, 0, c, size), x = cell_avg_q(s, 5, 0, c, size);
    for (int l = 0; l < s->n_lines; ++l) {
        double es = cell_avg_q(s, 0, l, c, size), cs = cell_avg_q(s, 1, l, c, size);
        double a0 = cell_lin(s, 2, l, c, size), idl = cell_lin(s, 3, l, c, size);
        double el, cl;
        line_eval(s->profile, s->lam[il], s->lam0[l], es, cs, a0, idl, u, &el, &cl);
        e += el;
        x += cl;
    }
    *eta = e;
    *chi = x;
}

/* ------------------------------------------------------------------ */
/* the march                                                           */
/* ------------------------------------------------------------------ */
/* ------------------------------------------------------------------ */
/* prefiltering (Sect. 5.1)                                            */
/* ------------------------------------------------------------------ */
/*
 * Prefiltered values of every cell of every level for one wavelength, from
 * the MIP-0 values eta0, chi0 [nvox].  For a level-m cell (side 2^m voxels)
 * and a signed axis (a, sign), radiation propagating along sign * e_a crosses
 * the cell along each of its (2^m)^(D-1) rows of MIP-0 voxels parallel to a.
 * Each row is solved exactly, voxel by voxel in the direction of propagation,
 * from I = 0 at its entry face: I <- I exp(-tau) + S (1 - exp(-tau)),
 * tau = chi ds0, and T_row = exp(-sum tau).  The cell's beam-averaged
 * transfer is Ibar = mean_rows I_row and 1 - Tbar = mean_rows (1 - T_row).
 * The equivalent homogeneous cell of side L = 2^m ds0 has the same transfer:
 * tau_eff = -ln(Tbar), chi_eff = tau_eff / L and, since its emergent
 * intensity is S_eff (1 - Tbar), eta_eff = S_eff chi_eff =
 * Ibar tau_eff / ((1 - Tbar) L), or Ibar / L when Tbar = 1.  Tbar = mean T_row
 * and 1 - Tbar = mean (1 - T_row) are summed separately (no cancellation at
 * either end); tau_eff = -ln(1 - (1 - Tbar)) while 1 - Tbar < 1/2, -ln(Tbar)
 * beyond, and, when every row is opaque enough for T_row to underflow
 * (Tbar = 0), the mean row optical depth (any such cell transmits nothing).
 * Output index:
 * (level offset + cell) * 2D + k, k = 2 a + (sign < 0).  Empty (inactive)
 * regions give zeros like the other level values.
 */
void orc_prefilter(const orc_scene* s, const double* eta0, const double* chi0, double* pf_eta, double* pf_chi)
{
    const int D = s->dim;
    const int K = 2 * D;
    for (int m = 0; m < s->n_levels; ++m) {
        const int side = 1 << m;
        const int32_t nc[3] = {s->n[0] >> m, D > 1 ? s->n[1] >> m : 1, D > 2 ? s->n[2] >> m : 1};
        const int64_t off = level_offset(s, m);
        for (int32_t cz = 0; cz < nc[2]; ++cz)
            for (int32_t cy = 0; cy < nc[1]; ++cy)
                for (int32_t cx = 0; cx < nc[0]; ++cx) {
                    const int32_t corner[3] = {cx * side, cy * side, cz * side};
                    const int64_t ci = cx + (int64_t)nc[0] * (cy + (int64_t)nc[1] * cz);
                    for (int a = 0; a < D; ++a)
                        for (int neg = 0; neg < 2; ++neg) {
                            /* the two axes across the rows (unused ones have extent 1) */
                            int b0 = -1, b1 = -1;
                            for (int b = 0; b < D; ++b)
                                if (b != a) {
                                    if (b0 < 0) b0 = b;
                                    else b1 = b;
                                }
                            const int e0 = b0 >= 0 ? side : 1, e1 = b1 >= 0 ? side : 1;
                            double sumI = 0.0, sumA = 0.0, sumT = 0.0, sumTau = 0.0;
                            for (int r1 = 0; r1 < e1; ++r1)
                                for (int r0 = 0; r0 < e0; ++r0) {
                                    double I = 0.0, tau_row = 0.0;
                                    for (int j = 0; j < side; ++j) {
                                        int32_t c[3] = {corner[0], corner[1], corner[2]};
                                        if (b0 >= 0) c[b0] += r0;
                                        if (b1 >= 0) c[b1] += r1;
                                        c[a] += neg ? side - 1 - j : j; /* entry face first */
                                        const int64_t v = vox_index(s, c);
                                        const double tau = chi0[v] * s->ds0;
                                        if (tau == 0.0) {
                                            I += eta0[v] * s->ds0;
                                        } else {
                                            I = I * exp(-tau) + (eta0[v] / chi0[v]) * (-expm1(-tau));
                                        }
                                        tau_row += tau;
                                    }
                                    sumI += I;
                                    sumA += -expm1(-tau_row);
                                    sumT += exp(-tau_row);
                                    sumTau += tau_row;
                                }
                            const double rows = (double)e0 * (double)e1;
                            const double Ibar = sumI / rows, absorbed = sumA / rows, Tbar = sumT / rows;
                            const double L = side * s->ds0;
                            double ce = 0.0, ee = 0.0;
                            if (absorbed > 0.0) {
                                const double tau_eff = absorbed < 0.5 ? -log1p(-absorbed)
                                                       : (Tbar > 0.0 ? -log(Tbar) : sumTau / rows);
                                ce = tau_eff / L;
                                ee = Ibar * tau_eff / (absorbed * L);
                            } else {
                                ee = Ibar / L;
                            }
                            const int k = 2 * a + neg;
                            pf_eta[(off + ci) * K + k] = ee;
                            pf_chi[(off + ci) * K + k] = ce;
                        }
                }
    }
}

/* Direction blend of a prefiltered cell: weights w_a^2 over the signed axes the
 * ray propagates along (normalised by their sum). */
static void cell_prefilter(const orc_scene* s, int il, int m, const int32_t c[3], const double* wd, double* eta,
                           double* chi)
{
    const int D = s->dim, K = 2 * D;
    const int64_t tot = orc_level_total(D, s->n, s->n_levels);
    const int64_t o = ((int64_t)il * tot + level_offset(s, m) + level_index(s, m, c)) * K;
    double e = 0.0, x = 0.0, ws = 0.0;
    for (int a = 0; a < D; ++a) {
        const double wa = wd[a] * wd[a];
        const int k = 2 * a + (wd[a] < 0.0);
        e += wa * s->pf_eta[o + k];
        x += wa * s->pf_chi[o + k];
        ws += wa;
    }
    *eta = e / ws;
    *chi = x / ws;
}

/*
 * For each ray r (probe voxel ray_vox[r], direction dirs[ray_dir[r]]) and each
 * wavelength il: I_out[r * n_lam + il] over the path interval [t1, t2] of the
 * ray (t1 = 0, t2 = infinity: the whole ray).  emis selects where a cell's
 * eta, chi come from (ORC_STATIC: st_eta/st_chi level grids; ORC_CLASSIC: line
 * model at the voxel, level 0 only; ORC_VELINTERP; ORC_CAV).  Each piece of the
 * ray's cell list is clipped to [t1, t2]; pieces left with no length are
 * dropped.  The recurrence starts at the far end of the interval from I0 if
 * the ray leaves the grid inside the interval (t1 < t_exit <= t2), else from 0
 * (the far field is another interval's).  T_out (nullable) receives the
 * transmittance of the interval, the product of exp(-tau) over its pieces.
 * nseg_out (nullable) receives the number of segments of each ray.
 */
static int march_rays(const orc_scene* s, int32_t emis, const int8_t* levels, const float* dirs, int64_t n_rays,
                      const int32_t* ray_vox, const int32_t* ray_dir, double t1, double t2, double* I_out,
                      double* T_out, int32_t n_threads, int32_t* nseg_out)
{
    const int D = s->dim;
    int cap = 0;
    for (int a = 0; a < D; ++a) cap += s->n[a];
    cap += 8;
    const int64_t tot = orc_level_total(D, s->n, s->n_levels);
    int err = 0;
    if (s->profile == ORC_VOIGT) weid_init();
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel
    {
        int32_t* sc = (int32_t*)malloc(sizeof(int32_t) * 3 * cap);
        double* sti = (double*)malloc(sizeof(double) * cap);
        double* sto = (double*)malloc(sizeof(double) * cap);
        int32_t* cell = (int32_t*)malloc(sizeof(int32_t) * 3 * cap);
        int32_t* lv = (int32_t*)malloc(sizeof(int32_t) * cap);
        double* ti = (double*)malloc(sizeof(double) * cap);
        double* to = (double*)malloc(sizeof(double) * cap);
        double* se = (double*)malloc(sizeof(double) * cap);
        double* sx = (double*)malloc(sizeof(double) * cap);
#pragma omp for schedule(dynamic, 16)
        for (int64_t r = 0; r < n_rays; ++r) {
            int64_t v = ray_vox[r];
            int32_t pv[3] = {(int32_t)(v % s->n[0]), (int32_t)((v / s->n[0]) % s->n[1]),
                             (int32_t)(v / ((int64_t)s->n[0] * s->n[1]))};
            const float* w = dirs + (int64_t)ray_dir[r] * D;
            float w3[3] = {0, 0, 0};
            double wd[3] = {0, 0, 0};
            double texit = INFINITY;
            for (int a = 0; a < D; ++a) {
                w3[a] = w[a];
                wd[a] = (double)w[a];
                /* the ray leaves the box through the first boundary plane it reaches */
                double te = INFINITY;
                if (wd[a] > 0) te = (pv[a] + 0.5) / wd[a];
                else if (wd[a] < 0) te = (pv[a] + 0.5 - s->n[a]) / wd[a];
                if (te < texit) texit = te;
            }
            int ns = orc_ray_segments(s, levels, pv, w3, cap, cell, lv, ti, to, sc, sti, sto, cap);
            if (ns < 0) {
#pragma omp atomic write
                err = 1;
                continue;
            }
            /* clip to [t1, t2] */
            int nc = 0;
            for (int i = 0; i < ns; ++i) {
                double a0 = ti[i] > t1 ? ti[i] : t1;
                double b0 = to[i] < t2 ? to[i] : t2;
                if (!(b0 > a0)) continue;
                for (int a = 0; a < 3; ++a) cell[3 * nc + a] = cell[3 * i + a];
                lv[nc] = lv[i];
                ti[nc] = a0;
                to[nc] = b0;
                ++nc;
            }
            ns = nc;
            const int exits = t1 < texit && texit <= t2;
            if (nseg_out) nseg_out[r] = ns;
            for (int il = 0; il < s->n_lam; ++il) {
                for (int i = 0; i < ns; ++i) {
                    const int32_t* c = cell + 3 * i;
                    int m = lv[i], size = 1 << m;
                    double e = 0.0, x = 0.0;
                    if (emis == ORC_STATIC || (emis == ORC_PREFILTER && m == 0)) {
                        int64_t o = (int64_t)il * tot + level_offset(s, m) + level_index(s, m, c);
                        e = s->st_eta[o];
                        x = s->st_chi[o];
                    } else if (emis == ORC_PREFILTER) {
                        cell_prefilter(s, il, m, c, wd, &e, &x);
                    } else if (emis == ORC_CLASSIC) {
                        double u = 0.0;
                        int64_t vv = vox_index(s, c);
                        for (int a = 0; a < D; ++a) u += (double)s->vel[a * nvox_of(s) + vv] * wd[a];
                        voxel_emis(s, vv, il, u, &e, &x);
                    } else if (emis == ORC_VELINTERP) {
                        cell_velinterp(s, c, size, wd, il, &e, &x);
                    } else {
                        cell_cav(s, c, size, wd, il, &e, &x);
                    }
                    se[i] = e;
                    sx[i] = x;
                }
                /* far end of the interval -> near end */
                double I = exits ? s->I0 : 0.0, T = 1.0;
                for (int i = ns - 1; i >= 0; --i) {
                    double len = (to[i] - ti[i]) * s->ds0;
                    if (sx[i] == 0.0) {
                        I += se[i] * len;
                    } else {
                        double tau = sx[i] * len;
                        I = I * exp(-tau) + (se[i] / sx[i]) * (-expm1(-tau));
                        T *= exp(-tau);
                    }
                }
                I_out[r * s->n_lam + il] = I;
                if (T_out) T_out[r * s->n_lam + il] = T;
            }
        }
        free(sc);
        free(sti);
        free(sto);
        free(cell);
        free(lv);
        free(ti);
        free(to);
        free(se);
        free(sx);
    }
    return err ? -1 : 0;
}

int orc_march(const orc_scene* s, int32_t emis, const int8_t* levels, const float* dirs, int64_t n_rays,
              const int32_t* ray_vox, const int32_t* ray_dir, double* I_out, int32_t n_threads,
              int32_t* nseg_out)
{
    return march_rays(s, emis, levels, dirs, n_rays, ray_vox, ray_dir, 0.0, INFINITY, I_out, NULL, n_threads,
                      nseg_out);
}

int orc_march_interval(const orc_scene* s, int32_t emis, const int8_t* levels, const float* dirs, int64_t n_rays,
                       const int32_t* ray_vox, const int32_t* ray_dir, double t1, double t2, double* I_out,
                       double* T_out, int32_t n_threads)
{
    if (!(t1 >= 0.0) || !(t2 >= t1)) return -2;
    return march_rays(s, emis, levels, dirs, n_rays, ray_vox, ray_dir, t1, t2, I_out, T_out, n_threads, NULL);
}

/* vectorised H(a, x) for tests */
void orc_voigt_h_vec(int64_t n, const double* a, const double* x, double* out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = orc_voigt_h(a[i], x[i]);
}
