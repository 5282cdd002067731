/*
 * Test infrastructure: exercises the FP64 oracle's entry points on seeded
 * random scenes so that the oracle can be built and run under AddressSanitizer
 * and UndefinedBehaviorSanitizer (tests/test_oracle_sanitize.py compiles this
 * file, which includes orc.c as one translation unit, with gcc).  It checks
 * only that every result is finite and that the calls succeed; the values
 * themselves are pinned by the Python tests.
 */
#include <stdio.h>

#include "orc.c"

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;

static double urand(void)
{
    /* splitmix64 */
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

static int check_finite(const double* x, int64_t n, const char* what)
{
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(x[i])) {
            fprintf(stderr, "%s: non-finite value at %lld\n", what, (long long)i);
            return 1;
        }
    return 0;
}

static int run_static(int dim, int N, int B, int L)
{
    orc_scene s;
    memset(&s, 0, sizeof(s));
    s.dim = dim;
    s.n[0] = s.n[1] = N;
    s.n[2] = dim > 2 ? N : 1;
    s.brick = B;
    s.n_levels = L;
    s.n_lam = 1;
    s.avg_mode = ORC_AVG_LINEAR;
    s.ds0 = 1.0;
    s.I0 = 0.3;
    const int64_t nv = nvox_of(&s);
    const int64_t tot = orc_level_total(dim, s.n, L);
    int64_t nb = 1;
    for (int a = 0; a < dim; ++a) nb *= N / B;
    double* eta0 = malloc(sizeof(double) * nv);
    double* chi0 = malloc(sizeof(double) * nv);
    uint8_t* act = malloc(nb);
    int8_t* lv = malloc(nb);
    double* st_e = malloc(sizeof(double) * tot);
    double* st_c = malloc(sizeof(double) * tot);
    for (int64_t b = 0; b < nb; ++b) act[b] = urand() < 0.7;
    for (int64_t v = 0; v < nv; ++v) {
        eta0[v] = 0.05 + urand();
        chi0[v] = 0.02 + 0.5 * urand();
    }
    int err = 0;
    orc_levels(&s, eta0, chi0, act, 1e-2, 0.25, -1, lv, st_e, st_c);
    s.st_eta = st_e;
    s.st_chi = st_c;
    const int nd = 5, nr = 200;
    float* dirs = malloc(sizeof(float) * nd * dim);
    for (int d = 0; d < nd; ++d) {
        double w[3] = {urand() - 0.5, urand() - 0.5, dim > 2 ? urand() - 0.5 : 0.0};
        double nrm = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        for (int a = 0; a < dim; ++a) dirs[d * dim + a] = (float)(w[a] / nrm);
    }
    int32_t* vox = malloc(sizeof(int32_t) * nr);
    int32_t* rd = malloc(sizeof(int32_t) * nr);
    for (int r = 0; r < nr; ++r) {
        vox[r] = (int32_t)(urand() * (double)nv);
        rd[r] = (int32_t)(urand() * nd);
    }
    double* I = malloc(sizeof(double) * nr);
    double* T = malloc(sizeof(double) * nr);
    const double ld[8] = {0.0, 3.0, 9.0, 27.0, INFINITY, INFINITY, INFINITY, INFINITY};
    for (int g = 0; g < 3; ++g) {
        s.level_dist = g == 0 ? NULL : ld;
        s.grade_mode = g == 2 ? ORC_GRADE_PATH : ORC_GRADE_ENTRY;
        err |= orc_march(&s, ORC_STATIC, lv, dirs, nr, vox, rd, I, 1, NULL) != 0;
        err |= check_finite(I, nr, "march");
        err |= orc_march(&s, ORC_STATIC, NULL, dirs, nr, vox, rd, I, 1, NULL) != 0;
        err |= check_finite(I, nr, "dense march");
        err |= orc_march_interval(&s, ORC_STATIC, lv, dirs, nr, vox, rd, 1.5, 6.0, I, T, 1) != 0;
        err |= check_finite(I, nr, "interval I") | check_finite(T, nr, "interval T");
    }
    free(eta0);
    free(chi0);
    free(act);
    free(lv);
    free(st_e);
    free(st_c);
    free(dirs);
    free(vox);
    free(rd);
    free(I);
    free(T);
    return err;
}

int main(void)
{
    int err = 0;
    err |= run_static(2, 32, 8, 4);
    err |= run_static(3, 16, 8, 4);
    double h = 0.0;
    for (int i = 0; i < 200; ++i) h += orc_voigt_h(1e-3 + urand(), 20.0 * (urand() - 0.5));
    err |= !isfinite(h);
    printf(err ? "sanitize check FAILED\n" : "sanitize check ok\n");
    return err;
}
