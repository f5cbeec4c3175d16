/*
 * sanitize_main.c -- driver that runs the CPU oracle (ray_oracle.c, included
 * as one translation unit) over rays of every model, so that it can be built
 * with the address and undefined-behaviour sanitizers on the host.
 *
 * TEST INFRASTRUCTURE ONLY: built and run by tests/test_oracle_sanitizers.py.
 * Exits 0 when every traced ray ends with a finite result and a known status.
 */
#include "ray_oracle.c"

#include <stdio.h>

static int run(or_params* p, int nrays, int nthreads, const char* name)
{
    const int nq = p->nsub < OR_MAX_SUB ? p->nsub : OR_MAX_SUB;
    const int w = p->nstokes + nq;
    double* al = (double*)malloc(sizeof(double) * nrays);
    double* be = (double*)malloc(sizeof(double) * nrays);
    double* S = (double*)malloc(sizeof(double) * nrays * w);
    ray_feat* ft = (ray_feat*)malloc(sizeof(ray_feat) * nrays);
    for (int i = 0; i < nrays; ++i) {
        al[i] = -18.0 + 36.0 * (i % 9) / 8.0 + 0.37 * (i / 9);
        be[i] = -17.0 + 34.0 * ((i * 7) % 11) / 10.0;
    }
    or_trace(p, nrays, al, be, S, ft, nthreads);
    int bad = 0;
    for (int i = 0; i < nrays; ++i) {
        for (int k = 0; k < w; ++k)
            if (!(S[(size_t)i * w + k] == S[(size_t)i * w + k])) bad++;
        if (ft[i].status < OR_OK || ft[i].status > OR_NAN || ft[i].status == OR_NAN) bad++;
    }
    printf("%-24s %d rays, %d problems\n", name, nrays, bad);
    free(al); free(be); free(S); free(ft);
    return bad;
}

int main(void)
{
    int bad = 0;
    or_params p;
    memset(&p, 0, sizeof(p));
    p.a = 0.94; p.r_cam = 1000.0; p.inc = 163.0 * OR_PI / 180.0; p.r_out = 1000.0; p.eps = 0.03;
    p.max_steps = 100000; p.nstokes = 4; p.model = OR_MODEL_THERMAL; p.freq = 230e9;
    p.L_cm = 5.906e11;
    double thermal[9] = { 2.0e6, 100.0, 10.0, 10.0, 1.3, 50.0, 1.1, 0.84, 1.0 };
    for (int i = 0; i < 9; ++i) p.mp[i] = thermal[i];
    bad += run(&p, 72, 2, "thermal IQUV");
    p.nstokes = 1;
    p.nsub = 4;
    bad += run(&p, 72, 2, "thermal I, subrings");
    p.nsub = 0;
    p.a = 0.0; p.inc = 17.0 * OR_PI / 180.0; p.model = OR_MODEL_TOYDISK;
    memset(p.mp, 0, sizeof(p.mp));
    p.mp[0] = 2.0; p.mp[1] = 0.3;
    bad += run(&p, 72, 2, "toy disk");
    /* small gridded snapshot: a smooth torus-like density, rotation, field */
    const int n1 = 12, n2 = 10, n3 = 8;
    float* g = (float*)malloc(sizeof(float) * 8 * n1 * n2 * n3);
    for (int k = 0; k < n3; ++k)
        for (int j = 0; j < n2; ++j)
            for (int i = 0; i < n1; ++i) {
                float* c = g + (((size_t)k * n2 + j) * n1 + i) * 8;
                const double r = exp(log(1.5) + (i + 0.5) * (log(60.0) - log(1.5)) / n1);
                const double th = mks_theta((j + 0.5) / n2, 0.3);
                const double rho = exp(-0.5 * (r - 12.0) * (r - 12.0) / 9.0 - 2.0 * cos(th) * cos(th)) + 1e-4;
                c[0] = (float)rho; c[1] = (float)(rho / (3.0 * r)); c[2] = -0.01f; c[3] = 0.0f;
                c[4] = (float)(0.5 / sqrt(r)); c[5] = 0.01f; c[6] = 0.0f; c[7] = (float)(0.1 * sqrt(rho / r));
            }
    p.a = 0.5; p.inc = 60.0 * OR_PI / 180.0; p.model = OR_MODEL_GRID; p.nstokes = 4;
    memset(p.mp, 0, sizeof(p.mp));
    p.mp[0] = 3e7; p.mp[1] = 20.0; p.mp[2] = 1.0; p.mp[3] = 13.0 / 9.0; p.mp[4] = 1.0; p.mp[5] = 50.0;
    p.mp[6] = log(1.5); p.mp[7] = (log(60.0) - log(1.5)) / n1; p.mp[8] = 0.3;
    p.mp[9] = n1; p.mp[10] = n2; p.mp[11] = n3;
    p.grid = g; p.n1 = n1; p.n2 = n2; p.n3 = n3; p.phi_cam = 0.7;
    bad += run(&p, 72, 2, "gridded snapshot IQUV");
    free(g);
    p.grid = 0;
    p.model = OR_MODEL_SCREEN_RING;
    memset(p.mp, 0, sizeof(p.mp));
    p.mp[0] = 5.0; p.mp[1] = 0.35; p.mp[2] = 0.05; p.mp[3] = 6.0;
    bad += run(&p, 72, 2, "screen ring");
    printf("%s\n", bad ? "PROBLEMS" : "OK");
    return bad ? 1 : 0;
}
