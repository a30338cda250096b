/*
 * Classical RK4 on the oracle's sparse generator (oracle; test
 * infrastructure only: the timed CPU baseline of the benchmark).
 *
 * Input: one problem's generator M_u (Eq. uvar-propagator) as CSR, exported
 * by oracle/cpu_timer.py from oracle.uvar, and its initial state. The
 * integrator is the paper's conventional RK4 (Sec. VII.E) written out as in
 * oracle/integrate.py:
 *     k1 = A y, k2 = A(y + h/2 k1), k3 = A(y + h/2 k2), k4 = A(y + h k3),
 *     y <- y + h/6 (k1 + 2 k2 + 2 k3 + k4),
 * complex double throughout, one sparse matrix-vector product per k, each
 * row summed in CSR order. Rows are split over OpenMP threads (static
 * schedule); no blocking or reordering beyond that.
 *
 * Usage: csr_rk4 DIR STEPS H THREADS
 *   DIR holds n_nnz.i64 (two int64: n, nnz), indptr.i64 (n+1), indices.i64
 *   (nnz), data.c128 (nnz complex), y0.c128 (n complex). Writes y.c128 (the
 *   final state) into DIR and prints one JSON line with the wall time of the
 *   RK4 loop (file input and output excluded) and the threads used.
 */
#include <complex.h>
#include <omp.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

static void *slurp(const char *dir, const char *name, size_t bytes) {
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE *f = fopen(path, "rb");
    if (!f) { fprintf(stderr, "cannot open %s\n", path); exit(2); }
    void *p = malloc(bytes ? bytes : 1);
    if (!p || fread(p, 1, bytes, f) != bytes) { fprintf(stderr, "short read %s\n", path); exit(2); }
    fclose(f);
    return p;
}

/* out = A x */
static void spmv(int64_t n, const int64_t *ip, const int64_t *ix, const double complex *a,
                 const double complex *x, double complex *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double complex s = 0;
        for (int64_t j = ip[i]; j < ip[i + 1]; ++j) s += a[j] * x[ix[j]];
        out[i] = s;
    }
}

/* out = y + c k */
static void axpy(int64_t n, const double complex *y, double c, const double complex *k, double complex *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = y[i] + c * k[i];
}

int main(int argc, char **argv) {
    if (argc != 5) { fprintf(stderr, "usage: csr_rk4 DIR STEPS H THREADS\n"); return 2; }
    const char *dir = argv[1];
    const long steps = atol(argv[2]);
    const double h = atof(argv[3]);
    const int threads = atoi(argv[4]);
    if (threads > 0) omp_set_num_threads(threads);
    int64_t *hdr = slurp(dir, "n_nnz.i64", 2 * sizeof(int64_t));
    const int64_t n = hdr[0], nnz = hdr[1];
    int64_t *ip = slurp(dir, "indptr.i64", (size_t)(n + 1) * sizeof(int64_t));
    int64_t *ix = slurp(dir, "indices.i64", (size_t)nnz * sizeof(int64_t));
    double complex *a = slurp(dir, "data.c128", (size_t)nnz * sizeof(double complex));
    double complex *y = slurp(dir, "y0.c128", (size_t)n * sizeof(double complex));
    double complex *k1 = malloc((size_t)n * sizeof *k1), *k2 = malloc((size_t)n * sizeof *k2);
    double complex *k3 = malloc((size_t)n * sizeof *k3), *k4 = malloc((size_t)n * sizeof *k4);
    double complex *t = malloc((size_t)n * sizeof *t);
    if (!k1 || !k2 || !k3 || !k4 || !t) { fprintf(stderr, "out of memory\n"); return 2; }
    int used = 1;
#pragma omp parallel
    {
#pragma omp single
        used = omp_get_num_threads();
    }
    struct timespec t0, t1;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    for (long s = 0; s < steps; ++s) {
        spmv(n, ip, ix, a, y, k1);
        axpy(n, y, 0.5 * h, k1, t);
        spmv(n, ip, ix, a, t, k2);
        axpy(n, y, 0.5 * h, k2, t);
        spmv(n, ip, ix, a, t, k3);
        axpy(n, y, h, k3, t);
        spmv(n, ip, ix, a, t, k4);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) y[i] = y[i] + (h / 6.0) * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    }
    clock_gettime(CLOCK_MONOTONIC, &t1);
    const double sec = (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
    char path[4096];
    snprintf(path, sizeof path, "%s/y.c128", dir);
    FILE *f = fopen(path, "wb");
    if (!f || fwrite(y, sizeof *y, (size_t)n, f) != (size_t)n) { fprintf(stderr, "cannot write %s\n", path); return 2; }
    fclose(f);
    printf("{\"n\": %lld, \"nnz\": %lld, \"steps\": %ld, \"threads\": %d, \"seconds\": %.9f}\n", (long long)n,
           (long long)nnz, steps, used, sec);
    return 0;
}
