/*
 * Sanitizer driver of the C oracle (built by the CPU tests together with
 * oracle/fea_oracle.c under -fsanitize=address,undefined). Reads a mesh
 * written by the test as raw arrays from directory argv[1]:
 *   sizes.i64   n_nodes, n_elems, conn_len
 *   types.u8 conn_ptr.i64 conn.i32 x.f64 y.f64 z.f64 young.f64 nu.f64
 *   nh.u8 u.f64 source.f64 (3 per element)
 * runs every oracle routine the tests use (graph, colouring, Algorithm 1
 * with |term| sums for three models, the OpenMP variants, the residual and
 * the subgrid scale) and writes their results to argv[1] for comparison.
 * Exit status 0 on success.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t or_graph_rows(int64_t, int64_t, const uint8_t *, const int64_t *, const int32_t *, int64_t *, int64_t *);
int or_graph_fill(int64_t, int64_t, const int64_t *, const int32_t *, const int64_t *, const int64_t *, int32_t *,
                  int32_t *, int64_t *, int32_t *);
int or_colour_greedy(int64_t, int64_t, const int64_t *, const int32_t *, int16_t *);
int64_t or_assemble(int64_t, int64_t, const uint8_t *, const int64_t *, const int32_t *, const double *,
                    const double *, const double *, int, const double *, const double *, const uint8_t *,
                    const double *, const double *, const int64_t *, const int64_t *, const int32_t *, double *,
                    double *, double *, double *);
int64_t or_assemble_omp(int, int64_t, int64_t, const uint8_t *, const int64_t *, const int32_t *, const double *,
                        const double *, const double *, int, const double *, const double *, const uint8_t *,
                        const double *, const double *, const int64_t *, const int64_t *, const int32_t *,
                        const int64_t *, const int32_t *, int, double *, double *);
int64_t or_residual(int64_t, int64_t, const uint8_t *, const int64_t *, const int32_t *, const double *,
                    const double *, const double *, const double *, const double *, const uint8_t *, const double *,
                    const double *, double *);
int64_t or_subscale(int64_t, const uint8_t *, const int64_t *, const int32_t *, const double *, const double *,
                    const double *, int, const double *, const double *, const double *, const double *, int64_t *,
                    double *);

static char dir[4096];

static void *load(const char *name, size_t bytes)
{
    char path[4200];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE *f = fopen(path, "rb");
    if (!f) { fprintf(stderr, "cannot open %s\n", path); exit(2); }
    void *p = malloc(bytes ? bytes : 1);
    if (bytes && fread(p, 1, bytes, f) != bytes) { fprintf(stderr, "short read %s\n", path); exit(2); }
    fclose(f);
    return p;
}

static void save(const char *name, const void *p, size_t bytes)
{
    char path[4200];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE *f = fopen(path, "wb");
    if (!f || fwrite(p, 1, bytes, f) != bytes) { fprintf(stderr, "cannot write %s\n", path); exit(2); }
    fclose(f);
}

int main(int argc, char **argv)
{
    if (argc < 2) return 2;
    snprintf(dir, sizeof dir, "%s", argv[1]);
    int64_t *sz = load("sizes.i64", 3 * sizeof(int64_t));
    const int64_t N = sz[0], E = sz[1], C = sz[2];
    uint8_t *types = load("types.u8", (size_t)E);
    int64_t *cptr = load("conn_ptr.i64", sizeof(int64_t) * (size_t)(E + 1));
    int32_t *conn = load("conn.i32", sizeof(int32_t) * (size_t)C);
    double *x = load("x.f64", 8 * (size_t)N), *y = load("y.f64", 8 * (size_t)N), *z = load("z.f64", 8 * (size_t)N);
    double *young = load("young.f64", 8 * (size_t)E), *nu = load("nu.f64", 8 * (size_t)E);
    uint8_t *nh = load("nh.u8", (size_t)E);
    double *u = load("u.f64", 8 * 3 * (size_t)N), *src = load("source.f64", 8 * 3 * (size_t)E);

    int64_t *row_ptr = malloc(sizeof(int64_t) * (size_t)(N + 1)), *map_ptr = malloc(sizeof(int64_t) * (size_t)(E + 1));
    if (or_graph_rows(N, E, types, cptr, conn, row_ptr, map_ptr) != 0) return 3;
    const int64_t nnz = row_ptr[N], ml = map_ptr[E];
    int32_t *col = malloc(4 * (size_t)nnz + 4), *e2nnz = malloc(4 * (size_t)ml + 4), *inv = malloc(4 * (size_t)ml + 4);
    int64_t *inv_ptr = malloc(8 * (size_t)(nnz + 1));
    if (or_graph_fill(N, E, cptr, conn, row_ptr, map_ptr, col, e2nnz, inv_ptr, inv) != 0) return 4;
    save("row_ptr.i64", row_ptr, 8 * (size_t)(N + 1));
    save("e2nnz.i32", e2nnz, 4 * (size_t)ml);
    save("inv.i32", inv, 4 * (size_t)ml);
    int16_t *colour = malloc(2 * (size_t)E + 2);
    const int nc = or_colour_greedy(N, E, cptr, conn, colour);
    if (nc <= 0) return 5;
    save("colour.i16", colour, 2 * (size_t)E);
    /* colour buckets, ascending element id within a colour */
    int64_t *bptr = calloc((size_t)nc + 1, sizeof(int64_t));
    int32_t *belem = malloc(4 * (size_t)E + 4);
    for (int64_t e = 0; e < E; ++e) bptr[colour[e] + 1]++;
    for (int c = 0; c < nc; ++c) bptr[c + 1] += bptr[c];
    int64_t *fill = malloc(8 * (size_t)nc);
    memcpy(fill, bptr, 8 * (size_t)nc);
    for (int64_t e = 0; e < E; ++e) belem[fill[colour[e]]++] = (int32_t)e;

    double *vals = malloc(8 * 9 * (size_t)nnz), *rhs = malloc(8 * 3 * (size_t)N);
    double *tv = malloc(8 * 9 * (size_t)nnz), *tr = malloc(8 * 3 * (size_t)N);
    /* Poisson, linear elasticity, neo-Hookean tangent (|term| sums too) */
    static const char *names[3][2] = {{"p_vals.f64", "p_rhs.f64"}, {"l_vals.f64", "l_rhs.f64"},
                                      {"n_vals.f64", "n_rhs.f64"}};
    for (int m = 0; m < 3; ++m) {
        const int model = m == 0 ? 0 : 1, B = m == 0 ? 1 : 3;
        double *s1 = malloc(8 * (size_t)E);
        for (int64_t e = 0; e < E; ++e) s1[e] = src[3 * e + 2];
        const double *s = m == 0 ? s1 : src;
        if (or_assemble(N, E, types, cptr, conn, x, y, z, model, young, nu, m == 2 ? nh : NULL, u, s, row_ptr,
                        map_ptr, e2nnz, vals, rhs, tv, tr) != 0)
            return 6;
        save(names[m][0], vals, 8 * (size_t)(nnz * B * B));
        save(names[m][1], rhs, 8 * (size_t)(N * B));
        free(s1);
    }
    for (int v = 1; v <= 2; ++v) {
        if (or_assemble_omp(v, N, E, types, cptr, conn, x, y, z, 1, young, nu, nh, u, src, row_ptr, map_ptr, e2nnz,
                            bptr, belem, nc, vals, rhs) != 0)
            return 7;
        save(v == 1 ? "omp_atomic_vals.f64" : "omp_colour_vals.f64", vals, 8 * 9 * (size_t)nnz);
    }
    if (or_residual(N, E, types, cptr, conn, x, y, z, young, nu, nh, u, src, rhs) != 0) return 8;
    save("residual.f64", rhs, 8 * 3 * (size_t)N);
    int64_t *gp = malloc(8 * (size_t)(E + 1));
    double *sub = malloc(8 * 3 * 8 * (size_t)E);
    if (or_subscale(E, types, cptr, conn, x, y, z, 1, young, nu, u, src, gp, sub) != 0) return 9;
    save("subscale.f64", sub, 8 * 3 * (size_t)gp[E]);
    free(types); free(cptr); free(conn); free(x); free(y); free(z); free(young); free(nu); free(nh); free(u);
    free(src); free(sz); free(row_ptr); free(map_ptr); free(col); free(e2nnz); free(inv); free(inv_ptr);
    free(colour); free(bptr); free(belem); free(fill); free(vals); free(rhs); free(tv); free(tr); free(gp); free(sub);
    return 0;
}
