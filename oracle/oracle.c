/*
 * oracle.c -- brute-force FP64 reference for the per-particle Voronoi
 * tessellation of a periodic (or bounded) point set.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP implementation.
 *
 * What it computes, and where the paper defines it:
 *   - Section 1 (definition): the cell of particle i is the region of space
 *     closer to x_i than to any other particle.  With periodic conditions
 *     (abstract; section 4) every periodic image x_j + L t counts as a
 *     particle.
 *   - Section 2 (after the buffer discussion): cell volume from the cell's
 *     facets; density = particle mass / cell volume; neighbours are the
 *     particles that share a facet with the cell.
 *   - Section 2 (gather step): outputs in input order, neighbour ids are the
 *     real particle ids.
 *   - Section 2 (boundary particles): a sub-volume is processed together with a
 *     buffer of surrounding particles; here such a sub-volume is a bounded box
 *     whose walls are the initial cell, and a cell that still touches a wall,
 *     or whose security ball leaves the box, is reported as incomplete.
 *
 * Algorithm (plain and slow on purpose; every step follows the definition):
 *   1. Start from the cube [-L/2, L/2]^3 around the seed (the bisectors of the
 *      seed with its own six nearest periodic images), or, for a bounded box,
 *      from the box itself.  The polytope is kept as a boundary representation:
 *      vertices and faces, each face a cyclic vertex list, counter-clockwise
 *      seen from outside, tagged with the particle that generated it.
 *   2. Clip by the bisector half-spaces { y : y.D <= |D|^2 / 2 } (D = minimum
 *      image vector from the seed to particle j) of the 64 nearest particles,
 *      nearest first; each face is clipped Sutherland-Hodgman style and the cut
 *      polygon becomes the new face.
 *   3. Scan ALL particles once more and clip by every j with |D_j| < 2 R not
 *      already applied, where R is the current largest vertex distance (R only
 *      shrinks, so one pass is exhaustive).  The result therefore does not depend on any search
 *      structure.  Periodic results are only claimed when 2R < L/2, where the
 *      minimum image is the only image that can matter.
 *   4. Each final vertex is recomputed from three of the planes that meet
 *      there (a vertex is equidistant from the seed and those particles) in
 *      extended precision, so rounding does not accumulate over the cuts.
 *   5. Volume by fan tetrahedra from the seed; face area and centroid by fan
 *      triangles; faces of (near) zero area are not facets.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC oracle.c -o liboracle.so -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_OK 0
#define ORA_ERR_ARG 1
#define ORA_ERR_NOMEM 2
#define ORA_ERR_CAPACITY 3
#define ORA_ERR_GEOMETRY 4

/* per-cell flag bits */
#define ORA_FLAG_WALL 1        /* a box face (own image / bounded wall) survived */
#define ORA_FLAG_INCOMPLETE 2  /* periodic: 2R >= L/2; bounded: ball(x,2R) leaves the box */
#define ORA_FLAG_CAPACITY 4    /* more faces than the caller's stride */

#define TAG_WALL(k) (-1 - (int64_t)(k)) /* k = 0..5 : -x,+x,-y,+y,-z,+z */
#define K_NEAREST 64

/* ------------------------------------------------------------------------ */
/* boundary representation of a convex polytope                              */

typedef struct {
    int nv, vcap;
    double *v; /* 3*vcap */
    int nf, fcap;
    int *fofs, *flen;
    int64_t *ftag;
    int nfv, fvcap;
    int *fv;
} poly;

typedef struct {
    poly a, b;          /* double buffer */
    double *s;          /* side values per vertex */
    int *cls, *map;     /* vertex class, old -> new index */
    int ecap, ne;       /* crossing-edge cache */
    int *ea, *eb, *eid;
    int *tmpi;          /* angle sort scratch */
    double *tmpd;
    int tcap;           /* capacity of s, cls, map, tmpi, tmpd */
} work;

static int grow_int(int **p, int *cap, int need) {
    if (need <= *cap) return 0;
    int c = *cap ? *cap : 64;
    while (c < need) c *= 2;
    int *q = (int *)realloc(*p, sizeof(int) * (size_t)c);
    if (!q) return -1;
    *p = q;
    *cap = c;
    return 0;
}

static int poly_reserve_v(poly *P, int nv) {
    if (nv <= P->vcap) return 0;
    int c = P->vcap ? P->vcap : 64;
    while (c < nv) c *= 2;
    double *q = (double *)realloc(P->v, sizeof(double) * 3 * (size_t)c);
    if (!q) return -1;
    P->v = q;
    P->vcap = c;
    return 0;
}

static int poly_reserve_f(poly *P, int nf) {
    if (nf <= P->fcap) return 0;
    int c = P->fcap ? P->fcap : 32;
    while (c < nf) c *= 2;
    int *o = (int *)realloc(P->fofs, sizeof(int) * (size_t)c);
    if (!o) return -1;
    P->fofs = o;
    int *l = (int *)realloc(P->flen, sizeof(int) * (size_t)c);
    if (!l) return -1;
    P->flen = l;
    int64_t *t = (int64_t *)realloc(P->ftag, sizeof(int64_t) * (size_t)c);
    if (!t) return -1;
    P->ftag = t;
    P->fcap = c;
    return 0;
}

/* grow every per-vertex scratch array of W to hold `need` entries, keeping contents */
static int work_reserve(work *W, int need) {
    if (need <= W->tcap) return 0;
    int c = W->tcap ? W->tcap : 64;
    while (c < need) c *= 2;
    double *s = (double *)realloc(W->s, sizeof(double) * (size_t)c);
    if (!s) return -1;
    W->s = s;
    int *x = (int *)realloc(W->cls, sizeof(int) * (size_t)c);
    if (!x) return -1;
    W->cls = x;
    x = (int *)realloc(W->map, sizeof(int) * (size_t)c);
    if (!x) return -1;
    W->map = x;
    x = (int *)realloc(W->tmpi, sizeof(int) * (size_t)c);
    if (!x) return -1;
    W->tmpi = x;
    double *t = (double *)realloc(W->tmpd, sizeof(double) * (size_t)c);
    if (!t) return -1;
    W->tmpd = t;
    W->tcap = c;
    return 0;
}

static void poly_free(poly *P) {
    free(P->v);
    free(P->fofs);
    free(P->flen);
    free(P->ftag);
    free(P->fv);
    memset(P, 0, sizeof(*P));
}

static void work_free(work *W) {
    poly_free(&W->a);
    poly_free(&W->b);
    free(W->s);
    free(W->cls);
    free(W->map);
    free(W->ea);
    free(W->eb);
    free(W->eid);
    free(W->tmpi);
    free(W->tmpd);
    memset(W, 0, sizeof(*W));
}

/* axis-aligned box [lo, hi] (seed-relative) as a polytope */
static int poly_box(poly *P, const double lo[3], const double hi[3]) {
    static const int faces[6][4] = {
        {0, 4, 6, 2}, /* -x */
        {1, 3, 7, 5}, /* +x */
        {0, 1, 5, 4}, /* -y */
        {2, 6, 7, 3}, /* +y */
        {0, 2, 3, 1}, /* -z */
        {4, 5, 7, 6}, /* +z */
    };
    if (poly_reserve_v(P, 8) || poly_reserve_f(P, 6) || grow_int(&P->fv, &P->fvcap, 24)) return -1;
    for (int k = 0; k < 8; ++k) {
        P->v[3 * k + 0] = (k & 1) ? hi[0] : lo[0];
        P->v[3 * k + 1] = (k & 2) ? hi[1] : lo[1];
        P->v[3 * k + 2] = (k & 4) ? hi[2] : lo[2];
    }
    P->nv = 8;
    P->nf = 6;
    P->nfv = 24;
    for (int f = 0; f < 6; ++f) {
        P->fofs[f] = 4 * f;
        P->flen[f] = 4;
        P->ftag[f] = TAG_WALL(f);
        for (int k = 0; k < 4; ++k) P->fv[4 * f + k] = faces[f][k];
    }
    return 0;
}

static double poly_rmax2(const poly *P) {
    double r2 = 0.0;
    for (int k = 0; k < P->nv; ++k) {
        const double *p = P->v + 3 * k;
        double d = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
        if (d > r2) r2 = d;
    }
    return r2;
}

/* new vertex on the crossing edge (a, b), shared by the two faces of the edge */
static int edge_vertex(work *W, poly *Q, const poly *P, int a, int b) {
    int lo = a < b ? a : b, hi = a < b ? b : a;
    for (int e = 0; e < W->ne; ++e)
        if (W->ea[e] == lo && W->eb[e] == hi) return W->eid[e];
    if (W->ne >= W->ecap) {
        int c = W->ecap ? 2 * W->ecap : 64;
        int *x = (int *)realloc(W->ea, sizeof(int) * (size_t)c);
        if (!x) return -1;
        W->ea = x;
        x = (int *)realloc(W->eb, sizeof(int) * (size_t)c);
        if (!x) return -1;
        W->eb = x;
        x = (int *)realloc(W->eid, sizeof(int) * (size_t)c);
        if (!x) return -1;
        W->eid = x;
        W->ecap = c;
    }
    /* interpolate from the kept end (class 0) to the removed end (class 2) */
    int in = (W->cls[a] == 0) ? a : b, out = (in == a) ? b : a;
    double si = W->s[in], so = W->s[out];
    double t = si / (si - so);
    if (poly_reserve_v(Q, Q->nv + 1)) return -1;
    const double *pi = P->v + 3 * in, *po = P->v + 3 * out;
    double *q = Q->v + 3 * Q->nv;
    for (int c = 0; c < 3; ++c) q[c] = pi[c] + t * (po[c] - pi[c]);
    int id = Q->nv++;
    W->ea[W->ne] = lo;
    W->eb[W->ne] = hi;
    W->eid[W->ne] = id;
    W->ne++;
    return id;
}

static int face_push(poly *Q, int vid) {
    if (grow_int(&Q->fv, &Q->fvcap, Q->nfv + 1)) return -1;
    Q->fv[Q->nfv++] = vid;
    return 0;
}

/*
 * Clip P by { y : n.y <= d } into Q.  Returns 1 if the polytope changed,
 * 0 if the plane cuts nothing, -1 on error.  Vertices with |n.y - d| <= tau
 * count as lying on the plane.
 */
static int poly_clip(work *W, poly *P, poly *Q, const double n[3], double d, int64_t tag, double tau) {
    if (work_reserve(W, P->nv)) return -1;
    int any_out = 0, any_keep = 0;
    for (int k = 0; k < P->nv; ++k) {
        const double *p = P->v + 3 * k;
        double s = n[0] * p[0] + n[1] * p[1] + n[2] * p[2] - d;
        W->s[k] = s;
        int c = (s > tau) ? 2 : ((s < -tau) ? 0 : 1);
        W->cls[k] = c;
        if (c == 2) any_out = 1; else any_keep = 1;
    }
    if (!any_out) return 0;
    if (!any_keep) return -1;

    Q->nv = 0;
    Q->nf = 0;
    Q->nfv = 0;
    if (poly_reserve_v(Q, P->nv)) return -1;
    for (int k = 0; k < P->nv; ++k) {
        if (W->cls[k] == 2) {
            W->map[k] = -1;
            continue;
        }
        W->map[k] = Q->nv;
        memcpy(Q->v + 3 * Q->nv, P->v + 3 * k, 3 * sizeof(double));
        Q->nv++;
    }
    W->ne = 0;

    for (int f = 0; f < P->nf; ++f) {
        int o = P->fofs[f], m = P->flen[f];
        int start = Q->nfv;
        for (int t = 0; t < m; ++t) {
            int a = P->fv[o + t], b = P->fv[o + (t + 1) % m];
            int ca = W->cls[a], cb = W->cls[b];
            if (ca != 2 && face_push(Q, W->map[a])) return -1;
            if ((ca == 0 && cb == 2) || (ca == 2 && cb == 0)) {
                int id = edge_vertex(W, Q, P, a, b);
                if (id < 0 || face_push(Q, id)) return -1;
            }
        }
        int len = Q->nfv - start;
        if (len >= 3) {
            if (poly_reserve_f(Q, Q->nf + 1)) return -1;
            Q->fofs[Q->nf] = start;
            Q->flen[Q->nf] = len;
            Q->ftag[Q->nf] = P->ftag[f];
            Q->nf++;
        } else {
            Q->nfv = start;
        }
    }

    /* the cut face: every kept vertex lying on the plane, ordered by angle */
    int cnt = 0;
    if (work_reserve(W, Q->nv)) return -1;
    for (int k = 0; k < P->nv; ++k)
        if (W->cls[k] == 1) W->tmpi[cnt++] = W->map[k];
    for (int e = 0; e < W->ne; ++e) W->tmpi[cnt++] = W->eid[e];
    if (cnt >= 3) {
        double c[3] = {0, 0, 0};
        for (int k = 0; k < cnt; ++k)
            for (int j = 0; j < 3; ++j) c[j] += Q->v[3 * W->tmpi[k] + j];
        for (int j = 0; j < 3; ++j) c[j] /= cnt;
        double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        double u[3] = {n[0] / nn, n[1] / nn, n[2] / nn};
        /* e1: any unit vector orthogonal to u; e2 = u x e1 */
        double a[3];
        if (fabs(u[0]) < 0.6) { a[0] = 1; a[1] = 0; a[2] = 0; }
        else { a[0] = 0; a[1] = 1; a[2] = 0; }
        double e1[3] = {a[1] * u[2] - a[2] * u[1], a[2] * u[0] - a[0] * u[2], a[0] * u[1] - a[1] * u[0]};
        double l1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
        for (int j = 0; j < 3; ++j) e1[j] /= l1;
        double e2[3] = {u[1] * e1[2] - u[2] * e1[1], u[2] * e1[0] - u[0] * e1[2], u[0] * e1[1] - u[1] * e1[0]};
        for (int k = 0; k < cnt; ++k) {
            const double *p = Q->v + 3 * W->tmpi[k];
            double r[3] = {p[0] - c[0], p[1] - c[1], p[2] - c[2]};
            W->tmpd[k] = atan2(r[0] * e2[0] + r[1] * e2[1] + r[2] * e2[2], r[0] * e1[0] + r[1] * e1[1] + r[2] * e1[2]);
        }
        /* insertion sort by angle (faces are small) */
        for (int i = 1; i < cnt; ++i) {
            double key = W->tmpd[i];
            int id = W->tmpi[i], j = i - 1;
            while (j >= 0 && W->tmpd[j] > key) {
                W->tmpd[j + 1] = W->tmpd[j];
                W->tmpi[j + 1] = W->tmpi[j];
                --j;
            }
            W->tmpd[j + 1] = key;
            W->tmpi[j + 1] = id;
        }
        if (poly_reserve_f(Q, Q->nf + 1)) return -1;
        Q->fofs[Q->nf] = Q->nfv;
        Q->flen[Q->nf] = cnt;
        Q->ftag[Q->nf] = tag;
        for (int k = 0; k < cnt; ++k)
            if (face_push(Q, W->tmpi[k])) return -1;
        Q->nf++;
    }
    return 1;
}

/* ------------------------------------------------------------------------ */
/* particle geometry                                                         */

typedef struct {
    int64_t n;
    const double *pos;   /* n x 3 */
    const int64_t *gid;  /* nullable: identity */
    double lo[3], hi[3], L[3];
    int periodic;
} world;

static void delta(const world *Wd, int64_t i, int64_t j, double D[3]) {
    for (int c = 0; c < 3; ++c) {
        double t = Wd->pos[3 * j + c] - Wd->pos[3 * i + c];
        if (Wd->periodic) t -= Wd->L[c] * nearbyint(t / Wd->L[c]);
        D[c] = t;
    }
}

/* max-heap of (d2, j) for the K nearest */
typedef struct {
    double d2;
    int64_t j;
} cand;

static int cand_less(const cand *a, const cand *b) {
    return (a->d2 < b->d2) || (a->d2 == b->d2 && a->j < b->j);
}

static void heap_push(cand *h, int *sz, int cap, cand c) {
    if (*sz < cap) {
        int k = (*sz)++;
        h[k] = c;
        while (k > 0) {
            int p = (k - 1) / 2;
            if (cand_less(&h[p], &h[k])) {
                cand t = h[p]; h[p] = h[k]; h[k] = t;
                k = p;
            } else break;
        }
    } else if (cand_less(&c, &h[0])) {
        h[0] = c;
        int k = 0;
        for (;;) {
            int l = 2 * k + 1, r = l + 1, m = k;
            if (l < *sz && cand_less(&h[m], &h[l])) m = l;
            if (r < *sz && cand_less(&h[m], &h[r])) m = r;
            if (m == k) break;
            cand t = h[m]; h[m] = h[k]; h[k] = t;
            k = m;
        }
    }
}

static int cmp_i64(const void *a, const void *b) {
    const int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

static int cmp_cand(const void *a, const void *b) {
    const cand *x = (const cand *)a, *y = (const cand *)b;
    if (cand_less(x, y)) return -1;
    if (cand_less(y, x)) return 1;
    return 0;
}

/*
 * Vertex refinement.  Every vertex of the final cell is a point equidistant
 * from the seed and the particles (or walls) of the faces that meet there.
 * Edge interpolation during clipping lets rounding errors accumulate from one
 * cut to the next, so each vertex is recomputed from three of its incident
 * face planes (the best-conditioned triple) by Cramer's rule in extended
 * precision.  Topology is untouched.
 */
#define REF_MAXF 8
static void plane_of(const world *Wd, int64_t i, int64_t tag, const double blo[3], const double bhi[3],
                     long double n[3], long double *d) {
    if (tag >= 0) {
        double D[3];
        delta(Wd, i, tag, D);
        for (int c = 0; c < 3; ++c) n[c] = D[c];
        *d = 0.5L * (n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    } else {
        int k = (int)(-1 - tag), a = k / 2;
        for (int c = 0; c < 3; ++c) n[c] = 0.0L;
        n[a] = (k & 1) ? 1.0L : -1.0L;
        *d = (k & 1) ? (long double)bhi[a] : -(long double)blo[a];
    }
}

static long double det3(const long double a[3], const long double b[3], const long double c[3]) {
    return a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) + a[2] * (b[0] * c[1] - b[1] * c[0]);
}

static int refine_vertices(const world *Wd, int64_t i, poly *P, const double blo[3], const double bhi[3]) {
    int *inc = (int *)malloc(sizeof(int) * (size_t)P->nv * REF_MAXF);
    int *cnt = (int *)calloc((size_t)P->nv, sizeof(int));
    long double *pl = (long double *)malloc(sizeof(long double) * 4 * (size_t)(P->nf > 0 ? P->nf : 1));
    if (!inc || !cnt || !pl) {
        free(inc);
        free(cnt);
        free(pl);
        return -1;
    }
    for (int f = 0; f < P->nf; ++f) {
        plane_of(Wd, i, P->ftag[f], blo, bhi, pl + 4 * f, pl + 4 * f + 3);
        for (int k = 0; k < P->flen[f]; ++k) {
            int v = P->fv[P->fofs[f] + k];
            if (cnt[v] < REF_MAXF) inc[v * REF_MAXF + cnt[v]++] = f;
        }
    }
    for (int v = 0; v < P->nv; ++v) {
        int m = cnt[v];
        if (m < 3) continue;
        long double best = 0.0L;
        int fa = -1, fb = -1, fc = -1;
        for (int a = 0; a < m; ++a)
            for (int b = a + 1; b < m; ++b)
                for (int c = b + 1; c < m; ++c) {
                    const int *q = inc + v * REF_MAXF;
                    long double dd = fabsl(det3(pl + 4 * q[a], pl + 4 * q[b], pl + 4 * q[c]));
                    if (dd > best) {
                        best = dd;
                        fa = q[a];
                        fb = q[b];
                        fc = q[c];
                    }
                }
        if (fa < 0) continue;
        const long double *A = pl + 4 * fa, *B = pl + 4 * fb, *C = pl + 4 * fc;
        long double det = det3(A, B, C);
        long double r[3] = {A[3], B[3], C[3]};
        for (int col = 0; col < 3; ++col) {
            long double a2[3] = {A[0], A[1], A[2]}, b2[3] = {B[0], B[1], B[2]}, c2[3] = {C[0], C[1], C[2]};
            a2[col] = r[0];
            b2[col] = r[1];
            c2[col] = r[2];
            P->v[3 * v + col] = (double)(det3(a2, b2, c2) / det);
        }
    }
    free(inc);
    free(cnt);
    free(pl);
    return 0;
}

/*
 * Build the cell of particle i into *out (which points at W->a or W->b).
 * Returns 0 on success.  *rmax2 receives the squared largest vertex distance,
 * *nplanes the number of particles with |D| < 2R (plus one), for the cost
 * model of the benchmark.
 */
static int build_cell(const world *Wd, int64_t i, work *W, poly **out, double tol, double *rmax2, int64_t *nplanes) {
    double blo[3], bhi[3];
    for (int c = 0; c < 3; ++c) {
        if (Wd->periodic) {
            blo[c] = -0.5 * Wd->L[c];
            bhi[c] = 0.5 * Wd->L[c];
        } else {
            blo[c] = Wd->lo[c] - Wd->pos[3 * i + c];
            bhi[c] = Wd->hi[c] - Wd->pos[3 * i + c];
        }
    }
    poly *P = &W->a, *Q = &W->b;
    if (poly_box(P, blo, bhi)) return ORA_ERR_NOMEM;

    /* pass A: the K nearest, nearest first */
    cand heap[K_NEAREST];
    int hs = 0;
    for (int64_t j = 0; j < Wd->n; ++j) {
        if (j == i) continue;
        double D[3];
        delta(Wd, i, j, D);
        cand c = {D[0] * D[0] + D[1] * D[1] + D[2] * D[2], j};
        heap_push(heap, &hs, K_NEAREST, c);
    }
    qsort(heap, (size_t)hs, sizeof(cand), cmp_cand);
    double r2 = poly_rmax2(P);
    int napplied = 0;
    for (int k = 0; k < hs; ++k) {
        if (heap[k].d2 >= 4.0 * r2 * (1.0 + 1e-9)) break;
        napplied = k + 1;
        double D[3];
        delta(Wd, i, heap[k].j, D);
        double dd = 0.5 * heap[k].d2;
        double tau = tol * sqrt(heap[k].d2) * sqrt(r2);
        int rc = poly_clip(W, P, Q, D, dd, heap[k].j, tau);
        if (rc < 0) return ORA_ERR_GEOMETRY;
        if (rc > 0) {
            poly *t = P; P = Q; Q = t;
            r2 = poly_rmax2(P);
        }
    }
    /* pass B: every particle, exhaustive.  A bisector already applied in pass A is
       skipped: the cell is an intersection of half-spaces, each taken once (a second
       cut by the same plane could only shave rounding slivers off its own face). */
    int64_t used[K_NEAREST];
    for (int k = 0; k < napplied; ++k) used[k] = heap[k].j;
    qsort(used, (size_t)napplied, sizeof(int64_t), cmp_i64);
    for (int64_t j = 0; j < Wd->n; ++j) {
        if (j == i) continue;
        if (napplied && bsearch(&j, used, (size_t)napplied, sizeof(int64_t), cmp_i64)) continue;
        double D[3];
        delta(Wd, i, j, D);
        double d2 = D[0] * D[0] + D[1] * D[1] + D[2] * D[2];
        if (d2 >= 4.0 * r2 * (1.0 + 1e-9)) continue;
        double tau = tol * sqrt(d2) * sqrt(r2);
        int rc = poly_clip(W, P, Q, D, 0.5 * d2, j, tau);
        if (rc < 0) return ORA_ERR_GEOMETRY;
        if (rc > 0) {
            poly *t = P; P = Q; Q = t;
            r2 = poly_rmax2(P);
        }
    }
    /* planes the security criterion had to examine (cost model only) */
    int64_t np = 1;
    for (int64_t j = 0; j < Wd->n; ++j) {
        if (j == i) continue;
        double D[3];
        delta(Wd, i, j, D);
        if (D[0] * D[0] + D[1] * D[1] + D[2] * D[2] < 4.0 * r2) np++;
    }
    *nplanes = np;
    if (refine_vertices(Wd, i, P, blo, bhi)) return ORA_ERR_NOMEM;
    *rmax2 = poly_rmax2(P);
    *out = P;
    return ORA_OK;
}

typedef struct {
    double area, cen[3];
} face_geom;

/* volume (seed at origin), and per-face area / centroid by fan triangles,
   accumulated in extended precision */
static double poly_measure(const poly *P, face_geom *fg) {
    long double vol = 0.0L;
    for (int f = 0; f < P->nf; ++f) {
        int o = P->fofs[f], m = P->flen[f];
        const double *w0 = P->v + 3 * P->fv[o];
        long double S[3] = {0, 0, 0}, C[3] = {0, 0, 0}, at = 0.0L;
        for (int k = 1; k + 1 < m; ++k) {
            const double *w1 = P->v + 3 * P->fv[o + k];
            const double *w2 = P->v + 3 * P->fv[o + k + 1];
            long double a[3] = {(long double)w1[0] - w0[0], (long double)w1[1] - w0[1], (long double)w1[2] - w0[2]};
            long double b[3] = {(long double)w2[0] - w0[0], (long double)w2[1] - w0[1], (long double)w2[2] - w0[2]};
            long double x[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
            for (int c = 0; c < 3; ++c) S[c] += x[c];
            long double ta = 0.5L * sqrtl(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
            for (int c = 0; c < 3; ++c) C[c] += ta * ((long double)w0[c] + w1[c] + w2[c]) / 3.0L;
            at += ta;
            /* tetrahedron (seed, w0, w1, w2) */
            vol += ((long double)w0[0] * ((long double)w1[1] * w2[2] - (long double)w1[2] * w2[1]) -
                    (long double)w0[1] * ((long double)w1[0] * w2[2] - (long double)w1[2] * w2[0]) +
                    (long double)w0[2] * ((long double)w1[0] * w2[1] - (long double)w1[1] * w2[0])) / 6.0L;
        }
        if (fg) {
            fg[f].area = (double)(0.5L * sqrtl(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]));
            for (int c = 0; c < 3; ++c) fg[f].cen[c] = at > 0 ? (double)(C[c] / at) : w0[c];
        }
    }
    return (double)vol;
}

/* ------------------------------------------------------------------------ */
/* exported entry points                                                    */

static int set_world(world *Wd, int64_t n, const double *pos, const int64_t *gid, const double *lo, const double *hi,
                     int periodic) {
    if (n < 1 || !pos || !lo || !hi) return ORA_ERR_ARG;
    Wd->n = n;
    Wd->pos = pos;
    Wd->gid = gid;
    Wd->periodic = periodic;
    for (int c = 0; c < 3; ++c) {
        Wd->lo[c] = lo[c];
        Wd->hi[c] = hi[c];
        Wd->L[c] = hi[c] - lo[c];
        if (!(Wd->L[c] > 0)) return ORA_ERR_ARG;
    }
    return ORA_OK;
}

/*
 * ora_cells: cells of the particles listed in query[0..nq).
 *   pos        n x 3 positions (FP64), gid optional global ids (else index)
 *   lo, hi     the box; periodic != 0 wraps it, else it is a bounded world
 *   tol        relative on-plane tolerance for the clipping side test
 *   area_eps   faces with area <= area_eps * V^(2/3) are not facets
 *   stride     capacity of the per-cell face arrays
 * outputs (per query q):
 *   vol[q], rmax[q], flags[q], nnb[q]
 *   topo[q*5 + {0..4}] = vertices, edges, faces (all, before the area filter),
 *                        largest vertex degree, planes examined (|D| < 2R, +1)
 *   nbr[q*stride + k]  neighbour global ids, ascending, self excluded
 *   farea[q*stride+k], fcen[(q*stride+k)*3 + c] (seed-relative), fdist[q*stride+k]
 */
int ora_cells(int64_t n, const double *pos, const int64_t *gid, const double *lo, const double *hi, int periodic,
              int64_t nq, const int64_t *query, double tol, double area_eps, int64_t stride, double *vol,
              double *rmax, int32_t *flags, int32_t *nnb, int64_t *topo, int64_t *nbr, double *farea, double *fcen,
              double *fdist, int nthreads) {
    world Wd;
    int rc = set_world(&Wd, n, pos, gid, lo, hi, periodic);
    if (rc) return rc;
    if (nq < 0 || (nq > 0 && !query) || stride < 1) return ORA_ERR_ARG;
    int err = ORA_OK;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        work W;
        memset(&W, 0, sizeof(W));
        face_geom *fg = NULL;
        int fgcap = 0;
        int64_t *ord = NULL;
#pragma omp for schedule(dynamic, 4)
        for (int64_t q = 0; q < nq; ++q) {
            int64_t i = query[q];
            if (i < 0 || i >= n) {
#pragma omp atomic write
                err = ORA_ERR_ARG;
                continue;
            }
            poly *P = NULL;
            double r2 = 0;
            int64_t np = 0;
            int c = build_cell(&Wd, i, &W, &P, tol, &r2, &np);
            if (c) {
#pragma omp atomic write
                err = c;
                continue;
            }
            if (P->nf > fgcap) {
                fgcap = 2 * P->nf;
                fg = (face_geom *)realloc(fg, sizeof(face_geom) * (size_t)fgcap);
                ord = (int64_t *)realloc(ord, sizeof(int64_t) * (size_t)fgcap);
            }
            double V = poly_measure(P, fg);
            int32_t fl = 0;
            double R = sqrt(r2);
            if (Wd.periodic) {
                for (int cc = 0; cc < 3; ++cc)
                    if (2.0 * R >= 0.5 * Wd.L[cc]) fl |= ORA_FLAG_INCOMPLETE;
            } else {
                for (int cc = 0; cc < 3; ++cc) {
                    double x = pos[3 * i + cc];
                    if (x - 2.0 * R < Wd.lo[cc] || x + 2.0 * R > Wd.hi[cc]) fl |= ORA_FLAG_INCOMPLETE;
                }
            }
            /* topology counts on the full polytope */
            int64_t edges2 = 0;
            int maxdeg = 0;
            {
                int *deg = (int *)calloc((size_t)P->nv, sizeof(int));
                for (int f = 0; f < P->nf; ++f) {
                    edges2 += P->flen[f];
                    for (int k = 0; k < P->flen[f]; ++k) deg[P->fv[P->fofs[f] + k]]++;
                }
                int used = 0;
                for (int k = 0; k < P->nv; ++k) {
                    if (deg[k] > maxdeg) maxdeg = deg[k];
                    if (deg[k] > 0) used++;
                }
                topo[5 * q + 0] = used;
                free(deg);
            }
            topo[5 * q + 1] = edges2 / 2;
            topo[5 * q + 2] = P->nf;
            topo[5 * q + 3] = maxdeg;
            topo[5 * q + 4] = np;
            /* facets: positive-area faces generated by other particles */
            double amin = area_eps * pow(fabs(V), 2.0 / 3.0);
            int cnt = 0;
            for (int f = 0; f < P->nf; ++f) {
                if (fg[f].area <= amin) continue;
                if (P->ftag[f] < 0) {
                    fl |= ORA_FLAG_WALL;
                    continue;
                }
                ord[cnt++] = f;
            }
            /* order by global id (insertion sort; lists are short) */
            for (int a = 1; a < cnt; ++a) {
                int64_t f = ord[a];
                int64_t g = gid ? gid[P->ftag[f]] : P->ftag[f];
                int b = a - 1;
                while (b >= 0) {
                    int64_t gb = gid ? gid[P->ftag[ord[b]]] : P->ftag[ord[b]];
                    if (gb <= g) break;
                    ord[b + 1] = ord[b];
                    --b;
                }
                ord[b + 1] = f;
            }
            if (cnt > stride) {
                fl |= ORA_FLAG_CAPACITY;
                cnt = (int)stride;
            }
            for (int k = 0; k < cnt; ++k) {
                int f = (int)ord[k];
                int64_t j = P->ftag[f];
                int64_t slot = q * stride + k;
                nbr[slot] = gid ? gid[j] : j;
                if (farea) farea[slot] = fg[f].area;
                if (fcen)
                    for (int cc = 0; cc < 3; ++cc) fcen[3 * slot + cc] = fg[f].cen[cc];
                if (fdist) {
                    double D[3];
                    delta(&Wd, i, j, D);
                    fdist[slot] = sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
                }
            }
            vol[q] = V;
            rmax[q] = R;
            flags[q] = fl;
            nnb[q] = cnt;
        }
        free(fg);
        free(ord);
        work_free(&W);
    }
    return err;
}

/*
 * ora_grid: exact volume average of the piecewise-constant Voronoi field over
 * a regular grid (section 2, optional grid output).  Voxel (a,b,c) is
 * [lo + (a,b,c) h, lo + (a+1,b+1,c+1) h), h = L / (nx,ny,nz); periodic boxes
 * wrap voxel indices.  grid[(a*ny + b)*nz + c] += value[i] * vol(cell_i ∩ voxel)
 * / vol(voxel), summed over the query cells (the caller zeroes grid).
 */
int ora_grid(int64_t n, const double *pos, const double *lo, const double *hi, int periodic, int64_t nq,
             const int64_t *query, const double *value, double tol, int nx, int ny, int nz, double *grid,
             int nthreads) {
    world Wd;
    int rc = set_world(&Wd, n, pos, NULL, lo, hi, periodic);
    if (rc) return rc;
    if (nx < 1 || ny < 1 || nz < 1 || !grid || !value) return ORA_ERR_ARG;
    int dims[3] = {nx, ny, nz};
    double h[3] = {Wd.L[0] / nx, Wd.L[1] / ny, Wd.L[2] / nz};
    double hv = h[0] * h[1] * h[2];
    int err = ORA_OK;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        work W;
        memset(&W, 0, sizeof(W));
        work V2;
        memset(&V2, 0, sizeof(V2));
#pragma omp for schedule(dynamic, 4)
        for (int64_t q = 0; q < nq; ++q) {
            int64_t i = query[q];
            poly *P = NULL;
            double r2;
            int64_t np;
            if (build_cell(&Wd, i, &W, &P, tol, &r2, &np)) {
#pragma omp atomic write
                err = ORA_ERR_GEOMETRY;
                continue;
            }
            double bmin[3], bmax[3];
            for (int c = 0; c < 3; ++c) {
                bmin[c] = 1e300;
                bmax[c] = -1e300;
            }
            for (int k = 0; k < P->nv; ++k)
                for (int c = 0; c < 3; ++c) {
                    double x = P->v[3 * k + c] + pos[3 * i + c];
                    if (x < bmin[c]) bmin[c] = x;
                    if (x > bmax[c]) bmax[c] = x;
                }
            int a0[3], a1[3];
            for (int c = 0; c < 3; ++c) {
                a0[c] = (int)floor((bmin[c] - Wd.lo[c]) / h[c]);
                a1[c] = (int)floor((bmax[c] - Wd.lo[c]) / h[c]);
            }
            for (int a = a0[0]; a <= a1[0]; ++a)
                for (int b = a0[1]; b <= a1[1]; ++b)
                    for (int c = a0[2]; c <= a1[2]; ++c) {
                        int idx[3] = {a, b, c};
                        int ok = 1;
                        double vlo[3], vhi[3];
                        for (int e = 0; e < 3; ++e) {
                            vlo[e] = Wd.lo[e] + idx[e] * h[e] - pos[3 * i + e];
                            vhi[e] = vlo[e] + h[e];
                            if (periodic) {
                                idx[e] %= dims[e];
                                if (idx[e] < 0) idx[e] += dims[e];
                            } else if (idx[e] < 0 || idx[e] >= dims[e]) {
                                ok = 0;
                            }
                        }
                        if (!ok) continue;
                        /* copy P and clip it by the six voxel walls */
                        poly *A = &V2.a, *B = &V2.b;
                        if (poly_reserve_v(A, P->nv) || poly_reserve_f(A, P->nf) ||
                            grow_int(&A->fv, &A->fvcap, P->nfv)) {
#pragma omp atomic write
                            err = ORA_ERR_NOMEM;
                            continue;
                        }
                        A->nv = P->nv;
                        A->nf = P->nf;
                        A->nfv = P->nfv;
                        memcpy(A->v, P->v, sizeof(double) * 3 * (size_t)P->nv);
                        memcpy(A->fofs, P->fofs, sizeof(int) * (size_t)P->nf);
                        memcpy(A->flen, P->flen, sizeof(int) * (size_t)P->nf);
                        memcpy(A->ftag, P->ftag, sizeof(int64_t) * (size_t)P->nf);
                        memcpy(A->fv, P->fv, sizeof(int) * (size_t)P->nfv);
                        int empty = 0;
                        for (int e = 0; e < 3 && !empty; ++e)
                            for (int sgn = 0; sgn < 2 && !empty; ++sgn) {
                                double nn[3] = {0, 0, 0};
                                double dd;
                                if (sgn == 0) { nn[e] = -1.0; dd = -vlo[e]; }
                                else { nn[e] = 1.0; dd = vhi[e]; }
                                int r = poly_clip(&V2, A, B, nn, dd, -100, 0.0);
                                if (r < 0) empty = 1; /* nothing left inside the voxel */
                                else if (r > 0) { poly *t = A; A = B; B = t; }
                            }
                        if (empty) continue;
                        double vol = poly_measure(A, NULL);
                        if (vol <= 0) continue;
                        double add = value[i] * vol / hv;
                        int64_t g = ((int64_t)idx[0] * ny + idx[1]) * nz + idx[2];
#pragma omp atomic
                        grid[g] += add;
                    }
        }
        work_free(&W);
        work_free(&V2);
    }
    return err;
}

/*
 * ora_structure: the full structure of cell i (the optional full structure
 * output: section 3, memory consumption; section 4): its vertices and its
 * faces as vertex loops.
 *   verts[3k..3k+2]   vertex k, absolute (seed + offset), k < *nv: every
 *                     vertex that lies on a face, in the polytope's order
 *   fid[f]            the id across face f: the neighbour's global id (gid,
 *                     else index), or -1 .. -6 for the walls -x, +x, -y, +y,
 *                     -z, +z; faces of area <= area_eps V^(2/3) are left out
 *                     and the rest are listed in ascending order of fid
 *   floff[f..f+1]     face f's loop in lverts (floff[0] = 0), vertex numbers
 *                     as in verts, counter-clockwise seen from outside
 *   *nv, *nf          vertex and face counts
 * Capacities vcap, fcap (floff holds fcap + 1) and lcap; ORA_ERR_CAPACITY if
 * one is too small.
 */
int ora_structure(int64_t n, const double *pos, const int64_t *gid, const double *lo, const double *hi, int periodic,
                  int64_t i, double tol, double area_eps, int64_t vcap, int64_t fcap, int64_t lcap, double *verts,
                  int64_t *nv, int64_t *fid, int64_t *floff, int64_t *nf, int32_t *lverts) {
    world Wd;
    int rc = set_world(&Wd, n, pos, gid, lo, hi, periodic);
    if (rc) return rc;
    if (i < 0 || i >= n || !verts || !nv || !fid || !floff || !nf || !lverts) return ORA_ERR_ARG;
    work W;
    memset(&W, 0, sizeof(W));
    poly *P = NULL;
    double r2;
    int64_t np;
    rc = build_cell(&Wd, i, &W, &P, tol, &r2, &np);
    face_geom *fg = NULL;
    int *num = NULL, *ord = NULL;
    if (!rc) {
        fg = (face_geom *)malloc(sizeof(face_geom) * (size_t)(P->nf > 0 ? P->nf : 1));
        num = (int *)malloc(sizeof(int) * (size_t)(P->nv > 0 ? P->nv : 1));
        ord = (int *)malloc(sizeof(int) * (size_t)(P->nf > 0 ? P->nf : 1));
        if (!fg || !num || !ord) rc = ORA_ERR_NOMEM;
    }
    if (!rc) {
        double V = poly_measure(P, fg);
        double amin = area_eps * pow(fabs(V), 2.0 / 3.0);
        /* vertices on some face, numbered in the polytope's order */
        for (int k = 0; k < P->nv; ++k) num[k] = -1;
        for (int f = 0; f < P->nf; ++f)
            for (int k = 0; k < P->flen[f]; ++k) num[P->fv[P->fofs[f] + k]] = 0;
        int64_t cntv = 0;
        for (int k = 0; k < P->nv; ++k)
            if (num[k] == 0) num[k] = (int)cntv++;
        /* kept faces, ascending by the id across them */
        int cnt = 0;
        for (int f = 0; f < P->nf; ++f)
            if (fg[f].area > amin) ord[cnt++] = f;
        for (int a = 1; a < cnt; ++a) {
            int f = ord[a];
            int64_t g = P->ftag[f] >= 0 && gid ? gid[P->ftag[f]] : P->ftag[f];
            int b = a - 1;
            while (b >= 0) {
                int64_t gb = P->ftag[ord[b]] >= 0 && gid ? gid[P->ftag[ord[b]]] : P->ftag[ord[b]];
                if (gb <= g) break;
                ord[b + 1] = ord[b];
                --b;
            }
            ord[b + 1] = f;
        }
        int64_t cntl = 0;
        for (int a = 0; a < cnt; ++a) cntl += P->flen[ord[a]];
        if (cntv > vcap || cnt > fcap || cntl > lcap) {
            rc = ORA_ERR_CAPACITY;
        } else {
            for (int k = 0; k < P->nv; ++k)
                if (num[k] >= 0)
                    for (int c = 0; c < 3; ++c) verts[3 * num[k] + c] = pos[3 * i + c] + P->v[3 * k + c];
            *nv = cntv;
            *nf = cnt;
            int64_t o = 0;
            floff[0] = 0;
            for (int a = 0; a < cnt; ++a) {
                int f = ord[a];
                int64_t t = P->ftag[f];
                fid[a] = t >= 0 && gid ? gid[t] : t;
                for (int k = 0; k < P->flen[f]; ++k) lverts[o++] = num[P->fv[P->fofs[f] + k]];
                floff[a + 1] = o;
            }
        }
    }
    free(fg);
    free(num);
    free(ord);
    work_free(&W);
    return rc;
}
