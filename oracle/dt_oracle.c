/*
 * CPU oracle for the Delaunay triangulations maintained by the kinetic
 * method (TEST INFRASTRUCTURE ONLY: nothing in the product path links,
 * loads or calls this file; only the tests, the smoke check and the CPU
 * baseline leg of the benchmark do).
 *
 * What it computes.  For a set S of distinct lattice points with global ids,
 * DT*(S) is the set of counter-clockwise triples (a,b,c) of S whose
 * circumcircle holds no other point of S, where a point exactly on a circle
 * is classified by an infinitesimal lift of every point on the paraboloid
 * z = x^2 + y^2 that grows with the point's id.  This is the empty
 * circumcircle definition of the Delaunay triangulation (Sec. I) made
 * unique for cocircular input, which the paper's uniqueness claim (Sec. I)
 * needs on an integer lattice.
 *
 * How.  From scratch, by incremental Bowyer-Watson insertion, the insertion
 * method the paper names (Sec. IV, "Insertion and Deletion"), with "ghost"
 * triangles joining every convex-hull edge to a vertex at infinity so that
 * points outside the current hull need no special case.  Arithmetic is exact
 * integer only: orient in int64, incircle in __int128, no floating-point
 * filter.  Points are inserted in the order given; the order changes the
 * running time only, never the result.  Nothing is shared with the GPU path.
 *
 * Parity pins: tests compare this code against the O(n^4) definition in
 * oracle/definition.py on small and degenerate inputs, against closed-form
 * examples, against scipy's Qhull on inputs in general position, and check
 * triangle counts, hull and local-Delaunay invariants.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;

#define INF_V (-1) /* the vertex at infinity */

/* ------------------------------------------------------------------ */
/* exact predicates                                                    */
/* ------------------------------------------------------------------ */

/* Twice the signed area of (a,b,c); > 0 when counter-clockwise.
 * |coordinate| < 2^24 so every product is < 2^48: exact in int64. */
int64_t oracle_orient(int64_t ax, int64_t ay, int64_t bx, int64_t by,
                      int64_t cx, int64_t cy) {
    return (bx - ax) * (cy - ay) - (by - ay) * (cx - ax);
}

/* Sign of the lifted determinant | a-d, |a-d|^2 ; b-d, ... ; c-d, ... |,
 * which for a counter-clockwise (a,b,c) is > 0 iff d lies strictly inside
 * the circle through a, b, c.  Computed exactly in 128-bit integers. */
int oracle_incircle_sign(int64_t ax, int64_t ay, int64_t bx, int64_t by,
                         int64_t cx, int64_t cy, int64_t dx, int64_t dy) {
    int64_t adx = ax - dx, ady = ay - dy;
    int64_t bdx = bx - dx, bdy = by - dy;
    int64_t cdx = cx - dx, cdy = cy - dy;
    i128 alift = (i128)adx * adx + (i128)ady * ady;
    i128 blift = (i128)bdx * bdx + (i128)bdy * bdy;
    i128 clift = (i128)cdx * cdx + (i128)cdy * cdy;
    i128 det = alift * ((i128)bdx * cdy - (i128)bdy * cdx)
             + blift * ((i128)cdx * ady - (i128)cdy * adx)
             + clift * ((i128)adx * bdy - (i128)ady * bdx);
    return (det > 0) - (det < 0);
}

static int sgn64(int64_t v) { return (v > 0) - (v < 0); }

/* Perturbed incircle.  When the exact determinant is zero, every point's
 * paraboloid height is raised by an infinitesimal that is larger the larger
 * the point's id; the determinant is linear in each height, so the point m
 * with the largest id decides, through the sign of the cofactor of its
 * height entry in the 4x4 lifted matrix with rows (x, y, x^2+y^2, 1) taken
 * in the order a, b, c, d:
 *   m = a : +orient(b, c, d)      m = b : -orient(a, c, d)
 *   m = c : +orient(a, b, d)      m = d : -orient(a, b, c)
 * The cofactor is never zero for distinct cocircular points (three distinct
 * points on a circle are not collinear). */
int oracle_incircle_star(int64_t ax, int64_t ay, int64_t ida,
                         int64_t bx, int64_t by, int64_t idb,
                         int64_t cx, int64_t cy, int64_t idc,
                         int64_t dx, int64_t dy, int64_t idd) {
    int s = oracle_incircle_sign(ax, ay, bx, by, cx, cy, dx, dy);
    if (s != 0) return s;
    int64_t m = ida;
    int which = 0;
    if (idb > m) { m = idb; which = 1; }
    if (idc > m) { m = idc; which = 2; }
    if (idd > m) { m = idd; which = 3; }
    switch (which) {
    case 0: return sgn64(oracle_orient(bx, by, cx, cy, dx, dy));
    case 1: return -sgn64(oracle_orient(ax, ay, cx, cy, dx, dy));
    case 2: return sgn64(oracle_orient(ax, ay, bx, by, dx, dy));
    default: return -sgn64(oracle_orient(ax, ay, bx, by, cx, cy));
    }
}

/* Ghost triangle (a, b, inf) stands for the open half-plane to the left of
 * a->b (the outside of hull edge b->a).  A new point q destroys it when q
 * lies in that half-plane, or on the line strictly between a and b. */
int oracle_ghost_conflict(int64_t ax, int64_t ay, int64_t bx, int64_t by,
                          int64_t qx, int64_t qy) {
    int64_t o = oracle_orient(ax, ay, bx, by, qx, qy);
    if (o > 0) return 1;
    if (o < 0) return 0;
    int64_t t1 = (qx - ax) * (bx - ax) + (qy - ay) * (by - ay);
    int64_t t2 = (qx - bx) * (ax - bx) + (qy - by) * (ay - by);
    return t1 > 0 && t2 > 0;
}

/* ------------------------------------------------------------------ */
/* triangulation store                                                 */
/* ------------------------------------------------------------------ */

typedef struct {
    int v[3];   /* point indices; a ghost has v[2] == INF_V */
    int nb[3];  /* triangle across the edge opposite v[i] */
    int dead;
} otri;

/* one boundary edge (a, b) of a cavity, seen counter-clockwise from inside,
 * with the surviving triangle `out` behind it and that triangle's edge index */
typedef struct { int a, b; long out; int out_e; } obnd;

typedef struct {
    const int64_t *x, *y, *id;
    long n;
    otri *t;
    long nt, cap;
    long *stack;   /* DFS stack of triangle indices */
    long scap;
    obnd *bnd;     /* cavity boundary edges */
    long bcap;
    long *start_of; /* fan lookup: boundary edge starting at vertex v (n+1 slots) */
} odt;

static int grow(void **p, long *cap, long need, size_t elem) {
    if (need <= *cap) return 0;
    long nc = *cap ? *cap : 64;
    while (nc < need) nc *= 2;
    void *q = realloc(*p, (size_t)nc * elem);
    if (!q) return -1;
    *p = q;
    *cap = nc;
    return 0;
}

static long new_tri(odt *d, int a, int b, int c) {
    if (grow((void **)&d->t, &d->cap, d->nt + 1, sizeof(otri))) return -1;
    otri *t = &d->t[d->nt];
    t->v[0] = a; t->v[1] = b; t->v[2] = c;
    t->nb[0] = t->nb[1] = t->nb[2] = -1;
    t->dead = 0;
    return d->nt++;
}

static int64_t orient_idx(const odt *d, int a, int b, int c) {
    return oracle_orient(d->x[a], d->y[a], d->x[b], d->y[b], d->x[c], d->y[c]);
}

/* Does inserting point q destroy triangle t? */
static int conflicts(const odt *d, const otri *t, int q) {
    if (t->v[2] == INF_V)
        return oracle_ghost_conflict(d->x[t->v[0]], d->y[t->v[0]],
                                     d->x[t->v[1]], d->y[t->v[1]], d->x[q], d->y[q]);
    int a = t->v[0], b = t->v[1], c = t->v[2];
    return oracle_incircle_star(d->x[a], d->y[a], d->id[a], d->x[b], d->y[b], d->id[b],
                                d->x[c], d->y[c], d->id[c], d->x[q], d->y[q], d->id[q]) > 0;
}

/* Find one triangle that q destroys: a visibility walk from `start`
 * (crossing any edge that has q strictly on its outer side), and a scan of
 * every live triangle if the walk has not ended after many steps. */
static long locate(const odt *d, long start, int q) {
    long cur = start;
    for (long hop = 0; hop < 4 * d->nt + 16; hop++) {
        const otri *t = &d->t[cur];
        if (t->v[2] == INF_V) {
            if (conflicts(d, t, q)) return cur;
            cur = t->nb[2]; /* back to the real triangle behind the hull edge */
            continue;
        }
        long next = -1;
        for (int i = 0; i < 3 && next < 0; i++)
            if (orient_idx(d, t->v[(i + 1) % 3], t->v[(i + 2) % 3], q) < 0) next = t->nb[i];
        if (next < 0) return cur; /* q in the closed triangle, so inside its circle */
        cur = next;
    }
    for (long i = 0; i < d->nt; i++)
        if (!d->t[i].dead && conflicts(d, &d->t[i], q)) return i;
    return -1;
}

static int edge_index(const otri *t, int a, int b) {
    /* index i such that edge (v[i+1], v[i+2]) == (a, b) */
    for (int i = 0; i < 3; i++)
        if (t->v[(i + 1) % 3] == a && t->v[(i + 2) % 3] == b) return i;
    return -1;
}

/* Insert point q; `hint` is a triangle to start the walk from.
 * Returns a live triangle incident to q, or -1 on failure. */
static long insert_point(odt *d, int q, long hint) {
    long seed = locate(d, hint, q);
    if (seed < 0) return -1;
    long nb = 0, sp = 0;
    if (grow((void **)&d->stack, &d->scap, 1, sizeof(long))) return -1;
    d->stack[sp++] = seed;
    d->t[seed].dead = 1;
    /* grow the conflict region by depth-first search over adjacency */
    while (sp > 0) {
        long ti = d->stack[--sp];
        for (int e = 0; e < 3; e++) {
            long o = d->t[ti].nb[e];
            if (d->t[o].dead) continue;
            if (conflicts(d, &d->t[o], q)) {
                d->t[o].dead = 1;
                if (grow((void **)&d->stack, &d->scap, sp + 1, sizeof(long))) return -1;
                d->stack[sp++] = o;
            } else {
                if (grow((void **)&d->bnd, &d->bcap, nb + 1, sizeof(obnd))) return -1;
                obnd *bd = &d->bnd[nb++];
                bd->a = d->t[ti].v[(e + 1) % 3];
                bd->b = d->t[ti].v[(e + 2) % 3];
                bd->out = o;
                bd->out_e = edge_index(&d->t[o], bd->b, bd->a);
            }
        }
    }
    /* fan: connect q to every boundary edge (a, b) */
    long first = d->nt;
    for (long i = 0; i < nb; i++) {
        int a = d->bnd[i].a, b = d->bnd[i].b;
        long nt;
        if (a == INF_V) nt = new_tri(d, b, q, INF_V);
        else if (b == INF_V) nt = new_tri(d, q, a, INF_V);
        else nt = new_tri(d, a, b, q);
        if (nt < 0) return -1;
        int e = edge_index(&d->t[nt], a, b);
        d->t[nt].nb[e] = (int)d->bnd[i].out;
        d->t[d->bnd[i].out].nb[d->bnd[i].out_e] = (int)nt;
        d->start_of[a == INF_V ? d->n : a] = nt;
    }
    /* the fan triangle on edge (a, b) meets, across (b, q), the one whose
     * boundary edge starts at b */
    for (long i = 0; i < nb; i++) {
        long ti = first + i;
        int b = d->bnd[i].b;
        long tj = d->start_of[b == INF_V ? d->n : b];
        int eb = edge_index(&d->t[ti], b, q);
        int ej = edge_index(&d->t[tj], q, b);
        if (eb < 0 || ej < 0) return -1;
        d->t[ti].nb[eb] = (int)tj;
        d->t[tj].nb[ej] = (int)ti;
    }
    return first;
}

typedef struct { int64_t x, y; } pxy;
static int cmp_pxy(const void *pa, const void *pb) {
    const pxy *a = pa, *b = pb;
    if (a->x != b->x) return a->x < b->x ? -1 : 1;
    if (a->y != b->y) return a->y < b->y ? -1 : 1;
    return 0;
}

typedef struct { int64_t a, b, c; } tri3;
static int cmp_tri3(const void *pa, const void *pb) {
    const tri3 *a = pa, *b = pb;
    if (a->a != b->a) return a->a < b->a ? -1 : 1;
    if (a->b != b->b) return a->b < b->b ? -1 : 1;
    if (a->c != b->c) return a->c < b->c ? -1 : 1;
    return 0;
}

static void odt_free(odt *d) {
    free(d->t); free(d->stack); free(d->bnd); free(d->start_of);
}

/*
 * oracle_dt: DT*(S) of n points.
 *   xy    int32 [n][2] coordinates in [0, 2^24)
 *   ids   int64 [n] distinct global ids (the perturbation order)
 *   out   int64 [cap][3] receives the real triangles as global ids, each
 *         counter-clockwise and rotated so that its smallest id comes first,
 *         the list sorted lexicographically
 * Returns the number of triangles (which may exceed cap: then only cap are
 * written), or -1 bad arguments, -2 coordinate out of range, -3 duplicate
 * point, -4 fewer than 3 points or all points collinear, -5 out of memory,
 * -8 internal failure.
 */
long oracle_dt(const int32_t *xy, const int64_t *ids, long n, int64_t *out, long cap) {
    if (!xy || !ids || n < 0 || (cap > 0 && !out)) return -1;
    if (n < 3) return -4;
    long rc = 0;
    int64_t *x = malloc(sizeof(int64_t) * n), *y = malloc(sizeof(int64_t) * n);
    pxy *srt = malloc(sizeof(pxy) * n);
    odt d;
    memset(&d, 0, sizeof d);
    if (!x || !y || !srt) { rc = -5; goto done; }
    for (long i = 0; i < n; i++) {
        if (xy[2 * i] < 0 || xy[2 * i] >= (1 << 24) || xy[2 * i + 1] < 0 ||
            xy[2 * i + 1] >= (1 << 24)) { rc = -2; goto done; }
        x[i] = xy[2 * i];
        y[i] = xy[2 * i + 1];
        srt[i].x = x[i];
        srt[i].y = y[i];
    }
    qsort(srt, n, sizeof(pxy), cmp_pxy);
    for (long i = 1; i < n; i++)
        if (srt[i].x == srt[i - 1].x && srt[i].y == srt[i - 1].y) { rc = -3; goto done; }

    d.x = x; d.y = y; d.id = ids; d.n = n;
    d.start_of = malloc(sizeof(long) * (n + 1));
    if (!d.start_of) { rc = -5; goto done; }

    /* first triangle: points 0, 1 and the first point not on their line */
    long k = -1;
    for (long i = 2; i < n; i++)
        if (orient_idx(&d, 0, 1, (int)i) != 0) { k = i; break; }
    if (k < 0) { rc = -4; goto done; }
    int a = 0, b = 1, c = (int)k;
    if (orient_idx(&d, a, b, c) < 0) { int s = a; a = b; b = s; }
    long t0 = new_tri(&d, a, b, c);
    long g0 = new_tri(&d, b, a, INF_V); /* outside of edge a->b */
    long g1 = new_tri(&d, c, b, INF_V);
    long g2 = new_tri(&d, a, c, INF_V);
    if (t0 < 0 || g0 < 0 || g1 < 0 || g2 < 0) { rc = -5; goto done; }
    /* real triangle: edge opposite a is (b,c) -> g1, opposite b is (c,a) -> g2,
     * opposite c is (a,b) -> g0 */
    d.t[t0].nb[0] = (int)g1; d.t[t0].nb[1] = (int)g2; d.t[t0].nb[2] = (int)g0;
    /* ghost (u, v, inf): nb[2] is the real triangle, nb[0] (edge v-inf) and
     * nb[1] (edge inf-u) are the neighbouring ghosts */
    d.t[g0].nb[2] = (int)t0; d.t[g0].nb[0] = (int)g2; d.t[g0].nb[1] = (int)g1;
    d.t[g1].nb[2] = (int)t0; d.t[g1].nb[0] = (int)g0; d.t[g1].nb[1] = (int)g2;
    d.t[g2].nb[2] = (int)t0; d.t[g2].nb[0] = (int)g1; d.t[g2].nb[1] = (int)g0;

    long hint = t0;
    for (long i = 2; i < n; i++) {
        if (i == k) continue;
        long r = insert_point(&d, (int)i, hint);
        if (r < 0) { rc = -8; goto done; }
        hint = r;
    }

    /* collect, canonicalise, sort */
    long cnt = 0;
    for (long i = 0; i < d.nt; i++)
        if (!d.t[i].dead && d.t[i].v[2] != INF_V) cnt++;
    tri3 *res = malloc(sizeof(tri3) * (cnt ? cnt : 1));
    if (!res) { rc = -5; goto done; }
    long j = 0;
    for (long i = 0; i < d.nt; i++) {
        const otri *t = &d.t[i];
        if (t->dead || t->v[2] == INF_V) continue;
        int64_t u0 = ids[t->v[0]], u1 = ids[t->v[1]], u2 = ids[t->v[2]];
        if (u1 < u0 && u1 < u2) { int64_t s = u0; u0 = u1; u1 = u2; u2 = s; }
        else if (u2 < u0 && u2 < u1) { int64_t s = u2; u2 = u1; u1 = u0; u0 = s; }
        res[j].a = u0; res[j].b = u1; res[j].c = u2;
        j++;
    }
    qsort(res, cnt, sizeof(tri3), cmp_tri3);
    for (long i = 0; i < cnt && i < cap; i++) {
        out[3 * i] = res[i].a;
        out[3 * i + 1] = res[i].b;
        out[3 * i + 2] = res[i].c;
    }
    free(res);
    rc = cnt;
done:
    free(x); free(y); free(srt);
    odt_free(&d);
    return rc;
}
