/*
 * h3d_oracle.c -- plain CPU FP64 oracle for the HODLR3D matrix-vector product.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library links, loads or calls
 * this file; only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header or constant with the GPU
 * path.
 *
 * What it computes, and where the paper defines it (Kandappan, Gujjula,
 * Ambikasaran, "HODLR3D: Hierarchical matrices for N-body problems in three
 * dimensions", arXiv 2307.16303):
 *
 *   dense reference   K(i,j) = f(|r_i - r_j|), K(i,i) = 0       Sec. 3.1, eq. (Laplace3D)
 *   octree            balanced octree on a cube B, subdivided   Sec. 2.1; Algorithm 1
 *                     until every leaf holds at most N_max points
 *   relations         V/E/F (share a vertex / edge / face),     Sec. 4, table of notations
 *                     W (no shared boundary)
 *   clan, lists       clan = siblings + children of the parent's
 *                     E and F neighbours; interaction list =
 *                     clan restricted to V and W                Sec. 4, table of notations;
 *                                                              Definition (HODLR3D admissibility)
 *   compression       ACA with tolerance eps on each admissible
 *                     block K(X,Y)                              Sec. 4.1, eq. (prank); Algorithm 1
 *   mat-vec           near field (self, E, F leaf blocks), then
 *                     low-rank applies level by level           Algorithm 2
 *   pivot + LU form   K(X,tau) R^-1 L^-1 K(sigma,Y) psi(Y) with
 *                     regenerated entries and the LU factors
 *                     of K(sigma,tau) taken from ACA            Sec. 4.1, eqs. (prank), (LR);
 *                                                              Algorithm 2, low-rank step
 *
 * Readings where the paper is silent (each is listed in the design notes of
 * the repository):
 *   - leaf rule: a leaf holds at most leaf_size points (Sec. 2.1 wording);
 *   - quantisation: half-open boxes, the upper face clamped into the last box;
 *   - ACA variant: partially pivoted, first row 0, Frobenius-norm stopping
 *     rule |u_k||v_k| <= tol |S_k|_F, ties in every argmax to the lowest index;
 *   - coincident distinct points contribute 0 (f(0) := 0);
 *   - the low-rank blocks are kept as explicit factors U V^T; in exact
 *     arithmetic this equals the pivot/LU form of eq. (prank), which
 *     oracle_apply_lu applies from the same ACA run;
 *   - the LU factors of K(sigma, tau) are read off the ACA factors at the
 *     pivots (L from U, unit-diagonal R from V), in ACA's pivot order.
 *
 * Floating point: compiled with -ffp-contract=off; every sum runs in index
 * order.  Point order inside a leaf: ascending original index.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_OK = 0, OR_EINVAL = 1, OR_ENOMEM = 2, OR_EDEPTH = 5 };
enum { REL_SELF = 0, REL_F = 1, REL_E = 2, REL_V = 3, REL_W = 4 };

/* ------------------------------------------------------------------ */
/* kernel functions: Sec. 3.1 lists 1/r, 1/r^4 and cos(r)/r; the     */
/* Laplace Green's function 1/(4 pi r) and the Yukawa exp(-k r)/r are */
/* the workloads this oracle is used on.                              */
/* ------------------------------------------------------------------ */
static double kfun(int kernel, double kp, double r)
{
    if (r == 0.0)
        return 0.0;
    switch (kernel) {
    case 0: /* Laplace 1/(4 pi r) */
        return 1.0 / (4.0 * M_PI * r);
    case 1: /* Yukawa exp(-kappa r)/r */
        return exp(-kp * r) / r;
    case 2: { /* 1/r^4 */
        double r2 = r * r;
        return 1.0 / (r2 * r2);
    }
    case 3: /* cos(kappa r)/r */
        return cos(kp * r) / r;
    default:
        return 0.0;
    }
}

static double pair_entry(int kernel, double kp, const double *a, const double *b)
{
    double dx = a[0] - b[0];
    double dy = a[1] - b[1];
    double dz = a[2] - b[2];
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    return kfun(kernel, kp, r);
}

/* ------------------------------------------------------------------ */
/* dense reference: y_i = sum_{j != i} f(|r_i - r_j|) x_j             */
/* ------------------------------------------------------------------ */
void oracle_kernel_eval(int kernel, double kp, const double *r, int64_t n, double *out)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = kfun(kernel, kp, r[i]);
}

/* points: n x 3 row-major; x: n x nrhs column-major (ld n); y likewise */
void oracle_dense_rows(const double *pts, int64_t n, int kernel, double kp,
                       const double *x, int64_t nrhs, const int64_t *rows,
                       int64_t nrows, double *out /* nrows x nrhs, ld nrows */)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < nrows; ++q) {
        int64_t i = rows[q];
        for (int64_t c = 0; c < nrhs; ++c) {
            double acc = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                if (j == i)
                    continue;
                acc += pair_entry(kernel, kp, pts + 3 * i, pts + 3 * j) * x[c * n + j];
            }
            out[c * nrows + q] = acc;
        }
    }
}

void oracle_dense_matvec(const double *pts, int64_t n, int kernel, double kp,
                         const double *x, int64_t nrhs, double *y)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t c = 0; c < nrhs; ++c) {
            double acc = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                if (j == i)
                    continue;
                acc += pair_entry(kernel, kp, pts + 3 * i, pts + 3 * j) * x[c * n + j];
            }
            y[c * n + i] = acc;
        }
    }
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int t)
{
#ifdef _OPENMP
    if (t > 0)
        omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* ------------------------------------------------------------------ */
/* ACA (Sec. 4.1, eq. (prank)), partially pivoted, on an entry oracle. */
/* ------------------------------------------------------------------ */
typedef double (*entry_fn)(const void *ctx, int64_t i, int64_t j);

/*
 * Compresses the m x n matrix given by K(i,j) into U (m x k) V^T (n x k).
 * U and V are column-major with leading dimensions m and n and room for kcap
 * columns.  Row and column pivots (the index sets sigma and tau of eq.
 * (prank)) are written to rowpiv/colpiv.  Returns the rank k; *capped is set
 * when the loop stopped at kcap < min(m,n) without meeting the tolerance.
 */
static int64_t aca_core(entry_fn K, const void *ctx, int64_t m, int64_t n,
                        double tol, int64_t kcap, double *U, double *V,
                        int64_t *rowpiv, int64_t *colpiv, int *capped, double *norm2)
{
    int64_t mn = m < n ? m : n;
    if (kcap > mn)
        kcap = mn;
    *capped = 0;
    *norm2 = 0.0;
    if (kcap <= 0)
        return 0;
    char *used_row = calloc((size_t)m, 1);
    char *used_col = calloc((size_t)n, 1);
    double *dots_u = malloc(sizeof(double) * (size_t)kcap);
    double *dots_v = malloc(sizeof(double) * (size_t)kcap);
    int64_t k = 0;
    double S2 = 0.0; /* running |S_k|_F^2 */
    int64_t i = 0;   /* first pivot row */
    for (;;) {
        /* residual of row i, written into the next V column */
        double *r = V + k * n;
        for (int64_t j = 0; j < n; ++j) {
            double v = K(ctx, i, j);
            for (int64_t l = 0; l < k; ++l)
                v -= U[l * m + i] * V[l * n + j];
            r[j] = v;
        }
        used_row[i] = 1;
        /* pivot column: largest |residual| over unused columns, lowest index on ties */
        int64_t jp = -1;
        double best = -1.0;
        for (int64_t j = 0; j < n; ++j) {
            if (used_col[j])
                continue;
            double a = fabs(r[j]);
            if (a > best) {
                best = a;
                jp = j;
            }
        }
        if (jp < 0 || best == 0.0) {
            /* this row is already reproduced exactly: move to the lowest unused row */
            int64_t nx = -1;
            for (int64_t ii = 0; ii < m; ++ii)
                if (!used_row[ii]) {
                    nx = ii;
                    break;
                }
            if (nx < 0)
                break;
            i = nx;
            continue;
        }
        double piv = r[jp];
        for (int64_t j = 0; j < n; ++j)
            r[j] = r[j] / piv;
        /* residual of column jp */
        double *u = U + k * m;
        for (int64_t ii = 0; ii < m; ++ii) {
            double v = K(ctx, ii, jp);
            for (int64_t l = 0; l < k; ++l)
                v -= U[l * m + ii] * V[l * n + jp];
            u[ii] = v;
        }
        used_col[jp] = 1;
        rowpiv[k] = i;
        colpiv[k] = jp;
        /* |S_k|_F^2 = |S_{k-1}|_F^2 + 2 sum_l (u_l.u_k)(v_l.v_k) + |u_k|^2 |v_k|^2 */
        double uu = 0.0, vv = 0.0;
        for (int64_t ii = 0; ii < m; ++ii)
            uu += u[ii] * u[ii];
        for (int64_t j = 0; j < n; ++j)
            vv += r[j] * r[j];
        for (int64_t l = 0; l < k; ++l) {
            double a = 0.0, b = 0.0;
            for (int64_t ii = 0; ii < m; ++ii)
                a += U[l * m + ii] * u[ii];
            for (int64_t j = 0; j < n; ++j)
                b += V[l * n + j] * r[j];
            dots_u[l] = a;
            dots_v[l] = b;
        }
        double cross = 0.0;
        for (int64_t l = 0; l < k; ++l)
            cross += dots_u[l] * dots_v[l];
        S2 = S2 + 2.0 * cross + uu * vv;
        k += 1;
        if (uu * vv <= tol * tol * S2)
            break;
        if (k == mn)
            break;
        if (k == kcap) {
            *capped = 1;
            break;
        }
        /* next pivot row: largest |u_k| over unused rows, lowest index on ties */
        int64_t ip = -1;
        best = -1.0;
        for (int64_t ii = 0; ii < m; ++ii) {
            if (used_row[ii])
                continue;
            double a = fabs(u[ii]);
            if (a > best) {
                best = a;
                ip = ii;
            }
        }
        if (ip < 0)
            break;
        i = ip;
    }
    free(used_row);
    free(used_col);
    free(dots_u);
    free(dots_v);
    *norm2 = S2;
    return k;
}

/* ACA on an explicit column-major matrix A (m x n, ld m). */
typedef struct {
    const double *A;
    int64_t m;
} dense_ctx;

static double dense_entry(const void *ctx, int64_t i, int64_t j)
{
    const dense_ctx *c = (const dense_ctx *)ctx;
    return c->A[j * c->m + i];
}

/* norm2 receives the running estimate |S_k|_F^2 at the stop */
int64_t oracle_aca_dense(const double *A, int64_t m, int64_t n, double tol,
                         int64_t kcap, double *U, double *V, int64_t *rowpiv,
                         int64_t *colpiv, int *capped, double *norm2)
{
    dense_ctx c = {A, m};
    return aca_core(dense_entry, &c, m, n, tol, kcap, U, V, rowpiv, colpiv, capped, norm2);
}

/* ------------------------------------------------------------------ */
/* HODLR3D structure                                                  */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    int kernel;
    double kp;
    int leaf_size;
    double tol;
    int max_depth;
    int64_t max_rank;
    double lo[3];
    double side;
    int L;
    int64_t *perm;    /* sorted position -> original index */
    double *sp;       /* sorted points, n x 3 */
    int64_t *leaf_off; /* 8^L + 1 */
    /* far blocks, ordered by (level, t, s) */
    int64_t nfar;
    int32_t *far_level;
    int64_t *far_t, *far_s;
    int64_t *far_rank;
    int64_t *far_uoff, *far_voff;
    int64_t *far_piv_off; /* offset into rowpiv/colpiv */
    int64_t *rowpiv, *colpiv;
    int64_t ncapped;
    double *U, *V;
    int64_t utot, vtot;
    /* near pairs (t, s, relation), ordered by (t, s) */
    int64_t nnear;
    int64_t *near_t, *near_s;
    int32_t *near_rel;
} oracle_h3d;

static int64_t pow8(int l) { return (int64_t)1 << (3 * l); }

static uint64_t morton_encode(uint64_t qx, uint64_t qy, uint64_t qz, int bits)
{
    uint64_t key = 0;
    for (int b = bits - 1; b >= 0; --b) {
        key = (key << 3) | (((qx >> b) & 1u) << 2) | (((qy >> b) & 1u) << 1) | ((qz >> b) & 1u);
    }
    return key;
}

static void morton_decode(uint64_t key, int bits, int64_t *qx, int64_t *qy, int64_t *qz)
{
    int64_t x = 0, y = 0, z = 0;
    for (int b = bits - 1; b >= 0; --b) {
        x = (x << 1) | (int64_t)((key >> (3 * b + 2)) & 1u);
        y = (y << 1) | (int64_t)((key >> (3 * b + 1)) & 1u);
        z = (z << 1) | (int64_t)((key >> (3 * b)) & 1u);
    }
    *qx = x;
    *qy = y;
    *qz = z;
}

uint64_t oracle_morton_encode(uint64_t qx, uint64_t qy, uint64_t qz, int bits)
{
    return morton_encode(qx, qy, qz, bits);
}

void oracle_morton_decode(uint64_t key, int bits, int64_t *q3)
{
    morton_decode(key, bits, q3, q3 + 1, q3 + 2);
}

/* Integer coordinate of a point at level l: floor((x - lo) * 2^l / side),
 * half-open boxes, upper face clamped into the last box. */
static int64_t quantize(double x, double lo, double side, int l)
{
    double scale = ldexp(1.0, l) / side;
    double t = floor((x - lo) * scale);
    int64_t nb = (int64_t)1 << l;
    if (!(t >= 0.0))
        return 0;
    if (t >= (double)nb)
        return nb - 1;
    return (int64_t)t;
}

static int64_t box_of_point(const oracle_h3d *h, const double *p, int l)
{
    int64_t qx = quantize(p[0], h->lo[0], h->side, l);
    int64_t qy = quantize(p[1], h->lo[1], h->side, l);
    int64_t qz = quantize(p[2], h->lo[2], h->side, l);
    return (int64_t)morton_encode((uint64_t)qx, (uint64_t)qy, (uint64_t)qz, l);
}

int oracle_relation(int64_t ax, int64_t ay, int64_t az, int64_t bx, int64_t by, int64_t bz)
{
    int64_t dx = llabs(ax - bx), dy = llabs(ay - by), dz = llabs(az - bz);
    int64_t mx = dx > dy ? dx : dy;
    if (dz > mx)
        mx = dz;
    if (mx == 0)
        return REL_SELF;
    if (mx >= 2)
        return REL_W;
    int64_t s = dx + dy + dz;
    if (s == 3)
        return REL_V;
    if (s == 2)
        return REL_E;
    return REL_F;
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* growable int64 vector */
typedef struct {
    int64_t *d;
    int64_t n, cap;
} ivec;

static int iv_push(ivec *v, int64_t x)
{
    if (v->n == v->cap) {
        int64_t nc = v->cap ? 2 * v->cap : 1024;
        int64_t *nd = realloc(v->d, sizeof(int64_t) * (size_t)nc);
        if (!nd)
            return 0;
        v->d = nd;
        v->cap = nc;
    }
    v->d[v->n++] = x;
    return 1;
}

static int64_t box_count(const oracle_h3d *h, int l, int64_t b)
{
    int64_t span = pow8(h->L - l);
    return h->leaf_off[(b + 1) * span] - h->leaf_off[b * span];
}

static int64_t box_start(const oracle_h3d *h, int l, int64_t b)
{
    return h->leaf_off[b * pow8(h->L - l)];
}

/* interaction list of box t at level l >= 1, sorted by s */
static int64_t interaction_list(const oracle_h3d *h, int l, int64_t t, int64_t *out)
{
    int64_t tx, ty, tz;
    morton_decode((uint64_t)t, l, &tx, &ty, &tz);
    int64_t px = tx >> 1, py = ty >> 1, pz = tz >> 1;
    int64_t np = (int64_t)1 << (l - 1);
    int64_t cnt = 0;
    for (int64_t qx = px - 1; qx <= px + 1; ++qx)
        for (int64_t qy = py - 1; qy <= py + 1; ++qy)
            for (int64_t qz = pz - 1; qz <= pz + 1; ++qz) {
                if (qx < 0 || qy < 0 || qz < 0 || qx >= np || qy >= np || qz >= np)
                    continue;
                int rp = oracle_relation(px, py, pz, qx, qy, qz);
                /* clan: siblings (children of the parent itself) and children
                 * of the parent's E and F neighbours */
                if (rp != REL_SELF && rp != REL_E && rp != REL_F)
                    continue;
                int64_t q = (int64_t)morton_encode((uint64_t)qx, (uint64_t)qy, (uint64_t)qz, l - 1);
                for (int64_t c = 0; c < 8; ++c) {
                    int64_t s = q * 8 + c;
                    if (s == t)
                        continue;
                    if (box_count(h, l, s) == 0)
                        continue;
                    int64_t sx, sy, sz;
                    morton_decode((uint64_t)s, l, &sx, &sy, &sz);
                    int rel = oracle_relation(tx, ty, tz, sx, sy, sz);
                    if (rel == REL_V || rel == REL_W)
                        out[cnt++] = s;
                }
            }
    qsort(out, (size_t)cnt, sizeof(int64_t), cmp_i64);
    return cnt;
}

/* near list of leaf t: itself and its E and F neighbours, sorted by s */
static int64_t near_list(const oracle_h3d *h, int64_t t, int64_t *out, int32_t *rel_out)
{
    int l = h->L;
    int64_t tx, ty, tz;
    morton_decode((uint64_t)t, l, &tx, &ty, &tz);
    int64_t nb = (int64_t)1 << l;
    int64_t cnt = 0;
    int64_t tmp[27];
    for (int64_t qx = tx - 1; qx <= tx + 1; ++qx)
        for (int64_t qy = ty - 1; qy <= ty + 1; ++qy)
            for (int64_t qz = tz - 1; qz <= tz + 1; ++qz) {
                if (qx < 0 || qy < 0 || qz < 0 || qx >= nb || qy >= nb || qz >= nb)
                    continue;
                int rel = oracle_relation(tx, ty, tz, qx, qy, qz);
                if (rel == REL_V)
                    continue;
                int64_t s = (int64_t)morton_encode((uint64_t)qx, (uint64_t)qy, (uint64_t)qz, l);
                if (box_count(h, l, s) == 0)
                    continue;
                tmp[cnt++] = s;
            }
    qsort(tmp, (size_t)cnt, sizeof(int64_t), cmp_i64);
    for (int64_t a = 0; a < cnt; ++a) {
        int64_t sx, sy, sz;
        out[a] = tmp[a];
        morton_decode((uint64_t)tmp[a], l, &sx, &sy, &sz);
        rel_out[a] = oracle_relation(tx, ty, tz, sx, sy, sz);
    }
    return cnt;
}

typedef struct {
    const oracle_h3d *h;
    int64_t t0, s0;
} block_ctx;

static double block_entry(const void *ctx, int64_t i, int64_t j)
{
    const block_ctx *c = (const block_ctx *)ctx;
    int64_t gi = c->t0 + i, gj = c->s0 + j;
    if (gi == gj)
        return 0.0;
    return pair_entry(c->h->kernel, c->h->kp, c->h->sp + 3 * gi, c->h->sp + 3 * gj);
}

void oracle_destroy(oracle_h3d *h)
{
    if (!h)
        return;
    free(h->perm);
    free(h->sp);
    free(h->leaf_off);
    free(h->far_level);
    free(h->far_t);
    free(h->far_s);
    free(h->far_rank);
    free(h->far_uoff);
    free(h->far_voff);
    free(h->far_piv_off);
    free(h->rowpiv);
    free(h->colpiv);
    free(h->U);
    free(h->V);
    free(h->near_t);
    free(h->near_s);
    free(h->near_rel);
    free(h);
}

/*
 * Builds the tree, the lists and (when compress != 0) the ACA factors.
 * box_side <= 0 selects the smallest enclosing cube (lo = componentwise
 * minimum, side = largest extent; side := 1 when every point coincides).
 */
int oracle_build(const double *pts, int64_t n, int kernel, double kp, int leaf_size,
                 double tol, int max_depth, int64_t max_rank, const double *box_lo,
                 double box_side, int compress, oracle_h3d **out)
{
    *out = NULL;
    if (n < 1 || leaf_size < 1 || !(tol > 0.0 && tol < 1.0) || max_depth < 0 || max_depth > 10)
        return OR_EINVAL;
    for (int64_t i = 0; i < 3 * n; ++i)
        if (!isfinite(pts[i]))
            return OR_EINVAL;
    oracle_h3d *h = calloc(1, sizeof(oracle_h3d));
    if (!h)
        return OR_ENOMEM;
    h->n = n;
    h->kernel = kernel;
    h->kp = kp;
    h->leaf_size = leaf_size;
    h->tol = tol;
    h->max_depth = max_depth;
    h->max_rank = max_rank;
    if (box_side > 0.0) {
        for (int a = 0; a < 3; ++a)
            h->lo[a] = box_lo[a];
        h->side = box_side;
        for (int64_t i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a) {
                double x = pts[3 * i + a];
                if (x < h->lo[a] || x > h->lo[a] + h->side) {
                    oracle_destroy(h);
                    return OR_EINVAL;
                }
            }
    } else {
        double mn[3], mx[3];
        for (int a = 0; a < 3; ++a)
            mn[a] = mx[a] = pts[a];
        for (int64_t i = 1; i < n; ++i)
            for (int a = 0; a < 3; ++a) {
                double x = pts[3 * i + a];
                if (x < mn[a])
                    mn[a] = x;
                if (x > mx[a])
                    mx[a] = x;
            }
        double side = 0.0;
        for (int a = 0; a < 3; ++a) {
            h->lo[a] = mn[a];
            if (mx[a] - mn[a] > side)
                side = mx[a] - mn[a];
        }
        h->side = side > 0.0 ? side : 1.0;
    }

    /* depth rule (Sec. 2.1): the smallest L at which no box holds more than leaf_size points */
    int64_t *box = malloc(sizeof(int64_t) * (size_t)n);
    int L = -1;
    for (int l = 0; l <= max_depth; ++l) {
        int64_t nbox = pow8(l);
        int64_t *cnt = calloc((size_t)nbox, sizeof(int64_t));
        int64_t mx = 0;
        for (int64_t i = 0; i < n; ++i) {
            box[i] = box_of_point(h, pts + 3 * i, l);
            int64_t c = ++cnt[box[i]];
            if (c > mx)
                mx = c;
        }
        free(cnt);
        if (mx <= leaf_size) {
            L = l;
            break;
        }
    }
    if (L < 0) {
        free(box);
        oracle_destroy(h);
        return OR_EDEPTH;
    }
    h->L = L;

    /* stable counting sort by leaf: points of a leaf keep ascending original index */
    int64_t nleaf = pow8(L);
    h->leaf_off = calloc((size_t)nleaf + 1, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i)
        h->leaf_off[box[i] + 1] += 1;
    for (int64_t b = 0; b < nleaf; ++b)
        h->leaf_off[b + 1] += h->leaf_off[b];
    int64_t *cursor = malloc(sizeof(int64_t) * (size_t)nleaf);
    memcpy(cursor, h->leaf_off, sizeof(int64_t) * (size_t)nleaf);
    h->perm = malloc(sizeof(int64_t) * (size_t)n);
    h->sp = malloc(sizeof(double) * 3 * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        int64_t pos = cursor[box[i]]++;
        h->perm[pos] = i;
    }
    for (int64_t p = 0; p < n; ++p)
        for (int a = 0; a < 3; ++a)
            h->sp[3 * p + a] = pts[3 * h->perm[p] + a];
    free(cursor);
    free(box);

    /* far blocks: for l = 1..L, every non-empty t, s in the interaction list of t */
    ivec fl = {0}, ft = {0}, fs = {0};
    int64_t list[160];
    for (int l = 1; l <= L; ++l) {
        int64_t nb = pow8(l);
        for (int64_t t = 0; t < nb; ++t) {
            if (box_count(h, l, t) == 0)
                continue;
            int64_t c = interaction_list(h, l, t, list);
            for (int64_t a = 0; a < c; ++a) {
                iv_push(&fl, l);
                iv_push(&ft, t);
                iv_push(&fs, list[a]);
            }
        }
    }
    h->nfar = fl.n;
    h->far_level = malloc(sizeof(int32_t) * (size_t)(fl.n + 1));
    for (int64_t b = 0; b < fl.n; ++b)
        h->far_level[b] = (int32_t)fl.d[b];
    free(fl.d);
    h->far_t = ft.d;
    h->far_s = fs.d;

    /* near pairs at the leaf level */
    ivec nt = {0}, ns = {0}, nr = {0};
    int32_t rels[27];
    for (int64_t t = 0; t < nleaf; ++t) {
        if (box_count(h, L, t) == 0)
            continue;
        int64_t c = near_list(h, t, list, rels);
        for (int64_t a = 0; a < c; ++a) {
            iv_push(&nt, t);
            iv_push(&ns, list[a]);
            iv_push(&nr, rels[a]);
        }
    }
    h->nnear = nt.n;
    h->near_t = nt.d;
    h->near_s = ns.d;
    h->near_rel = malloc(sizeof(int32_t) * (size_t)(nr.n + 1));
    for (int64_t a = 0; a < nr.n; ++a)
        h->near_rel[a] = (int32_t)nr.d[a];
    free(nr.d);

    h->far_rank = calloc((size_t)h->nfar + 1, sizeof(int64_t));
    h->far_uoff = calloc((size_t)h->nfar + 1, sizeof(int64_t));
    h->far_voff = calloc((size_t)h->nfar + 1, sizeof(int64_t));
    h->far_piv_off = calloc((size_t)h->nfar + 1, sizeof(int64_t));
    if (!compress) {
        *out = h;
        return OR_OK;
    }

    /* ACA on every admissible block (Algorithm 1); blocks are independent */
    double **Ub = calloc((size_t)h->nfar + 1, sizeof(double *));
    double **Vb = calloc((size_t)h->nfar + 1, sizeof(double *));
    int64_t **Rp = calloc((size_t)h->nfar + 1, sizeof(int64_t *));
    int64_t **Cp = calloc((size_t)h->nfar + 1, sizeof(int64_t *));
    int64_t ncapped = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : ncapped)
    for (int64_t b = 0; b < h->nfar; ++b) {
        int l = h->far_level[b];
        int64_t m = box_count(h, l, h->far_t[b]);
        int64_t nn = box_count(h, l, h->far_s[b]);
        int64_t kcap = m < nn ? m : nn;
        if (max_rank > 0 && max_rank < kcap)
            kcap = max_rank;
        double *U = malloc(sizeof(double) * (size_t)(m * kcap));
        double *V = malloc(sizeof(double) * (size_t)(nn * kcap));
        int64_t *rp = malloc(sizeof(int64_t) * (size_t)kcap);
        int64_t *cp = malloc(sizeof(int64_t) * (size_t)kcap);
        block_ctx ctx = {h, box_start(h, l, h->far_t[b]), box_start(h, l, h->far_s[b])};
        int capped = 0;
        double norm2 = 0.0;
        int64_t k = aca_core(block_entry, &ctx, m, nn, tol, kcap, U, V, rp, cp, &capped, &norm2);
        ncapped += capped;
        h->far_rank[b] = k;
        Ub[b] = U;
        Vb[b] = V;
        Rp[b] = rp;
        Cp[b] = cp;
    }
    h->ncapped = ncapped;
    int64_t ut = 0, vt = 0, pt = 0;
    for (int64_t b = 0; b < h->nfar; ++b) {
        int l = h->far_level[b];
        h->far_uoff[b] = ut;
        h->far_voff[b] = vt;
        h->far_piv_off[b] = pt;
        ut += box_count(h, l, h->far_t[b]) * h->far_rank[b];
        vt += box_count(h, l, h->far_s[b]) * h->far_rank[b];
        pt += h->far_rank[b];
    }
    h->far_uoff[h->nfar] = ut;
    h->far_voff[h->nfar] = vt;
    h->far_piv_off[h->nfar] = pt;
    h->utot = ut;
    h->vtot = vt;
    h->U = malloc(sizeof(double) * (size_t)(ut + 1));
    h->V = malloc(sizeof(double) * (size_t)(vt + 1));
    h->rowpiv = malloc(sizeof(int64_t) * (size_t)(pt + 1));
    h->colpiv = malloc(sizeof(int64_t) * (size_t)(pt + 1));
    for (int64_t b = 0; b < h->nfar; ++b) {
        int l = h->far_level[b];
        int64_t m = box_count(h, l, h->far_t[b]);
        int64_t nn = box_count(h, l, h->far_s[b]);
        int64_t k = h->far_rank[b];
        memcpy(h->U + h->far_uoff[b], Ub[b], sizeof(double) * (size_t)(m * k));
        memcpy(h->V + h->far_voff[b], Vb[b], sizeof(double) * (size_t)(nn * k));
        memcpy(h->rowpiv + h->far_piv_off[b], Rp[b], sizeof(int64_t) * (size_t)k);
        memcpy(h->colpiv + h->far_piv_off[b], Cp[b], sizeof(int64_t) * (size_t)k);
        free(Ub[b]);
        free(Vb[b]);
        free(Rp[b]);
        free(Cp[b]);
    }
    free(Ub);
    free(Vb);
    free(Rp);
    free(Cp);
    *out = h;
    return OR_OK;
}

/* Replaces the factors by externally supplied ones (same block order,
 * U_b m x k and V_b n x k column-major, concatenated). */
int oracle_set_factors(oracle_h3d *h, const int64_t *ranks, const double *U, const double *V)
{
    int64_t ut = 0, vt = 0;
    for (int64_t b = 0; b < h->nfar; ++b) {
        int l = h->far_level[b];
        h->far_rank[b] = ranks[b];
        h->far_uoff[b] = ut;
        h->far_voff[b] = vt;
        ut += box_count(h, l, h->far_t[b]) * ranks[b];
        vt += box_count(h, l, h->far_s[b]) * ranks[b];
    }
    h->far_uoff[h->nfar] = ut;
    h->far_voff[h->nfar] = vt;
    free(h->U);
    free(h->V);
    h->U = malloc(sizeof(double) * (size_t)(ut + 1));
    h->V = malloc(sizeof(double) * (size_t)(vt + 1));
    if (!h->U || !h->V)
        return OR_ENOMEM;
    memcpy(h->U, U, sizeof(double) * (size_t)ut);
    memcpy(h->V, V, sizeof(double) * (size_t)vt);
    h->utot = ut;
    h->vtot = vt;
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Mat-vec (Algorithm 2) and its adjoint                              */
/* ------------------------------------------------------------------ */
static void near_block_apply(const oracle_h3d *h, int64_t t, int64_t s, const double *xp,
                             double *yp, int adjoint)
{
    int L = h->L;
    int64_t t0 = box_start(h, L, t), m = box_count(h, L, t);
    int64_t s0 = box_start(h, L, s), nn = box_count(h, L, s);
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < nn; ++j) {
            int64_t gi = t0 + i, gj = s0 + j;
            double k = (gi == gj) ? 0.0 : pair_entry(h->kernel, h->kp, h->sp + 3 * gi, h->sp + 3 * gj);
            if (!adjoint)
                yp[gi] += k * xp[gj];
            else
                yp[gj] += k * xp[gi];
        }
}

static void far_block_apply(const oracle_h3d *h, int64_t b, const double *xp, double *yp,
                            int adjoint, double *z)
{
    int l = h->far_level[b];
    int64_t t0 = box_start(h, l, h->far_t[b]), m = box_count(h, l, h->far_t[b]);
    int64_t s0 = box_start(h, l, h->far_s[b]), nn = box_count(h, l, h->far_s[b]);
    int64_t k = h->far_rank[b];
    const double *U = h->U + h->far_uoff[b];
    const double *V = h->V + h->far_voff[b];
    if (!adjoint) {
        /* y_t += U (V^T x_s) */
        for (int64_t c = 0; c < k; ++c) {
            double a = 0.0;
            for (int64_t j = 0; j < nn; ++j)
                a += V[c * nn + j] * xp[s0 + j];
            z[c] = a;
        }
        for (int64_t i = 0; i < m; ++i) {
            double a = 0.0;
            for (int64_t c = 0; c < k; ++c)
                a += U[c * m + i] * z[c];
            yp[t0 + i] += a;
        }
    } else {
        /* y_s += V (U^T x_t) */
        for (int64_t c = 0; c < k; ++c) {
            double a = 0.0;
            for (int64_t i = 0; i < m; ++i)
                a += U[c * m + i] * xp[t0 + i];
            z[c] = a;
        }
        for (int64_t j = 0; j < nn; ++j) {
            double a = 0.0;
            for (int64_t c = 0; c < k; ++c)
                a += V[c * nn + j] * z[c];
            yp[s0 + j] += a;
        }
    }
}

/* ------------------------------------------------------------------ */
/* The paper's storage form (Sec. 4.1, eqs. (prank) and (LR); the      */
/* low-rank step of Algorithm 2): per block only the pivots sigma (rows */
/* of X), tau (columns of Y) and the LU factors of K(sigma, tau) are    */
/* kept; a product regenerates K(sigma, Y) and K(X, tau) and applies    */
/* K(X,tau) R^-1 L^-1 K(sigma,Y) psi(Y) by forward and backward         */
/* substitution.                                                        */
/* ------------------------------------------------------------------ */

/*
 * LU factors of K(sigma, tau) for block b, taken from the ACA factors as a
 * by-product (Sec. 4.1): with the pivots in the order ACA chose them,
 *   L[a][l] = u_l[sigma_a]  (a >= l; lower triangular, diagonal = the pivots)
 *   R[l][c] = v_l[tau_c]    (c >  l; R has a unit diagonal, v_l[tau_l] = 1)
 * since u_l vanishes on the earlier pivot rows and v_l on the earlier pivot
 * columns, K(sigma, tau) = U(sigma,:) V(tau,:)^T = L R.  Packed into one
 * k x k column-major matrix: L on and below the diagonal, R above it.
 */
static void block_lu(const oracle_h3d *h, int64_t b, double *LU)
{
    int l = h->far_level[b];
    int64_t m = box_count(h, l, h->far_t[b]);
    int64_t nn = box_count(h, l, h->far_s[b]);
    int64_t k = h->far_rank[b];
    const double *U = h->U + h->far_uoff[b];
    const double *V = h->V + h->far_voff[b];
    const int64_t *sig = h->rowpiv + h->far_piv_off[b];
    const int64_t *tau = h->colpiv + h->far_piv_off[b];
    for (int64_t c = 0; c < k; ++c)         /* column c */
        for (int64_t a = 0; a < k; ++a) {   /* row a */
            if (a >= c)
                LU[c * k + a] = U[c * m + sig[a]];   /* L[a][c] = u_c[sigma_a] */
            else
                LU[c * k + a] = V[a * nn + tau[c]];  /* R[a][c] = v_a[tau_c] */
        }
}

/* the packed LU factors of every block, concatenated (k_b^2 values each) */
void oracle_export_lu(const oracle_h3d *h, double *out)
{
    int64_t off = 0;
    for (int64_t b = 0; b < h->nfar; ++b) {
        block_lu(h, b, out + off);
        off += h->far_rank[b] * h->far_rank[b];
    }
}

/* K(X, tau) R^-1 L^-1 K(sigma, Y) applied to x_s (forward), or its transpose
 * K(sigma,Y)^T L^-T R^-T K(X,tau)^T applied to x_t (adjoint); LU is the
 * packed k x k matrix of block_lu, w a k-vector of workspace. */
static void far_block_apply_lu(const oracle_h3d *h, int64_t b, const double *LU, const double *xp,
                               double *yp, int adjoint, double *w)
{
    int l = h->far_level[b];
    int64_t t0 = box_start(h, l, h->far_t[b]), m = box_count(h, l, h->far_t[b]);
    int64_t s0 = box_start(h, l, h->far_s[b]), nn = box_count(h, l, h->far_s[b]);
    int64_t k = h->far_rank[b];
    const int64_t *sig = h->rowpiv + h->far_piv_off[b];
    const int64_t *tau = h->colpiv + h->far_piv_off[b];
    block_ctx ctx = {h, t0, s0};
    if (!adjoint) {
        /* w = K(sigma, Y) x(Y) */
        for (int64_t a = 0; a < k; ++a) {
            double acc = 0.0;
            for (int64_t j = 0; j < nn; ++j)
                acc += block_entry(&ctx, sig[a], j) * xp[s0 + j];
            w[a] = acc;
        }
        /* w = L^-1 w: forward substitution */
        for (int64_t a = 0; a < k; ++a) {
            double acc = w[a];
            for (int64_t c = 0; c < a; ++c)
                acc -= LU[c * k + a] * w[c];
            w[a] = acc / LU[a * k + a];
        }
        /* w = R^-1 w: backward substitution, unit diagonal */
        for (int64_t a = k - 1; a >= 0; --a) {
            double acc = w[a];
            for (int64_t c = a + 1; c < k; ++c)
                acc -= LU[c * k + a] * w[c];
            w[a] = acc;
        }
        /* y(X) += K(X, tau) w */
        for (int64_t i = 0; i < m; ++i) {
            double acc = 0.0;
            for (int64_t c = 0; c < k; ++c)
                acc += block_entry(&ctx, i, tau[c]) * w[c];
            yp[t0 + i] += acc;
        }
    } else {
        /* w = K(X, tau)^T x(X) */
        for (int64_t c = 0; c < k; ++c) {
            double acc = 0.0;
            for (int64_t i = 0; i < m; ++i)
                acc += block_entry(&ctx, i, tau[c]) * xp[t0 + i];
            w[c] = acc;
        }
        /* w = R^-T w: forward substitution with the unit lower R^T */
        for (int64_t a = 0; a < k; ++a) {
            double acc = w[a];
            for (int64_t c = 0; c < a; ++c)
                acc -= LU[a * k + c] * w[c];
            w[a] = acc;
        }
        /* w = L^-T w: backward substitution with the upper L^T */
        for (int64_t a = k - 1; a >= 0; --a) {
            double acc = w[a];
            for (int64_t c = a + 1; c < k; ++c)
                acc -= LU[a * k + c] * w[c];
            w[a] = acc / LU[a * k + a];
        }
        /* y(Y) += K(sigma, Y)^T w */
        for (int64_t j = 0; j < nn; ++j) {
            double acc = 0.0;
            for (int64_t a = 0; a < k; ++a)
                acc += block_entry(&ctx, sig[a], j) * w[a];
            yp[s0 + j] += acc;
        }
    }
}

/*
 * y = K~ x (adjoint = 0) or y = K~^T x (adjoint = 1); x, y: n x nrhs,
 * column-major, original point order.  near != 0 includes the dense leaf
 * blocks, far != 0 the low-rank blocks (both set for the full product).
 */
static int apply_form(const oracle_h3d *h, const double *x, int64_t nrhs, double *y,
                      int adjoint, int near, int far, int lu_form)
{
    int64_t n = h->n;
    double *xp = malloc(sizeof(double) * (size_t)n);
    double *yp = malloc(sizeof(double) * (size_t)n);
    int64_t kmax = 1;
    for (int64_t b = 0; b < h->nfar; ++b)
        if (h->far_rank[b] > kmax)
            kmax = h->far_rank[b];
    double *z = malloc(sizeof(double) * (size_t)kmax);
    double *LU = lu_form ? malloc(sizeof(double) * (size_t)(kmax * kmax)) : NULL;
    if (!xp || !yp || !z || (lu_form && !LU)) {
        free(xp);
        free(yp);
        free(z);
        free(LU);
        return OR_ENOMEM;
    }
    for (int64_t c = 0; c < nrhs; ++c) {
        for (int64_t p = 0; p < n; ++p) {
            xp[p] = x[c * n + h->perm[p]];
            yp[p] = 0.0;
        }
        if (near) {
            /* Algorithm 2: per leaf, the self block, then E blocks, then F blocks */
            int64_t a = 0;
            while (a < h->nnear) {
                int64_t t = h->near_t[a];
                int64_t e = a;
                while (e < h->nnear && h->near_t[e] == t)
                    ++e;
                static const int order[3] = {REL_SELF, REL_E, REL_F};
                for (int o = 0; o < 3; ++o)
                    for (int64_t q = a; q < e; ++q)
                        if (h->near_rel[q] == order[o])
                            near_block_apply(h, t, h->near_s[q], xp, yp, adjoint);
                a = e;
            }
        }
        if (far) {
            /* low-rank part, level 1..L, targets in Morton order, lists ascending */
            for (int64_t b = 0; b < h->nfar; ++b) {
                if (lu_form) {
                    block_lu(h, b, LU);
                    far_block_apply_lu(h, b, LU, xp, yp, adjoint, z);
                } else {
                    far_block_apply(h, b, xp, yp, adjoint, z);
                }
            }
        }
        for (int64_t p = 0; p < n; ++p)
            y[c * n + h->perm[p]] = yp[p];
    }
    free(xp);
    free(yp);
    free(z);
    free(LU);
    return OR_OK;
}

int oracle_apply(const oracle_h3d *h, const double *x, int64_t nrhs, double *y, int adjoint,
                 int near, int far)
{
    return apply_form(h, x, nrhs, y, adjoint, near, far, 0);
}

/* As oracle_apply, with every low-rank block applied in the pivot + LU form
 * of Sec. 4.1 (entries of K(sigma,Y) and K(X,tau) regenerated). */
int oracle_apply_lu(const oracle_h3d *h, const double *x, int64_t nrhs, double *y, int adjoint,
                    int near, int far)
{
    return apply_form(h, x, nrhs, y, adjoint, near, far, 1);
}

/* ------------------------------------------------------------------ */
/* accessors                                                          */
/* ------------------------------------------------------------------ */
int oracle_depth(const oracle_h3d *h) { return h->L; }
int64_t oracle_num_far(const oracle_h3d *h) { return h->nfar; }
int64_t oracle_num_near(const oracle_h3d *h) { return h->nnear; }
int64_t oracle_num_capped(const oracle_h3d *h) { return h->ncapped; }
int64_t oracle_factor_len(const oracle_h3d *h, int which) { return which == 0 ? h->utot : h->vtot; }
void oracle_box(const oracle_h3d *h, double *lo_side)
{
    lo_side[0] = h->lo[0];
    lo_side[1] = h->lo[1];
    lo_side[2] = h->lo[2];
    lo_side[3] = h->side;
}

void oracle_export_tree(const oracle_h3d *h, int64_t *perm, int64_t *leaf_off)
{
    memcpy(perm, h->perm, sizeof(int64_t) * (size_t)h->n);
    memcpy(leaf_off, h->leaf_off, sizeof(int64_t) * (size_t)(pow8(h->L) + 1));
}

/* far table: level, t, s, m, n, rank per block */
void oracle_export_far(const oracle_h3d *h, int64_t *level, int64_t *t, int64_t *s, int64_t *m,
                       int64_t *nn, int64_t *rank)
{
    for (int64_t b = 0; b < h->nfar; ++b) {
        int l = h->far_level[b];
        level[b] = l;
        t[b] = h->far_t[b];
        s[b] = h->far_s[b];
        m[b] = box_count(h, l, h->far_t[b]);
        nn[b] = box_count(h, l, h->far_s[b]);
        rank[b] = h->far_rank[b];
    }
}

void oracle_export_near(const oracle_h3d *h, int64_t *t, int64_t *s, int64_t *rel)
{
    for (int64_t a = 0; a < h->nnear; ++a) {
        t[a] = h->near_t[a];
        s[a] = h->near_s[a];
        rel[a] = h->near_rel[a];
    }
}

void oracle_export_factors(const oracle_h3d *h, double *U, double *V)
{
    memcpy(U, h->U, sizeof(double) * (size_t)h->utot);
    memcpy(V, h->V, sizeof(double) * (size_t)h->vtot);
}

/* pivots of each block: rows (local to t) and columns (local to s), concatenated */
void oracle_export_pivots(const oracle_h3d *h, int64_t *rowpiv, int64_t *colpiv)
{
    int64_t pt = h->far_piv_off[h->nfar];
    memcpy(rowpiv, h->rowpiv, sizeof(int64_t) * (size_t)pt);
    memcpy(colpiv, h->colpiv, sizeof(int64_t) * (size_t)pt);
}

/* dense entries of block b (m x n column-major), for SVD checks */
void oracle_block_dense(const oracle_h3d *h, int64_t b, double *out)
{
    int l = h->far_level[b];
    int64_t m = box_count(h, l, h->far_t[b]);
    int64_t nn = box_count(h, l, h->far_s[b]);
    block_ctx ctx = {h, box_start(h, l, h->far_t[b]), box_start(h, l, h->far_s[b])};
    for (int64_t j = 0; j < nn; ++j)
        for (int64_t i = 0; i < m; ++i)
            out[j * m + i] = block_entry(&ctx, i, j);
}
