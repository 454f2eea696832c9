/*
 * dcrf_oracle.c -- plain, slow, FP64 CPU oracle for the filter-based pairwise
 * messages of a dense CRF with Gaussian pairwise potentials, after
 * Desmaison, Bunel, Kohli, Torr and Kumar, "Efficient Continuous Relaxations
 * for Dense CRF" (ECCV 2016).
 *
 * TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library. It shares no code,
 * header, table or constant generator with the GPU library; it is written
 * from the paper and from the mathematics of the permutohedral lattice.
 *
 * Two operators are defined here:
 *
 *  1. The exact Gaussian sum of the filter-based method (Sec. 3, eq. fb, with
 *     the kernel of eq. gaussiankernel):
 *         out_a = sum_b exp(-|f_a - f_b|^2 / 2) * in_b .
 *
 *  2. A reference permutohedral-lattice filter. The paper uses the filter of
 *     Adams et al. (Sec. 3 "Filter-based Method", App. A) and gives none of its
 *     details; what follows is written from the lattice mathematics:
 *       - elevate f (dimension d) onto the hyperplane sum(x) = 0 of R^{d+1}
 *         with an orthonormal basis, scaled by s = (d+1) sqrt(2/3) so that the
 *         splat-blur-slice chain has unit variance per feature direction;
 *       - find the remainder-0 point of the lattice (d+1)A*_d closest to x and
 *         the simplex of the Delaunay triangulation that contains x, with its
 *         d+1 vertices and barycentric weights;
 *       - splat: V[v] += b * in (only vertices with b > 0 are created);
 *       - blur: for j = 0..d, V'[v] = V[v]/2 + (V[v+u_j] + V[v-u_j])/4 with
 *         u_j = (d+1) e_j - 1 and missing vertices read as 0 (out of place);
 *       - slice: out_a = gamma_d * sum_k b_k V[v_k], where
 *         gamma_d = (4 pi / 3)^{d/2} sqrt(d+1) makes the response to a uniform
 *         density equal to the Gaussian integral (2 pi)^{d/2} times that
 *         density (vertex cell volume (d+1)^{d-1/2} / s^d in feature units).
 *     The adjoint of the chain is the same splat and slice with the blur run
 *     in the order j = d..0.
 *
 * Floating point: every step is FP64. Build with -ffp-contract=off so that no
 * multiply-add is fused: the lattice coordinates decide which vertices exist,
 * and a reader of the code should be able to say exactly what was rounded.
 */

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXD 8

/* ------------------------------------------------------------------------- */
/* 1. Exact Gaussian sum (Sec. 3, eq. fb and eq. gaussiankernel).            */
/* ------------------------------------------------------------------------- */

/*
 * out[a*C + c] = sum_b exp(-|fa_a - fb_b|^2 / 2) * vb[b*C + c]
 * for a in [0, na), b in [0, nb). With exclude_same_index != 0 the term b == a
 * is skipped (the "b != a" of eq. labelling-energy); that only makes sense when
 * the two point sets are the same.
 */
void or_gauss_exact(int na, const double *fa, int nb, const double *fb, int d,
                    int C, const double *vb, double *out,
                    int exclude_same_index)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int a = 0; a < na; ++a) {
        double *o = out + (size_t)a * C;
        for (int c = 0; c < C; ++c) o[c] = 0.0;
        for (int b = 0; b < nb; ++b) {
            if (exclude_same_index && b == a) continue;
            double r2 = 0.0;
            for (int j = 0; j < d; ++j) {
                double t = fa[(size_t)a * d + j] - fb[(size_t)b * d + j];
                r2 += t * t;
            }
            double k = exp(-0.5 * r2);
            const double *v = vb + (size_t)b * C;
            for (int c = 0; c < C; ++c) o[c] += k * v[c];
        }
    }
}

/* ------------------------------------------------------------------------- */
/* 2. Reference permutohedral lattice.                                       */
/* ------------------------------------------------------------------------- */

/* Elevation matrix E (d+1 x d) times the scale s = (d+1) sqrt(2/3).
 * Column j of the orthonormal basis is (1,...,1, -(j+1), 0,...,0) with j+1
 * leading ones, divided by sqrt((j+1)(j+2)). */
static void elevation_matrix(int d, double E[OR_MAXD][OR_MAXD])
{
    double s = (double)(d + 1) * sqrt(2.0 / 3.0);
    for (int i = 0; i <= d; ++i)
        for (int j = 0; j < d; ++j) {
            double cj = s / sqrt((double)((j + 1) * (j + 2)));
            if (i <= j)
                E[i][j] = cj;
            else if (i == j + 1)
                E[i][j] = -(double)(j + 1) * cj;
            else
                E[i][j] = 0.0;
        }
}

/* x = E f, summed in the order j = 0..d-1. */
void or_elevate(int d, const double *f, double *x)
{
    double E[OR_MAXD][OR_MAXD];
    elevation_matrix(d, E);
    for (int i = 0; i <= d; ++i) {
        double acc = 0.0;
        for (int j = 0; j < d; ++j) acc += E[i][j] * f[j];
        x[i] = acc;
    }
}

/* rank[i] = position of coordinate i when delta is sorted in descending
 * order, equal values ordered by lower coordinate index first. */
static void rank_descending(int n, const double *delta, int *rank)
{
    for (int i = 0; i < n; ++i) {
        int r = 0;
        for (int j = 0; j < n; ++j)
            if (delta[j] > delta[i] || (delta[j] == delta[i] && j < i)) ++r;
        rank[i] = r;
    }
}

/*
 * The simplex of the lattice (d+1)A*_d that contains the elevated point x.
 * vert[k*(d+1) + i] = coordinate i of vertex k (k = 0..d), b[k] = its
 * barycentric weight.
 */
void or_simplex(int d, const double *x, int *vert, double *b)
{
    const int D1 = d + 1;
    double c[OR_MAXD], delta[OR_MAXD], y[OR_MAXD];
    int rank[OR_MAXD];
    long sum = 0;

    /* nearest multiple of d+1, coordinate by coordinate */
    for (int i = 0; i < D1; ++i) {
        c[i] = (double)D1 * floor(x[i] / (double)D1 + 0.5);
        sum += (long)llround(c[i]) / D1;
    }
    for (int i = 0; i < D1; ++i) delta[i] = x[i] - c[i];
    rank_descending(D1, delta, rank);

    /* bring the coordinate sum back to zero (Conway and Sloane's decoding of
     * A*_d): move the coordinates that were rounded the farthest */
    if (sum != 0) {
        for (int i = 0; i < D1; ++i) {
            if (sum > 0 && rank[i] >= D1 - sum) c[i] -= (double)D1;
            if (sum < 0 && rank[i] < -sum) c[i] += (double)D1;
        }
        for (int i = 0; i < D1; ++i) delta[i] = x[i] - c[i];
        rank_descending(D1, delta, rank);
    }

    /* barycentric weights from the sorted offsets y_0 >= ... >= y_d */
    for (int i = 0; i < D1; ++i) y[rank[i]] = delta[i];
    b[0] = 1.0 - (y[0] - y[d]) / (double)D1;
    for (int p = 0; p < d; ++p) b[d - p] = (y[p] - y[p + 1]) / (double)D1;

    /* vertex k: coordinate i moves by k, or by k - (d+1) when its rank is
     * among the last k */
    for (int k = 0; k < D1; ++k)
        for (int i = 0; i < D1; ++i)
            vert[k * D1 + i] = (int)llround(c[i]) + k - (rank[i] > d - k ? D1 : 0);
}

/* ---- a small open-addressing hash map: d integer coordinates -> id ---- */

typedef struct {
    int d;
    size_t cap;        /* power of two */
    int *keys;         /* cap x d */
    int *ids;          /* cap, -1 = empty */
} or_map;

static uint64_t hash_coords(int d, const int *k)
{
    uint64_t h = 1469598103934665603ULL;
    for (int i = 0; i < d; ++i) {
        h ^= (uint64_t)(uint32_t)k[i];
        h *= 1099511628211ULL;
    }
    return h;
}

static void map_init(or_map *m, int d, size_t expected)
{
    size_t cap = 16;
    while (cap < 2 * expected + 16) cap <<= 1;
    m->d = d;
    m->cap = cap;
    m->keys = (int *)malloc(cap * (size_t)d * sizeof(int));
    m->ids = (int *)malloc(cap * sizeof(int));
    for (size_t i = 0; i < cap; ++i) m->ids[i] = -1;
}

static void map_free(or_map *m)
{
    free(m->keys);
    free(m->ids);
}

/* returns the id of key k; inserts it with id *next (then ++*next) if absent
 * and insert != 0, else returns -1 when absent */
static int map_find(or_map *m, const int *k, int insert, int *next)
{
    size_t i = hash_coords(m->d, k) & (m->cap - 1);
    for (;;) {
        if (m->ids[i] < 0) {
            if (!insert) return -1;
            memcpy(m->keys + i * m->d, k, (size_t)m->d * sizeof(int));
            m->ids[i] = (*next)++;
            return m->ids[i];
        }
        if (memcmp(m->keys + i * m->d, k, (size_t)m->d * sizeof(int)) == 0)
            return m->ids[i];
        i = (i + 1) & (m->cap - 1);
    }
}

typedef struct {
    int d, n, nv;
    int *pix_vid;      /* n x (d+1): vertex id, -1 where the weight is 0 */
    double *pix_w;     /* n x (d+1): barycentric weight */
    int *vkey;         /* nv x d: first d coordinates of each vertex */
    int *nbr;          /* nv x (d+1) x 2: id of v + u_j, v - u_j, or -1 */
} or_lattice;

/* Build the lattice of n points with features f (n x d). */
or_lattice *or_lattice_build(int n, int d, const double *f)
{
    const int D1 = d + 1;
    or_lattice *L = (or_lattice *)calloc(1, sizeof(or_lattice));
    L->d = d;
    L->n = n;
    L->pix_vid = (int *)malloc((size_t)n * D1 * sizeof(int));
    L->pix_w = (double *)malloc((size_t)n * D1 * sizeof(double));
    L->vkey = (int *)malloc((size_t)n * D1 * d * sizeof(int) + sizeof(int));
    or_map m;
    map_init(&m, d, (size_t)n * D1);
    int next = 0;
    for (int a = 0; a < n; ++a) {
        double x[OR_MAXD], b[OR_MAXD];
        int vert[OR_MAXD * OR_MAXD];
        or_elevate(d, f + (size_t)a * d, x);
        or_simplex(d, x, vert, b);
        for (int k = 0; k < D1; ++k) {
            L->pix_w[(size_t)a * D1 + k] = b[k];
            if (b[k] > 0.0) {
                int before = next;
                int id = map_find(&m, vert + k * D1, 1, &next);
                if (id == before && next == before + 1)
                    memcpy(L->vkey + (size_t)id * d, vert + k * D1,
                           (size_t)d * sizeof(int));
                L->pix_vid[(size_t)a * D1 + k] = id;
            } else {
                L->pix_vid[(size_t)a * D1 + k] = -1;
            }
        }
    }
    L->nv = next;
    /* neighbours along +-u_j; u_j has d at coordinate j and -1 elsewhere,
     * u_d has -1 on all of the first d coordinates */
    L->nbr = (int *)malloc((size_t)(next > 0 ? next : 1) * D1 * 2 * sizeof(int));
    for (int v = 0; v < next; ++v) {
        for (int j = 0; j < D1; ++j) {
            int kp[OR_MAXD], km[OR_MAXD];
            for (int i = 0; i < d; ++i) {
                int u = (i == j) ? d : -1;
                kp[i] = L->vkey[(size_t)v * d + i] + u;
                km[i] = L->vkey[(size_t)v * d + i] - u;
            }
            L->nbr[((size_t)v * D1 + j) * 2 + 0] = map_find(&m, kp, 0, NULL);
            L->nbr[((size_t)v * D1 + j) * 2 + 1] = map_find(&m, km, 0, NULL);
        }
    }
    map_free(&m);
    return L;
}

void or_lattice_free(or_lattice *L)
{
    if (!L) return;
    free(L->pix_vid);
    free(L->pix_w);
    free(L->vkey);
    free(L->nbr);
    free(L);
}

int or_lattice_nv(const or_lattice *L) { return L->nv; }

/* per-point vertex ids and weights, n x (d+1) each */
void or_lattice_points(const or_lattice *L, int *vid, double *w)
{
    size_t cnt = (size_t)L->n * (L->d + 1);
    memcpy(vid, L->pix_vid, cnt * sizeof(int));
    memcpy(w, L->pix_w, cnt * sizeof(double));
}

/* first d coordinates of every vertex, nv x d */
void or_lattice_keys(const or_lattice *L, int *keys)
{
    memcpy(keys, L->vkey, (size_t)L->nv * L->d * sizeof(int));
}

/* neighbour table, nv x (d+1) x 2 */
void or_lattice_neighbours(const or_lattice *L, int *nbr)
{
    memcpy(nbr, L->nbr, (size_t)L->nv * (L->d + 1) * 2 * sizeof(int));
}

/* V (nv x C) = sum over points of b * in (n x C). The channels are
 * independent: threads take whole channels, and every V[v][c] receives its
 * terms in the order of the points, as in a serial loop. */
void or_lattice_splat(const or_lattice *L, int C, const double *in, double *V)
{
    const int D1 = L->d + 1;
    memset(V, 0, (size_t)L->nv * C * sizeof(double));
#pragma omp parallel for schedule(static) if (C > 1 && (size_t)L->n * C > 4096)
    for (int c = 0; c < C; ++c)
        for (int a = 0; a < L->n; ++a)
            for (int k = 0; k < D1; ++k) {
                int v = L->pix_vid[(size_t)a * D1 + k];
                if (v < 0) continue;
                double b = L->pix_w[(size_t)a * D1 + k];
                V[(size_t)v * C + c] += b * in[(size_t)a * C + c];
            }
}

/* one blur pass along u_j, out of place */
static void blur_pass(const or_lattice *L, int j, int C, const double *V,
                      double *W)
{
    const int D1 = L->d + 1;
#pragma omp parallel for schedule(static) if ((size_t)L->nv * C > 16384)
    for (int v = 0; v < L->nv; ++v) {
        int np = L->nbr[((size_t)v * D1 + j) * 2 + 0];
        int nm = L->nbr[((size_t)v * D1 + j) * 2 + 1];
        for (int c = 0; c < C; ++c) {
            double vp = np >= 0 ? V[(size_t)np * C + c] : 0.0;
            double vm = nm >= 0 ? V[(size_t)nm * C + c] : 0.0;
            W[(size_t)v * C + c] = 0.5 * V[(size_t)v * C + c] + 0.25 * (vp + vm);
        }
    }
}

/* all d+1 passes, j = 0..d (reverse != 0: j = d..0); V is overwritten */
void or_lattice_blur(const or_lattice *L, int C, double *V, int reverse)
{
    const int D1 = L->d + 1;
    size_t cnt = (size_t)L->nv * C;
    double *W = (double *)malloc((cnt ? cnt : 1) * sizeof(double));
    for (int p = 0; p < D1; ++p) {
        int j = reverse ? (D1 - 1 - p) : p;
        blur_pass(L, j, C, V, W);
        memcpy(V, W, cnt * sizeof(double));
    }
    free(W);
}

/* out (n x C) = sum_k b_k V[v_k]   (no calibration factor) */
void or_lattice_slice(const or_lattice *L, int C, const double *V, double *out)
{
    const int D1 = L->d + 1;
#pragma omp parallel for schedule(static) if ((size_t)L->n * C > 16384)
    for (int a = 0; a < L->n; ++a) {
        for (int c = 0; c < C; ++c) out[(size_t)a * C + c] = 0.0;
        for (int k = 0; k < D1; ++k) {
            int v = L->pix_vid[(size_t)a * D1 + k];
            if (v < 0) continue;
            double b = L->pix_w[(size_t)a * D1 + k];
            for (int c = 0; c < C; ++c)
                out[(size_t)a * C + c] += b * V[(size_t)v * C + c];
        }
    }
}

double or_lattice_gamma(int d)
{
    return pow(4.0 * M_PI / 3.0, 0.5 * d) * sqrt((double)(d + 1));
}

/* out = gamma_d * slice(blur(splat(in))) ; reverse != 0 gives the adjoint */
void or_lattice_filter(const or_lattice *L, int C, const double *in,
                       double *out, int reverse)
{
    size_t cnt = (size_t)L->nv * C;
    double *V = (double *)malloc((cnt ? cnt : 1) * sizeof(double));
    or_lattice_splat(L, C, in, V);
    or_lattice_blur(L, C, V, reverse);
    or_lattice_slice(L, C, V, out);
    double g = or_lattice_gamma(L->d);
    for (size_t i = 0; i < (size_t)L->n * C; ++i) out[i] *= g;
    free(V);
}

/* ------------------------------------------------------------------------- */
/* 3. The two triangular sums of the LP subgradient by divide and conquer.   */
/* ------------------------------------------------------------------------- */

/*
 * For one order of the N pixels (order[p] = pixel at position p), the sums of
 * eq. grad_lp
 *     U[c]  = sum over pixels a after c  of Kbar_ac,
 *     Lo[c] = sum over pixels a before c of Kbar_ac,
 * with Kbar = sum_m w_m K_m, by the divide and conquer of App. E: every node
 * [lo, hi) of level l (lo = floor(n N / 2^l), split at
 * mid = floor((2n+1) N / 2^(l+1))) filters the indicator of its left half and
 * of its right half over the node's own points, with one reference lattice
 * per kernel built on those points; the right indicator read at the left half
 * adds to U, the left indicator read at the right half adds to Lo. Levels
 * l = 0 .. ceil(log2 N) - 1. The nodes of a level hold disjoint pixels, so they
 * are independent; within a node the kernels are added in the order m = 0..nk-1
 * (acc = acc + w_m * filter_m), and the levels in increasing order.
 * feats[m]: N x dims[m] features of kernel m (pixel-indexed).
 */
void or_lp_dnc_lattice(int N, int nk, const int *dims, const double *const *feats,
                       const double *w, const int *order, double *U, double *Lo)
{
    for (int a = 0; a < N; ++a) U[a] = Lo[a] = 0.0;
    int levels = 0;
    while ((1LL << levels) < (long long)N) ++levels;
    for (int l = 0; l < levels; ++l) {
        const long long nn = 1LL << l;
#pragma omp parallel for schedule(dynamic, 1)
        for (long long n = 0; n < nn; ++n) {
            const long long lo = (n * N) >> l, hi = ((n + 1) * N) >> l;
            const long long mid = ((2 * n + 1) * N) >> (l + 1);
            if (!(lo < mid && mid < hi)) continue;
            const int np = (int)(hi - lo), nl = (int)(mid - lo);
            double *ind = (double *)calloc((size_t)np * 2, sizeof(double));
            double *acc = (double *)calloc((size_t)np * 2, sizeof(double));
            double *out = (double *)malloc((size_t)np * 2 * sizeof(double));
            for (int i = 0; i < np; ++i) ind[(size_t)i * 2 + (i < nl ? 0 : 1)] = 1.0;
            for (int m = 0; m < nk; ++m) {
                const int d = dims[m];
                double *f = (double *)malloc((size_t)np * d * sizeof(double));
                for (int i = 0; i < np; ++i)
                    memcpy(f + (size_t)i * d, feats[m] + (size_t)order[lo + i] * d,
                           (size_t)d * sizeof(double));
                or_lattice *Lt = or_lattice_build(np, d, f);
                or_lattice_filter(Lt, 2, ind, out, 0);
                for (int i = 0; i < np * 2; ++i) acc[i] += w[m] * out[i];
                or_lattice_free(Lt);
                free(f);
            }
            for (int i = 0; i < nl; ++i) U[order[lo + i]] += acc[(size_t)i * 2 + 1];
            for (int i = nl; i < np; ++i) Lo[order[lo + i]] += acc[(size_t)i * 2 + 0];
            free(ind);
            free(acc);
            free(out);
        }
    }
}
