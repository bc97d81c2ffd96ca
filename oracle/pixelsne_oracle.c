/*
 * PixelSNE CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 implementation of what PixelSNE computes (Kim et al.,
 * "PixelSNE: Visualizing Fast with Just Enough Precision via Pixel-Aligned
 * Stochastic Neighbor Embedding", arXiv:1611.02568).  It exists to check the
 * GPU library; only the tests, the smoke check and the benchmark's CPU
 * baseline may load it.  It shares no code, header or constant table with
 * the GPU path.
 *
 * Every step follows the paper's order and notation:
 *   - high-dimensional affinities P from a Gaussian kernel at a perplexity
 *     (Section 3.2) over k nearest neighbours (Section 3.3);
 *   - pixel coordinates z with 0 <= z < r (Eq. 1-2);
 *   - the pixel-aligned quadtree (P-Quadtree, Section 4.1): the root is the
 *     fixed screen, cells split down to unit pixels, each cell holds its
 *     boundary (Eq. 6), member count and centre of mass (Eq. 7-8);
 *   - Barnes-Hut repulsion by depth-first traversal with the opening
 *     criterion (Eq. 11), leaf stop (Section 4.1, "Bounded tree depth");
 *   - q in terms of z with the scale factors beta (Eq. 12-13) and the
 *     gradient of Eq. 5 in the pixel frame;
 *   - screen-driven scaling (Section 4.2).
 *
 * Readings where the paper is silent or garbled (each one is listed in the
 * design notes): the opening test compares the cell diagonal with the
 * unsquared distance; the test runs in the true (beta-weighted) metric; the
 * leaf that holds point i excludes i itself; the tree root is [0, 2^L)^2 with
 * unit-pixel leaves; pixel = clamp(floor(z), 0, r-1); optimiser constants are
 * the usual Barnes-Hut-SNE ones (eta 200, momentum 0.5 -> 0.8 at 250, gains
 * +0.2 / x0.8 floored at 0.01, exaggeration 12 for 250 iterations).
 *
 * Centre-of-mass sums and Z use compensated (Neumaier) summation so that the
 * oracle's sums are accurate to a few ulp regardless of order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2

int orc_version(void) { return 3; }

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* ------------------------------------------------------------------ */
/* compensated summation                                               */
/* ------------------------------------------------------------------ */
typedef struct { double s, c; } csum;
static inline void cs_add(csum* a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static inline double cs_get(const csum* a) { return a->s + a->c; }

/* ------------------------------------------------------------------ */
/* k nearest neighbours, brute force (replaces the VP / RP trees of     */
/* Section 3.3 and 4.3).  Squared Euclidean distance in FP64; the       */
/* point itself is excluded; ties go to the smaller index.              */
/* ------------------------------------------------------------------ */
static inline int knn_less(double da, int32_t ja, double db, int32_t jb) {
    return da < db || (da == db && ja < jb);
}

/* max-heap on (d, j) */
static void heap_sift_down(double* d, int32_t* j, int m, int pos) {
    for (;;) {
        int l = 2 * pos + 1, r = l + 1, big = pos;
        if (l < m && knn_less(d[big], j[big], d[l], j[l])) big = l;
        if (r < m && knn_less(d[big], j[big], d[r], j[r])) big = r;
        if (big == pos) return;
        double td = d[pos]; d[pos] = d[big]; d[big] = td;
        int32_t tj = j[pos]; j[pos] = j[big]; j[big] = tj;
        pos = big;
    }
}
static void heap_sift_up(double* d, int32_t* j, int pos) {
    while (pos > 0) {
        int p = (pos - 1) / 2;
        if (!knn_less(d[p], j[p], d[pos], j[pos])) return;
        double td = d[pos]; d[pos] = d[p]; d[p] = td;
        int32_t tj = j[pos]; j[pos] = j[p]; j[p] = tj;
        pos = p;
    }
}

/* rows == NULL: all n rows.  Outputs idx/d2 are [nrows][k], ascending. */
int orc_knn(const double* X, int64_t n, int32_t D, int32_t k, const int64_t* rows,
            int64_t nrows, int32_t* idx_out, double* d2_out) {
    if (!X || n < 2 || D < 1 || k < 1 || k > n - 1) return ORC_EINVAL;
    if (!rows) nrows = n;
    int64_t q;
#pragma omp parallel for schedule(dynamic, 4)
    for (q = 0; q < nrows; q++) {
        int64_t i = rows ? rows[q] : q;
        double* hd = d2_out + q * k;
        int32_t* hj = idx_out + q * k;
        int m = 0;
        const double* xi = X + i * (int64_t)D;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            const double* xj = X + j * (int64_t)D;
            double s = 0.0;
            for (int t = 0; t < D; t++) { double e = xi[t] - xj[t]; s += e * e; }
            if (m < k) {
                hd[m] = s; hj[m] = (int32_t)j; heap_sift_up(hd, hj, m); m++;
            } else if (knn_less(s, (int32_t)j, hd[0], hj[0])) {
                hd[0] = s; hj[0] = (int32_t)j; heap_sift_down(hd, hj, m, 0);
            }
        }
        /* heap sort into ascending order */
        for (int e = m - 1; e > 0; e--) {
            double td = hd[0]; hd[0] = hd[e]; hd[e] = td;
            int32_t tj = hj[0]; hj[0] = hj[e]; hj[e] = tj;
            heap_sift_down(hd, hj, e, 0);
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Approximate k nearest neighbours (Section 4.3: the K-NNG of          */
/* LargeVis): a few random-projection trees give every point candidate  */
/* neighbours (the other points of its leaf); then, since the neighbours */
/* of a point's neighbours are likely its neighbours too, a few rounds   */
/* replace each point's list by the best k of the list and its          */
/* neighbours' lists (every round reads the previous round's lists).    */
/*                                                                      */
/* A tree splits a set of points (a range of a permutation, in order)   */
/* by the hyperplane halfway between two of its points a and b, chosen  */
/* by a counter-based generator: point i goes right iff                 */
/*   sum_d (x_id - (x_ad + x_bd) / 2) (x_ad - x_bd) > 0                 */
/* (FP64, terms in order of d, no fused multiply-add); the split keeps   */
/* the order inside each side.  If a side would hold fewer than k + 1    */
/* points (equal points, or a plane near the edge), or below level 48,   */
/* the range is cut in the middle instead, so that with leaf_size >=     */
/* 2k + 2 every leaf offers each of its points at least k candidates.    */
/* Ranges of at most leaf_size points are leaves.  The generator is     */
/* SplitMix64 (Steele, Lea and Flood, 2014) keyed by seed, tree, level  */
/* and the range's first position: a = h0 mod m, b = h1 mod (m - 1),     */
/* b += 1 if b >= a.  Lists are the best k by (d^2, index), distinct,   */
/* self excluded.                                                       */
/* ------------------------------------------------------------------ */
static inline uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

static uint64_t rp_draw(uint64_t seed, int32_t tree, int32_t level, int64_t a, int which) {
    uint64_t x = splitmix64(seed ^ (uint64_t)(uint32_t)tree);
    x = splitmix64(x ^ (uint64_t)(uint32_t)level);
    return splitmix64(x ^ (((uint64_t)a << 1) | (uint64_t)which));
}

static double sqdist(const double* X, int32_t D, int64_t i, int64_t j) {
    const double* a = X + i * (int64_t)D;
    const double* b = X + j * (int64_t)D;
    double s = 0.0;
    for (int t = 0; t < D; t++) { double e = a[t] - b[t]; s += e * e; }
    return s;
}

/* keep the best k of a sorted list (ascending (d, j)); no duplicates */
static void list_insert(double* ld, int32_t* lj, int32_t* m, int32_t k, double d, int32_t j) {
    if (*m == k && !knn_less(d, j, ld[k - 1], lj[k - 1])) return;
    for (int32_t q = 0; q < *m; q++) if (lj[q] == j) return;
    int32_t pos = *m < k ? *m : k - 1;
    while (pos > 0 && knn_less(d, j, ld[pos - 1], lj[pos - 1])) {
        ld[pos] = ld[pos - 1]; lj[pos] = lj[pos - 1]; pos--;
    }
    ld[pos] = d; lj[pos] = j;
    if (*m < k) (*m)++;
}

#define RP_MAX_LEVEL 48

int orc_knn_approx(const double* X, int64_t n, int32_t D, int32_t k, int32_t n_trees,
                   int32_t leaf_size, int32_t explore, uint64_t seed, int32_t* idx_out,
                   double* d2_out) {
    if (!X || n < 2 || D < 1 || k < 1 || k > n - 1 || n_trees < 1 || leaf_size < 2 * k + 2 ||
        explore < 0 || n >= ((int64_t)1 << 31))
        return ORC_EINVAL;
    int64_t* perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* tmp = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* seg = (int64_t*)malloc(sizeof(int64_t) * 2 * (size_t)n);    /* (a, b) pairs */
    int64_t* seg2 = (int64_t*)malloc(sizeof(int64_t) * 2 * (size_t)n);
    unsigned char* side = (unsigned char*)malloc((size_t)n);
    double* ld = (double*)malloc(sizeof(double) * (size_t)n * k);
    int32_t* lj = (int32_t*)malloc(sizeof(int32_t) * (size_t)n * k);
    double* nd = (double*)malloc(sizeof(double) * (size_t)n * k);
    int32_t* nj = (int32_t*)malloc(sizeof(int32_t) * (size_t)n * k);
    int32_t* lm = (int32_t*)calloc((size_t)n, sizeof(int32_t));
    int32_t* nm = (int32_t*)calloc((size_t)n, sizeof(int32_t));
    int rc = ORC_OK;
    if (!perm || !tmp || !seg || !seg2 || !side || !ld || !lj || !nd || !nj || !lm || !nm) {
        rc = ORC_ENOMEM;
        goto done;
    }
    for (int32_t tr = 0; tr < n_trees; tr++) {
        for (int64_t i = 0; i < n; i++) perm[i] = i;
        int64_t ns = 1;
        seg[0] = 0; seg[1] = n;
        for (int32_t level = 0;; level++) {
            int64_t ns2 = 0, split = 0;
            for (int64_t s = 0; s < ns; s++) {
                const int64_t a = seg[2 * s], b = seg[2 * s + 1], m = b - a;
                if (m <= leaf_size) {                  /* a leaf: keep */
                    seg2[2 * ns2] = a; seg2[2 * ns2 + 1] = b; ns2++;
                    continue;
                }
                split = 1;
                int64_t nl = 0;
                if (level < RP_MAX_LEVEL) {
                    int64_t ia = (int64_t)(rp_draw(seed, tr, level, a, 0) % (uint64_t)m);
                    int64_t ib = (int64_t)(rp_draw(seed, tr, level, a, 1) % (uint64_t)(m - 1));
                    if (ib >= ia) ib++;
                    const double* xa = X + perm[a + ia] * (int64_t)D;
                    const double* xb = X + perm[a + ib] * (int64_t)D;
                    for (int64_t p = a; p < b; p++) {
                        const double* xi = X + perm[p] * (int64_t)D;
                        double acc = 0.0;
                        for (int d = 0; d < D; d++) {
                            double mid = (xa[d] + xb[d]) * 0.5;
                            double v = xa[d] - xb[d];
                            acc += (xi[d] - mid) * v;
                        }
                        side[p] = acc > 0.0;
                        nl += side[p] ? 0 : 1;
                    }
                }
                if (nl < k + 1 || m - nl < k + 1) {
                    nl = m / 2;                        /* cut in the middle, order kept */
                } else {
                    int64_t l = a, r = a + nl;
                    for (int64_t p = a; p < b; p++) {
                        if (side[p]) tmp[r++] = perm[p];
                        else tmp[l++] = perm[p];
                    }
                    for (int64_t p = a; p < b; p++) perm[p] = tmp[p];
                }
                seg2[2 * ns2] = a; seg2[2 * ns2 + 1] = a + nl; ns2++;
                seg2[2 * ns2] = a + nl; seg2[2 * ns2 + 1] = b; ns2++;
            }
            int64_t* sw = seg; seg = seg2; seg2 = sw;
            ns = ns2;
            if (!split) break;
        }
        /* leaf mates are candidates */
        int64_t s;
#pragma omp parallel for schedule(dynamic, 16)
        for (s = 0; s < ns; s++) {
            const int64_t a = seg[2 * s], b = seg[2 * s + 1];
            for (int64_t p = a; p < b; p++) {
                const int64_t i = perm[p];
                for (int64_t q = a; q < b; q++) {
                    if (q == p) continue;
                    const int64_t j = perm[q];
                    list_insert(ld + i * k, lj + i * k, &lm[i], k, sqdist(X, D, i, j), (int32_t)j);
                }
            }
        }
    }
    for (int32_t e = 0; e < explore; e++) {
        int64_t i;
#pragma omp parallel for schedule(dynamic, 64)
        for (i = 0; i < n; i++) {
            double* od = nd + i * k;
            int32_t* oj = nj + i * k;
            int32_t om = lm[i];
            for (int32_t q = 0; q < om; q++) { od[q] = ld[i * k + q]; oj[q] = lj[i * k + q]; }
            for (int32_t a = 0; a < lm[i]; a++) {
                const int64_t j = lj[i * k + a];
                for (int32_t c = 0; c < lm[j]; c++) {
                    const int64_t l = lj[j * k + c];
                    if (l == i) continue;
                    list_insert(od, oj, &om, k, sqdist(X, D, i, l), (int32_t)l);
                }
            }
            nm[i] = om;
        }
        double* sd = ld; ld = nd; nd = sd;
        int32_t* sj = lj; lj = nj; nj = sj;
        int32_t* sm = lm; lm = nm; nm = sm;
    }
    {
        int64_t i;
        for (i = 0; i < n; i++) {
            if (lm[i] < k) { rc = ORC_EINVAL; goto done; }   /* cannot happen: see above */
            for (int32_t q = 0; q < k; q++) {
                idx_out[i * k + q] = lj[i * k + q];
                d2_out[i * k + q] = ld[i * k + q];
            }
        }
    }
done:
    free(perm); free(tmp); free(seg); free(seg2); free(side);
    free(ld); free(lj); free(nd); free(nj); free(lm); free(nm);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Perplexity calibration (Section 3.2): for each row find the          */
/* Gaussian precision b_i with entropy H(P_i) = ln(u) (natural log),   */
/* p_{j|i} = exp(-b_i * delta_j) / sum, delta_j = d2_ij - min_j d2_ij   */
/* (the shift cancels in the normalisation).  Bisection that doubles / */
/* halves b until the root is bracketed, from b = 1; stops when         */
/* |H - ln u| < tol or after max_iter evaluations.                      */
/* ------------------------------------------------------------------ */
int orc_perplexity(const double* d2, int64_t nrows, int32_t k, double perplexity, double tol,
                   int32_t max_iter, double* P_out, double* beta_out, int32_t* iters_out) {
    if (!d2 || !P_out || nrows < 1 || k < 1 || !(perplexity > 0)) return ORC_EINVAL;
    const double target = log(perplexity);
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < nrows; i++) {
        const double* d = d2 + i * k;
        double* p = P_out + i * k;
        double dmin = d[0];
        for (int j = 1; j < k; j++) if (d[j] < dmin) dmin = d[j];
        double b = 1.0, lo = 0.0, hi = 0.0;
        int have_lo = 0, have_hi = 0, it;
        double S = 0.0;
        for (it = 0; it < max_iter; it++) {
            S = 0.0; double SD = 0.0;
            for (int j = 0; j < k; j++) {
                double dj = d[j] - dmin;
                double e = exp(-b * dj);
                p[j] = e; S += e; SD += dj * e;
            }
            double H = log(S) + b * SD / S;
            if (fabs(H - target) < tol || it == max_iter - 1) break;
            if (H > target) {              /* too flat: sharpen */
                lo = b; have_lo = 1;
                b = have_hi ? 0.5 * (b + hi) : 2.0 * b;
            } else {                       /* too peaked: flatten */
                hi = b; have_hi = 1;
                b = have_lo ? 0.5 * (b + lo) : 0.5 * b;
            }
        }
        for (int j = 0; j < k; j++) p[j] /= S;
        if (beta_out) beta_out[i] = b;
        if (iters_out) iters_out[i] = it + 1;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Symmetrisation: p_ij = (p_{j|i} + p_{i|j}) / (2n) over the union of  */
/* the directed kNN edges, zero diagonal, CSR with ascending columns.   */
/* Both entries of a pair are formed from the same two summands, so the */
/* result is exactly symmetric.  Returns nnz (< 0 on error).  Call once */
/* with col == NULL to size the arrays.                                 */
/* ------------------------------------------------------------------ */
typedef struct { int32_t r, c; double v; } coo_t;
static int coo_cmp(const void* a, const void* b) {
    const coo_t* x = (const coo_t*)a; const coo_t* y = (const coo_t*)b;
    if (x->r != y->r) return x->r < y->r ? -1 : 1;
    if (x->c != y->c) return x->c < y->c ? -1 : 1;
    return 0;
}

int64_t orc_symmetrize(const int32_t* idx, const double* Pc, int64_t n, int32_t k,
                       int64_t* row_ptr, int32_t* col, double* val, int64_t cap) {
    if (!idx || !Pc || n < 2 || k < 1) return ORC_EINVAL;
    int64_t m = 2 * n * (int64_t)k;
    coo_t* e = (coo_t*)malloc(sizeof(coo_t) * (size_t)m);
    if (!e) return ORC_ENOMEM;
    for (int64_t i = 0; i < n; i++)
        for (int t = 0; t < k; t++) {
            int32_t j = idx[i * k + t];
            double v = Pc[i * k + t];
            e[2 * (i * k + t)] = (coo_t){(int32_t)i, j, v};
            e[2 * (i * k + t) + 1] = (coo_t){j, (int32_t)i, v};
        }
    qsort(e, (size_t)m, sizeof(coo_t), coo_cmp);
    int64_t nnz = 0;
    for (int64_t a = 0; a < m;) {
        int64_t b = a + 1;
        while (b < m && e[b].r == e[a].r && e[b].c == e[a].c) b++;
        if (e[a].r != e[a].c) nnz++;
        a = b;
    }
    if (col) {
        if (cap < nnz || !row_ptr || !val) { free(e); return ORC_EINVAL; }
        for (int64_t i = 0; i <= n; i++) row_ptr[i] = 0;
        int64_t w = 0;
        for (int64_t a = 0; a < m;) {
            int64_t b = a + 1;
            while (b < m && e[b].r == e[a].r && e[b].c == e[a].c) b++;
            if (e[a].r != e[a].c) {
                /* at most two summands (i->j and j->i), added once */
                double s = e[a].v;
                for (int64_t c = a + 1; c < b; c++) s += e[c].v;
                col[w] = e[a].c;
                val[w] = s / (2.0 * (double)n);
                row_ptr[e[a].r + 1]++;
                w++;
            }
            a = b;
        }
        for (int64_t i = 0; i < n; i++) row_ptr[i + 1] += row_ptr[i];
    }
    free(e);
    return nnz;
}

/* ------------------------------------------------------------------ */
/* Pixel assignment and Morton keys (Eq. 1-2, Section 4.1).             */
/* pixel = clamp(floor(z), 0, r - 1); key interleaves x in even bits    */
/* and y in odd bits, so the child index is 2*ybit + xbit (NW, NE, SW,  */
/* SE with y pointing down the screen).                                 */
/* ------------------------------------------------------------------ */
static inline int32_t pixel_of(double z, int32_t r) {
    double f = floor(z);
    if (!(f >= 0.0)) return 0;           /* also catches NaN */
    if (f > (double)(r - 1)) return r - 1;
    return (int32_t)f;
}

static inline uint32_t morton2(uint32_t px, uint32_t py, int L) {
    uint32_t key = 0;
    for (int b = 0; b < L; b++) {
        key |= ((px >> b) & 1u) << (2 * b);
        key |= ((py >> b) & 1u) << (2 * b + 1);
    }
    return key;
}

static int log2_exact(int32_t r) {
    if (r < 2 || (r & (r - 1))) return -1;
    int L = 0;
    while ((1 << L) < r) L++;
    return L;
}

int orc_morton(const double* z, int64_t n, int32_t r, uint32_t* key) {
    int L = log2_exact(r);
    if (L < 0 || L > 16) return ORC_EINVAL;
    for (int64_t i = 0; i < n; i++)
        key[i] = morton2((uint32_t)pixel_of(z[2 * i], r), (uint32_t)pixel_of(z[2 * i + 1], r), L);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* P-Quadtree (Section 4.1).  Built by assigning each point, in index   */
/* order, from the root down to its unit pixel; every cell on the way   */
/* counts the point and accumulates its coordinates for the centre of  */
/* mass (Eq. 8).                                                        */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t child[4];
    int32_t level;
    uint32_t prefix;        /* P-Quadtree: Morton prefix of the cell */
    uint64_t prefix64;      /* D-Quadtree: Morton prefix on the 2^32 grid */
    int64_t count;
    csum sx, sy;
    int64_t first;          /* D-Quadtree leaf: first member point (-1: none) */
} onode;

typedef struct {
    int32_t r, L;
    int32_t kind;           /* 0: P-Quadtree (pixel leaves), 1: D-Quadtree */
    int32_t Lmax;           /* deepest level: L, or 32 for the D-Quadtree */
    int64_t n, nnodes, cap;
    onode* nodes;
    int32_t* leaf_of;       /* node id of each point's leaf */
    int64_t* next;          /* D-Quadtree: next member of the same leaf (-1: last) */
} otree;

static inline int is_leaf(const onode* nd) {
    return nd->child[0] < 0 && nd->child[1] < 0 && nd->child[2] < 0 && nd->child[3] < 0;
}

static int32_t tree_new_node(otree* t, int32_t level, uint32_t prefix) {
    if (t->nnodes == t->cap) {
        int64_t nc = t->cap ? 2 * t->cap : 1024;
        onode* p = (onode*)realloc(t->nodes, sizeof(onode) * (size_t)nc);
        if (!p) return -1;
        t->nodes = p; t->cap = nc;
    }
    onode* c = &t->nodes[t->nnodes];
    memset(c, 0, sizeof(*c));
    c->child[0] = c->child[1] = c->child[2] = c->child[3] = -1;
    c->level = level; c->prefix = prefix;
    c->first = -1;
    return (int32_t)t->nnodes++;
}

void orc_tree_free(void* h) {
    otree* t = (otree*)h;
    if (!t) return;
    free(t->nodes); free(t->leaf_of); free(t->next); free(t);
}

void* orc_tree_build(const double* z, int64_t n, int32_t r) {
    int L = log2_exact(r);
    if (!z || n < 1 || L < 0 || L > 16) return NULL;
    otree* t = (otree*)calloc(1, sizeof(otree));
    if (!t) return NULL;
    t->r = r; t->L = L; t->n = n;
    t->kind = 0; t->Lmax = L;
    t->leaf_of = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!t->leaf_of || tree_new_node(t, 0, 0) != 0) { orc_tree_free(t); return NULL; }
    for (int64_t i = 0; i < n; i++) {
        double zx = z[2 * i], zy = z[2 * i + 1];
        uint32_t px = (uint32_t)pixel_of(zx, r), py = (uint32_t)pixel_of(zy, r);
        int32_t c = 0;
        for (int l = 0;; l++) {
            onode* nd = &t->nodes[c];
            nd->count++;
            cs_add(&nd->sx, zx);
            cs_add(&nd->sy, zy);
            if (l == L) break;
            int sh = L - 1 - l;           /* bit that splits this cell */
            int q = (int)(((py >> sh) & 1u) << 1 | ((px >> sh) & 1u));
            int32_t ch = nd->child[q];
            if (ch < 0) {
                uint32_t pre = (nd->prefix << 2) | (uint32_t)q;
                ch = tree_new_node(t, l + 1, pre);
                if (ch < 0) { orc_tree_free(t); return NULL; }
                t->nodes[c].child[q] = ch;   /* nodes may have moved */
            }
            c = ch;
        }
        t->leaf_of[i] = c;
    }
    return t;
}

/* ------------------------------------------------------------------ */
/* D-Quadtree of Barnes-Hut-SNE (Section 3.3): the root spans the data, */
/* [min y_d, max y_d + eps) per axis (Eq. 9-10), and cells split into  */
/* four equal quadrants as points are assigned one by one, until every  */
/* leaf holds at most one point.  The root is the screen's frame: the   */
/* scaling of Section 4.2 maps [min, max + eps) onto [0, r), so in the  */
/* pixel frame the root is [0, r)^2.  Cell boundaries are kept exact on */
/* a 2^32 x 2^32 grid over the root (q = floor(z 2^(32 - L)); child     */
/* index 2 ybit + xbit as for the P-Quadtree); points that fall in one  */
/* grid cell cannot be told apart there and share a leaf at level 32.   */
/* Each cell counts its points and sums their coordinates (Eq. 7-8).    */
/* ------------------------------------------------------------------ */
static inline uint32_t grid32(double z, int L) {
    double f = floor(ldexp(z, 32 - L));
    if (!(f >= 0.0)) return 0;
    if (f > 4294967295.0) return 4294967295u;
    return (uint32_t)f;
}

static inline int quadrant(uint32_t qx, uint32_t qy, int level) {
    int sh = 31 - level;                  /* bit that splits a cell of this level */
    return (int)(((qy >> sh) & 1u) << 1 | ((qx >> sh) & 1u));
}

void* orc_dtree_build(const double* z, int64_t n, int32_t r) {
    int L = log2_exact(r);
    if (!z || n < 1 || L < 0 || L > 16) return NULL;
    otree* t = (otree*)calloc(1, sizeof(otree));
    if (!t) return NULL;
    t->r = r; t->L = L; t->n = n;
    t->kind = 1; t->Lmax = 32;
    t->leaf_of = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    t->next = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    if (!t->leaf_of || !t->next || tree_new_node(t, 0, 0) != 0) { orc_tree_free(t); return NULL; }
    for (int64_t i = 0; i < n; i++) {
        const double zx = z[2 * i], zy = z[2 * i + 1];
        const uint32_t qx = grid32(zx, L), qy = grid32(zy, L);
        int32_t c = 0;
        for (;;) {
            onode* nd = &t->nodes[c];
            nd->count++;
            cs_add(&nd->sx, zx);
            cs_add(&nd->sy, zy);
            if (is_leaf(nd)) {
                if (nd->first < 0) {                       /* empty leaf */
                    nd->first = i; t->next[i] = -1;
                    break;
                }
                const int64_t f = nd->first;
                const uint32_t fx = grid32(z[2 * f], L), fy = grid32(z[2 * f + 1], L);
                if (nd->level == 32 || (fx == qx && fy == qy)) {
                    /* same grid cell: the leaf keeps both (members in order) */
                    int64_t j = f;
                    while (t->next[j] >= 0) j = t->next[j];
                    t->next[j] = i; t->next[i] = -1;
                    break;
                }
                /* split: the leaf's members (one grid position) move to
                 * their quadrant child; then i continues below */
                const int level = nd->level;
                const uint64_t pre = nd->prefix64;
                const int qf = quadrant(fx, fy, level);
                int32_t ch = tree_new_node(t, level + 1, 0);
                if (ch < 0) { orc_tree_free(t); return NULL; }
                nd = &t->nodes[c];                           /* nodes may have moved */
                onode* cn = &t->nodes[ch];
                cn->prefix64 = (pre << 2) | (uint64_t)qf;
                cn->first = f;
                for (int64_t j = f; j >= 0; j = t->next[j]) {
                    cn->count++;
                    cs_add(&cn->sx, z[2 * j]);
                    cs_add(&cn->sy, z[2 * j + 1]);
                }
                nd->first = -1;
                nd->child[qf] = ch;
            }
            const int q = quadrant(qx, qy, nd->level);
            int32_t ch = nd->child[q];
            if (ch < 0) {
                const uint64_t pre = (nd->prefix64 << 2) | (uint64_t)q;
                const int level = nd->level;
                ch = tree_new_node(t, level + 1, 0);
                if (ch < 0) { orc_tree_free(t); return NULL; }
                t->nodes[ch].prefix64 = pre;
                t->nodes[c].child[q] = ch;
            }
            c = ch;
        }
    }
    /* each point's leaf, after all the splits */
    for (int64_t c = 0; c < t->nnodes; c++)
        if (is_leaf(&t->nodes[c]))
            for (int64_t j = t->nodes[c].first; j >= 0; j = t->next[j]) t->leaf_of[j] = (int32_t)c;
    return t;
}

int32_t orc_tree_depth(const void* h) { return ((const otree*)h)->Lmax; }
int64_t orc_tree_num_nodes(const void* h) { return ((const otree*)h)->nnodes; }

/* number of occupied cells at each level 0..Lmax */
int orc_tree_level_sizes(const void* h, int64_t* sizes) {
    const otree* t = (const otree*)h;
    for (int l = 0; l <= t->Lmax; l++) sizes[l] = 0;
    for (int64_t c = 0; c < t->nnodes; c++) sizes[t->nodes[c].level]++;
    return ORC_OK;
}

typedef struct { uint32_t prefix; int64_t id; } pref_t;
static int pref_cmp(const void* a, const void* b) {
    const pref_t* x = (const pref_t*)a; const pref_t* y = (const pref_t*)b;
    return x->prefix < y->prefix ? -1 : (x->prefix > y->prefix ? 1 : 0);
}

/* cells of one level of a D-Quadtree ascending by prefix: prefix on the
 * 2^32 grid, count, sums */
typedef struct { uint64_t prefix; int64_t id; } pref64_t;
static int pref64_cmp(const void* a, const void* b) {
    const pref64_t* x = (const pref64_t*)a; const pref64_t* y = (const pref64_t*)b;
    return x->prefix < y->prefix ? -1 : (x->prefix > y->prefix ? 1 : 0);
}

int orc_tree_level64(const void* h, int32_t level, uint64_t* prefix, int64_t* count, double* sum) {
    const otree* t = (const otree*)h;
    if (level < 0 || level > t->Lmax) return ORC_EINVAL;
    int64_t m = 0;
    for (int64_t c = 0; c < t->nnodes; c++) if (t->nodes[c].level == level) m++;
    pref64_t* v = (pref64_t*)malloc(sizeof(pref64_t) * (size_t)(m ? m : 1));
    if (!v) return ORC_ENOMEM;
    m = 0;
    for (int64_t c = 0; c < t->nnodes; c++)
        if (t->nodes[c].level == level) { v[m].prefix = t->nodes[c].prefix64; v[m].id = c; m++; }
    qsort(v, (size_t)m, sizeof(pref64_t), pref64_cmp);
    for (int64_t a = 0; a < m; a++) {
        const onode* nd = &t->nodes[v[a].id];
        if (prefix) prefix[a] = nd->prefix64;
        if (count) count[a] = nd->count;
        if (sum) { sum[2 * a] = cs_get(&nd->sx); sum[2 * a + 1] = cs_get(&nd->sy); }
    }
    free(v);
    return ORC_OK;
}

/* cells of one level ascending by Morton prefix: prefix, count, sums */
int orc_tree_level(const void* h, int32_t level, uint32_t* prefix, int64_t* count, double* sum) {
    const otree* t = (const otree*)h;
    if (level < 0 || level > t->L || t->kind != 0) return ORC_EINVAL;
    int64_t m = 0;
    for (int64_t c = 0; c < t->nnodes; c++) if (t->nodes[c].level == level) m++;
    pref_t* v = (pref_t*)malloc(sizeof(pref_t) * (size_t)(m ? m : 1));
    if (!v) return ORC_ENOMEM;
    m = 0;
    for (int64_t c = 0; c < t->nnodes; c++)
        if (t->nodes[c].level == level) { v[m].prefix = t->nodes[c].prefix; v[m].id = c; m++; }
    qsort(v, (size_t)m, sizeof(pref_t), pref_cmp);
    for (int64_t a = 0; a < m; a++) {
        const onode* nd = &t->nodes[v[a].id];
        if (prefix) prefix[a] = nd->prefix;
        if (count) count[a] = nd->count;
        if (sum) { sum[2 * a] = cs_get(&nd->sx); sum[2 * a + 1] = cs_get(&nd->sy); }
    }
    free(v);
    return ORC_OK;
}

/* stable order of points by Morton key (ties by index) */
typedef struct { uint32_t key; int64_t i; } kp_t;
static int kp_cmp(const void* a, const void* b) {
    const kp_t* x = (const kp_t*)a; const kp_t* y = (const kp_t*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->i < y->i ? -1 : (x->i > y->i ? 1 : 0);
}

int orc_sorted_order(const double* z, int64_t n, int32_t r, uint32_t* key_sorted, int64_t* perm) {
    int L = log2_exact(r);
    if (L < 0) return ORC_EINVAL;
    kp_t* v = (kp_t*)malloc(sizeof(kp_t) * (size_t)n);
    if (!v) return ORC_ENOMEM;
    for (int64_t i = 0; i < n; i++) {
        v[i].key = morton2((uint32_t)pixel_of(z[2 * i], r), (uint32_t)pixel_of(z[2 * i + 1], r), L);
        v[i].i = i;
    }
    qsort(v, (size_t)n, sizeof(kp_t), kp_cmp);
    for (int64_t s = 0; s < n; s++) {
        if (key_sorted) key_sorted[s] = v[s].key;
        if (perm) perm[s] = v[s].i;
    }
    free(v);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Barnes-Hut repulsion on the P-Quadtree (Eq. 5 second term, Eq. 11,  */
/* Eq. 12).  For point i, depth-first from the root, children in order  */
/* 0..3.  At a cell with side w (pixels) and representative point c:    */
/*   dz = z_i - c,  d2 = beta1 dz1^2 + beta2 dz2^2   (Eq. 12 metric)    */
/*   diag2 = w^2 (beta1 + beta2)                      (cell diagonal^2)  */
/*   a leaf is always used; an inner cell is used iff                    */
/*   diag2 < theta^2 * d2  (diagonal / distance < theta), else recurse.  */
/* predicate 0 evaluates that test in FP64; predicate 1 in FP32: z_i, c, */
/* w, beta and theta^2 rounded to FP32, each axis scaled by             */
/* r_d = sqrt(beta_d) rounded to FP32, then                              */
/*   (w*w)*(b1+b2) < th2*(dx*dx + dy*dy),                                */
/*   dx = z_i1*r_1 - c_1*r_1,  dy = z_i2*r_2 - c_2*r_2,                  */
/* each operation rounded to FP32 in that order (no fused multiply-add;  */
/* the library's FP32 path takes the same decision).  The forces of a    */
/* used cell are FP64 either way.                                        */
/* A used cell adds m*w_ic to Z_i and m*w_ic^2*dz to R_i, w = 1/(1+d2).  */
/* m = N_c, except in the leaf holding i: m = N_c - 1 and c is the mean */
/* of the other points (the cell centre in CELL_CENTER mode); skipped   */
/* when m = 0.                                                          */
/* com_mode 0: centre of mass (Eq. 8); 1: geometric cell centre         */
/* (Section 4.1, which uses it in place of the centre of mass).        */
/* visits counts every cell reached by the traversal.                    */
/* ------------------------------------------------------------------ */
/* rows == NULL: every point, outputs indexed by point; otherwise outputs are
 * indexed by position in rows[0..nrows). */
int orc_repulsion_rows(const void* h, const double* z, const double* beta, double theta,
                       int32_t com_mode, int32_t predicate, const int64_t* rows, int64_t nrows,
                       double* R, double* Zi, int64_t* visits) {
    const otree* t = (const otree*)h;
    if (!t || !z || !beta || !(theta >= 0.0) || theta >= 1.0) return ORC_EINVAL;
    if (predicate != 0 && predicate != 1) return ORC_EINVAL;
    if (t->kind == 1 && com_mode == 1) return ORC_EINVAL;   /* D-Quadtree: centres of mass only */
    const int L = t->L;
    const double b1 = beta[0], b2 = beta[1], th2 = theta * theta;
    /* single-precision operands of the FP32 opening test */
    const float b1f = (float)b1, b2f = (float)b2, th2f = (float)th2, bsf = b1f + b2f;
    const float r1f = (float)sqrt(b1), r2f = (float)sqrt(b2);
    if (!rows) nrows = t->n;
    int64_t q;
#pragma omp parallel for schedule(dynamic, 64)
    for (q = 0; q < nrows; q++) {
        const int64_t i = rows ? rows[q] : q;
        const double zx = z[2 * i], zy = z[2 * i + 1];
        const int32_t own = t->leaf_of[i];
        double rx = 0.0, ry = 0.0, zsum = 0.0;
        int64_t nv = 0;
        int32_t stack[4 * 36];          /* 3 per level below the root, 33 levels at most */
        int sp = 0;
        stack[sp++] = 0;
        while (sp > 0) {
            const int32_t c = stack[--sp];
            const onode* nd = &t->nodes[c];
            nv++;
            const double w = ldexp(1.0, L - nd->level);   /* side in pixels */
            double m = (double)nd->count, cx, cy;
            if (com_mode == 1) {
                uint32_t x0 = 0, y0 = 0;
                for (int b = 0; b < nd->level; b++) {
                    x0 |= ((nd->prefix >> (2 * b)) & 1u) << b;
                    y0 |= ((nd->prefix >> (2 * b + 1)) & 1u) << b;
                }
                cx = (double)x0 * w + 0.5 * w;
                cy = (double)y0 * w + 0.5 * w;
            } else {
                cx = cs_get(&nd->sx) / m;
                cy = cs_get(&nd->sy) / m;
            }
            int use;
            if (is_leaf(nd)) {
                use = 1;
                if (c == own) {
                    m -= 1.0;
                    if (m <= 0.0) continue;
                    if (com_mode != 1) {
                        cx = (cs_get(&nd->sx) - zx) / m;
                        cy = (cs_get(&nd->sy) - zy) / m;
                    }
                }
            } else if (predicate == 0) {
                double dx = zx - cx, dy = zy - cy;
                double d2 = b1 * dx * dx + b2 * dy * dy;
                double diag2 = w * w * (b1 + b2);
                use = diag2 < th2 * d2;
            } else {
                /* the same test in single precision: operands rounded to
                 * FP32, the axes scaled by sqrt(beta) in FP32, every
                 * operation rounded to FP32 in this order */
                float dxf = (float)zx * r1f - (float)cx * r1f;
                float dyf = (float)zy * r2f - (float)cy * r2f;
                float wf = (float)w;
                float d2f = dxf * dxf + dyf * dyf;
                float diag2f = (wf * wf) * bsf;
                use = diag2f < th2f * d2f;
            }
            if (use) {
                double dx = zx - cx, dy = zy - cy;
                double d2 = b1 * dx * dx + b2 * dy * dy;
                double qij = 1.0 / (1.0 + d2);
                zsum += m * qij;
                rx += m * qij * qij * dx;
                ry += m * qij * qij * dy;
            } else {
                for (int ch = 3; ch >= 0; ch--)
                    if (nd->child[ch] >= 0) stack[sp++] = nd->child[ch];
            }
        }
        R[2 * q] = rx; R[2 * q + 1] = ry;
        Zi[q] = zsum;
        if (visits) visits[q] = nv;
    }
    return ORC_OK;
}

int orc_repulsion(const void* h, const double* z, const double* beta, double theta,
                  int32_t com_mode, int32_t predicate, double* R, double* Zi, int64_t* visits) {
    return orc_repulsion_rows(h, z, beta, theta, com_mode, predicate, NULL, 0, R, Zi, visits);
}

/* Z = sum_i Z_i, compensated, in index order */
double orc_sum(const double* v, int64_t n) {
    csum a = {0, 0};
    for (int64_t i = 0; i < n; i++) cs_add(&a, v[i]);
    return cs_get(&a);
}

/* ------------------------------------------------------------------ */
/* Attraction (Eq. 5 first term over the sparse P of Section 3.3):      */
/* A_i = sum_{j in row i} p_ij w_ij (z_i - z_j), w from Eq. 12.         */
/* ------------------------------------------------------------------ */
int orc_attraction_rows(const double* z, int64_t n, const double* beta, const int64_t* row_ptr,
                        const int32_t* col, const double* val, const int64_t* rows,
                        int64_t nrows, double* A) {
    if (!z || !beta || !row_ptr || !col || !val || !A) return ORC_EINVAL;
    const double b1 = beta[0], b2 = beta[1];
    if (!rows) nrows = n;
    int64_t q;
#pragma omp parallel for schedule(static)
    for (q = 0; q < nrows; q++) {
        const int64_t i = rows ? rows[q] : q;
        double ax = 0.0, ay = 0.0;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; e++) {
            int32_t j = col[e];
            double dx = z[2 * i] - z[2 * (int64_t)j], dy = z[2 * i + 1] - z[2 * (int64_t)j + 1];
            double qij = 1.0 / (1.0 + b1 * dx * dx + b2 * dy * dy);
            ax += val[e] * qij * dx;
            ay += val[e] * qij * dy;
        }
        A[2 * q] = ax; A[2 * q + 1] = ay;
    }
    return ORC_OK;
}

int orc_attraction(const double* z, int64_t n, const double* beta, const int64_t* row_ptr,
                   const int32_t* col, const double* val, double* A) {
    return orc_attraction_rows(z, n, beta, row_ptr, col, val, NULL, 0, A);
}

/* ------------------------------------------------------------------ */
/* Screen-driven scaling (Section 4.2): per axis                        */
/*   gamma_d = max_i zh_d - min_i zh_d + eps,                            */
/*   z_d = r (zh_d - min_i zh_d) / gamma_d.                              */
/* Writes z, gamma[2], zmin[2].                                          */
/* ------------------------------------------------------------------ */
int orc_normalize(const double* zh, int64_t n, int32_t r, double eps, double* z,
                  double* gamma, double* zmin) {
    if (!zh || !z || n < 1) return ORC_EINVAL;
    for (int d = 0; d < 2; d++) {
        double lo = zh[d], hi = zh[d];
        for (int64_t i = 1; i < n; i++) {
            double v = zh[2 * i + d];
            if (v < lo) lo = v;
            if (v > hi) hi = v;
        }
        double g = hi - lo + eps;
        for (int64_t i = 0; i < n; i++) z[2 * i + d] = (double)r * (zh[2 * i + d] - lo) / g;
        if (gamma) gamma[d] = g;
        if (zmin) zmin[d] = lo;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Gradient in the pixel frame.  With y = s * z (per axis) and          */
/* beta_d = s_d^2, Eq. 5 becomes dC/dy_i,d = 4 s_d B_i,d with            */
/*   B_i = alpha * A_i - R_i / Z,                                        */
/* alpha the early-exaggeration factor on P.                            */
/* Outputs B (and optionally A, R, Z_i, visits, Z).                      */
/* ------------------------------------------------------------------ */
int orc_gradient(const double* z, int64_t n, int32_t r, const double* s, double theta,
                 int32_t com_mode, int32_t predicate, int32_t tree, double alpha,
                 const int64_t* row_ptr, const int32_t* col,
                 const double* val, double* B, double* A_out, double* R_out, double* Zi_out,
                 int64_t* visits, double* Z_out) {
    double beta[2] = {s[0] * s[0], s[1] * s[1]};
    void* h = tree == 1 ? orc_dtree_build(z, n, r) : orc_tree_build(z, n, r);
    if (!h) return ORC_ENOMEM;
    double* A = A_out ? A_out : (double*)malloc(sizeof(double) * 2 * (size_t)n);
    double* R = R_out ? R_out : (double*)malloc(sizeof(double) * 2 * (size_t)n);
    double* Zi = Zi_out ? Zi_out : (double*)malloc(sizeof(double) * (size_t)n);
    int rc = ORC_ENOMEM;
    if (A && R && Zi) {
        rc = orc_repulsion(h, z, beta, theta, com_mode, predicate, R, Zi, visits);
        if (rc == ORC_OK) rc = orc_attraction(z, n, beta, row_ptr, col, val, A);
        if (rc == ORC_OK) {
            double Z = orc_sum(Zi, n);
            if (Z_out) *Z_out = Z;
            for (int64_t i = 0; i < 2 * n; i++) B[i] = alpha * A[i] - R[i] / Z;
        }
    }
    if (!A_out) free(A);
    if (!R_out) free(R);
    if (!Zi_out) free(Zi);
    orc_tree_free(h);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Optimisation loop.  Per iteration t (0-based):                        */
/*   B from the current z (above);                                      */
/*   gains: g += 0.2 where sign(B) != sign(u), else g *= 0.8; g >= gmin; */
/*   u = mu_t u - eta g B;  zh = z + u;                                  */
/*   screen scaling of zh -> z, s *= gamma / r, u *= r / gamma.          */
/* The pixel-frame step equals a y-frame step on dC/dy / 4 because     */
/* y = s z and the gradient carries the factor s (Eq. 12-13).           */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t r;
    double theta;
    int32_t com_mode;
    double eta, mom0, mom1;
    int32_t mom_switch;
    double exaggeration;
    int32_t exag_iters;
    double min_gain, eps;
    int32_t predicate;   /* opening test: 0 FP64, 1 FP32 (see orc_repulsion_rows) */
    int32_t tree;        /* 0: P-Quadtree, 1: D-Quadtree (orc_dtree_build) */
} orc_params;

static inline double sgn(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

int orc_iterate(const orc_params* p, int64_t n, const int64_t* row_ptr, const int32_t* col,
                const double* val, double* z, double* u, double* g, double* s, int32_t t0,
                int32_t n_iter, double* Z_hist) {
    if (!p || !z || !u || !g || !s) return ORC_EINVAL;
    double* B = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    double* zh = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    if (!B || !zh) { free(B); free(zh); return ORC_ENOMEM; }
    int rc = ORC_OK;
    for (int32_t it = 0; it < n_iter; it++) {
        int32_t t = t0 + it;
        double alpha = t < p->exag_iters ? p->exaggeration : 1.0;
        double mu = t < p->mom_switch ? p->mom0 : p->mom1;
        double Z;
        rc = orc_gradient(z, n, p->r, s, p->theta, p->com_mode, p->predicate, p->tree, alpha,
                          row_ptr, col, val, B,
                          NULL, NULL, NULL, NULL, &Z);
        if (rc != ORC_OK) break;
        if (Z_hist) Z_hist[it] = Z;
        for (int64_t e = 0; e < 2 * n; e++) {
            double gn = (sgn(B[e]) != sgn(u[e])) ? g[e] + 0.2 : g[e] * 0.8;
            if (gn < p->min_gain) gn = p->min_gain;
            g[e] = gn;
            u[e] = mu * u[e] - p->eta * gn * B[e];
            zh[e] = z[e] + u[e];
        }
        double gamma[2], zmin[2];
        orc_normalize(zh, n, p->r, p->eps, z, gamma, zmin);
        for (int d = 0; d < 2; d++) {
            s[d] *= gamma[d] / (double)p->r;
            for (int64_t i = 0; i < n; i++) u[2 * i + d] *= (double)p->r / gamma[d];
        }
    }
    free(B); free(zh);
    return rc;
}

/* ------------------------------------------------------------------ */
/* KL objective (Eq. 4) with q from Eq. 12 and the exact normaliser:    */
/*   C = sum_nnz p ln p - sum_nnz p ln w_ij + ln Z,  Z = sum_{i!=j} w_ij */
/* over all ordered pairs (O(n^2)).  P must sum to 1.                    */
/* ------------------------------------------------------------------ */
double orc_kl(const double* z, int64_t n, const double* s, const int64_t* row_ptr,
              const int32_t* col, const double* val) {
    const double b1 = s[0] * s[0], b2 = s[1] * s[1];
    double* zrow = (double*)malloc(sizeof(double) * (size_t)n);
    if (!zrow) return NAN;
    int64_t i;
#pragma omp parallel for schedule(dynamic, 16)
    for (i = 0; i < n; i++) {
        csum a = {0, 0};
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            double dx = z[2 * i] - z[2 * j], dy = z[2 * i + 1] - z[2 * j + 1];
            cs_add(&a, 1.0 / (1.0 + b1 * dx * dx + b2 * dy * dy));
        }
        zrow[i] = cs_get(&a);
    }
    double Z = orc_sum(zrow, n);
    csum c = {0, 0};
    for (i = 0; i < n; i++)
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; e++) {
            int32_t j = col[e];
            double p = val[e];
            if (p <= 0.0) continue;
            double dx = z[2 * i] - z[2 * (int64_t)j], dy = z[2 * i + 1] - z[2 * (int64_t)j + 1];
            double w = 1.0 / (1.0 + b1 * dx * dx + b2 * dy * dy);
            cs_add(&c, p * log(p) - p * log(w));
        }
    free(zrow);
    return cs_get(&c) + log(Z);
}

/* ================================================================== */
/* The 3-D case (Section 1, footnote: the approach extends to 3-D      */
/* embeddings).  The screen becomes a cube of r^3 voxels, the          */
/* P-Quadtree an octree of fixed depth L = log2 r (L <= 10) with unit- */
/* voxel leaves, the Morton key interleaves x, y, z in bits 3b, 3b+1,  */
/* 3b+2 (child index 4 zbit + 2 ybit + xbit), and every per-axis step  */
/* (scaling, beta, the metric of the opening test) runs over three     */
/* axes: diag^2 = w^2 (b1 + b2 + b3), d^2 = sum_d b_d dz_d^2.  The     */
/* opening test is FP64.  State arrays are [n][3].                     */
/* ================================================================== */
typedef struct {
    int32_t child[8];
    int32_t level;
    uint32_t prefix;
    int64_t count;
    csum s[3];
} onode3;

typedef struct {
    int32_t r, L;
    int64_t n, nnodes, cap;
    onode3* nodes;
    int32_t* leaf_of;
} otree3;

static int32_t tree3_new_node(otree3* t, int32_t level, uint32_t prefix) {
    if (t->nnodes == t->cap) {
        int64_t nc = t->cap ? 2 * t->cap : 1024;
        onode3* p = (onode3*)realloc(t->nodes, sizeof(onode3) * (size_t)nc);
        if (!p) return -1;
        t->nodes = p; t->cap = nc;
    }
    onode3* c = &t->nodes[t->nnodes];
    memset(c, 0, sizeof(*c));
    for (int q = 0; q < 8; q++) c->child[q] = -1;
    c->level = level; c->prefix = prefix;
    return (int32_t)t->nnodes++;
}

void orc_tree3_free(void* h) {
    otree3* t = (otree3*)h;
    if (!t) return;
    free(t->nodes); free(t->leaf_of); free(t);
}

static inline uint32_t morton3(uint32_t px, uint32_t py, uint32_t pz, int L) {
    uint32_t key = 0;
    for (int b = 0; b < L; b++) {
        key |= ((px >> b) & 1u) << (3 * b);
        key |= ((py >> b) & 1u) << (3 * b + 1);
        key |= ((pz >> b) & 1u) << (3 * b + 2);
    }
    return key;
}

/* each point, in index order, from the root down to its voxel */
void* orc_tree3_build(const double* z, int64_t n, int32_t r) {
    int L = log2_exact(r);
    if (!z || n < 1 || L < 0 || L > 10) return NULL;
    otree3* t = (otree3*)calloc(1, sizeof(otree3));
    if (!t) return NULL;
    t->r = r; t->L = L; t->n = n;
    t->leaf_of = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!t->leaf_of || tree3_new_node(t, 0, 0) != 0) { orc_tree3_free(t); return NULL; }
    for (int64_t i = 0; i < n; i++) {
        uint32_t p[3];
        for (int d = 0; d < 3; d++) p[d] = (uint32_t)pixel_of(z[3 * i + d], r);
        int32_t c = 0;
        for (int l = 0;; l++) {
            onode3* nd = &t->nodes[c];
            nd->count++;
            for (int d = 0; d < 3; d++) cs_add(&nd->s[d], z[3 * i + d]);
            if (l == L) break;
            int sh = L - 1 - l;
            int q = (int)(((p[2] >> sh) & 1u) << 2 | ((p[1] >> sh) & 1u) << 1 | ((p[0] >> sh) & 1u));
            int32_t ch = nd->child[q];
            if (ch < 0) {
                uint32_t pre = (nd->prefix << 3) | (uint32_t)q;
                ch = tree3_new_node(t, l + 1, pre);
                if (ch < 0) { orc_tree3_free(t); return NULL; }
                t->nodes[c].child[q] = ch;
            }
            c = ch;
        }
        t->leaf_of[i] = c;
    }
    return t;
}

int orc_tree3_level_sizes(const void* h, int64_t* sizes) {
    const otree3* t = (const otree3*)h;
    for (int l = 0; l <= t->L; l++) sizes[l] = 0;
    for (int64_t c = 0; c < t->nnodes; c++) sizes[t->nodes[c].level]++;
    return ORC_OK;
}

int orc_tree3_level(const void* h, int32_t level, uint32_t* prefix, int64_t* count, double* sum) {
    const otree3* t = (const otree3*)h;
    if (level < 0 || level > t->L) return ORC_EINVAL;
    int64_t m = 0;
    for (int64_t c = 0; c < t->nnodes; c++) if (t->nodes[c].level == level) m++;
    pref_t* v = (pref_t*)malloc(sizeof(pref_t) * (size_t)(m ? m : 1));
    if (!v) return ORC_ENOMEM;
    m = 0;
    for (int64_t c = 0; c < t->nnodes; c++)
        if (t->nodes[c].level == level) { v[m].prefix = t->nodes[c].prefix; v[m].id = c; m++; }
    qsort(v, (size_t)m, sizeof(pref_t), pref_cmp);
    for (int64_t a = 0; a < m; a++) {
        const onode3* nd = &t->nodes[v[a].id];
        if (prefix) prefix[a] = nd->prefix;
        if (count) count[a] = nd->count;
        if (sum) for (int d = 0; d < 3; d++) sum[3 * a + d] = cs_get(&nd->s[d]);
    }
    free(v);
    return ORC_OK;
}

/* Barnes-Hut repulsion on the octree: as orc_repulsion_rows in three
 * dimensions (FP64 opening test, own-voxel exclusion, mass centres). */
int orc_repulsion3(const void* h, const double* z, const double* beta, double theta,
                   double* R, double* Zi, int64_t* visits) {
    const otree3* t = (const otree3*)h;
    if (!t || !z || !beta || !(theta >= 0.0) || theta >= 1.0) return ORC_EINVAL;
    const int L = t->L;
    const double th2 = theta * theta;
    const double bs = beta[0] + beta[1] + beta[2];
    int64_t i;
#pragma omp parallel for schedule(dynamic, 64)
    for (i = 0; i < t->n; i++) {
        const double* zi = z + 3 * i;
        const int32_t own = t->leaf_of[i];
        double r3[3] = {0.0, 0.0, 0.0}, zs = 0.0;
        int64_t nv = 0;
        int32_t stack[8 * 12];
        int sp = 0;
        stack[sp++] = 0;
        while (sp > 0) {
            const int32_t c = stack[--sp];
            const onode3* nd = &t->nodes[c];
            nv++;
            const double w = ldexp(1.0, L - nd->level);
            double m = (double)nd->count, cc[3];
            for (int d = 0; d < 3; d++) cc[d] = cs_get(&nd->s[d]) / m;
            int use;
            if (nd->level == L) {
                use = 1;
                if (c == own) {
                    m -= 1.0;
                    if (m <= 0.0) continue;
                    for (int d = 0; d < 3; d++) cc[d] = (cs_get(&nd->s[d]) - zi[d]) / m;
                }
            } else {
                double d2 = 0.0;
                for (int d = 0; d < 3; d++) { double e = zi[d] - cc[d]; d2 += beta[d] * e * e; }
                use = w * w * bs < th2 * d2;
            }
            if (use) {
                double e[3], d2 = 0.0;
                for (int d = 0; d < 3; d++) { e[d] = zi[d] - cc[d]; d2 += beta[d] * e[d] * e[d]; }
                double q = 1.0 / (1.0 + d2);
                zs += m * q;
                for (int d = 0; d < 3; d++) r3[d] += m * q * q * e[d];
            } else {
                for (int ch = 7; ch >= 0; ch--)
                    if (nd->child[ch] >= 0) stack[sp++] = nd->child[ch];
            }
        }
        for (int d = 0; d < 3; d++) R[3 * i + d] = r3[d];
        Zi[i] = zs;
        if (visits) visits[i] = nv;
    }
    return ORC_OK;
}

int orc_gradient3(const double* z, int64_t n, int32_t r, const double* s, double theta,
                  double alpha, const int64_t* row_ptr, const int32_t* col, const double* val,
                  double* B, double* A, double* R, double* Zi, int64_t* visits, double* Z_out) {
    const double beta[3] = {s[0] * s[0], s[1] * s[1], s[2] * s[2]};
    void* h = orc_tree3_build(z, n, r);
    if (!h) return ORC_ENOMEM;
    int rc = orc_repulsion3(h, z, beta, theta, R, Zi, visits);
    orc_tree3_free(h);
    if (rc != ORC_OK) return rc;
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; i++) {
        double a[3] = {0.0, 0.0, 0.0};
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; e++) {
            const int64_t j = col[e];
            double dz[3], d2 = 0.0;
            for (int d = 0; d < 3; d++) { dz[d] = z[3 * i + d] - z[3 * j + d]; d2 += beta[d] * dz[d] * dz[d]; }
            const double q = 1.0 / (1.0 + d2);
            for (int d = 0; d < 3; d++) a[d] += val[e] * q * dz[d];
        }
        for (int d = 0; d < 3; d++) A[3 * i + d] = a[d];
    }
    const double Z = orc_sum(Zi, n);
    if (Z_out) *Z_out = Z;
    for (int64_t e = 0; e < 3 * n; e++) B[e] = alpha * A[e] - R[e] / Z;
    return ORC_OK;
}

/* the optimisation loop of orc_iterate over three axes */
int orc_iterate3(const orc_params* p, int64_t n, const int64_t* row_ptr, const int32_t* col,
                 const double* val, double* z, double* u, double* g, double* s, int32_t t0,
                 int32_t n_iter) {
    if (!p || !z || !u || !g || !s) return ORC_EINVAL;
    double* B = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    double* A = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    double* R = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    double* Zi = (double*)malloc(sizeof(double) * (size_t)n);
    double* zh = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    int rc = (B && A && R && Zi && zh) ? ORC_OK : ORC_ENOMEM;
    for (int32_t it = 0; it < n_iter && rc == ORC_OK; it++) {
        const int32_t t = t0 + it;
        const double alpha = t < p->exag_iters ? p->exaggeration : 1.0;
        const double mu = t < p->mom_switch ? p->mom0 : p->mom1;
        double Z;
        rc = orc_gradient3(z, n, p->r, s, p->theta, alpha, row_ptr, col, val, B, A, R, Zi, NULL, &Z);
        if (rc != ORC_OK) break;
        for (int64_t e = 0; e < 3 * n; e++) {
            double gn = (sgn(B[e]) != sgn(u[e])) ? g[e] + 0.2 : g[e] * 0.8;
            if (gn < p->min_gain) gn = p->min_gain;
            g[e] = gn;
            u[e] = mu * u[e] - p->eta * gn * B[e];
            zh[e] = z[e] + u[e];
        }
        for (int d = 0; d < 3; d++) {
            double lo = zh[d], hi = zh[d];
            for (int64_t i = 1; i < n; i++) {
                const double v = zh[3 * i + d];
                if (v < lo) lo = v;
                if (v > hi) hi = v;
            }
            const double gam = hi - lo + p->eps;
            for (int64_t i = 0; i < n; i++) {
                z[3 * i + d] = (double)p->r * (zh[3 * i + d] - lo) / gam;
                u[3 * i + d] *= (double)p->r / gam;
            }
            s[d] *= gam / (double)p->r;
        }
    }
    free(B); free(A); free(R); free(Zi); free(zh);
    return rc;
}

/* normalisation of an initial 3-D embedding: z, gamma[3], zmin[3] */
int orc_normalize3(const double* zh, int64_t n, int32_t r, double eps, double* z, double* gamma,
                   double* zmin) {
    if (!zh || !z || n < 1) return ORC_EINVAL;
    for (int d = 0; d < 3; d++) {
        double lo = zh[d], hi = zh[d];
        for (int64_t i = 1; i < n; i++) {
            const double v = zh[3 * i + d];
            if (v < lo) lo = v;
            if (v > hi) hi = v;
        }
        const double gam = hi - lo + eps;
        for (int64_t i = 0; i < n; i++) z[3 * i + d] = (double)r * (zh[3 * i + d] - lo) / gam;
        if (gamma) gamma[d] = gam;
        if (zmin) zmin[d] = lo;
    }
    return ORC_OK;
}

/* KL (Eq. 4) of a 3-D embedding with the exact normaliser */
double orc_kl3(const double* z, int64_t n, const double* s, const int64_t* row_ptr,
               const int32_t* col, const double* val) {
    const double b[3] = {s[0] * s[0], s[1] * s[1], s[2] * s[2]};
    double* zrow = (double*)malloc(sizeof(double) * (size_t)n);
    if (!zrow) return NAN;
    int64_t i;
#pragma omp parallel for schedule(dynamic, 16)
    for (i = 0; i < n; i++) {
        csum a = {0, 0};
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            double d2 = 0.0;
            for (int d = 0; d < 3; d++) { double e = z[3 * i + d] - z[3 * j + d]; d2 += b[d] * e * e; }
            cs_add(&a, 1.0 / (1.0 + d2));
        }
        zrow[i] = cs_get(&a);
    }
    double Z = orc_sum(zrow, n);
    csum c = {0, 0};
    for (i = 0; i < n; i++)
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; e++) {
            const int64_t j = col[e];
            const double p = val[e];
            if (p <= 0.0) continue;
            double d2 = 0.0;
            for (int d = 0; d < 3; d++) { double ee = z[3 * i + d] - z[3 * j + d]; d2 += b[d] * ee * ee; }
            cs_add(&c, p * log(p) + p * log(1.0 + d2));
        }
    free(zrow);
    return cs_get(&c) + log(Z);
}
