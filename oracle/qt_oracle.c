/*
 * CPU oracle for the quadtree block-sparse matrix multiply C = A*B.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark build, load or call this file. The GPU
 * library never links or calls it, and the two share no code.
 *
 * It follows Rubensson & Rudberg (arXiv:1501.07800) as plainly as possible:
 *
 *   - Matrix representation (Sec. 3.1, "Matrix" chunk type): a quadtree whose
 *     internal nodes hold four children; a zero submatrix is a NIL child at
 *     any level; every level halves the dimension of the level above, so the
 *     padded side is leaf * 2^L; nodes carry no global offsets.
 *   - Leaf type (Sec. 4.1): a block-sparse leaf, a two-dimensional lb x lb
 *     table of b x b blocks in which only nonzero blocks are allocated.
 *   - Multiply (Sec. 3, Algorithm 1): if either operand is NIL the product is
 *     NIL; at the leaf level the leaf multiply runs; otherwise
 *     C_mn = add(mul(A_m1, B_1n), mul(A_m2, B_2n)) for m, n in {1, 2} and the
 *     four results are assembled into one node (createFromIds, Sec. 3.2).
 *   - Add (Sec. 3, Algorithm 2): both present -> recurse (or leaf add);
 *     otherwise the one that is present, or NIL. Also exported on its own
 *     (qo_add) for the standalone C = A + B.
 *   - Leaf multiply (Sec. 4.1, Fig. 2): every product A(i,k) B(k,j) of two
 *     present blocks is added into block (i,j) of the result; here as plain
 *     triple loops, k ascending, each block product summed over t ascending
 *     in a local fp64 variable and then added into the result block.
 *
 * Readings where the paper is silent:
 *   - A leaf product with no block products, and a node whose four children
 *     are all NIL, are NIL (zero submatrices are never stored, Sec. 3.1).
 *   - Only structural sparsity is detected: a result block stays present
 *     even if its values cancel to zero.
 *   - Inside a block, entries are stored row-major.
 *   - A repeated (I, J) in the input is an error, not a sum.
 *
 * Compile: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no FMA
 * contraction, so every product and sum rounds separately).
 *
 * Counters kept for the analysis of Sec. 5: multiply tasks with both operands
 * present, per level (the C_l of Eq. 1-3), add tasks with both operands
 * present, per level, and the number of leaf block products.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define QO_OK 0
#define QO_ERR_ARG 1
#define QO_ERR_SHAPE 2
#define QO_ERR_DUPLICATE 3
#define QO_ERR_OOM 4

#define QO_MAX_LEVELS 48

typedef struct qo_node qo_node;
struct qo_node {
    int is_leaf;
    qo_node *child[4];   /* internal: quadrant (m, n) at index 2*m + n; NULL is NIL */
    double **blk;        /* leaf: lb*lb blocks, row-major (i*lb + j); NULL = zero block */
    double n2;           /* input trees: squared Frobenius norm of the submatrix */
    double *bn2;         /* input leaves: squared Frobenius norm of every block (lb*lb) */
};

typedef struct {
    int b;               /* block size */
    int lb;              /* blocks per leaf side */
    int L;               /* leaf level (root is level 0) */
    int use_abs;         /* multiply |A| by |B| (for error bounds) */
    double tau2;         /* norm threshold squared: drop what has ||A|| ||B|| < tau (0: none) */
    int par_levels;      /* spawn OpenMP tasks above this depth */
    int64_t mul_tasks[QO_MAX_LEVELS];
    int64_t add_tasks[QO_MAX_LEVELS];
    int64_t block_products;
    int64_t leaf_block_adds;
    int64_t pruned_tasks[QO_MAX_LEVELS];   /* multiply tasks dropped by the norm threshold */
    int64_t pruned_products;               /* block products dropped by it */
} qo_ctx;

typedef struct {
    int64_t nnz;
    int32_t *I, *J;
    double *V;
    int b, lb, L;
    int64_t mul_tasks[QO_MAX_LEVELS];
    int64_t add_tasks[QO_MAX_LEVELS];
    int64_t block_products;
    int64_t leaf_block_adds;
    int64_t nodes_per_level[QO_MAX_LEVELS];   /* non-NIL nodes of C per level */
    int64_t pruned_tasks[QO_MAX_LEVELS];
    int64_t pruned_products;
} qo_result;

/* ------------------------------------------------------------------ trees */

static qo_node *node_new(int is_leaf, int lb) {
    qo_node *n = (qo_node *)calloc(1, sizeof(qo_node));
    if (!n) return NULL;
    n->is_leaf = is_leaf;
    if (is_leaf) {
        n->blk = (double **)calloc((size_t)lb * lb, sizeof(double *));
        if (!n->blk) { free(n); return NULL; }
    }
    return n;
}

/* Squared Frobenius norm of a b x b block: the squares of its entries summed
 * in row-major order. */
static double block_norm2(const double *x, int b) {
    double s = 0.0;
    for (int e = 0; e < b * b; ++e) s += x[e] * x[e];
    return s;
}

/* Free a tree. Input trees point into caller memory (own_blocks = 0). */
static void tree_free(qo_node *n, int lb, int own_blocks) {
    if (!n) return;
    if (n->is_leaf) {
        if (own_blocks)
            for (int q = 0; q < lb * lb; ++q) free(n->blk[q]);
        free(n->blk);
        free(n->bn2);
    } else {
        for (int c = 0; c < 4; ++c) tree_free(n->child[c], lb, own_blocks);
    }
    free(n);
}

/*
 * Build the subtree covering block rows [r0, r0+side) and columns
 * [c0, c0+side) from the blocks listed in idx[0..cnt). An empty range is NIL.
 */
static qo_node *tree_build(const int32_t *I, const int32_t *J, const double *V,
                           int b, int lb, int64_t *idx, int64_t cnt,
                           int64_t r0, int64_t c0, int64_t side, int *err) {
    if (cnt == 0) return NULL;
    if (side == lb) {
        qo_node *n = node_new(1, lb);
        if (!n) { *err = QO_ERR_OOM; return NULL; }
        n->bn2 = (double *)calloc((size_t)lb * lb, sizeof(double));
        if (!n->bn2) { tree_free(n, lb, 0); *err = QO_ERR_OOM; return NULL; }
        for (int64_t t = 0; t < cnt; ++t) {
            int64_t i = I[idx[t]] - r0, j = J[idx[t]] - c0;
            n->blk[i * lb + j] = (double *)(V + (size_t)idx[t] * b * b);
        }
        /* norms: every block's, and the leaf's as their sum (row-major block order) */
        for (int q = 0; q < lb * lb; ++q)
            if (n->blk[q]) {
                n->bn2[q] = block_norm2(n->blk[q], b);
                n->n2 += n->bn2[q];
            }
        return n;
    }
    int64_t half = side / 2;
    int64_t *part = (int64_t *)malloc((size_t)cnt * sizeof(int64_t));
    if (!part) { *err = QO_ERR_OOM; return NULL; }
    int64_t fill = 0;
    int64_t begin[4];
    for (int q = 0; q < 4; ++q) {
        begin[q] = fill;
        for (int64_t t = 0; t < cnt; ++t) {
            int m = (I[idx[t]] - r0) >= half;
            int nn = (J[idx[t]] - c0) >= half;
            if (2 * m + nn == q) part[fill++] = idx[t];
        }
    }
    qo_node *n = node_new(0, lb);
    if (!n) { free(part); *err = QO_ERR_OOM; return NULL; }
    int any = 0;
    for (int q = 0; q < 4; ++q) {
        int64_t e = (q < 3) ? begin[q + 1] : fill;
        int m = q >> 1, nn = q & 1;
        n->child[q] = tree_build(I, J, V, b, lb, part + begin[q], e - begin[q],
                                 r0 + m * half, c0 + nn * half, half, err);
        if (*err) break;
        any |= (n->child[q] != NULL);
    }
    free(part);
    if (*err || !any) { tree_free(n, lb, 0); return NULL; }
    for (int q = 0; q < 4; ++q)   /* a node's squared norm: the sum of its children's */
        if (n->child[q]) n->n2 += n->child[q]->n2;
    return n;
}

/* -------------------------------------------------------------- leaf ops */

/* X += A_blk * B_blk for b x b row-major blocks; each entry of the block
 * product is summed over t ascending in a local variable first. */
static void block_mul_add(double *X, const double *A, const double *B, int b, int use_abs) {
    for (int r = 0; r < b; ++r)
        for (int c = 0; c < b; ++c) {
            double s = 0.0;
            for (int t = 0; t < b; ++t) {
                double a = A[r * b + t], x = B[t * b + c];
                if (use_abs) { a = fabs(a); x = fabs(x); }
                s += a * x;
            }
            X[r * b + c] += s;
        }
}

static qo_node *leaf_multiply(qo_ctx *ctx, const qo_node *A, const qo_node *B, int *err) {
    int lb = ctx->lb, b = ctx->b;
    qo_node *X = node_new(1, lb);
    if (!X) { *err = QO_ERR_OOM; return NULL; }
    int64_t prods = 0, pruned = 0;
    int any = 0;
    for (int i = 0; i < lb; ++i)
        for (int j = 0; j < lb; ++j)
            for (int k = 0; k < lb; ++k) {
                const double *a = A->blk[i * lb + k], *x = B->blk[k * lb + j];
                if (!a || !x) continue;
                /* a block product of negligible norm is dropped (with tau = 0, none) */
                if (A->bn2[i * lb + k] * B->bn2[k * lb + j] < ctx->tau2) { ++pruned; continue; }
                double **dst = &X->blk[i * lb + j];
                if (!*dst) {
                    *dst = (double *)calloc((size_t)b * b, sizeof(double));
                    if (!*dst) { *err = QO_ERR_OOM; tree_free(X, lb, 1); return NULL; }
                }
                block_mul_add(*dst, a, x, b, ctx->use_abs);
                ++prods;
                any = 1;
            }
#pragma omp atomic
    ctx->block_products += prods;
#pragma omp atomic
    ctx->pruned_products += pruned;
    if (!any) { tree_free(X, lb, 1); return NULL; }
    return X;
}

/* X = X + Y for leaves; X and Y are temporaries: Y's storage is consumed. */
static void leaf_add_into(qo_ctx *ctx, qo_node *X, qo_node *Y) {
    int lb = ctx->lb, bb = ctx->b * ctx->b;
    int64_t adds = 0;
    for (int q = 0; q < lb * lb; ++q) {
        if (!Y->blk[q]) continue;
        if (!X->blk[q]) {
            X->blk[q] = Y->blk[q];
        } else {
            for (int e = 0; e < bb; ++e) X->blk[q][e] += Y->blk[q][e];
            free(Y->blk[q]);
            ++adds;
        }
        Y->blk[q] = NULL;
    }
#pragma omp atomic
    ctx->leaf_block_adds += adds;
    tree_free(Y, lb, 1);
}

/* ------------------------------------------------------ Algorithm 2: add */

/* C = X + Y where X and Y are temporaries owned by the caller (consumed). */
static qo_node *qt_add(qo_ctx *ctx, int level, qo_node *X, qo_node *Y) {
    if (X && Y) {
#pragma omp atomic
        ctx->add_tasks[level] += 1;
        if (level == ctx->L) {
            leaf_add_into(ctx, X, Y);
            return X;
        }
        for (int q = 0; q < 4; ++q) {
            X->child[q] = qt_add(ctx, level + 1, X->child[q], Y->child[q]);
            Y->child[q] = NULL;
        }
        free(Y);
        return X;   /* a sum of two non-NIL nodes keeps at least one child */
    }
    if (X) return X;
    if (Y) return Y;
    return NULL;
}

/* ------------------------------------------------- Algorithm 1: multiply */

static qo_node *qt_mul(qo_ctx *ctx, int level, const qo_node *A, const qo_node *B, int *err) {
    if (!A || !B) return NULL;                       /* fallback: NIL */
    /* a product of negligible norm is NIL as well: every block product below
     * has a norm product at most this one (with tau = 0, nothing is dropped) */
    if (A->n2 * B->n2 < ctx->tau2) {
#pragma omp atomic
        ctx->pruned_tasks[level] += 1;
        return NULL;
    }
#pragma omp atomic
    ctx->mul_tasks[level] += 1;
    if (level == ctx->L) return leaf_multiply(ctx, A, B, err);

    qo_node *Y[4][2];
    int spawn = level < ctx->par_levels;
    for (int m = 0; m < 2; ++m)
        for (int n = 0; n < 2; ++n)
            for (int k = 0; k < 2; ++k) {
                const qo_node *a = A->child[2 * m + k];
                const qo_node *x = B->child[2 * k + n];
                qo_node **dst = &Y[2 * m + n][k];
                int *e = err;
                if (spawn) {
#pragma omp task firstprivate(a, x, dst, e) shared(ctx)
                    *dst = qt_mul(ctx, level + 1, a, x, e);
                } else {
                    *dst = qt_mul(ctx, level + 1, a, x, e);
                }
            }
    if (spawn) {
#pragma omp taskwait
    }
    qo_node *C = node_new(0, ctx->lb);
    if (!C) *err = QO_ERR_OOM;
    int any = 0;
    for (int q = 0; q < 4; ++q) {
        qo_node *s = qt_add(ctx, level + 1, Y[q][0], Y[q][1]);
        if (C) C->child[q] = s; else tree_free(s, ctx->lb, 1);
        any |= (s != NULL);
    }
    if (!C) return NULL;
    if (!any) { free(C); return NULL; }              /* createFromIds of four NILs */
    return C;
}

/* ------------------------------------------------------------ emitting */

typedef struct { int32_t I, J; double *p; } qo_entry;

typedef struct { qo_entry *e; int64_t n, cap; int err; } qo_list;

static void list_push(qo_list *l, int32_t I, int32_t J, double *p) {
    if (l->n == l->cap) {
        int64_t cap = l->cap ? 2 * l->cap : 1024;
        qo_entry *e = (qo_entry *)realloc(l->e, (size_t)cap * sizeof(qo_entry));
        if (!e) { l->err = QO_ERR_OOM; return; }
        l->e = e; l->cap = cap;
    }
    l->e[l->n].I = I; l->e[l->n].J = J; l->e[l->n].p = p; l->n++;
}

static void collect(const qo_node *n, int level, int L, int lb, int64_t r0, int64_t c0,
                    int64_t side, qo_list *out, int64_t *nodes_per_level) {
    if (!n) return;
    nodes_per_level[level] += 1;
    if (n->is_leaf) {
        for (int i = 0; i < lb; ++i)
            for (int j = 0; j < lb; ++j)
                if (n->blk[i * lb + j])
                    list_push(out, (int32_t)(r0 + i), (int32_t)(c0 + j), n->blk[i * lb + j]);
        return;
    }
    int64_t half = side / 2;
    for (int q = 0; q < 4; ++q)
        collect(n->child[q], level + 1, L, lb, r0 + (q >> 1) * half, c0 + (q & 1) * half,
                half, out, nodes_per_level);
}

static int cmp_entry(const void *x, const void *y) {
    const qo_entry *a = (const qo_entry *)x, *b = (const qo_entry *)y;
    if (a->I != b->I) return a->I < b->I ? -1 : 1;
    if (a->J != b->J) return a->J < b->J ? -1 : 1;
    return 0;
}

static int cmp_pos(const void *x, const void *y) {
    int64_t a = *(const int64_t *)x, b = *(const int64_t *)y;
    return (a > b) - (a < b);
}

/* ------------------------------------------------------------ interface */

/* Check one operand's block list: range and duplicates. */
static int validate(int64_t nbr, int64_t nbc, int64_t nnz, const int32_t *I, const int32_t *J) {
    if (nnz < 0 || (nnz > 0 && (!I || !J))) return QO_ERR_ARG;
    for (int64_t t = 0; t < nnz; ++t)
        if (I[t] < 0 || I[t] >= nbr || J[t] < 0 || J[t] >= nbc) return QO_ERR_ARG;
    if (nnz < 2) return QO_OK;
    int64_t *pos = (int64_t *)malloc((size_t)nnz * sizeof(int64_t));
    if (!pos) return QO_ERR_OOM;
    for (int64_t t = 0; t < nnz; ++t) pos[t] = (int64_t)I[t] * nbc + J[t];
    qsort(pos, (size_t)nnz, sizeof(int64_t), cmp_pos);
    int rc = QO_OK;
    for (int64_t t = 1; t < nnz; ++t)
        if (pos[t] == pos[t - 1]) { rc = QO_ERR_DUPLICATE; break; }
    free(pos);
    return rc;
}

static int is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

/*
 * C = A * B (or |A| * |B| when use_abs != 0).
 * Dimensions are scalar; b is the block size, leaf the leaf dimension
 * (a power-of-two multiple of b). On success *out holds the result.
 *
 * tau > 0 makes it the norm-thresholded product the paper's conclusions
 * point to (storing each submatrix's Frobenius norm in the quadtree, after
 * Bock and Challacombe): every node of the input trees carries its squared
 * Frobenius norm, a multiply task whose operands have ||A|| ||B|| < tau is
 * NIL, and at the leaves every block product with ||A(i,k)|| ||B(k,j)|| < tau
 * is left out (compared as squares). A node's norm bounds the norm of every
 * block below it, so the task rule never drops a block product the block
 * rule would keep: C(I,J) is the sum over the K with ||A(I,K)|| ||B(K,J)|| >=
 * tau, present iff one such K exists. tau = 0 is the exact product.
 */
int qo_multiply(int64_t a_rows, int64_t a_cols, int64_t a_nnz,
                const int32_t *Ia, const int32_t *Ja, const double *Va,
                int64_t b_rows, int64_t b_cols, int64_t b_nnz,
                const int32_t *Ib, const int32_t *Jb, const double *Vb,
                int b, int leaf, int use_abs, double tau, int par_levels, qo_result **out) {
    *out = NULL;
    if (b <= 0 || leaf <= 0 || a_rows < 0 || a_cols < 0 || b_rows < 0 || b_cols < 0)
        return QO_ERR_ARG;
    if (a_rows % b || a_cols % b || b_rows % b || b_cols % b || leaf % b) return QO_ERR_SHAPE;
    if (!is_pow2(leaf / b)) return QO_ERR_SHAPE;
    if (a_cols != b_rows) return QO_ERR_SHAPE;
    int lb = leaf / b;
    int64_t nbr_a = a_rows / b, nbc_a = a_cols / b, nbr_b = b_rows / b, nbc_b = b_cols / b;
    int rc = validate(nbr_a, nbc_a, a_nnz, Ia, Ja);
    if (rc) return rc;
    rc = validate(nbr_b, nbc_b, b_nnz, Ib, Jb);
    if (rc) return rc;

    /* common padded side: lb * 2^L blocks covering every dimension */
    int64_t need = nbr_a;
    if (nbc_a > need) need = nbc_a;
    if (nbc_b > need) need = nbc_b;
    int L = 0;
    int64_t side = lb;
    while (side < need) { side *= 2; ++L; }
    if (L + 1 >= QO_MAX_LEVELS) return QO_ERR_SHAPE;

    qo_result *res = (qo_result *)calloc(1, sizeof(qo_result));
    if (!res) return QO_ERR_OOM;
    res->b = b; res->lb = lb; res->L = L;

    int err = QO_OK;
    int64_t *ia = (int64_t *)malloc((size_t)(a_nnz + 1) * sizeof(int64_t));
    int64_t *ib = (int64_t *)malloc((size_t)(b_nnz + 1) * sizeof(int64_t));
    if (!ia || !ib) { free(ia); free(ib); free(res); return QO_ERR_OOM; }
    for (int64_t t = 0; t < a_nnz; ++t) ia[t] = t;
    for (int64_t t = 0; t < b_nnz; ++t) ib[t] = t;
    qo_node *A = tree_build(Ia, Ja, Va, b, lb, ia, a_nnz, 0, 0, side, &err);
    qo_node *B = err ? NULL : tree_build(Ib, Jb, Vb, b, lb, ib, b_nnz, 0, 0, side, &err);
    free(ia); free(ib);
    if (err) { tree_free(A, lb, 0); tree_free(B, lb, 0); free(res); return err; }

    qo_ctx ctx;
    memset(&ctx, 0, sizeof(ctx));
    if (!(tau >= 0.0)) { tree_free(A, lb, 0); tree_free(B, lb, 0); free(res); return QO_ERR_ARG; }
    ctx.b = b; ctx.lb = lb; ctx.L = L; ctx.use_abs = use_abs; ctx.par_levels = par_levels;
    ctx.tau2 = tau * tau;
    qo_node *C = NULL;
#pragma omp parallel
#pragma omp single
    C = qt_mul(&ctx, 0, A, B, &err);
    tree_free(A, lb, 0);
    tree_free(B, lb, 0);
    if (err) { tree_free(C, lb, 1); free(res); return err; }

    qo_list lst = {0};
    collect(C, 0, L, lb, 0, 0, side, &lst, res->nodes_per_level);
    if (lst.err) { free(lst.e); tree_free(C, lb, 1); free(res); return lst.err; }
    qsort(lst.e, (size_t)lst.n, sizeof(qo_entry), cmp_entry);
    res->nnz = lst.n;
    res->I = (int32_t *)malloc((size_t)(lst.n + 1) * sizeof(int32_t));
    res->J = (int32_t *)malloc((size_t)(lst.n + 1) * sizeof(int32_t));
    res->V = (double *)malloc((size_t)(lst.n + 1) * b * b * sizeof(double));
    if (!res->I || !res->J || !res->V) {
        free(res->I); free(res->J); free(res->V); free(lst.e); tree_free(C, lb, 1); free(res);
        return QO_ERR_OOM;
    }
    for (int64_t t = 0; t < lst.n; ++t) {
        res->I[t] = lst.e[t].I;
        res->J[t] = lst.e[t].J;
        memcpy(res->V + (size_t)t * b * b, lst.e[t].p, (size_t)b * b * sizeof(double));
    }
    free(lst.e);
    tree_free(C, lb, 1);
    memcpy(res->mul_tasks, ctx.mul_tasks, sizeof(ctx.mul_tasks));
    memcpy(res->add_tasks, ctx.add_tasks, sizeof(ctx.add_tasks));
    memcpy(res->pruned_tasks, ctx.pruned_tasks, sizeof(ctx.pruned_tasks));
    res->block_products = ctx.block_products;
    res->leaf_block_adds = ctx.leaf_block_adds;
    res->pruned_products = ctx.pruned_products;
    *out = res;
    return QO_OK;
}

/* Deep copy of an input tree into owned blocks (Algorithm 2 consumes its
 * operands, which are temporaries of Algorithm 1 in the multiply). */
static qo_node *tree_clone(const qo_node *n, int lb, int b, int *err) {
    if (!n) return NULL;
    qo_node *c = node_new(n->is_leaf, lb);
    if (!c) { *err = QO_ERR_OOM; return NULL; }
    if (n->is_leaf) {
        for (int q = 0; q < lb * lb; ++q) {
            if (!n->blk[q]) continue;
            c->blk[q] = (double *)malloc((size_t)b * b * sizeof(double));
            if (!c->blk[q]) { *err = QO_ERR_OOM; tree_free(c, lb, 1); return NULL; }
            memcpy(c->blk[q], n->blk[q], (size_t)b * b * sizeof(double));
        }
    } else {
        for (int q = 0; q < 4; ++q) {
            c->child[q] = tree_clone(n->child[q], lb, b, err);
            if (*err) { tree_free(c, lb, 1); return NULL; }
        }
    }
    return c;
}

/* C = A + B by Algorithm 2 (both operands rows x cols, same b and leaf). */
int qo_add(int64_t rows, int64_t cols, int64_t a_nnz, const int32_t *Ia, const int32_t *Ja, const double *Va,
           int64_t b_nnz, const int32_t *Ib, const int32_t *Jb, const double *Vb, int b, int leaf,
           qo_result **out) {
    *out = NULL;
    if (b <= 0 || leaf <= 0 || rows < 0 || cols < 0) return QO_ERR_ARG;
    if (rows % b || cols % b || leaf % b || !is_pow2(leaf / b)) return QO_ERR_SHAPE;
    int lb = leaf / b;
    int64_t nbr = rows / b, nbc = cols / b;
    int rc = validate(nbr, nbc, a_nnz, Ia, Ja);
    if (rc) return rc;
    rc = validate(nbr, nbc, b_nnz, Ib, Jb);
    if (rc) return rc;
    int64_t need = nbr > nbc ? nbr : nbc, side = lb;
    int L = 0;
    while (side < need) { side *= 2; ++L; }
    if (L + 1 >= QO_MAX_LEVELS) return QO_ERR_SHAPE;
    qo_result *res = (qo_result *)calloc(1, sizeof(qo_result));
    if (!res) return QO_ERR_OOM;
    res->b = b; res->lb = lb; res->L = L;
    int err = QO_OK;
    int64_t *ia = (int64_t *)malloc((size_t)(a_nnz + 1) * sizeof(int64_t));
    int64_t *ib = (int64_t *)malloc((size_t)(b_nnz + 1) * sizeof(int64_t));
    if (!ia || !ib) { free(ia); free(ib); free(res); return QO_ERR_OOM; }
    for (int64_t t = 0; t < a_nnz; ++t) ia[t] = t;
    for (int64_t t = 0; t < b_nnz; ++t) ib[t] = t;
    qo_node *A = tree_build(Ia, Ja, Va, b, lb, ia, a_nnz, 0, 0, side, &err);
    qo_node *B = err ? NULL : tree_build(Ib, Jb, Vb, b, lb, ib, b_nnz, 0, 0, side, &err);
    free(ia); free(ib);
    qo_node *X = err ? NULL : tree_clone(A, lb, b, &err);
    qo_node *Y = err ? NULL : tree_clone(B, lb, b, &err);
    tree_free(A, lb, 0);
    tree_free(B, lb, 0);
    if (err) { tree_free(X, lb, 1); tree_free(Y, lb, 1); free(res); return err; }
    qo_ctx ctx;
    memset(&ctx, 0, sizeof(ctx));
    ctx.b = b; ctx.lb = lb; ctx.L = L;
    qo_node *C = qt_add(&ctx, 0, X, Y);
    qo_list lst = {0};
    collect(C, 0, L, lb, 0, 0, side, &lst, res->nodes_per_level);
    if (lst.err) { free(lst.e); tree_free(C, lb, 1); free(res); return lst.err; }
    qsort(lst.e, (size_t)lst.n, sizeof(qo_entry), cmp_entry);
    res->nnz = lst.n;
    res->I = (int32_t *)malloc((size_t)(lst.n + 1) * sizeof(int32_t));
    res->J = (int32_t *)malloc((size_t)(lst.n + 1) * sizeof(int32_t));
    res->V = (double *)malloc((size_t)(lst.n + 1) * b * b * sizeof(double));
    if (!res->I || !res->J || !res->V) {
        free(res->I); free(res->J); free(res->V); free(lst.e); tree_free(C, lb, 1); free(res);
        return QO_ERR_OOM;
    }
    for (int64_t t = 0; t < lst.n; ++t) {
        res->I[t] = lst.e[t].I;
        res->J[t] = lst.e[t].J;
        memcpy(res->V + (size_t)t * b * b, lst.e[t].p, (size_t)b * b * sizeof(double));
    }
    free(lst.e);
    tree_free(C, lb, 1);
    memcpy(res->add_tasks, ctx.add_tasks, sizeof(ctx.add_tasks));
    res->leaf_block_adds = ctx.leaf_block_adds;
    *out = res;
    return QO_OK;
}

int64_t qo_result_nnz(const qo_result *r) { return r->nnz; }

int qo_result_levels(const qo_result *r) { return r->L + 1; }

void qo_result_copy(const qo_result *r, int32_t *I, int32_t *J, double *V) {
    memcpy(I, r->I, (size_t)r->nnz * sizeof(int32_t));
    memcpy(J, r->J, (size_t)r->nnz * sizeof(int32_t));
    memcpy(V, r->V, (size_t)r->nnz * r->b * r->b * sizeof(double));
}

/* Counters: mul/add tasks and C nodes per level (levels 0..L), then
 * stats[0] = block products, stats[1] = leaf block additions. */
void qo_result_stats(const qo_result *r, int64_t *mul_tasks, int64_t *add_tasks,
                     int64_t *nodes, int64_t *stats) {
    for (int l = 0; l <= r->L; ++l) {
        mul_tasks[l] = r->mul_tasks[l];
        add_tasks[l] = r->add_tasks[l];
        nodes[l] = r->nodes_per_level[l];
    }
    stats[0] = r->block_products;
    stats[1] = r->leaf_block_adds;
}

/* Multiply tasks dropped by the norm threshold per level, and block products. */
void qo_result_pruned(const qo_result *r, int64_t *tasks, int64_t *products) {
    for (int l = 0; l <= r->L; ++l) tasks[l] = r->pruned_tasks[l];
    *products = r->pruned_products;
}

void qo_result_free(qo_result *r) {
    if (!r) return;
    free(r->I); free(r->J); free(r->V);
    free(r);
}

/* OpenMP thread count used by qo_multiply (n <= 0 leaves it unchanged);
 * returns the count now in effect. */
int qo_threads(int n) {
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}
