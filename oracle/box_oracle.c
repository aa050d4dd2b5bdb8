/*
 * Reference oracle for the lattice convolution sum -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  The product (HIP) path never calls it,
 * links it, or shares code with it.
 *
 * What it computes (plain definitions, FP64 throughout):
 *
 *   f(x)        = sum over stored lattice sites n of c_n * phi(x - n)
 *                                           (the convolution sum, Sec. 1, Eq. 1)
 *   grad f(x)   = sum_n c_n * grad phi(x - n)
 *                   (derivatives of the spline, Sec. 3: the sub-region
 *                    polynomials may be differentiated)
 *   dL/dc_n     = sum_i g_i * phi(x_i - n),   dL/dx_i = g_i * grad f(x_i)
 *
 * with phi(y) = |det L| * M_Xi(y + Xi*1/2), the centred box spline of the
 * direction matrix Xi normalised so that its lattice translates sum to one.
 * The paper leaves normalisation and centring unstated; this reading makes
 * f(c == 1) == 1.
 *
 * The evaluation is the "naive" approach of Sec. 1: one evaluation of phi per
 * candidate lattice site, each locating its own polynomial piece.  phi is
 * evaluated by the de Boor--Hollig--Riemenschneider box-spline recurrence
 * (C. de Boor, K. Hollig, S. Riemenschneider, "Box Splines", 1993; C. de Boor,
 * "On the evaluation of box splines", 1993):
 *
 *   (#Xi - s) M_Xi(z) = sum_{xi in Xi} [ t_xi M_{Xi\xi}(z)
 *                                        + (1 - t_xi) M_{Xi\xi}(z - xi) ]
 *
 * for any t with Xi t = z (here the least-norm t), terminating at a square
 * Xi = B with M_B = 1/|det B| on the half-open parallelepiped B[0,1)^s.
 * Terms whose Xi\xi no longer spans R^s are singular measures and are dropped.
 * Face ties of the parallelepipeds are resolved by a fixed generic direction v
 * (a face point is inside iff z + eps*v is inside for small eps > 0), which
 * makes every level of the recurrence the v-directional limit of itself.
 * That needs every term to see a face that several parallelepipeds share in
 * the same way: z is rounded once to the grid 2^-48 Z^s (a move of at most
 * 2^-49 per coordinate) and the side tests are done exactly, in integers, as
 * adj(B) w against 0 and det(B).
 *
 * Gradients use the directional-derivative identity
 *   D_xi M_Xi(z) = M_{Xi\xi}(z) - M_{Xi\xi}(z - xi)
 * for s independent directions, followed by an s x s solve.  Hessians apply
 * it twice: grad(D_xi M_Xi) = grad M_{Xi\xi}(z) - grad M_{Xi\xi}(z - xi),
 * the inner gradients by the same solve on Xi\xi, then H = A^{-1} R with A
 * the s chosen directions as rows and R the rows grad(D_xi M_Xi).  This needs
 * Xi with every two directions removed still spanning (C^1 box splines and
 * smoother), where the sub-region polynomials' second derivatives are the
 * classical ones off the knot planes.
 *
 * Stored coefficients are described per Cartesian coset (the lookup of Sec. 4.1
 * is one memory array per Cartesian coset): coset m holds the sites
 * n = D * (i, j, k) + l_m, i in [0, dims[0]), ..., in C order [k][j][i]
 * (i fastest).  Sites outside the stored range contribute zero.
 *
 * Limits: s in {2, 3}; at most 8 distinct directions, multiplicity <= 15,
 * direction entries in [-2, 2], support inside |z_i| < 16.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXD 8   /* distinct directions */
#define ORC_QBITS 48 /* arguments of M are rounded to the grid 2^-ORC_QBITS */
#define ORC_ZMAX 16.0 /* every support lies in |z_i| < ORC_ZMAX (checked at set-up) */
#define ORC_MAXC 8   /* cosets */
#define MEMO_BITS 12
#define MEMO_SIZE (1u << MEMO_BITS)

typedef struct {
    int s;                    /* dimension */
    int nd;                   /* number of distinct directions (up to sign) */
    int dir[ORC_MAXD][3];     /* distinct directions */
    int mult0[ORC_MAXD];      /* their multiplicities in Xi */
    double centre[3];         /* Xi * 1 / 2 */
    double detL;              /* |det L| */
    double halfwidth[3];      /* support half-width per axis */
    double v[3];              /* generic tie-break direction */
} orc_spline;

typedef struct {
    uint64_t key;
    uint32_t gen;
    double val;
} memo_entry;

typedef struct {
    memo_entry *tab;
    uint32_t gen;
} memo_t;

/* ---------------------------------------------------------------- helpers */

static double det3(const double a[3][3]) {
    return a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1])
         - a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0])
         + a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
}

static double detn(int s, const double a[3][3]) {
    if (s == 2) return a[0][0] * a[1][1] - a[0][1] * a[1][0];
    return det3(a);
}

/* Solve a x = b (s <= 3) by Cramer's rule.  Returns 0 if singular. */
static int solve(int s, const double a[3][3], const double b[3], double x[3]) {
    double d = detn(s, a);
    if (d == 0.0) return 0;
    for (int c = 0; c < s; ++c) {
        double m[3][3];
        for (int i = 0; i < s; ++i)
            for (int j = 0; j < s; ++j) m[i][j] = (j == c) ? b[i] : a[i][j];
        x[c] = detn(s, m) / d;
    }
    return 1;
}

/* Gram matrix sum_d mult_d dir_d dir_d^T; the directions span R^s iff it is
 * nonsingular. Integer entries, so the determinant test is exact. */
static void gram(const orc_spline *sp, const int *mult, double g[3][3]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) g[i][j] = 0.0;
    for (int d = 0; d < sp->nd; ++d) {
        if (!mult[d]) continue;
        for (int i = 0; i < sp->s; ++i)
            for (int j = 0; j < sp->s; ++j)
                g[i][j] += (double)mult[d] * sp->dir[d][i] * sp->dir[d][j];
    }
}

static int spans(const orc_spline *sp, const int *mult) {
    double g[3][3];
    gram(sp, mult, g);
    return detn(sp->s, g) != 0.0;
}

static uint64_t memo_key(const orc_spline *sp, const int *mult, const int *shift) {
    uint64_t k = 0;
    for (int d = 0; d < sp->nd; ++d) k = (k << 4) | (uint64_t)(mult[d] & 15);
    for (int i = 0; i < 3; ++i) k = (k << 7) | (uint64_t)((shift[i] + 64) & 127);
    return k;
}

static int memo_get(memo_t *m, uint64_t key, double *val) {
    uint32_t h = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> (64 - MEMO_BITS));
    for (uint32_t p = 0; p < MEMO_SIZE; ++p) {
        memo_entry *e = &m->tab[(h + p) & (MEMO_SIZE - 1)];
        if (e->gen != m->gen) return 0;
        if (e->key == key) { *val = e->val; return 1; }
    }
    return 0;
}

static void memo_put(memo_t *m, uint64_t key, double val) {
    uint32_t h = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> (64 - MEMO_BITS));
    for (uint32_t p = 0; p < MEMO_SIZE; ++p) {
        memo_entry *e = &m->tab[(h + p) & (MEMO_SIZE - 1)];
        if (e->gen != m->gen) { e->gen = m->gen; e->key = key; e->val = val; return; }
    }
    /* table full: value is simply not cached */
}

/* ------------------------------------------------------- the recurrence */

/* M_{Xi(mult)}(z - shift); the directions with positive multiplicity span. */
static double box_M(const orc_spline *sp, const int *mult, const int *shift,
                    const double *z, memo_t *memo) {
    const int s = sp->s;
    double w[3] = {0, 0, 0};
    int n = 0;
    for (int i = 0; i < s; ++i) w[i] = z[i] - (double)shift[i];
    for (int d = 0; d < sp->nd; ++d) n += mult[d];

    /* The support is the zonotope sum_d mult_d [0,1] dir_d; its bounding box
     * is a cheap exact-zero test. */
    for (int i = 0; i < s; ++i) {
        double lo = 0.0, hi = 0.0;
        for (int d = 0; d < sp->nd; ++d) {
            double e = (double)mult[d] * sp->dir[d][i];
            if (e < 0) lo += e; else hi += e;
        }
        if (w[i] < lo || w[i] > hi) return 0.0;
    }

    if (n == s) {
        /* Square basis: the normalised indicator of B[0,1)^s. */
        double B[3][3];
        int c = 0;
        for (int d = 0; d < sp->nd; ++d)
            if (mult[d]) {
                for (int i = 0; i < s; ++i) B[i][c] = sp->dir[d][i];
                ++c;
            }
        /* u = B^-1 w = adj(B) w / det(B) with w on the grid 2^-48 Z^s:
         * |w| < 2 ORC_ZMAX = 2^5 makes w 2^48 an exact 53-bit integer and,
         * with |adj(B)| <= 8, the numerators exact in 64 bits, so u in
         * (0,1), u == 0 and u == 1 are decided exactly; a tie takes the
         * side of v. */
        int64_t Bi[3][3], adj[3][3], wq[3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) Bi[i][j] = (i < s && j < s) ? (int64_t)B[i][j] : (i == j);
        for (int i = 0; i < s; ++i) wq[i] = (int64_t)ldexp(w[i], ORC_QBITS);
        if (s == 2) {
            adj[0][0] = Bi[1][1]; adj[0][1] = -Bi[0][1];
            adj[1][0] = -Bi[1][0]; adj[1][1] = Bi[0][0];
        } else {
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    const int r0 = (j + 1) % 3, r1 = (j + 2) % 3, c0 = (i + 1) % 3, c1 = (i + 2) % 3;
                    adj[i][j] = Bi[r0][c0] * Bi[r1][c1] - Bi[r0][c1] * Bi[r1][c0];
                }
        }
        int64_t det = 0;
        for (int j = 0; j < s; ++j) det += Bi[0][j] * adj[j][0];
        if (det == 0) return 0.0;
        const int64_t sg = det > 0 ? 1 : -1;
        const int64_t one = sg * det * ((int64_t)1 << ORC_QBITS);
        for (int i = 0; i < s; ++i) {
            int64_t num = 0;
            double nv = 0.0;
            for (int j = 0; j < s; ++j) {
                num += adj[i][j] * wq[j];
                nv += (double)adj[i][j] * sp->v[j];
            }
            num *= sg;
            nv *= (double)sg;
            if (num > 0 && num < one) continue;
            if (num == 0 && nv > 0.0) continue;
            if (num == one && nv < 0.0) continue;
            return 0.0;
        }
        return 1.0 / (double)(sg * det);
    }

    uint64_t key = memo_key(sp, mult, shift);
    double cached;
    if (memo_get(memo, key, &cached)) return cached;

    /* Least-norm t with Xi t = w:  t_xi = xi . a,  (Xi Xi^T) a = w. */
    double G[3][3], a[3] = {0, 0, 0};
    gram(sp, mult, G);
    solve(s, G, w, a);

    int sub[ORC_MAXD];
    double acc = 0.0;
    for (int d = 0; d < sp->nd; ++d) {
        if (!mult[d]) continue;
        memcpy(sub, mult, sizeof(int) * sp->nd);
        sub[d] -= 1;
        if (!spans(sp, sub)) continue;
        double t = 0.0;
        for (int i = 0; i < s; ++i) t += sp->dir[d][i] * a[i];
        int sh2[3] = {shift[0], shift[1], shift[2]};
        for (int i = 0; i < s; ++i) sh2[i] += sp->dir[d][i];
        double m0 = box_M(sp, sub, shift, z, memo);
        double m1 = box_M(sp, sub, sh2, z, memo);
        acc += (double)mult[d] * (t * m0 + (1.0 - t) * m1);
    }
    double val = acc / (double)(n - s);
    memo_put(memo, key, val);
    return val;
}

/* z = y + centre rounded to the grid 2^-ORC_QBITS Z^s; 0 if some |z_i| is
 * so large that z is outside the support of every spline handled here. */
static int grid_arg(const orc_spline *sp, const double *y, double z[3]) {
    for (int i = 0; i < 3; ++i) z[i] = 0.0;
    for (int i = 0; i < sp->s; ++i) {
        const double v = y[i] + sp->centre[i];
        if (!(fabs(v) < ORC_ZMAX)) return 0;
        z[i] = ldexp(nearbyint(ldexp(v, ORC_QBITS)), -ORC_QBITS);
    }
    return 1;
}

/* phi(y) and optionally its gradient. */
static double phi_eval(const orc_spline *sp, const double *y, double *grad, memo_t *memo) {
    const int s = sp->s;
    double z[3] = {0, 0, 0};
    int zero[3] = {0, 0, 0};
    if (!grid_arg(sp, y, z)) {
        if (grad)
            for (int i = 0; i < s; ++i) grad[i] = 0.0;
        return 0.0;
    }
    memo->gen++;
    if (memo->gen == 0) { memset(memo->tab, 0, sizeof(memo_entry) * MEMO_SIZE); memo->gen = 1; }
    double val = sp->detL * box_M(sp, sp->mult0, zero, z, memo);
    if (grad) {
        /* Directional derivatives along s independent directions whose
         * removal keeps Xi spanning, then solve for the gradient. */
        double A[3][3], b[3];
        int rows = 0;
        int sub[ORC_MAXD];
        for (int d = 0; d < sp->nd && rows < s; ++d) {
            memcpy(sub, sp->mult0, sizeof(int) * sp->nd);
            sub[d] -= 1;
            if (!spans(sp, sub)) continue;
            /* keep only directions independent of the rows chosen so far */
            double T[3][3];
            for (int r = 0; r < rows; ++r)
                for (int i = 0; i < s; ++i) T[r][i] = A[r][i];
            for (int i = 0; i < s; ++i) T[rows][i] = sp->dir[d][i];
            if (rows + 1 == s) {
                if (detn(s, T) == 0.0) continue;
            } else if (rows == 1 && s == 3) {
                double cx = T[0][1] * T[1][2] - T[0][2] * T[1][1];
                double cy = T[0][2] * T[1][0] - T[0][0] * T[1][2];
                double cz = T[0][0] * T[1][1] - T[0][1] * T[1][0];
                if (cx == 0.0 && cy == 0.0 && cz == 0.0) continue;
            }
            int sh[3] = {0, 0, 0};
            for (int i = 0; i < s; ++i) sh[i] = sp->dir[d][i];
            double m0 = box_M(sp, sub, zero, z, memo);
            double m1 = box_M(sp, sub, sh, z, memo);
            for (int i = 0; i < s; ++i) A[rows][i] = sp->dir[d][i];
            b[rows] = sp->detL * (m0 - m1);
            ++rows;
        }
        double g[3] = {0, 0, 0};
        if (rows == s) solve(s, A, b, g);
        for (int i = 0; i < s; ++i) grad[i] = g[i];
    }
    return val;
}

/* Up to s directions of Xi(mult), mutually independent, whose removal keeps
 * Xi spanning; their indices in dirs, their vectors as the rows of A. */
static int pick_dirs(const orc_spline *sp, const int *mult, int dirs[3], double A[3][3]) {
    const int s = sp->s;
    int rows = 0;
    int sub[ORC_MAXD];
    for (int d = 0; d < sp->nd && rows < s; ++d) {
        if (!mult[d]) continue;
        memcpy(sub, mult, sizeof(int) * sp->nd);
        sub[d] -= 1;
        if (!spans(sp, sub)) continue;
        double T[3][3];
        for (int r = 0; r < rows; ++r)
            for (int i = 0; i < s; ++i) T[r][i] = A[r][i];
        for (int i = 0; i < s; ++i) T[rows][i] = sp->dir[d][i];
        if (rows + 1 == s) {
            if (detn(s, T) == 0.0) continue;
        } else if (rows == 1 && s == 3) {
            double cx = T[0][1] * T[1][2] - T[0][2] * T[1][1];
            double cy = T[0][2] * T[1][0] - T[0][0] * T[1][2];
            double cz = T[0][0] * T[1][1] - T[0][1] * T[1][0];
            if (cx == 0.0 && cy == 0.0 && cz == 0.0) continue;
        }
        for (int i = 0; i < s; ++i) A[rows][i] = sp->dir[d][i];
        dirs[rows++] = d;
    }
    return rows;
}

/* grad M_{Xi(mult)}(z - shift) by s directional derivatives; 0 if Xi(mult)
 * has no s usable directions. */
static int box_grad(const orc_spline *sp, const int *mult, const int *shift, const double *z,
                    memo_t *memo, double g[3]) {
    const int s = sp->s;
    int dirs[3];
    double A[3][3], b[3];
    if (pick_dirs(sp, mult, dirs, A) != s) return 0;
    int sub[ORC_MAXD];
    for (int r = 0; r < s; ++r) {
        const int d = dirs[r];
        memcpy(sub, mult, sizeof(int) * sp->nd);
        sub[d] -= 1;
        int sh[3] = {shift[0], shift[1], shift[2]};
        for (int i = 0; i < s; ++i) sh[i] += sp->dir[d][i];
        b[r] = box_M(sp, sub, shift, z, memo) - box_M(sp, sub, sh, z, memo);
    }
    g[0] = g[1] = g[2] = 0.0;
    return solve(s, A, b, g);
}

/* phi(y), grad phi and the Hessian of phi (s x s, row-major); 0 if the
 * Hessian is not available for this Xi. */
static int phi_hess(const orc_spline *sp, const double *y, double *val, double *grad,
                    double *hess, memo_t *memo) {
    const int s = sp->s;
    *val = phi_eval(sp, y, grad, memo);
    double z[3] = {0, 0, 0};
    int zero[3] = {0, 0, 0};
    if (!grid_arg(sp, y, z)) {
        for (int i = 0; i < s * s; ++i) hess[i] = 0.0;
        return 1;
    }
    int dirs[3];
    double A[3][3], R[3][3];
    if (pick_dirs(sp, sp->mult0, dirs, A) != s) return 0;
    int sub[ORC_MAXD];
    for (int r = 0; r < s; ++r) {
        const int d = dirs[r];
        memcpy(sub, sp->mult0, sizeof(int) * sp->nd);
        sub[d] -= 1;
        int sh[3] = {0, 0, 0};
        for (int i = 0; i < s; ++i) sh[i] = sp->dir[d][i];
        double g0[3], g1[3];
        if (!box_grad(sp, sub, zero, z, memo, g0) || !box_grad(sp, sub, sh, z, memo, g1)) return 0;
        for (int i = 0; i < s; ++i) R[r][i] = sp->detL * (g0[i] - g1[i]);
    }
    /* A H = R, column by column */
    for (int j = 0; j < s; ++j) {
        double b[3], h[3] = {0, 0, 0};
        for (int r = 0; r < s; ++r) b[r] = R[r][j];
        if (!solve(s, A, b, h)) return 0;
        for (int i = 0; i < s; ++i) hess[i * s + j] = h[i];
    }
    return 1;
}

/* ----------------------------------------------------------- set-up */

/* Xi: s x n row-major, columns are directions.  L: s x s. */
static int spline_init(orc_spline *sp, int s, int n, const int *Xi, const int *L) {
    if (s < 2 || s > 3 || n < s) return -1;
    memset(sp, 0, sizeof(*sp));
    sp->s = s;
    for (int j = 0; j < n; ++j) {
        int col[3] = {0, 0, 0};
        for (int i = 0; i < s; ++i) col[i] = Xi[i * n + j];
        /* canonical sign: first nonzero entry positive (phi is centred, so
         * the sign of a direction does not change it; the centre is taken
         * from the original columns below) */
        int sg = 0;
        for (int i = 0; i < s && !sg; ++i) sg = (col[i] > 0) - (col[i] < 0);
        if (sg == 0) return -2;
        int c[3] = {0, 0, 0};
        for (int i = 0; i < s; ++i) c[i] = col[i] * sg;
        int found = -1;
        for (int d = 0; d < sp->nd; ++d) {
            int same = 1;
            for (int i = 0; i < s; ++i) same &= (sp->dir[d][i] == c[i]);
            if (same) { found = d; break; }
        }
        if (found < 0) {
            if (sp->nd == ORC_MAXD) return -3;
            found = sp->nd++;
            for (int i = 0; i < s; ++i) sp->dir[found][i] = c[i];
        }
        if (++sp->mult0[found] > 15) return -3;
    }
    if (!spans(sp, sp->mult0)) return -4;
    /* centre and half-width from the canonical (sign-normalised) columns:
     * centring removes the dependence on direction signs */
    for (int i = 0; i < s; ++i) {
        double c = 0.0, h = 0.0;
        for (int d = 0; d < sp->nd; ++d) {
            c += 0.5 * sp->mult0[d] * sp->dir[d][i];
            h += 0.5 * sp->mult0[d] * abs(sp->dir[d][i]);
        }
        sp->centre[i] = c;
        sp->halfwidth[i] = h;
        /* the uncentred support spans [c - h, c + h]; the exact face tests
         * need it inside |z| < ORC_ZMAX, and |adj(B)| <= 8 needs small
         * direction entries */
        if (fabs(c) + h >= ORC_ZMAX) return -6;
    }
    for (int d = 0; d < sp->nd; ++d)
        for (int i = 0; i < s; ++i)
            if (abs(sp->dir[d][i]) > 2) return -6;
    double Lm[3][3];
    for (int i = 0; i < s; ++i)
        for (int j = 0; j < s; ++j) Lm[i][j] = L[i * s + j];
    sp->detL = fabs(detn(s, Lm));
    if (sp->detL == 0.0) return -5;
    sp->v[0] = 0.8731;
    sp->v[1] = 0.3419;
    sp->v[2] = 0.1257;
    return 0;
}

static memo_t memo_new(void) {
    memo_t m;
    m.tab = (memo_entry *)calloc(MEMO_SIZE, sizeof(memo_entry));
    m.gen = 0;
    return m;
}

typedef struct {
    int n_cosets;
    int D[3];
    int shift[ORC_MAXC][3];
    int64_t dims[3];
    int64_t per_coset;
} orc_layout;

static int layout_init(orc_layout *ly, int s, int n_cosets, const int *D,
                       const int *shifts, const int64_t *dims) {
    if (n_cosets < 1 || n_cosets > ORC_MAXC) return -1;
    memset(ly, 0, sizeof(*ly));
    ly->n_cosets = n_cosets;
    ly->per_coset = 1;
    for (int i = 0; i < 3; ++i) {
        ly->D[i] = (i < s) ? D[i] : 1;
        ly->dims[i] = (i < s) ? dims[i] : 1;
        if (ly->D[i] <= 0 || ly->dims[i] < 0) return -2;
        ly->per_coset *= ly->dims[i];
    }
    for (int m = 0; m < n_cosets; ++m)
        for (int i = 0; i < 3; ++i) ly->shift[m][i] = (i < s) ? shifts[m * s + i] : 0;
    return 0;
}

/* Visit every stored site n that can influence x (or every stored site when
 * brute is set), calling back with its flat index and phi, grad phi. */
typedef void (*site_cb)(void *ctx, int64_t flat, double phi, const double *gphi);

static void visit_sites(const orc_spline *sp, const orc_layout *ly, const double *x,
                        int brute, int want_grad, memo_t *memo, site_cb cb, void *ctx) {
    const int s = sp->s;
    for (int m = 0; m < ly->n_cosets; ++m) {
        int64_t lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        for (int i = 0; i < 3; ++i) {
            if (i >= s) { lo[i] = 0; hi[i] = 0; continue; }
            if (brute) { lo[i] = 0; hi[i] = ly->dims[i] - 1; continue; }
            double a = (x[i] - sp->halfwidth[i] - ly->shift[m][i]) / ly->D[i];
            double b = (x[i] + sp->halfwidth[i] - ly->shift[m][i]) / ly->D[i];
            if (!(a == a) || !(b == b)) { lo[i] = 1; hi[i] = 0; continue; }
            if (a < -1e15) a = -1e15;
            if (b > 1e15) b = 1e15;
            lo[i] = (int64_t)ceil(a);
            hi[i] = (int64_t)floor(b);
            if (lo[i] < 0) lo[i] = 0;
            if (hi[i] > ly->dims[i] - 1) hi[i] = ly->dims[i] - 1;
        }
        for (int64_t k = lo[2]; k <= hi[2]; ++k)
            for (int64_t j = lo[1]; j <= hi[1]; ++j)
                for (int64_t i = lo[0]; i <= hi[0]; ++i) {
                    int64_t idx[3] = {i, j, k};
                    double y[3] = {0, 0, 0}, g[3] = {0, 0, 0};
                    for (int a = 0; a < s; ++a)
                        y[a] = x[a] - (double)(ly->D[a] * idx[a] + ly->shift[m][a]);
                    double p = phi_eval(sp, y, want_grad ? g : NULL, memo);
                    int64_t flat = m * ly->per_coset + (k * ly->dims[1] + j) * ly->dims[0] + i;
                    cb(ctx, flat, p, g);
                }
    }
}

typedef struct {
    const double *coef;
    double f;
    double g[3];
} eval_ctx;

static void eval_cb(void *vctx, int64_t flat, double phi, const double *gphi) {
    eval_ctx *c = (eval_ctx *)vctx;
    double cn = c->coef[flat];
    c->f += cn * phi;
    c->g[0] += cn * gphi[0];
    c->g[1] += cn * gphi[1];
    c->g[2] += cn * gphi[2];
}

typedef struct {
    double *acc;
    double gi;
} bwd_ctx;

static void bwd_cb(void *vctx, int64_t flat, double phi, const double *gphi) {
    (void)gphi;
    bwd_ctx *c = (bwd_ctx *)vctx;
    c->acc[flat] += c->gi * phi;
}

/* ------------------------------------------------------- exported API */

/* phi and grad phi at npts points y (npts x s).  grad may be NULL. */
int orc_phi(int s, int n, const int *Xi, const int *L, int64_t npts, const double *y,
            double *out, double *grad) {
    orc_spline sp;
    int rc = spline_init(&sp, s, n, Xi, L);
    if (rc) return rc;
    int err = 0;
#pragma omp parallel
    {
        memo_t memo = memo_new();
        if (!memo.tab) {
#pragma omp atomic write
            err = -10;
        } else {
#pragma omp for schedule(dynamic, 64)
            for (int64_t p = 0; p < npts; ++p) {
                double g[3] = {0, 0, 0};
                out[p] = phi_eval(&sp, y + p * s, grad ? g : NULL, &memo);
                if (grad)
                    for (int i = 0; i < s; ++i) grad[p * s + i] = g[i];
            }
        }
        free(memo.tab);
    }
    return err;
}

/* f (and optionally grad f) at npts points x (npts x s, FP64).
 * coef: n_cosets * prod(dims) values, coset-major, each C order. */
int orc_eval(int s, int n, const int *Xi, const int *L, int n_cosets, const int *D,
             const int *shifts, const int64_t *dims, const double *coef, int64_t npts,
             const double *x, double *f, double *grad, int brute) {
    orc_spline sp;
    orc_layout ly;
    int rc = spline_init(&sp, s, n, Xi, L);
    if (rc) return rc;
    rc = layout_init(&ly, s, n_cosets, D, shifts, dims);
    if (rc) return rc - 20;
    int err = 0;
#pragma omp parallel
    {
        memo_t memo = memo_new();
        if (!memo.tab) {
#pragma omp atomic write
            err = -10;
        } else {
#pragma omp for schedule(dynamic, 16)
            for (int64_t p = 0; p < npts; ++p) {
                eval_ctx c;
                memset(&c, 0, sizeof(c));
                c.coef = coef;
                visit_sites(&sp, &ly, x + p * s, brute, grad != NULL, &memo, eval_cb, &c);
                f[p] = c.f;
                if (grad)
                    for (int i = 0; i < s; ++i) grad[p * s + i] = c.g[i];
            }
        }
        free(memo.tab);
    }
    return err;
}

/* f, grad f and the Hessian of f (npts x s x s) at npts points x; returns
 * -30 when the Hessian is not available for this Xi (two directions whose
 * removal stops Xi spanning). */
int orc_eval_hess(int s, int n, const int *Xi, const int *L, int n_cosets, const int *D,
                  const int *shifts, const int64_t *dims, const double *coef, int64_t npts,
                  const double *x, double *f, double *grad, double *hess) {
    orc_spline sp;
    orc_layout ly;
    int rc = spline_init(&sp, s, n, Xi, L);
    if (rc) return rc;
    rc = layout_init(&ly, s, n_cosets, D, shifts, dims);
    if (rc) return rc - 20;
    int err = 0;
#pragma omp parallel
    {
        memo_t memo = memo_new();
        if (!memo.tab) {
#pragma omp atomic write
            err = -10;
        } else {
#pragma omp for schedule(dynamic, 16)
            for (int64_t p = 0; p < npts; ++p) {
                const double *xp = x + p * s;
                double fa = 0.0, ga[3] = {0, 0, 0}, ha[9] = {0};
                for (int m = 0; m < ly.n_cosets; ++m) {
                    int64_t lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
                    int empty = 0;
                    for (int i = 0; i < s; ++i) {
                        double a = (xp[i] - sp.halfwidth[i] - ly.shift[m][i]) / ly.D[i];
                        double b = (xp[i] + sp.halfwidth[i] - ly.shift[m][i]) / ly.D[i];
                        if (!(a == a) || !(b == b)) { empty = 1; break; }
                        if (a < -1e15) a = -1e15;
                        if (b > 1e15) b = 1e15;
                        lo[i] = (int64_t)ceil(a);
                        hi[i] = (int64_t)floor(b);
                        if (lo[i] < 0) lo[i] = 0;
                        if (hi[i] > ly.dims[i] - 1) hi[i] = ly.dims[i] - 1;
                    }
                    if (empty) continue;
                    for (int64_t k = lo[2]; k <= hi[2]; ++k)
                        for (int64_t j = lo[1]; j <= hi[1]; ++j)
                            for (int64_t i = lo[0]; i <= hi[0]; ++i) {
                                int64_t idx[3] = {i, j, k};
                                double y[3] = {0, 0, 0}, g[3] = {0, 0, 0}, h[9] = {0}, v = 0.0;
                                for (int a = 0; a < s; ++a)
                                    y[a] = xp[a] - (double)(ly.D[a] * idx[a] + ly.shift[m][a]);
                                if (!phi_hess(&sp, y, &v, g, h, &memo)) {
#pragma omp atomic write
                                    err = -30;
                                }
                                const double cn = coef[m * ly.per_coset + (k * ly.dims[1] + j) * ly.dims[0] + i];
                                fa += cn * v;
                                for (int a = 0; a < s; ++a) ga[a] += cn * g[a];
                                for (int a = 0; a < s * s; ++a) ha[a] += cn * h[a];
                            }
                }
                f[p] = fa;
                for (int a = 0; a < s; ++a) grad[p * s + a] = ga[a];
                for (int a = 0; a < s * s; ++a) hess[p * s * s + a] = ha[a];
            }
        }
        free(memo.tab);
    }
    return err;
}

/* dL/dc_n = sum_i g_i phi(x_i - n) for every stored site (same layout as the
 * coefficients).  Each thread scatters into a private FP64 array; the arrays
 * are then summed in thread order. */
int orc_backward_coef(int s, int n, const int *Xi, const int *L, int n_cosets, const int *D,
                      const int *shifts, const int64_t *dims, int64_t npts, const double *x,
                      const double *g, double *dLdc) {
    orc_spline sp;
    orc_layout ly;
    int rc = spline_init(&sp, s, n, Xi, L);
    if (rc) return rc;
    rc = layout_init(&ly, s, n_cosets, D, shifts, dims);
    if (rc) return rc - 20;
    const int64_t total = ly.per_coset * n_cosets;
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    double *bufs = (double *)calloc((size_t)total * nthreads, sizeof(double));
    if (!bufs) return -10;
    int err = 0;
#pragma omp parallel num_threads(nthreads)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        memo_t memo = memo_new();
        if (!memo.tab) {
#pragma omp atomic write
            err = -10;
        } else {
            bwd_ctx c;
            c.acc = bufs + (size_t)tid * total;
#pragma omp for schedule(static)
            for (int64_t p = 0; p < npts; ++p) {
                c.gi = g[p];
                visit_sites(&sp, &ly, x + p * s, 0, 0, &memo, bwd_cb, &c);
            }
        }
        free(memo.tab);
    }
    for (int64_t k = 0; k < total; ++k) {
        double acc = 0.0;
        for (int t = 0; t < nthreads; ++t) acc += bufs[(size_t)t * total + k];
        dLdc[k] = acc;
    }
    free(bufs);
    return err;
}

/* Threads the oracle uses (for reporting). */
int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
