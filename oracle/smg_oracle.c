/*
 * smg_oracle.c -- plain FP64 CPU oracle for the SMG-preconditioned Krylov
 * solvers of Bouwmeester, Dougherty and Knyazev, "Nonsymmetric multigrid
 * preconditioning for conjugate gradient methods" (arXiv 1212.6680).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; it exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark can compare the GPU library against a slow,
 * obviously correct implementation.  It shares no code, header or table with
 * the GPU library.
 *
 * What it computes:
 *   - the model problem of Section 2: the 7-point negative Laplacian on an
 *     nx*ny*nz brick with homogeneous Dirichlet boundary, per-axis
 *     coefficients cx, cy, cz (the paper uses unit grid size, c = 1);
 *   - the SMG V-cycle used as a preconditioner (Section 3: plane relaxation
 *     as the smoother at every level of a V-cycle, independent pre- and
 *     post-smoothing counts).  The paper does not spell out SMG's internals;
 *     the reading implemented here is:
 *       * semicoarsening in z by two, coarse planes = odd fine planes,
 *         linear prolongation P, restriction P^T, Galerkin coarse operator
 *         P^T A P (the "restriction and prolongation pair" that keeps the
 *         balanced cycle symmetric, Section 1);
 *       * zebra plane relaxation in correction form, pre-smoothing colour
 *         order F (even) then C (odd), post-smoothing in the reverse order;
 *       * each plane solve is one 2D V-cycle built by the same rules in y
 *         (x-lines, zebra line relaxation, Galerkin), whose coarsest level is
 *         one exact line solve (Thomas algorithm); the 2D cycles inherit the
 *         3D smoothing counts unless told otherwise;
 *   - Algorithm 1 of Section 2 with beta from equation (1) (standard PCG),
 *     equation (2) (flexible PCG) or beta = 0 (PSD).
 *
 * Layout: index i + nx*(j + ny*k), x fastest.  Every routine is FP64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* Model problem operator (Section 2): y = A x, 7-point, Dirichlet.          */
/* ------------------------------------------------------------------------- */
void oracle_matvec(int nx, int ny, int nz, double cx, double cy, double cz,
                   const double *x, double *y)
{
    const double diag = 2.0 * cx + 2.0 * cy + 2.0 * cz;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = (size_t)i + (size_t)nx * ((size_t)j + (size_t)ny * k);
                double v = diag * x[c];
                if (i > 0) v -= cx * x[c - 1];
                if (i < nx - 1) v -= cx * x[c + 1];
                if (j > 0) v -= cy * x[c - nx];
                if (j < ny - 1) v -= cy * x[c + nx];
                if (k > 0) v -= cz * x[c - (size_t)nx * ny];
                if (k < nz - 1) v -= cz * x[c + (size_t)nx * ny];
                y[c] = v;
            }
}

/* ------------------------------------------------------------------------- */
/* Blocks of the form a*S + b*I, S = tridiag(-1, 2, -1) along x (lines) or   */
/* S = T2 = cx*Tx (x) I + cy*I (x) Ty (planes).                               */
/* ------------------------------------------------------------------------- */

/* out -= (a*Tx + b*I) v  on one x-line of length nx */
static void line_block_sub(int nx, double a, double b, const double *v, double *out)
{
    for (int i = 0; i < nx; ++i) {
        double t = 2.0 * v[i];
        if (i > 0) t -= v[i - 1];
        if (i < nx - 1) t -= v[i + 1];
        out[i] -= a * t + b * v[i];
    }
}

/* out -= (a*T2 + b*I) v  on one nx*ny plane */
static void plane_block_sub(int nx, int ny, double cx, double cy, double a, double b,
                            const double *v, double *out)
{
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)i + (size_t)nx * j;
            double tx = 2.0 * v[c], ty = 2.0 * v[c];
            if (i > 0) tx -= v[c - 1];
            if (i < nx - 1) tx -= v[c + 1];
            if (j > 0) ty -= v[c - nx];
            if (j < ny - 1) ty -= v[c + nx];
            out[c] -= a * (cx * tx + cy * ty) + b * v[c];
        }
}

/* Exact solve of (a*Tx + b*I) u = f by the Thomas algorithm (the block is
 * SPD, so elimination without pivoting is stable).  work has nx entries. */
void oracle_line_solve(int nx, double a, double b, const double *f, double *u, double *work)
{
    const double diag = 2.0 * a + b, off = -a;
    double m = diag;
    work[0] = off / m;
    u[0] = f[0] / m;
    for (int i = 1; i < nx; ++i) {
        m = diag - off * work[i - 1];
        work[i] = off / m;
        u[i] = (f[i] - off * u[i - 1]) / m;
    }
    for (int i = nx - 2; i >= 0; --i) u[i] -= work[i] * u[i + 1];
}

/* Galerkin coarsening of a block-tridiagonal operator with diagonal blocks
 * D_f = Da[f]*S + Db[f]*I (f < n) and couplings O_f = Oa[f]*S + Ob[f]*I
 * between f and f+1 (f < n-1), under the linear prolongation whose coarse
 * point K sits on fine point 2K+1 and reaches 2K and 2K+2 with weight 1/2.
 * Since P acts on the block index only, P^T A P stays in span{S, I}:
 *   D^c_K = 1/4 D_{2K} + D_{2K+1} + 1/4 D_{2K+2} + O_{2K} + O_{2K+1}
 *   O^c_K = 1/2 O_{2K+1} + 1/4 D_{2K+2} + 1/2 O_{2K+2}
 * with every term that names a missing fine block dropped. */
static int galerkin(int n, const double *Da, const double *Db, const double *Oa,
                    const double *Ob, double *cDa, double *cDb, double *cOa, double *cOb)
{
    int nc = n / 2;
    for (int K = 0; K < nc; ++K) {
        int f0 = 2 * K, f1 = 2 * K + 1, f2 = 2 * K + 2;
        cDa[K] = 0.25 * Da[f0] + Da[f1] + Oa[f0];
        cDb[K] = 0.25 * Db[f0] + Db[f1] + Ob[f0];
        if (f2 < n) {
            cDa[K] += 0.25 * Da[f2] + Oa[f1];
            cDb[K] += 0.25 * Db[f2] + Ob[f1];
        }
        if (K + 1 < nc) {
            cOa[K] = 0.5 * Oa[f1] + 0.25 * Da[f2] + 0.5 * Oa[f2];
            cOb[K] = 0.5 * Ob[f1] + 0.25 * Db[f2] + 0.5 * Ob[f2];
        }
    }
    return nc;
}

/* ------------------------------------------------------------------------- */
/* Hierarchies                                                               */
/* ------------------------------------------------------------------------- */
typedef struct {          /* one 2D level of a plane hierarchy */
    int ny;               /* number of x-lines */
    double *La, *Lb;      /* L_j = La[j]*Tx + Lb[j]*I            (ny)   */
    double *Va, *Vb;      /* V_j = Va[j]*Tx + Vb[j]*I, j <-> j+1  (ny-1) */
} level2_t;

typedef struct {
    int nlev;
    level2_t *lev;
} plane_hier_t;

typedef struct {          /* one 3D level */
    int nz;
    double *Ca, *Cb;      /* C_K = Ca[K]*T2 + Cb[K]*I             (nz)   */
    double *Ua, *Ub;      /* U_K = Ua[K]*T2 + Ub[K]*I, K <-> K+1  (nz-1) */
    plane_hier_t *ph;     /* plane-solve hierarchy of every plane        */
    double *x, *b, *r;    /* level vectors                              */
} level3_t;

typedef struct {          /* per-thread scratch for one plane solve */
    double **x, **b, **r; /* per 2D level, nx*ny_l each */
    double *rk, *yk, *tmp;
} ws2_t;

typedef struct oracle_smg {
    int nx, ny, nz;
    double cx, cy, cz;
    int pre, post, ipre, ipost, order;
    int nlev;
    level3_t *lev;
    int nthreads;
    ws2_t *ws;
} oracle_smg;

static double *zalloc(size_t n) { return (double *)calloc(n ? n : 1, sizeof(double)); }

static int levels_of(int n)
{
    int L = 1;
    while (n > 1) { n /= 2; ++L; }
    return L;
}

/* 2D hierarchy of the plane operator Q = alpha*T2 + beta*I.  Restricted to
 * x-line j, Q has diagonal block alpha*cx*Tx + (2*alpha*cy + beta)*I and
 * couplings -alpha*cy*I to lines j-1 and j+1. */
static void build_plane_hier(plane_hier_t *h, int ny, double cx, double cy, double alpha, double beta)
{
    h->nlev = levels_of(ny);
    h->lev = (level2_t *)calloc((size_t)h->nlev, sizeof(level2_t));
    level2_t *f = &h->lev[0];
    f->ny = ny;
    f->La = zalloc(ny); f->Lb = zalloc(ny); f->Va = zalloc(ny); f->Vb = zalloc(ny);
    for (int j = 0; j < ny; ++j) {
        f->La[j] = alpha * cx;
        f->Lb[j] = 2.0 * alpha * cy + beta;
        f->Va[j] = 0.0;
        f->Vb[j] = -alpha * cy;
    }
    for (int l = 1; l < h->nlev; ++l) {
        level2_t *p = &h->lev[l - 1], *c = &h->lev[l];
        int nc = p->ny / 2;
        c->La = zalloc(nc); c->Lb = zalloc(nc); c->Va = zalloc(nc); c->Vb = zalloc(nc);
        c->ny = galerkin(p->ny, p->La, p->Lb, p->Va, p->Vb, c->La, c->Lb, c->Va, c->Vb);
    }
}

static void free_plane_hier(plane_hier_t *h)
{
    for (int l = 0; l < h->nlev; ++l) {
        free(h->lev[l].La); free(h->lev[l].Lb); free(h->lev[l].Va); free(h->lev[l].Vb);
    }
    free(h->lev);
}

/* ------------------------------------------------------------------------- */
/* 2D V-cycle on one plane (the plane solve of the 3D smoother)              */
/* ------------------------------------------------------------------------- */

/* r_j = b_j - (Q x)_j for one line */
static void resid_line(const oracle_smg *S, const level2_t *L, int j, const double *b,
                       const double *x, double *r)
{
    const int nx = S->nx;
    memcpy(r, b + (size_t)nx * j, sizeof(double) * nx);
    line_block_sub(nx, L->La[j], L->Lb[j], x + (size_t)nx * j, r);
    if (j > 0) line_block_sub(nx, L->Va[j - 1], L->Vb[j - 1], x + (size_t)nx * (j - 1), r);
    if (j < L->ny - 1) line_block_sub(nx, L->Va[j], L->Vb[j], x + (size_t)nx * (j + 1), r);
}

/* one zebra half-sweep over the lines of one colour, correction form:
 * x_j += L_j^{-1} (b - Q x)_j */
static void sweep2(const oracle_smg *S, const level2_t *L, int colour, const double *b,
                   double *x, ws2_t *w)
{
    const int nx = S->nx;
    double *r = w->tmp + nx, *u = w->tmp + 2 * (size_t)nx;
    for (int j = colour; j < L->ny; j += 2) {
        resid_line(S, L, j, b, x, r);
        oracle_line_solve(nx, L->La[j], L->Lb[j], r, u, w->tmp);
        for (int i = 0; i < nx; ++i) x[(size_t)nx * j + i] += u[i];
    }
}

static void vcycle2(const oracle_smg *S, const plane_hier_t *h, int l, const double *b,
                    double *x, ws2_t *w)
{
    const int nx = S->nx;
    const level2_t *L = &h->lev[l];
    const int first = S->order == 0 ? 0 : 1, second = 1 - first;
    if (L->ny == 1) {                       /* coarsest: one exact line solve */
        oracle_line_solve(nx, L->La[0], L->Lb[0], b, x, w->tmp);
        return;
    }
    memset(x, 0, sizeof(double) * (size_t)nx * L->ny);
    for (int s = 0; s < S->ipre; ++s) {
        sweep2(S, L, first, b, x, w);
        sweep2(S, L, second, b, x, w);
    }
    /* residual, restriction P^T */
    double *r = w->r[l];
    for (int j = 0; j < L->ny; ++j) resid_line(S, L, j, b, x, r + (size_t)nx * j);
    const int nc = L->ny / 2;
    double *bc = w->b[l + 1], *xc = w->x[l + 1];
    for (int J = 0; J < nc; ++J)
        for (int i = 0; i < nx; ++i) {
            double v = 0.5 * r[(size_t)nx * (2 * J) + i] + r[(size_t)nx * (2 * J + 1) + i];
            if (2 * J + 2 < L->ny) v += 0.5 * r[(size_t)nx * (2 * J + 2) + i];
            bc[(size_t)nx * J + i] = v;
        }
    vcycle2(S, h, l + 1, bc, xc, w);
    /* prolongation P, correction */
    for (int J = 0; J < nc; ++J)
        for (int i = 0; i < nx; ++i) {
            double v = xc[(size_t)nx * J + i];
            x[(size_t)nx * (2 * J) + i] += 0.5 * v;
            x[(size_t)nx * (2 * J + 1) + i] += v;
            if (2 * J + 2 < L->ny) x[(size_t)nx * (2 * J + 2) + i] += 0.5 * v;
        }
    for (int s = 0; s < S->ipost; ++s) {
        sweep2(S, L, second, b, x, w);
        sweep2(S, L, first, b, x, w);
    }
}

/* ------------------------------------------------------------------------- */
/* 3D V-cycle                                                                */
/* ------------------------------------------------------------------------- */

/* r_k = b_k - (A_l x)_k for one plane k of level l */
static void resid_plane(const oracle_smg *S, const level3_t *L, int k, const double *b,
                        const double *x, double *r)
{
    const int nx = S->nx, ny = S->ny;
    const size_t pl = (size_t)nx * ny;
    memcpy(r, b + pl * k, sizeof(double) * pl);
    plane_block_sub(nx, ny, S->cx, S->cy, L->Ca[k], L->Cb[k], x + pl * k, r);
    if (k > 0) plane_block_sub(nx, ny, S->cx, S->cy, L->Ua[k - 1], L->Ub[k - 1], x + pl * (k - 1), r);
    if (k < L->nz - 1) plane_block_sub(nx, ny, S->cx, S->cy, L->Ua[k], L->Ub[k], x + pl * (k + 1), r);
}

static ws2_t *thread_ws(oracle_smg *S)
{
#ifdef _OPENMP
    return &S->ws[omp_get_thread_num()];
#else
    return &S->ws[0];
#endif
}

/* zebra plane relaxation over one colour, correction form:
 * x_k += V2_k(b - A x)_k with V2_k one 2D V-cycle of plane k's operator */
static void sweep3(oracle_smg *S, level3_t *L, int colour, const double *b, double *x)
{
    const size_t pl = (size_t)S->nx * S->ny;
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = colour; k < L->nz; k += 2) {
        ws2_t *w = thread_ws(S);
        resid_plane(S, L, k, b, x, w->rk);
        vcycle2(S, &L->ph[k], 0, w->rk, w->yk, w);
        for (size_t c = 0; c < pl; ++c) x[pl * k + c] += w->yk[c];
    }
}

static void vcycle3(oracle_smg *S, int l, const double *b, double *x)
{
    level3_t *L = &S->lev[l];
    const size_t pl = (size_t)S->nx * S->ny;
    const int first = S->order == 0 ? 0 : 1, second = 1 - first;
    if (L->nz == 1) {                       /* coarsest: one plane solve */
        ws2_t *w = &S->ws[0];
        vcycle2(S, &L->ph[0], 0, b, x, w);
        return;
    }
    memset(x, 0, sizeof(double) * pl * L->nz);
    for (int s = 0; s < S->pre; ++s) {
        sweep3(S, L, first, b, x);
        sweep3(S, L, second, b, x);
    }
    level3_t *C = &S->lev[l + 1];
#pragma omp parallel for schedule(static)
    for (int k = 0; k < L->nz; ++k) resid_plane(S, L, k, b, x, L->r + pl * k);
#pragma omp parallel for schedule(static)
    for (int K = 0; K < C->nz; ++K)
        for (size_t c = 0; c < pl; ++c) {
            double v = 0.5 * L->r[pl * (2 * K) + c] + L->r[pl * (2 * K + 1) + c];
            if (2 * K + 2 < L->nz) v += 0.5 * L->r[pl * (2 * K + 2) + c];
            C->b[pl * K + c] = v;
        }
    vcycle3(S, l + 1, C->b, C->x);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < L->nz; ++k) {
        /* fine plane k receives coarse K = (k-1)/2 with weight 1 when k is
         * odd, and coarse K = k/2 - 1 and K = k/2 with weight 1/2 when even */
        for (size_t c = 0; c < pl; ++c) {
            double v;
            if (k % 2 == 1) {
                v = C->x[pl * (k / 2) + c];
            } else {
                v = 0.0;
                if (k / 2 - 1 >= 0) v += 0.5 * C->x[pl * (k / 2 - 1) + c];
                if (k / 2 < C->nz) v += 0.5 * C->x[pl * (k / 2) + c];
            }
            x[pl * k + c] += v;
        }
    }
    for (int s = 0; s < S->post; ++s) {
        sweep3(S, L, second, b, x);
        sweep3(S, L, first, b, x);
    }
}

/* ------------------------------------------------------------------------- */
/* Public SMG interface                                                      */
/* ------------------------------------------------------------------------- */
oracle_smg *oracle_smg_create(int nx, int ny, int nz, double cx, double cy, double cz,
                              int pre, int post, int ipre, int ipost, int order)
{
    if (nx < 1 || ny < 1 || nz < 1 || pre < 0 || post < 0) return NULL;
    oracle_smg *S = (oracle_smg *)calloc(1, sizeof(oracle_smg));
    S->nx = nx; S->ny = ny; S->nz = nz;
    S->cx = cx; S->cy = cy; S->cz = cz;
    S->pre = pre; S->post = post;
    S->ipre = ipre < 0 ? pre : ipre;
    S->ipost = ipost < 0 ? post : ipost;
    S->order = order;
    S->nlev = levels_of(nz);
    S->lev = (level3_t *)calloc((size_t)S->nlev, sizeof(level3_t));
    const size_t pl = (size_t)nx * ny;
    /* fine level: C_k = T2 + 2cz I, U_k = -cz I (7-point operator) */
    level3_t *f = &S->lev[0];
    f->nz = nz;
    f->Ca = zalloc(nz); f->Cb = zalloc(nz); f->Ua = zalloc(nz); f->Ub = zalloc(nz);
    for (int k = 0; k < nz; ++k) {
        f->Ca[k] = 1.0; f->Cb[k] = 2.0 * cz;
        f->Ua[k] = 0.0; f->Ub[k] = -cz;
    }
    for (int l = 1; l < S->nlev; ++l) {
        level3_t *p = &S->lev[l - 1], *c = &S->lev[l];
        int nc = p->nz / 2;
        c->Ca = zalloc(nc); c->Cb = zalloc(nc); c->Ua = zalloc(nc); c->Ub = zalloc(nc);
        c->nz = galerkin(p->nz, p->Ca, p->Cb, p->Ua, p->Ub, c->Ca, c->Cb, c->Ua, c->Ub);
    }
    for (int l = 0; l < S->nlev; ++l) {
        level3_t *L = &S->lev[l];
        L->ph = (plane_hier_t *)calloc((size_t)L->nz, sizeof(plane_hier_t));
        for (int k = 0; k < L->nz; ++k) build_plane_hier(&L->ph[k], ny, cx, cy, L->Ca[k], L->Cb[k]);
        if (l > 0) { L->x = zalloc(pl * L->nz); L->b = zalloc(pl * L->nz); }
        L->r = zalloc(pl * L->nz);
    }
#ifdef _OPENMP
    S->nthreads = omp_get_max_threads();
#else
    S->nthreads = 1;
#endif
    S->ws = (ws2_t *)calloc((size_t)S->nthreads, sizeof(ws2_t));
    const int n2 = levels_of(ny);
    for (int t = 0; t < S->nthreads; ++t) {
        ws2_t *w = &S->ws[t];
        w->x = (double **)calloc((size_t)n2, sizeof(double *));
        w->b = (double **)calloc((size_t)n2, sizeof(double *));
        w->r = (double **)calloc((size_t)n2, sizeof(double *));
        int nyl = ny;
        for (int l = 0; l < n2; ++l) {
            w->x[l] = zalloc((size_t)nx * nyl);
            w->b[l] = zalloc((size_t)nx * nyl);
            w->r[l] = zalloc((size_t)nx * nyl);
            nyl /= 2;
        }
        w->rk = zalloc(pl); w->yk = zalloc(pl); w->tmp = zalloc(3 * (size_t)nx);
    }
    return S;
}

void oracle_smg_destroy(oracle_smg *S)
{
    if (!S) return;
    const int n2 = levels_of(S->ny);
    for (int t = 0; t < S->nthreads; ++t) {
        ws2_t *w = &S->ws[t];
        for (int l = 0; l < n2; ++l) { free(w->x[l]); free(w->b[l]); free(w->r[l]); }
        free(w->x); free(w->b); free(w->r); free(w->rk); free(w->yk); free(w->tmp);
    }
    free(S->ws);
    for (int l = 0; l < S->nlev; ++l) {
        level3_t *L = &S->lev[l];
        for (int k = 0; k < L->nz; ++k) free_plane_hier(&L->ph[k]);
        free(L->ph); free(L->Ca); free(L->Cb); free(L->Ua); free(L->Ub);
        free(L->x); free(L->b); free(L->r);
    }
    free(S->lev);
    free(S);
}

/* s = B r : one V-cycle from a zero initial guess */
void oracle_smg_apply(oracle_smg *S, const double *r, double *s) { vcycle3(S, 0, r, s); }

int oracle_smg_nlevels(const oracle_smg *S) { return S->nlev; }
int oracle_smg_level_nz(const oracle_smg *S, int l) { return S->lev[l].nz; }

/* 3D level coefficients: out = {Ca[K], Cb[K], Ua[K], Ub[K]} (Ua/Ub are 0
 * for the last plane, which has no upper neighbour) */
void oracle_smg_plane_coef(const oracle_smg *S, int l, int K, double *out)
{
    const level3_t *L = &S->lev[l];
    out[0] = L->Ca[K]; out[1] = L->Cb[K];
    out[2] = K < L->nz - 1 ? L->Ua[K] : 0.0;
    out[3] = K < L->nz - 1 ? L->Ub[K] : 0.0;
}

int oracle_smg_plane_nlevels(const oracle_smg *S, int l, int K) { return S->lev[l].ph[K].nlev; }
int oracle_smg_plane_level_ny(const oracle_smg *S, int l, int K, int l2) { return S->lev[l].ph[K].lev[l2].ny; }

/* 2D level coefficients of plane K of 3D level l: {La, Lb, Va, Vb} of line j */
void oracle_smg_line_coef(const oracle_smg *S, int l, int K, int l2, int j, double *out)
{
    const level2_t *L = &S->lev[l].ph[K].lev[l2];
    out[0] = L->La[j]; out[1] = L->Lb[j];
    out[2] = j < L->ny - 1 ? L->Va[j] : 0.0;
    out[3] = j < L->ny - 1 ? L->Vb[j] : 0.0;
}

/* One 2D V-cycle (the plane solve) of plane K at 3D level l on a single
 * plane right-hand side b (nx*ny), result in x. */
void oracle_smg_plane_solve(oracle_smg *S, int l, int K, const double *b, double *x)
{
    vcycle2(S, &S->lev[l].ph[K], 0, b, x, &S->ws[0]);
}

/* ------------------------------------------------------------------------- */
/* Algorithm 1 (Section 2): PCG with beta from (1), flexible PCG with (2),   */
/* PSD with beta = 0.  T is the SMG V-cycle, or the identity when S is NULL. */
/* ------------------------------------------------------------------------- */
static double dot(size_t n, const double *a, const double *b)
{
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (size_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

enum { ORACLE_PCG = 0, ORACLE_FPCG = 1, ORACLE_PSD = 2 };

/* Returns 0 converged, 1 max_iter reached, -4 breakdown (non-finite scalar).
 * Stopping test: ||r_k||_2 <= rtol ||b||_2 on the recursive residual, or,
 * with stop_c, sqrt|(s_k, r_k)| <= rtol sqrt|(T b, b)| (the C-norm ratio
 * plotted in Figs. 2 and 5), tested as soon as s_k = T r_k is formed.
 * hist (nullable, max_iter+1 entries) receives ||r_k||_2/||b||_2 for
 * k = 0..iters; histC (nullable, max_iter+1 entries) receives
 * sqrt|(s_k, r_k)| / sqrt|(T b, b)| for every k at which s_k was formed. */
int oracle_krylov(oracle_smg *S, int method, int nx, int ny, int nz, double cx, double cy,
                  double cz, const double *b, double *x, double rtol, int stop_c, int max_iter,
                  double *hist, double *histC, int *iters_out, double *rel_out,
                  double *true_rel_out)
{
    const size_t n = (size_t)nx * ny * nz;
    double *r = zalloc(n), *s = zalloc(n), *p = zalloc(n), *q = zalloc(n), *rp = zalloc(n);
    int status = 1, k = 0, cconv = 0;
    oracle_matvec(nx, ny, nz, cx, cy, cz, x, q);
    for (size_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
    const double bnorm = sqrt(dot(n, b, b));
    const double bden = bnorm > 0.0 ? bnorm : 1.0;
    double rel = sqrt(dot(n, r, r)) / bden;
    double cden = 0.0;
    if (histC || stop_c) {                        /* (T b, b) for the C-norm */
        if (S) oracle_smg_apply(S, b, s); else memcpy(s, b, n * sizeof(double));
        cden = sqrt(fabs(dot(n, s, b)));
        if (cden == 0.0) cden = 1.0;
    }
    if (hist) hist[0] = rel;
    double sr_prev = 0.0;
    for (k = 0; k < max_iter && (stop_c || rel > rtol); ++k) {
        if (S) oracle_smg_apply(S, r, s); else memcpy(s, r, n * sizeof(double));
        const double sr = dot(n, s, r);
        if (histC) histC[k] = sqrt(fabs(sr)) / cden;
        if (stop_c && !(sqrt(fabs(sr)) / cden > rtol)) { cconv = 1; break; }
        double beta = 0.0;
        if (k > 0 && method == ORACLE_PCG) beta = sr / sr_prev;                       /* (1) */
        if (k > 0 && method == ORACLE_FPCG) beta = (sr - dot(n, s, rp)) / sr_prev;    /* (2) */
        if (!isfinite(beta)) { status = -4; break; }
        if (k == 0 || method == ORACLE_PSD) memcpy(p, s, n * sizeof(double));
        else
            for (size_t i = 0; i < n; ++i) p[i] = s[i] + beta * p[i];
        oracle_matvec(nx, ny, nz, cx, cy, cz, p, q);
        const double alpha = sr / dot(n, p, q);
        if (!isfinite(alpha)) { status = -4; break; }
        if (method == ORACLE_FPCG) memcpy(rp, r, n * sizeof(double));
        for (size_t i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        sr_prev = sr;
        rel = sqrt(dot(n, r, r)) / bden;
        if (hist) hist[k + 1] = rel;
    }
    if (status == 1 && (stop_c ? cconv : rel <= rtol)) status = 0;
    oracle_matvec(nx, ny, nz, cx, cy, cz, x, q);
    for (size_t i = 0; i < n; ++i) q[i] = b[i] - q[i];
    if (true_rel_out) *true_rel_out = sqrt(dot(n, q, q)) / bden;
    if (rel_out) *rel_out = rel;
    if (iters_out) *iters_out = k;
    free(r); free(s); free(p); free(q); free(rp);
    return status;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the parallel loops from here on (for timing the oracle on one
 * core beside all of them). */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
