/*
 * pd_oracle.c -- plain, slow FP64 CPU oracle for the bond-based PMB peridynamics step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline of the benchmark may load this library.  It shares no code, header,
 * table or constant with the HIP library; the two meet only through the seeded
 * input generators (module pd_inputs).
 *
 * Built with gcc -O2 -ffp-contract=off (no FMA contraction, no fast-math) so the
 * rounding sequence of every expression below is the one written.  Parallel loops
 * run over rows only; each row's arithmetic and summation order is fixed, so any
 * thread count gives bitwise the same result.
 *
 * What it computes (paper: "PeriPy - a high performance OpenCL peridynamics package"):
 *   family          H_i = { j != i : |x_j - x_i| <= delta }            (Eq. family; self excluded)
 *   kinematics      xi = x_j - x_i, eta = u_j - u_i                    (Sec. 2.1)
 *   stretch         s = (|eta + xi| - |xi|) / |xi|                     (Eq. microelastic)
 *   PMB force       f = c s mu (eta + xi)/|eta + xi|, c = 18K/(pi d^4) (Eq. simpleBond, Sec. 2.2)
 *   breaking        mu = 0 for ever once s >= s_c                      (Eq. mu; the paper's bond
 *                   kernel keeps a bond only while s < s0, and a bond that breaks contributes
 *                   nothing in the pass that breaks it: Algorithm 2)
 *   node force      F_i = sum_j f(eta_ij, xi_ij) V_j + b_i             (Eq. discrete EOM, beta = 1)
 *   damage          phi_i = 1 - sum_j mu_ij V_j / sum_j V_j            (Sec. 2.2, local damage)
 *   integrators     velocity Verlet (Eqs. Velocity_Verlet1-3), Euler-Cromer and forward Euler
 *                   (the integrator classes listed in Sec. 3.6; their update rules are not printed).
 *   damage laws     n-linear softening laws (the laws made of linear spline pieces of
 *                   Sec. 3.6; trilinear in Sec. 6, bilinear in Sec. 7) per bond class, with
 *                   irreversibility through the largest stretch a bond has reached (Sec. 2.2
 *                   reading: the bond follows the secant to the origin once it has softened)
 *   corrections     a conical micromodulus c (1 - |xi|/delta), partial volumes beta(|xi|) of
 *                   neighbours cut by the horizon, and the volume-method surface correction
 *                   lambda_ij = 2 V0 / (V_i + V_j) over family volumes (Sec. 2.5)
 *   quasi-static    prescribed displacements ramped by a fifth-order polynomial in time with
 *   loading         zero initial velocity and acceleration (Examples 2 and 3, Secs. 6-7), and
 *                   'no-failure zones': bonds of flagged nodes never break (Secs. 5.1, 6, 7).
 *   adjoint         reverse-mode derivative of an Euler-Cromer run with the break schedule
 *                   frozen, w.r.t. per-slot stiffness and body-force magnitude.
 *   state-based     the ordinary state-based linear peridynamic solid (Sec. 8.2, after Silling
 *                   et al. 2007): weighted volume m_i = sum_j omega |xi|^2 V_j, dilation
 *                   theta_i = (3/m_i) sum_j omega |xi| e_ij V_j over intact bonds, extension
 *                   e = |xi + eta| - |xi|, scalar force state t_ij = (3 K theta_i / m_i) omega |xi|
 *                   + (15 G / m_i) omega (e - theta_i |xi| / 3), node force sum_j (t_ij + t_ji)
 *                   M_ij V_j with M = (xi + eta)/|xi + eta|; influence function omega = 1.  Two
 *                   passes per force evaluation: breaking and dilation, then the force.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define PDO_EC 0
#define PDO_VV 1
#define PDO_FE 2

#define PDO_MAXB 8  /* breakpoints per damage law */

#define PDO_FREE 0
#define PDO_DISP 1
#define PDO_VEL 2

typedef struct pdo_problem {
    int64_t n;
    const double *x;         /* n*3 reference coordinates (row-major) */
    const double *vol;       /* n   lumped node volumes */
    const int64_t *row_ptr;  /* n+1 CSR row starts */
    const int32_t *col;      /* nnz neighbour ids, ascending within each row */
    const double *kslot;     /* nnz per-slot micromodulus, or NULL: every slot uses c */
    double c;                /* constant micromodulus */
    double s0;               /* critical stretch */
    double rho;              /* density */
    double eta;              /* dynamic-relaxation damping coefficient */
    double dt;               /* time step */
    const double *bhat;      /* n*3 body-force direction field, or NULL */
    double bmag;             /* body-force magnitude: b_i = bmag * bhat_i */
    const uint8_t *bc_kind;  /* n*3: PDO_FREE / PDO_DISP / PDO_VEL, or NULL (no constraints) */
    const uint8_t *bc_sched; /* n*3: 0 -> g(t) = 1, 1 -> g(t) = t, 2 -> fifth-order ramp over ramp_T */
    const double *bc_val;    /* n*3 amplitudes A */
    int32_t scheme;          /* PDO_EC / PDO_VV / PDO_FE */
    int32_t nthreads;        /* <= 0: library default */
    double ramp_T;           /* duration of the fifth-order ramp (schedule 2) */
    const uint8_t *nofail;   /* n or NULL: 1 = no-failure zone, bonds touching the node never break
                                and their damage state does not change */
    /* Damage laws.  ncls = 0: the brittle law with s0 above.  Otherwise class k has
     * cls_nb[k] breakpoints s_0 < s_1 < ... < s_last (cls_s[k * PDO_MAXB + .]) with force
     * ratios r_0 = 1, ..., r_last = 0 (cls_r): the bond force of a monotonic pull is
     * c s up to s_0, then c s_0 times the linear interpolation of the ratios, and the
     * bond is broken from s_last on (one breakpoint: the brittle law with s0 = s_0). */
    int32_t ncls;
    int32_t pad2_;
    const int32_t *cls_nb;
    const double *cls_s;
    const double *cls_r;
    const uint8_t *slot_cls; /* nnz class of each slot, or NULL: class 0 */
    /* Stiffness corrections, each a factor on the slot's stiffness, applied in this order:
     * micro = 1: conical micromodulus max(0, 1 - |xi|/delta); pvol = 1: partial volume
     * beta(|xi|) = 1 up to delta - dx/2, linear down to 0 at delta + dx/2; surf = 1:
     * lambda_ij = 2 V0 / (V_i + V_j) with famvol[] the family volumes and v0 their maximum
     * (pdo_family_volumes). */
    int32_t micro;
    int32_t pvol;
    double delta;
    double pv_dx;
    int32_t surf;
    int32_t pad3_;
    const double *famvol;
    double v0;
    /* model = 1: the ordinary state-based linear solid with bulk modulus K and shear
     * modulus G in place of the PMB bond force (c, kslot, damage laws and corrections are
     * not used); m[] the weighted volumes (pdo_weighted_volumes); theta[] (n) receives the
     * dilation of every node in each force evaluation. */
    int32_t model;
    int32_t pad4_;
    double K;
    double G;
    const double *m;
    double *theta;
} pdo_problem;

typedef struct pdo_state {
    double *u;               /* n*3 displacement */
    double *v;               /* n*3 velocity */
    double *a;               /* n*3 acceleration (velocity Verlet) */
    uint8_t *broken;         /* nnz: 1 once the slot's bond is broken */
    int32_t *break_step;     /* nnz or NULL: pass index at which a slot broke */
    const int32_t *frozen;   /* nnz or NULL: replay, slot alive in pass k iff k < frozen[b] */
    int64_t step;            /* number of completed time steps */
    int32_t a_valid;         /* velocity Verlet: a holds the acceleration of the current u */
    int32_t pad_;
    double *smax;            /* nnz (with damage laws): the largest stretch a slot has reached
                                beyond its elastic limit, 0 while it has not */
} pdo_state;

static void set_threads(const pdo_problem *P)
{
#ifdef _OPENMP
    if (P->nthreads > 0) omp_set_num_threads(P->nthreads);
#else
    (void)P;
#endif
}

/* ------------------------------------------------------------------ family (Eq. family) */

static int within_horizon(const double *x, int64_t i, int64_t j, double d2max)
{
    double a = x[3 * j + 0] - x[3 * i + 0];
    double b = x[3 * j + 1] - x[3 * i + 1];
    double c = x[3 * j + 2] - x[3 * i + 2];
    double d2 = a * a + b * b;
    d2 = d2 + c * c;
    return d2 <= d2max;
}

/* Brute force O(n^2).  With col == NULL only row_ptr is filled; returns nnz. */
int64_t pdo_family_brute(int64_t n, const double *x, double delta, int64_t *row_ptr, int32_t *col)
{
    double d2max = delta * delta;
    if (col == NULL) {
        row_ptr[0] = 0;
        for (int64_t i = 0; i < n; ++i) {
            int64_t cnt = 0;
            for (int64_t j = 0; j < n; ++j)
                if (j != i && within_horizon(x, i, j, d2max)) ++cnt;
            row_ptr[i + 1] = row_ptr[i] + cnt;
        }
        return row_ptr[n];
    }
    for (int64_t i = 0; i < n; ++i) {
        int64_t w = row_ptr[i];
        for (int64_t j = 0; j < n; ++j)
            if (j != i && within_horizon(x, i, j, d2max)) col[w++] = (int32_t)j;
    }
    return row_ptr[n];
}

/* Cell list with cells at least delta wide; rows sorted ascending.  Same contract. */
typedef struct cellgrid {
    double lo[3];
    double h;
    int64_t dim[3];
    int64_t *start;  /* ncell+1 */
    int64_t *items;  /* n, node ids grouped by cell, ascending within a cell */
} cellgrid;

static int64_t cell_coord(const cellgrid *g, double v, int d)
{
    int64_t c = (int64_t)floor((v - g->lo[d]) / g->h);
    if (c < 0) c = 0;
    if (c >= g->dim[d]) c = g->dim[d] - 1;
    return c;
}

static void grid_build(cellgrid *g, int64_t n, const double *x, double delta)
{
    double hi[3];
    for (int d = 0; d < 3; ++d) { g->lo[d] = x[d]; hi[d] = x[d]; }
    for (int64_t i = 1; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            if (x[3 * i + d] < g->lo[d]) g->lo[d] = x[3 * i + d];
            if (x[3 * i + d] > hi[d]) hi[d] = x[3 * i + d];
        }
    /* cells a hair wider than delta, so that rounding in the cell coordinate can
     * never put two nodes within delta of each other two cells apart */
    g->h = delta > 0 ? delta * (1.0 + 1e-9) : 1.0;
    int64_t ncell = 1;
    for (int d = 0; d < 3; ++d) {
        g->dim[d] = (int64_t)floor((hi[d] - g->lo[d]) / g->h) + 1;
        ncell *= g->dim[d];
    }
    g->start = calloc((size_t)ncell + 1, sizeof(int64_t));
    g->items = malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *cid = malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        int64_t cx = cell_coord(g, x[3 * i], 0), cy = cell_coord(g, x[3 * i + 1], 1),
                cz = cell_coord(g, x[3 * i + 2], 2);
        cid[i] = (cz * g->dim[1] + cy) * g->dim[0] + cx;
        g->start[cid[i] + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) g->start[c + 1] += g->start[c];
    int64_t *fill = malloc((size_t)ncell * sizeof(int64_t) + 1);
    memcpy(fill, g->start, (size_t)ncell * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) g->items[fill[cid[i]]++] = i;
    free(fill);
    free(cid);
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

int64_t pdo_family_cells(int64_t n, const double *x, double delta, int64_t *row_ptr, int32_t *col)
{
    cellgrid g;
    double d2max = delta * delta;
    grid_build(&g, n, x, delta);
    if (col == NULL) row_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t cx = cell_coord(&g, x[3 * i], 0), cy = cell_coord(&g, x[3 * i + 1], 1),
                cz = cell_coord(&g, x[3 * i + 2], 2);
        int64_t w = col ? row_ptr[i] : 0;
        for (int64_t z = cz - 1; z <= cz + 1; ++z) {
            if (z < 0 || z >= g.dim[2]) continue;
            for (int64_t y = cy - 1; y <= cy + 1; ++y) {
                if (y < 0 || y >= g.dim[1]) continue;
                for (int64_t xx = cx - 1; xx <= cx + 1; ++xx) {
                    if (xx < 0 || xx >= g.dim[0]) continue;
                    int64_t c = (z * g.dim[1] + y) * g.dim[0] + xx;
                    for (int64_t p = g.start[c]; p < g.start[c + 1]; ++p) {
                        int64_t j = g.items[p];
                        if (j == i || !within_horizon(x, i, j, d2max)) continue;
                        if (col) col[w] = (int32_t)j;
                        ++w;
                    }
                }
            }
        }
        if (col)
            qsort(col + row_ptr[i], (size_t)(w - row_ptr[i]), sizeof(int32_t), cmp_i32);
        else
            row_ptr[i + 1] = row_ptr[i] + w;
    }
    free(g.start);
    free(g.items);
    return row_ptr[n];
}

/* ------------------------------------------------------------------ bond forces */

/* Secant ratio of damage law k at a stretch sm beyond its elastic limit s_0 (and below
 * s_last): the law's force c s_0 rho(sm), rho interpolated linearly between breakpoints,
 * divided by the elastic force c sm. */
static double law_ratio(const pdo_problem *P, int k, double sm)
{
    const double *sb = P->cls_s + k * PDO_MAXB, *rb = P->cls_r + k * PDO_MAXB;
    int seg = 0;
    while (seg + 2 < P->cls_nb[k] && sm >= sb[seg + 1]) ++seg;
    double rho = rb[seg] + (rb[seg + 1] - rb[seg]) * ((sm - sb[seg]) / (sb[seg + 1] - sb[seg]));
    return (sb[0] * rho) / sm;
}

static int slot_class(const pdo_problem *P, int64_t b) { return P->slot_cls ? P->slot_cls[b] : 0; }

/* Partial volume of a neighbour at reference distance L: the share of its cubic cell
 * (side dx, centred on it) inside the horizon, approximated linearly across the shell
 * delta - dx/2 .. delta + dx/2. */
static double partial_volume(const pdo_problem *P, double L)
{
    const double h = 0.5 * P->pv_dx;
    if (L <= P->delta - h) return 1.0;
    if (L >= P->delta + h) return 0.0;
    return (P->delta + h - L) / P->pv_dx;
}

static double bond_length(const double *x, int64_t i, int64_t j)
{
    double a = x[3 * j + 0] - x[3 * i + 0];
    double b = x[3 * j + 1] - x[3 * i + 1];
    double c = x[3 * j + 2] - x[3 * i + 2];
    return sqrt((a * a + b * b) + c * c);
}

/* Family volumes V_i = sum over H_i of beta_ij V_j (beta = 1 without partial volumes);
 * returns their maximum, the volume of a complete family. */
double pdo_family_volumes(const pdo_problem *P, double *famvol)
{
    double vmax = 0.0;
    for (int64_t i = 0; i < P->n; ++i) {
        double v = 0.0;
        for (int64_t b = P->row_ptr[i]; b < P->row_ptr[i + 1]; ++b) {
            const int64_t j = P->col[b];
            v += (P->pvol ? partial_volume(P, bond_length(P->x, i, j)) : 1.0) * P->vol[j];
        }
        famvol[i] = v;
        if (v > vmax) vmax = v;
    }
    return vmax;
}

/* Weighted volumes of the state-based model, m_i = sum over the whole family H_i of
 * omega |xi|^2 V_j with omega = 1 (reference configuration, bonds broken or not). */
void pdo_weighted_volumes(const pdo_problem *P, double *m)
{
    for (int64_t i = 0; i < P->n; ++i) {
        double acc = 0.0;
        for (int64_t b = P->row_ptr[i]; b < P->row_ptr[i + 1]; ++b) {
            const double L = bond_length(P->x, i, P->col[b]);
            acc += L * L * P->vol[P->col[b]];
        }
        m[i] = acc;
    }
}

/* Damage of a slot under the damage laws: 1 broken, 1 - secant ratio once softened. */
static double slot_damage(const pdo_problem *P, const uint8_t *broken, const double *smax, int64_t b)
{
    if (broken[b]) return 1.0;
    if (P->ncls > 0 && smax && smax[b] > 0.0) return 1.0 - law_ratio(P, slot_class(P, b), smax[b]);
    return 0.0;
}

/* Force density of every node for displacement u, in pass k (the index of the time
 * level u belongs to).  Without a frozen schedule, a slot whose stretch reaches s0
 * is marked broken (and its pass recorded) and contributes nothing; with a frozen
 * schedule, the slot is alive in pass k iff k < frozen[b]. */
static void lps_force(const pdo_problem *P, pdo_state *S, const double *u, int64_t k, double *F);

void pdo_force(const pdo_problem *P, pdo_state *S, const double *u, int64_t k, double *F)
{
    const double *x = P->x;
    set_threads(P);
    if (P->model == 1) {
        lps_force(P, S, u, k, F);
        return;
    }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < P->n; ++i) {
        double f0 = 0.0, f1 = 0.0, f2 = 0.0;
        for (int64_t b = P->row_ptr[i]; b < P->row_ptr[i + 1]; ++b) {
            if (S->frozen) {
                if (!(k < (int64_t)S->frozen[b])) continue;
            } else if (S->broken[b]) {
                continue;
            }
            int64_t j = P->col[b];
            double xi0 = x[3 * j + 0] - x[3 * i + 0];
            double xi1 = x[3 * j + 1] - x[3 * i + 1];
            double xi2 = x[3 * j + 2] - x[3 * i + 2];
            double y0 = xi0 + (u[3 * j + 0] - u[3 * i + 0]);
            double y1 = xi1 + (u[3 * j + 1] - u[3 * i + 1]);
            double y2 = xi2 + (u[3 * j + 2] - u[3 * i + 2]);
            double r = sqrt((y0 * y0 + y1 * y1) + y2 * y2);
            double L = sqrt((xi0 * xi0 + xi1 * xi1) + xi2 * xi2);
            double s = (r - L) / L;
            const int unbreakable = P->nofail && (P->nofail[i] || P->nofail[j]);
            double w = 1.0;  /* secant ratio of a softened bond */
            if (P->ncls > 0) {
                const int cl = slot_class(P, b);
                const double s_first = P->cls_s[cl * PDO_MAXB];
                const double s_last = P->cls_s[cl * PDO_MAXB + P->cls_nb[cl] - 1];
                if (S->frozen || unbreakable) {  /* damage state as it stands */
                    if (S->smax[b] > 0.0) w = law_ratio(P, cl, S->smax[b]);
                } else {
                    double sm = s > S->smax[b] ? s : S->smax[b];
                    if (sm >= s_last) {
                        S->broken[b] = 1;
                        if (S->break_step) S->break_step[b] = (int32_t)k;
                        continue;
                    }
                    if (sm > s_first) {
                        S->smax[b] = sm;
                        w = law_ratio(P, cl, sm);
                    }
                }
            } else if (!S->frozen && !unbreakable && s >= P->s0) {
                S->broken[b] = 1;
                if (S->break_step) S->break_step[b] = (int32_t)k;
                continue;
            }
            double kb = P->kslot ? P->kslot[b] : P->c;
            if (P->micro == 1) {
                const double m = 1.0 - L / P->delta;
                kb = kb * (m > 0.0 ? m : 0.0);
            }
            if (P->pvol) kb = kb * partial_volume(P, L);
            if (P->surf) kb = kb * ((2.0 * P->v0) / (P->famvol[i] + P->famvol[j]));
            double scal = (((kb * s) * w) * P->vol[j]) / r;
            f0 += scal * y0;
            f1 += scal * y1;
            f2 += scal * y2;
        }
        if (P->bhat) {
            f0 += P->bmag * P->bhat[3 * i + 0];
            f1 += P->bmag * P->bhat[3 * i + 1];
            f2 += P->bmag * P->bhat[3 * i + 2];
        }
        F[3 * i + 0] = f0;
        F[3 * i + 1] = f1;
        F[3 * i + 2] = f2;
    }
}

/* Deformed bond of slot (i, j): y = xi + eta, its length r and the reference length L. */
static void deformed_bond(const double *x, const double *u, int64_t i, int64_t j, double y[3], double *r, double *L)
{
    double xi[3];
    for (int d = 0; d < 3; ++d) {
        xi[d] = x[3 * j + d] - x[3 * i + d];
        y[d] = xi[d] + (u[3 * j + d] - u[3 * i + d]);
    }
    *r = sqrt((y[0] * y[0] + y[1] * y[1]) + y[2] * y[2]);
    *L = sqrt((xi[0] * xi[0] + xi[1] * xi[1]) + xi[2] * xi[2]);
}

/* The state-based force density (see the header), in pass k.  First pass: a slot whose
 * stretch e / |xi| reaches s0 breaks (as in the bond-based model: outside no-failure
 * zones, never with a frozen schedule), then the dilation of every node sums the bonds
 * still intact.  Second pass: every intact bond adds (t_ij + t_ji) M_ij V_j, t_ji formed
 * with node j's dilation and weighted volume. */
static void lps_force(const pdo_problem *P, pdo_state *S, const double *u, int64_t k, double *F)
{
    const double *x = P->x;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < P->n; ++i) {
        double acc = 0.0;
        for (int64_t b = P->row_ptr[i]; b < P->row_ptr[i + 1]; ++b) {
            if (S->frozen) {
                if (!(k < (int64_t)S->frozen[b])) continue;
            } else if (S->broken[b]) {
                continue;
            }
            const int64_t j = P->col[b];
            double y[3], r, L;
            deformed_bond(x, u, i, j, y, &r, &L);
            const double e = r - L;
            const int unbreakable = P->nofail && (P->nofail[i] || P->nofail[j]);
            if (!S->frozen && !unbreakable && e / L >= P->s0) {
                S->broken[b] = 1;
                if (S->break_step) S->break_step[b] = (int32_t)k;
                continue;
            }
            acc += L * e * P->vol[j];  /* omega = 1 */
        }
        P->theta[i] = 3.0 * acc / P->m[i];
    }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < P->n; ++i) {
        double f[3] = {0.0, 0.0, 0.0};
        for (int64_t b = P->row_ptr[i]; b < P->row_ptr[i + 1]; ++b) {
            if (S->frozen) {
                if (!(k < (int64_t)S->frozen[b])) continue;
            } else if (S->broken[b]) {
                continue;
            }
            const int64_t j = P->col[b];
            double y[3], r, L;
            deformed_bond(x, u, i, j, y, &r, &L);
            const double e = r - L;
            const double th_i = P->theta[i], th_j = P->theta[j];
            const double t_ij = (3.0 * P->K * th_i / P->m[i]) * L + (15.0 * P->G / P->m[i]) * (e - th_i * L / 3.0);
            const double t_ji = (3.0 * P->K * th_j / P->m[j]) * L + (15.0 * P->G / P->m[j]) * (e - th_j * L / 3.0);
            const double scal = (t_ij + t_ji) * P->vol[j] / r;
            for (int d = 0; d < 3; ++d) f[d] += scal * y[d];
        }
        for (int d = 0; d < 3; ++d) {
            if (P->bhat) f[d] += P->bmag * P->bhat[3 * i + d];
            F[3 * i + d] = f[d];
        }
    }
}

/* ------------------------------------------------------------------ boundary conditions */

static int bc_kind(const pdo_problem *P, int64_t i, int d)
{
    return P->bc_kind ? P->bc_kind[3 * i + d] : PDO_FREE;
}

/* Time schedules g(t) of a prescribed quantity and their derivatives:
 *   0: g = 1;   1: g = t;
 *   2: the fifth-order ramp from 0 to 1 over [0, T] whose first and second derivatives
 *      vanish at both ends, g = tau^3 (10 - 15 tau + 6 tau^2) with tau = t / T, and g = 1
 *      from T on (the boundary displacement ramp of Secs. 6-7). */
static double sched_g(const pdo_problem *P, int sched, double t)
{
    if (sched == 1) return t;
    if (sched == 2) {
        if (t >= P->ramp_T) return 1.0;
        double tau = t / P->ramp_T;
        return tau * tau * tau * (10.0 - 15.0 * tau + 6.0 * tau * tau);
    }
    return 1.0;
}

static double sched_dg(const pdo_problem *P, int sched, double t)
{
    if (sched == 1) return 1.0;
    if (sched == 2) {
        if (t >= P->ramp_T) return 0.0;
        double tau = t / P->ramp_T;
        return 30.0 * tau * tau * (1.0 - tau) * (1.0 - tau) / P->ramp_T;
    }
    return 0.0;
}

/* Prescribed velocity of a constrained component at time t. */
static double bc_velocity(const pdo_problem *P, int64_t i, int d, double t)
{
    double A = P->bc_val[3 * i + d];
    int sc = P->bc_sched[3 * i + d];
    if (P->bc_kind[3 * i + d] == PDO_DISP) return A * sched_dg(P, sc, t);
    return A * sched_g(P, sc, t);
}

/* Prescribed displacement at time t; uprev is the component's displacement one step earlier. */
static double bc_displacement(const pdo_problem *P, int64_t i, int d, double t, double uprev)
{
    double A = P->bc_val[3 * i + d];
    int sc = P->bc_sched[3 * i + d];
    if (P->bc_kind[3 * i + d] == PDO_DISP) return A * sched_g(P, sc, t);
    return uprev + P->dt * (A * sched_g(P, sc, t));
}

/* ------------------------------------------------------------------ time integration */

static int64_t nnz_of(const pdo_problem *P) { return P->row_ptr[P->n]; }

/* One step k -> k+1.  Returns 0. */
static int step_once(const pdo_problem *P, pdo_state *S, double *F, double *unew)
{
    const int64_t n = P->n;
    const int64_t k = S->step;
    const double dt = P->dt;
    const double t1 = (double)(k + 1) * dt;

    if (P->scheme == PDO_EC || P->scheme == PDO_FE) {
        pdo_force(P, S, S->u, k, F);
        for (int64_t i = 0; i < n; ++i)
            for (int d = 0; d < 3; ++d) {
                int64_t q = 3 * i + d;
                double a = (F[q] - P->eta * S->v[q]) / P->rho;
                double u0 = S->u[q];
                double un, vn;
                if (P->scheme == PDO_EC) {
                    vn = S->v[q] + dt * a;
                    un = u0 + dt * vn;
                } else {
                    un = u0 + dt * S->v[q];
                    vn = S->v[q] + dt * a;
                }
                if (bc_kind(P, i, d) != PDO_FREE) {
                    vn = bc_velocity(P, i, d, t1);
                    un = bc_displacement(P, i, d, t1, u0);
                }
                S->u[q] = un;
                S->v[q] = vn;
            }
        S->step = k + 1;
        return 0;
    }

    /* velocity Verlet (Eqs. Velocity_Verlet1-3): position, force at the new position, velocity */
    if (!S->a_valid) {
        pdo_force(P, S, S->u, k, F);
        for (int64_t i = 0; i < n; ++i)
            for (int d = 0; d < 3; ++d) {
                int64_t q = 3 * i + d;
                S->a[q] = bc_kind(P, i, d) != PDO_FREE ? 0.0 : (F[q] - P->eta * S->v[q]) / P->rho;
            }
        S->a_valid = 1;
    }
    const double half_dt = 0.5 * dt;
    const double half_dt2 = 0.5 * dt * dt;
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            int64_t q = 3 * i + d;
            double un = (S->u[q] + dt * S->v[q]) + half_dt2 * S->a[q];
            if (bc_kind(P, i, d) != PDO_FREE) un = bc_displacement(P, i, d, t1, S->u[q]);
            unew[q] = un;
        }
    pdo_force(P, S, unew, k + 1, F);
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            int64_t q = 3 * i + d;
            double vhalf = S->v[q] + half_dt * S->a[q];
            double an = (F[q] - P->eta * vhalf) / P->rho;
            double vn = S->v[q] + half_dt * (S->a[q] + an);
            if (bc_kind(P, i, d) != PDO_FREE) {
                vn = bc_velocity(P, i, d, t1);
                an = 0.0;
            }
            S->u[q] = unew[q];
            S->v[q] = vn;
            S->a[q] = an;
        }
    S->step = k + 1;
    return 0;
}

/* Advance nsteps steps.  Returns 0, or -1 if the state became non-finite (the
 * step index is left at the first non-finite step). */
int pdo_run(const pdo_problem *P, pdo_state *S, int64_t nsteps)
{
    const int64_t n3 = 3 * P->n;
    double *F = malloc((size_t)(n3 > 0 ? n3 : 1) * sizeof(double));
    double *unew = malloc((size_t)(n3 > 0 ? n3 : 1) * sizeof(double));
    int rc = 0;
    for (int64_t s = 0; s < nsteps; ++s) {
        step_once(P, S, F, unew);
        for (int64_t q = 0; q < n3; ++q)
            if (!isfinite(S->u[q]) || !isfinite(S->v[q])) { rc = -1; break; }
        if (rc) break;
    }
    free(F);
    free(unew);
    return rc;
}

/* ------------------------------------------------------------------ damage */

/* phi_i = 1 - sum_j (1 - d_ij) V_j / sum_j V_j over the initial family: d = 1 for a
 * broken bond, 1 - secant ratio for a softened one (smax may be NULL: brittle), 0
 * otherwise.  With the brittle law this is 1 - sum_j mu_ij V_j / sum_j V_j. */
void pdo_damage(const pdo_problem *P, const uint8_t *broken, const double *smax, double *phi)
{
    for (int64_t i = 0; i < P->n; ++i) {
        double num = 0.0, den = 0.0;
        for (int64_t b = P->row_ptr[i]; b < P->row_ptr[i + 1]; ++b) {
            double vj = P->vol[P->col[b]];
            den += vj;
            const double d = slot_damage(P, broken, smax, b);
            if (d == 0.0)
                num += vj;
            else if (d < 1.0)
                num += (1.0 - d) * vj;
        }
        phi[i] = den > 0.0 ? 1.0 - num / den : 0.0;
    }
}

/* ------------------------------------------------------------------ adjoint (Euler-Cromer) */

/* out = J_F(u)^T nu in pass k with the frozen schedule, written as the literal
 * transpose of the Jacobian: every slot b = (i, j) has dF_i/du_j = k_b V_j K_b and
 * dF_i/du_i -= k_b V_j K_b, K_b = (1/L - 1/r) I + y y^T / r^3 (the derivative of
 * y/L - y/r with respect to y).  Single-threaded scatter. */
void pdo_apply_jt(const pdo_problem *P, const int32_t *frozen, const double *u, int64_t k,
                  const double *nu, double *out)
{
    const double *x = P->x;
    memset(out, 0, (size_t)(3 * P->n) * sizeof(double));
    for (int64_t i = 0; i < P->n; ++i) {
        for (int64_t b = P->row_ptr[i]; b < P->row_ptr[i + 1]; ++b) {
            if (!(k < (int64_t)frozen[b])) continue;
            int64_t j = P->col[b];
            double xi[3], y[3];
            for (int d = 0; d < 3; ++d) {
                xi[d] = x[3 * j + d] - x[3 * i + d];
                y[d] = xi[d] + (u[3 * j + d] - u[3 * i + d]);
            }
            double r = sqrt((y[0] * y[0] + y[1] * y[1]) + y[2] * y[2]);
            double L = sqrt((xi[0] * xi[0] + xi[1] * xi[1]) + xi[2] * xi[2]);
            double kb = P->kslot ? P->kslot[b] : P->c;
            double w = kb * P->vol[j];
            double diag = 1.0 / L - 1.0 / r;
            double r3 = r * r * r;
            /* (K_b nu_i) */
            double yn = y[0] * nu[3 * i + 0] + y[1] * nu[3 * i + 1] + y[2] * nu[3 * i + 2];
            for (int d = 0; d < 3; ++d) {
                double kn = diag * nu[3 * i + d] + y[d] * yn / r3;
                out[3 * j + d] += w * kn;   /* (dF_i/du_j)^T nu_i */
                out[3 * i + d] -= w * kn;   /* (dF_i/du_i)^T nu_i */
            }
        }
    }
}

/* Gradient of L = sum over sensors of |u^T - target|^2 after nsteps Euler-Cromer
 * steps from (u0, v0) at step index step0, with the break schedule frozen.  The
 * caller passes dL/du^T for the m sensor nodes (m*3).  Outputs the gradient with
 * respect to every slot's stiffness (grad_k, nnz; the problem must carry kslot)
 * and with respect to the body-force magnitude (grad_A).  The whole trajectory is
 * stored.  Returns 0, or -1 on allocation failure. */
int pdo_adjoint_ec(const pdo_problem *P, const int32_t *frozen, int64_t nsteps,
                   const double *u0, const double *v0, int64_t step0,
                   int64_t m, const int64_t *sensors, const double *dLdu,
                   double *grad_k, double *grad_A)
{
    const int64_t n = P->n, n3 = 3 * n, nnz = nnz_of(P);
    const double dt = P->dt;
    double *traj = malloc((size_t)(nsteps > 0 ? nsteps : 1) * (size_t)n3 * sizeof(double));
    double *F = malloc((size_t)(n3 > 0 ? n3 : 1) * sizeof(double));
    double *unew = malloc((size_t)(n3 > 0 ? n3 : 1) * sizeof(double));
    double *lu = calloc((size_t)(n3 > 0 ? n3 : 1), sizeof(double));
    double *lv = calloc((size_t)(n3 > 0 ? n3 : 1), sizeof(double));
    double *nu = malloc((size_t)(n3 > 0 ? n3 : 1) * sizeof(double));
    double *jt = malloc((size_t)(n3 > 0 ? n3 : 1) * sizeof(double));
    if (!traj || !F || !unew || !lu || !lv || !nu || !jt) {
        free(traj); free(F); free(unew); free(lu); free(lv); free(nu); free(jt);
        return -1;
    }
    pdo_problem Q = *P;
    Q.scheme = PDO_EC;
    pdo_state S;
    memset(&S, 0, sizeof S);
    S.u = malloc((size_t)(n3 > 0 ? n3 : 1) * sizeof(double));
    S.v = malloc((size_t)(n3 > 0 ? n3 : 1) * sizeof(double));
    S.frozen = frozen;
    S.step = step0;
    memcpy(S.u, u0, (size_t)n3 * sizeof(double));
    memcpy(S.v, v0, (size_t)n3 * sizeof(double));
    for (int64_t s = 0; s < nsteps; ++s) {
        memcpy(traj + (size_t)s * n3, S.u, (size_t)n3 * sizeof(double));
        step_once(&Q, &S, F, unew);
    }
    for (int64_t p = 0; p < m; ++p)
        for (int d = 0; d < 3; ++d) lu[3 * sensors[p] + d] += dLdu[3 * p + d];
    memset(grad_k, 0, (size_t)nnz * sizeof(double));
    double gA = 0.0;
    double *gAi = calloc((size_t)(n > 0 ? n : 1), sizeof(double));  /* per-node load-gradient terms */
    if (!gAi) {
        free(traj); free(F); free(unew); free(lu); free(lv); free(nu); free(jt);
        free(S.u); free(S.v);
        return -1;
    }
    set_threads(P);
    const double h = dt / P->rho;
    const double damp = 1.0 - dt * P->eta / P->rho;
    for (int64_t s = nsteps - 1; s >= 0; --s) {
        const int64_t k = step0 + s;
        const double *u = traj + (size_t)s * n3;
        /* nu = adjoint of the unconstrained new velocity.  A prescribed component
         * passes nothing to the new velocity; a displacement-controlled one passes
         * nothing back to u^k either, a velocity-controlled one (u' = u + dt V) does. */
        for (int64_t i = 0; i < n; ++i)
            for (int d = 0; d < 3; ++d) {
                int64_t q = 3 * i + d;
                int kind = bc_kind(P, i, d);
                if (kind == PDO_FREE) {
                    nu[q] = lv[q] + dt * lu[q];
                } else {
                    nu[q] = 0.0;
                    if (kind == PDO_DISP) lu[q] = 0.0;
                }
            }
        /* parameter gradients: dF_i/dk_b = V_j s y / r, dF_i/dA = bhat_i (rows in parallel:
         * each row updates only its own slots; the load terms are summed in node order below) */
#pragma omp parallel for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i) {
            for (int64_t b = P->row_ptr[i]; b < P->row_ptr[i + 1]; ++b) {
                if (!(k < (int64_t)frozen[b])) continue;
                int64_t j = P->col[b];
                double xi[3], y[3];
                for (int d = 0; d < 3; ++d) {
                    xi[d] = P->x[3 * j + d] - P->x[3 * i + d];
                    y[d] = xi[d] + (u[3 * j + d] - u[3 * i + d]);
                }
                double r = sqrt((y[0] * y[0] + y[1] * y[1]) + y[2] * y[2]);
                double L = sqrt((xi[0] * xi[0] + xi[1] * xi[1]) + xi[2] * xi[2]);
                double sv = ((r - L) / L) * P->vol[j] / r;
                grad_k[b] += h * sv * (y[0] * nu[3 * i] + y[1] * nu[3 * i + 1] + y[2] * nu[3 * i + 2]);
            }
            gAi[i] = P->bhat ? h * (P->bhat[3 * i] * nu[3 * i] + P->bhat[3 * i + 1] * nu[3 * i + 1] +
                                    P->bhat[3 * i + 2] * nu[3 * i + 2])
                             : 0.0;
        }
        if (P->bhat)
            for (int64_t i = 0; i < n; ++i) gA += gAi[i];
        pdo_apply_jt(P, frozen, u, k, nu, jt);
        for (int64_t q = 0; q < n3; ++q) {
            lu[q] = lu[q] + h * jt[q];
            lv[q] = damp * nu[q];
        }
    }
    *grad_A = gA;
    free(gAi);
    free(traj); free(F); free(unew); free(lu); free(lv); free(nu); free(jt);
    free(S.u); free(S.v);
    return 0;
}
