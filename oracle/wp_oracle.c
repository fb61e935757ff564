/*
 * wp_oracle.c -- plain FP64 CPU oracle for the wave-propagation patch update.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or table with the HIP library and is written for reading, not speed.
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math), so
 * every product and sum is rounded as written.
 *
 * What it computes (Davis & LeVeque, Sec. 3 "Numerical Methods", and the
 * high-resolution wave-propagation method it cites, LeVeque 1997 / LeVeque
 * 2002 ch. 6, 9, 15, 20-21):
 *   - at every cell edge a Riemann problem splits the jump (wave form) or the
 *     flux difference (f-wave form) into waves W^p with speeds s^p, giving the
 *     fluctuations A^-dQ (waves with s<0) and A^+dQ (s>0);
 *   - second-order correction fluxes  Ftilde = 1/2 sum_p |s|(1-dt/dx|s|) Wlim
 *     (f-wave form: sgn(s) instead of |s|), Wlim = phi(theta) W with the MC
 *     limiter phi(theta) = max(0, min((1+theta)/2, 2, 2 theta)) and
 *     theta = (W_upwind . W)/(W . W);
 *   - in 2D the transverse Riemann problem: each normal fluctuation is split
 *     into up- and down-going parts with the eigenvectors of the neighbouring
 *     cells, and 1/2 dt/dx of them is subtracted from the transverse
 *     correction fluxes;
 *   - the cell update
 *       Q^{n+1} = Q - dt/dx [A+dQ_{i-1/2} + A-dQ_{i+1/2}]
 *                   - dt/dy [B+dQ_{j-1/2} + B-dQ_{j+1/2}]
 *                   - dt/dx [F_{i+1/2} - F_{i-1/2}] - dt/dy [G_{j+1/2} - G_{j-1/2}].
 *
 * Equations: variable-coefficient acoustics q_t + A(x)q_x (+ B(x)q_y) = 0 in
 * non-conservative wave form (Sec. 5.1, 5.2 coefficient matrices); its
 * time-reversed adjoint q~_t - (A^T q~)_x - (B^T q~)_y = 0 in f-wave form
 * (Sec. 2 adjoint equation, Sec. 4 time reversal); nonlinear shallow water
 * (eq. swe, Sec. 5.3) with a well-balanced f-wave Roe solver; and the
 * linearised shallow-water adjoint (Sec. 5.3 linearised system).
 *
 * Array layout: every field is (nx+4) x (ny+4) with two ghost layers,
 * row-major, x fastest; a state is m such fields back to back.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NG 2
#define MAXM 3
#define MAXW 3

typedef struct {
    int nx, ny, NX, NY;
} grid_t;

static inline long gidx(const grid_t *g, int i, int j) {
    return (long)(i + NG) + (long)(j + NG) * g->NX;
}

/* ------------------------------------------------------------------------ */
/* Boundary conditions (Sec. 5.1 walls; Sec. 5.2.3 outflow; ghost-cell      */
/* methodology, Sec. 1/3).  x-direction ghosts for the interior rows first, */
/* then y-direction ghosts for every column including the x ghosts, so that */
/* corner ghosts are defined.                                                */
/*   0 extrapolation: ghost = nearest interior cell                         */
/*   1 wall: mirror image, normal velocity negated                           */
/*   2 periodic                                                              */
/* ------------------------------------------------------------------------ */
static void fill_ghosts_field(const grid_t *g, double *f, const int bc[4], double sx, double sy)
{
    int nx = g->nx, ny = g->ny;
    for (int j = 0; j < ny; j++) {
        for (int k = 1; k <= NG; k++) {
            long lo = gidx(g, -k, j), hi = gidx(g, nx - 1 + k, j);
            switch (bc[0]) {
            case 0: f[lo] = f[gidx(g, 0, j)]; break;
            case 1: f[lo] = sx * f[gidx(g, k - 1, j)]; break;
            default: f[lo] = f[gidx(g, nx - k, j)]; break;
            }
            switch (bc[1]) {
            case 0: f[hi] = f[gidx(g, nx - 1, j)]; break;
            case 1: f[hi] = sx * f[gidx(g, nx - k, j)]; break;
            default: f[hi] = f[gidx(g, k - 1, j)]; break;
            }
        }
    }
    for (int i = -NG; i < nx + NG; i++) {
        for (int k = 1; k <= NG; k++) {
            long lo = gidx(g, i, -k), hi = gidx(g, i, ny - 1 + k);
            switch (bc[2]) {
            case 0: f[lo] = f[gidx(g, i, 0)]; break;
            case 1: f[lo] = sy * f[gidx(g, i, k - 1)]; break;
            default: f[lo] = f[gidx(g, i, ny - k)]; break;
            }
            switch (bc[3]) {
            case 0: f[hi] = f[gidx(g, i, ny - 1)]; break;
            case 1: f[hi] = sy * f[gidx(g, i, ny - k)]; break;
            default: f[hi] = f[gidx(g, i, k - 1)]; break;
            }
        }
    }
}

/* 1D ghost fill of a field of length nx+4 (same rules, x only). */
static void fill_ghosts_1d(int nx, double *f, int bclo, int bchi, double sx)
{
    for (int k = 1; k <= NG; k++) {
        int lo = NG - k, hi = NG + nx - 1 + k;
        if (bclo == 0) f[lo] = f[NG];
        else if (bclo == 1) f[lo] = sx * f[NG + k - 1];
        else f[lo] = f[NG + nx - k];
        if (bchi == 0) f[hi] = f[NG + nx - 1];
        else if (bchi == 1) f[hi] = sx * f[NG + nx - k];
        else f[hi] = f[NG + k - 1];
    }
}

/* Fill ghosts of an m-component state; component `ucomp` changes sign at an
 * x wall and `vcomp` at a y wall (-1: none). */
void or_fill_ghosts(int m, int nx, int ny, double *q, const int *bc, int ucomp, int vcomp)
{
    grid_t g = {nx, ny, nx + 2 * NG, ny + 2 * NG};
    long n = (long)g.NX * g.NY;
    for (int k = 0; k < m; k++)
        fill_ghosts_field(&g, q + k * n, bc, k == ucomp ? -1.0 : 1.0, k == vcomp ? -1.0 : 1.0);
}

/* ------------------------------------------------------------------------ */
/* Riemann solvers.  Each returns, for one edge between cell l (left/below) */
/* and cell r (right/above) in direction dir (0 = x, 1 = y):                */
/*   nw waves wave[p][k], speeds s[p], fluctuations amdq, apdq.             */
/* aux per cell: acoustics {Z, c, rho, K}; swe {B}; lswe {hbar, c}.          */
/* ------------------------------------------------------------------------ */
#define NAUX 4

typedef struct {
    int m, nw, fwave;
    void (*rp)(int dir, const double *ql, const double *qr, const double *al, const double *ar,
               double wave[MAXW][MAXM], double s[MAXW], double *amdq, double *apdq, double g);
    /* transverse split of the fluctuation d, which lives in cell `own`, into
     * the parts crossing the edge to the `lo` neighbour (bm, negative speeds)
     * and to the `hi` neighbour (bp), along direction tdir.  ql/qr/al/ar are
     * the two cells of the normal edge the fluctuation came from. */
    void (*tsplit)(int tdir, const double *d, const double *alo, const double *aown, const double *ahi,
                   const double *ql, const double *qr, const double *al, const double *ar,
                   double *bm, double *bp, double g);
} solver_t;

static void split_fluct(int m, int nw, double wave[MAXW][MAXM], const double s[MAXW], double *amdq, double *apdq)
{
    for (int k = 0; k < m; k++) { amdq[k] = 0.0; apdq[k] = 0.0; }
    for (int p = 0; p < nw; p++) {
        for (int k = 0; k < m; k++) {
            if (s[p] < 0.0) amdq[k] += wave[p][k];
            else if (s[p] > 0.0) apdq[k] += wave[p][k];
            else { amdq[k] += 0.5 * wave[p][k]; apdq[k] += 0.5 * wave[p][k]; }
        }
    }
}

/* --- forward acoustics, wave form (Sec. 5.1/5.2 matrices A, B) ----------- */
/* x-edge: dQ = W1 + W2, W1 = a1 (-Z_l, 1, 0) at speed -c_l,
 *                        W2 = a2 ( Z_r, 1, 0) at speed +c_r.                */
static void rp_acou_fwd(int dir, const double *ql, const double *qr, const double *al, const double *ar,
                        double wave[MAXW][MAXM], double s[MAXW], double *amdq, double *apdq, double g)
{
    (void)g;
    int n = dir == 0 ? 1 : 2, t = dir == 0 ? 2 : 1;
    double Zl = al[0], Zr = ar[0];
    double dp = qr[0] - ql[0], dun = qr[n] - ql[n];
    double a1 = (-dp + Zr * dun) / (Zl + Zr);
    double a2 = (dp + Zl * dun) / (Zl + Zr);
    wave[0][0] = -a1 * Zl; wave[0][n] = a1; wave[0][t] = 0.0;
    wave[1][0] = a2 * Zr;  wave[1][n] = a2; wave[1][t] = 0.0;
    s[0] = -al[1];
    s[1] = ar[1];
    for (int k = 0; k < 3; k++) { amdq[k] = s[0] * wave[0][k]; apdq[k] = s[1] * wave[1][k]; }
}

/* transverse: d lives in cell own; split at the lo edge with eigenvectors
 * (-Z_lo, .., 1) [into lo, speed -c_lo] and (Z_own, .., 1); at the hi edge with
 * (-Z_own, .., 1) and (Z_hi, .., 1) [into hi, speed +c_hi]. */
static void ts_acou_fwd(int tdir, const double *d, const double *alo, const double *aown, const double *ahi,
                        const double *ql, const double *qr, const double *al, const double *ar,
                        double *bm, double *bp, double g)
{
    (void)ql; (void)qr; (void)al; (void)ar; (void)g;
    int n = tdir == 0 ? 1 : 2, t = tdir == 0 ? 2 : 1;
    double Zlo = alo[0], Zo = aown[0], Zhi = ahi[0];
    double bmin = (-d[0] + Zo * d[n]) / (Zlo + Zo);
    double bplus = (d[0] + Zo * d[n]) / (Zo + Zhi);
    double sm = -alo[1], sp = ahi[1];
    bm[0] = sm * bmin * (-Zlo); bm[n] = sm * bmin; bm[t] = 0.0;
    bp[0] = sp * bplus * Zhi;   bp[n] = sp * bplus; bp[t] = 0.0;
}

/* --- adjoint acoustics, time reversed, f-wave form (Sec. 2, 4) ----------- */
/* flux of the reversed adjoint: f = -A^T q = -(u/rho, K p, 0) in x,
 * g = -B^T q = -(v/rho, 0, K p) in y.  Eigenvectors of -A^T: (1, Z, 0) at
 * speed -c and (1, -Z, 0) at speed +c.
 * dF = b1 (1, Z_l, 0) + b2 (1, -Z_r, 0). */
static void rp_acou_adj(int dir, const double *ql, const double *qr, const double *al, const double *ar,
                        double wave[MAXW][MAXM], double s[MAXW], double *amdq, double *apdq, double g)
{
    (void)g;
    int n = dir == 0 ? 1 : 2, t = dir == 0 ? 2 : 1;
    double Zl = al[0], Zr = ar[0];
    double f1l = -ql[n] / al[2], f1r = -qr[n] / ar[2];
    double f2l = -al[3] * ql[0], f2r = -ar[3] * qr[0];
    double df1 = f1r - f1l, df2 = f2r - f2l;
    double b1 = (Zr * df1 + df2) / (Zl + Zr);
    double b2 = (Zl * df1 - df2) / (Zl + Zr);
    wave[0][0] = b1; wave[0][n] = b1 * Zl;  wave[0][t] = 0.0;
    wave[1][0] = b2; wave[1][n] = -b2 * Zr; wave[1][t] = 0.0;
    s[0] = -al[1];
    s[1] = ar[1];
    for (int k = 0; k < 3; k++) { amdq[k] = wave[0][k]; apdq[k] = wave[1][k]; }
}

/* lo edge: d = g1 (1, Z_lo) + g2 (1, -Z_own)  -> down part -c_lo g1 (1, Z_lo)
 * hi edge: d = g1 (1, Z_own) + g2 (1, -Z_hi)  -> up part  +c_hi g2 (1, -Z_hi) */
static void ts_acou_adj(int tdir, const double *d, const double *alo, const double *aown, const double *ahi,
                        const double *ql, const double *qr, const double *al, const double *ar,
                        double *bm, double *bp, double g)
{
    (void)ql; (void)qr; (void)al; (void)ar; (void)g;
    int n = tdir == 0 ? 1 : 2, t = tdir == 0 ? 2 : 1;
    double Zlo = alo[0], Zo = aown[0], Zhi = ahi[0];
    double gm = (Zo * d[0] + d[n]) / (Zlo + Zo);
    double gp = (Zo * d[0] - d[n]) / (Zo + Zhi);
    double sm = -alo[1], sp = ahi[1];
    bm[0] = sm * gm; bm[n] = sm * gm * Zlo;  bm[t] = 0.0;
    bp[0] = sp * gp; bp[n] = -sp * gp * Zhi; bp[t] = 0.0;
}

/* --- shallow water, f-wave Roe solver, well balanced (eq. swe) ----------- */
/* State (eta, hu, hv), h = eta - B.  x-edge Roe state h_bar, u_hat, v_hat,
 * c_hat = sqrt(g h_bar).  The flux difference minus the bathymetry source,
 *   delta = (d(hu), d(hu^2) + g h_bar d(eta), d(huv)),
 * uses 1/2 g (h_r^2 - h_l^2) + g h_bar dB = g h_bar d(eta), so a lake at rest
 * gives delta = 0 exactly.  Speeds u-c, u, u+c; eigenvectors (1, u-c, v),
 * (0, 0, 1), (1, u+c, v).  The y-edge is the same with x and y swapped. */
static void roe_state(int dir, const double *ql, const double *qr, const double *al, const double *ar, double g,
                      double *un, double *ut, double *c, double *hbar, double *hl, double *hr)
{
    int n = dir == 0 ? 1 : 2, t = dir == 0 ? 2 : 1;
    *hl = ql[0] - al[0];
    *hr = qr[0] - ar[0];
    double sl = sqrt(*hl), sr = sqrt(*hr);
    double unl = ql[n] / *hl, unr = qr[n] / *hr, utl = ql[t] / *hl, utr = qr[t] / *hr;
    *hbar = 0.5 * (*hl + *hr);
    *un = (sl * unl + sr * unr) / (sl + sr);
    *ut = (sl * utl + sr * utr) / (sl + sr);
    *c = sqrt(g * *hbar);
}

static void rp_swe(int dir, const double *ql, const double *qr, const double *al, const double *ar,
                   double wave[MAXW][MAXM], double s[MAXW], double *amdq, double *apdq, double g)
{
    int n = dir == 0 ? 1 : 2, t = dir == 0 ? 2 : 1;
    double un, ut, c, hbar, hl, hr;
    roe_state(dir, ql, qr, al, ar, g, &un, &ut, &c, &hbar, &hl, &hr);
    double d1 = qr[n] - ql[n];
    double d2 = (qr[n] * (qr[n] / hr) - ql[n] * (ql[n] / hl)) + g * hbar * (qr[0] - ql[0]);
    double d3 = qr[n] * (qr[t] / hr) - ql[n] * (ql[t] / hl);
    double s1 = un - c, s3 = un + c;
    double b1 = ((un + c) * d1 - d2) / (2.0 * c);
    double b3 = (d2 - (un - c) * d1) / (2.0 * c);
    double b2 = d3 - ut * d1;
    wave[0][0] = b1; wave[0][n] = b1 * s1; wave[0][t] = b1 * ut;
    wave[1][0] = 0.0; wave[1][n] = 0.0; wave[1][t] = b2;
    wave[2][0] = b3; wave[2][n] = b3 * s3; wave[2][t] = b3 * ut;
    s[0] = s1; s[1] = un; s[2] = s3;
    split_fluct(3, 3, wave, s, amdq, apdq);
}

/* transverse (constant-state split): decompose d with the eigenvectors of the
 * transverse direction at the Roe state of the normal edge the fluctuation
 * came from; B-d = sum over negative speeds of speed * strength * vector. */
static void ts_swe(int tdir, const double *d, const double *alo, const double *aown, const double *ahi,
                   const double *ql, const double *qr, const double *al, const double *ar,
                   double *bm, double *bp, double g)
{
    (void)alo; (void)aown; (void)ahi;
    int ndir = 1 - tdir;
    double un, ut, c, hbar, hl, hr;
    roe_state(ndir, ql, qr, al, ar, g, &un, &ut, &c, &hbar, &hl, &hr);
    /* velocity components along tdir (vt) and along the other axis (vo) */
    double vt = ut, vo = un;
    int kt = tdir == 0 ? 1 : 2, ko = tdir == 0 ? 2 : 1;
    double g1 = ((vt + c) * d[0] - d[kt]) / (2.0 * c);
    double g3 = (d[kt] - (vt - c) * d[0]) / (2.0 * c);
    double g2 = d[ko] - vo * d[0];
    double lam[3] = {vt - c, vt, vt + c};
    double r[3][3];
    r[0][0] = 1.0; r[0][kt] = vt - c; r[0][ko] = vo;
    r[1][0] = 0.0; r[1][kt] = 0.0;    r[1][ko] = 1.0;
    r[2][0] = 1.0; r[2][kt] = vt + c; r[2][ko] = vo;
    double str[3] = {g1, g2, g3};
    for (int k = 0; k < 3; k++) { bm[k] = 0.0; bp[k] = 0.0; }
    for (int p = 0; p < 3; p++)
        for (int k = 0; k < 3; k++) {
            double v = lam[p] * str[p] * r[p][k];
            if (lam[p] < 0.0) bm[k] += v; else bp[k] += v;
        }
}

/* --- linearised shallow-water adjoint, time reversed, f-wave ------------- */
/* Linearised system (Sec. 5.3): A = [[0,1,0],[g hbar,0,0],[0,0,0]], hbar = -B.
 * Reversed adjoint flux f = -A^T q = (-g hbar mu, -eta, 0); eigenvectors of
 * -A^T: (c, 1, 0) at speed -c, (-c, 1, 0) at speed +c. */
static void rp_lswe_adj(int dir, const double *ql, const double *qr, const double *al, const double *ar,
                        double wave[MAXW][MAXM], double s[MAXW], double *amdq, double *apdq, double g)
{
    int n = dir == 0 ? 1 : 2, t = dir == 0 ? 2 : 1;
    double cl = al[1], cr = ar[1];
    double f1l = -g * al[0] * ql[n], f1r = -g * ar[0] * qr[n];
    double f2l = -ql[0], f2r = -qr[0];
    double df1 = f1r - f1l, df2 = f2r - f2l;
    double b1 = (df1 + cr * df2) / (cl + cr);
    double b2 = (cl * df2 - df1) / (cl + cr);
    wave[0][0] = b1 * cl;  wave[0][n] = b1; wave[0][t] = 0.0;
    wave[1][0] = -b2 * cr; wave[1][n] = b2; wave[1][t] = 0.0;
    s[0] = -cl;
    s[1] = cr;
    for (int k = 0; k < 3; k++) { amdq[k] = wave[0][k]; apdq[k] = wave[1][k]; }
}

/* lo edge: d = g1 (c_lo, 1) + g2 (-c_own, 1)  -> -c_lo g1 (c_lo, 1)
 * hi edge: d = g1 (c_own, 1) + g2 (-c_hi, 1)  -> +c_hi g2 (-c_hi, 1) */
static void ts_lswe_adj(int tdir, const double *d, const double *alo, const double *aown, const double *ahi,
                        const double *ql, const double *qr, const double *al, const double *ar,
                        double *bm, double *bp, double g)
{
    (void)ql; (void)qr; (void)al; (void)ar; (void)g;
    int n = tdir == 0 ? 1 : 2, t = tdir == 0 ? 2 : 1;
    double clo = alo[1], co = aown[1], chi = ahi[1];
    double gm = (d[0] + co * d[n]) / (clo + co);
    double gp = (co * d[n] - d[0]) / (co + chi);
    bm[0] = -clo * gm * clo; bm[n] = -clo * gm; bm[t] = 0.0;
    bp[0] = -chi * gp * chi; bp[n] = chi * gp;  bp[t] = 0.0;
}

static const solver_t SOLVERS[4] = {
    {3, 2, 0, rp_acou_fwd, ts_acou_fwd},
    {3, 2, 1, rp_acou_adj, ts_acou_adj},
    {3, 3, 1, rp_swe, ts_swe},
    {3, 2, 1, rp_lswe_adj, ts_lswe_adj},
};

/* ------------------------------------------------------------------------ */
/* MC limiter on a vector wave (dot-product theta)                          */
/* ------------------------------------------------------------------------ */
static double mc_phi(double theta)
{
    double a = fmin(0.5 * (1.0 + theta), 2.0);
    a = fmin(a, 2.0 * theta);
    return fmax(0.0, a);
}

static double limiter_factor(int m, const double *w, const double *wup, int limiter)
{
    if (limiter == 0) return 1.0; /* unlimited Lax-Wendroff */
    double a = 0.0, b = 0.0;
    for (int k = 0; k < m; k++) { a += wup[k] * w[k]; b += w[k] * w[k]; }
    if (b == 0.0) return 0.0;
    return mc_phi(a / b);
}

/* ------------------------------------------------------------------------ */
/* Generic 2D step on a ghosted patch.                                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    double *wx, *sx, *amx, *apx, *wy, *sy, *amy, *apy, *F, *G;
    long cap;
} work_t;

static work_t WORK = {0};

static void work_reserve(long ncell)
{
    if (WORK.cap >= ncell) return;
    free(WORK.wx); free(WORK.sx); free(WORK.amx); free(WORK.apx);
    free(WORK.wy); free(WORK.sy); free(WORK.amy); free(WORK.apy);
    free(WORK.F); free(WORK.G);
    WORK.wx = malloc(sizeof(double) * ncell * MAXW * MAXM);
    WORK.wy = malloc(sizeof(double) * ncell * MAXW * MAXM);
    WORK.sx = malloc(sizeof(double) * ncell * MAXW);
    WORK.sy = malloc(sizeof(double) * ncell * MAXW);
    WORK.amx = malloc(sizeof(double) * ncell * MAXM);
    WORK.apx = malloc(sizeof(double) * ncell * MAXM);
    WORK.amy = malloc(sizeof(double) * ncell * MAXM);
    WORK.apy = malloc(sizeof(double) * ncell * MAXM);
    WORK.F = malloc(sizeof(double) * ncell * MAXM);
    WORK.G = malloc(sizeof(double) * ncell * MAXM);
    WORK.cap = ncell;
}

static inline void load_cell(const grid_t *g, const double *f, int m, int i, int j, double *out)
{
    long n = (long)g->NX * g->NY, id = gidx(g, i, j);
    for (int k = 0; k < m; k++) out[k] = f[k * n + id];
}

/*
 * One step of the unsplit 2D wave-propagation method.
 *   which: 0 forward acoustics, 1 adjoint acoustics, 2 shallow water,
 *          3 linearised shallow-water adjoint
 *   q, qn: ghosted states (q ghosts filled); qn interior is written
 *   aux:   NAUX ghosted fields
 *   order: 1 = Godunov only, 2 = with correction fluxes
 * Returns the largest Courant number |s| dt/dx over the edges of the interior
 * cells (max over both directions).
 */
double or_step2d(int which, int nx, int ny, double dtdx, double dtdy, double g,
                 const double *aux, const double *q, double *qn,
                 int order, int limiter, int transverse)
{
    const solver_t *S = &SOLVERS[which];
    grid_t gr = {nx, ny, nx + 2 * NG, ny + 2 * NG};
    const int m = S->m, nw = S->nw;
    long ncell = (long)gr.NX * gr.NY;
    work_reserve(ncell);
    double *wx = WORK.wx, *sx = WORK.sx, *amx = WORK.amx, *apx = WORK.apx;
    double *wy = WORK.wy, *sy = WORK.sy, *amy = WORK.amy, *apy = WORK.apy;
    double *F = WORK.F, *G = WORK.G;
    double cfl = 0.0;

    /* normal solves at x-edges (i-1/2, j): i in [-1, nx+1], j in [-1, ny] */
#pragma omp parallel for schedule(static)
    for (int j = -1; j <= ny; j++) {
        for (int i = -1; i <= nx + 1; i++) {
            double ql[MAXM], qr[MAXM], al[NAUX], ar[NAUX], wave[MAXW][MAXM], s[MAXW];
            load_cell(&gr, q, m, i - 1, j, ql); load_cell(&gr, q, m, i, j, qr);
            load_cell(&gr, aux, NAUX, i - 1, j, al); load_cell(&gr, aux, NAUX, i, j, ar);
            long e = gidx(&gr, i, j);
            S->rp(0, ql, qr, al, ar, wave, s, amx + e * MAXM, apx + e * MAXM, g);
            for (int p = 0; p < nw; p++) {
                sx[e * MAXW + p] = s[p];
                for (int k = 0; k < m; k++) wx[(e * MAXW + p) * MAXM + k] = wave[p][k];
            }
        }
    }
    /* normal solves at y-edges (i, j-1/2): i in [-1, nx], j in [-1, ny+1] */
#pragma omp parallel for schedule(static)
    for (int j = -1; j <= ny + 1; j++) {
        for (int i = -1; i <= nx; i++) {
            double ql[MAXM], qr[MAXM], al[NAUX], ar[NAUX], wave[MAXW][MAXM], s[MAXW];
            load_cell(&gr, q, m, i, j - 1, ql); load_cell(&gr, q, m, i, j, qr);
            load_cell(&gr, aux, NAUX, i, j - 1, al); load_cell(&gr, aux, NAUX, i, j, ar);
            long e = gidx(&gr, i, j);
            S->rp(1, ql, qr, al, ar, wave, s, amy + e * MAXM, apy + e * MAXM, g);
            for (int p = 0; p < nw; p++) {
                sy[e * MAXW + p] = s[p];
                for (int k = 0; k < m; k++) wy[(e * MAXW + p) * MAXM + k] = wave[p][k];
            }
        }
    }
    /* Courant number over the edges of interior cells */
    for (int j = 0; j < ny; j++)
        for (int i = 0; i <= nx; i++)
            for (int p = 0; p < nw; p++) cfl = fmax(cfl, fabs(sx[gidx(&gr, i, j) * MAXW + p]) * dtdx);
    if (ny > 1 || dtdy > 0.0)
        for (int j = 0; j <= ny; j++)
            for (int i = 0; i < nx; i++)
                for (int p = 0; p < nw; p++) cfl = fmax(cfl, fabs(sy[gidx(&gr, i, j) * MAXW + p]) * dtdy);

    /* second-order correction fluxes F at x-edges i in [0,nx], rows [0,ny-1]
     * and G at y-edges j in [0,ny], columns [0,nx-1] */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; j++) {
        for (int i = 0; i <= nx; i++) {
            long e = gidx(&gr, i, j);
            double *Fe = F + e * MAXM;
            for (int k = 0; k < m; k++) Fe[k] = 0.0;
            if (order < 2) continue;
            for (int p = 0; p < nw; p++) {
                double s = sx[e * MAXW + p];
                long eu = s > 0.0 ? gidx(&gr, i - 1, j) : gidx(&gr, i + 1, j);
                const double *w = wx + (e * MAXW + p) * MAXM, *wu = wx + (eu * MAXW + p) * MAXM;
                double phi = limiter_factor(m, w, wu, limiter);
                double as = fabs(s);
                double coef = S->fwave ? (s > 0.0 ? 1.0 : (s < 0.0 ? -1.0 : 0.0)) : as;
                for (int k = 0; k < m; k++) Fe[k] += 0.5 * coef * (1.0 - dtdx * as) * (phi * w[k]);
            }
        }
    }
#pragma omp parallel for schedule(static)
    for (int j = 0; j <= ny; j++) {
        for (int i = 0; i < nx; i++) {
            long e = gidx(&gr, i, j);
            double *Ge = G + e * MAXM;
            for (int k = 0; k < m; k++) Ge[k] = 0.0;
            if (order < 2) continue;
            for (int p = 0; p < nw; p++) {
                double s = sy[e * MAXW + p];
                long eu = s > 0.0 ? gidx(&gr, i, j - 1) : gidx(&gr, i, j + 1);
                const double *w = wy + (e * MAXW + p) * MAXM, *wu = wy + (eu * MAXW + p) * MAXM;
                double phi = limiter_factor(m, w, wu, limiter);
                double as = fabs(s);
                double coef = S->fwave ? (s > 0.0 ? 1.0 : (s < 0.0 ? -1.0 : 0.0)) : as;
                for (int k = 0; k < m; k++) Ge[k] += 0.5 * coef * (1.0 - dtdy * as) * (phi * w[k]);
            }
        }
    }

    if (transverse) {
        /* x-edge fluctuations into G.  A+dQ_{i-1/2,j} lives in cell (i,j),
         * A-dQ_{i-1/2,j} in cell (i-1,j); each is split at the two y-edges of
         * its cell.  Serial over rows (scatter). */
        for (int j = -1; j <= ny; j++) {
            for (int i = 0; i <= nx; i++) {
                long e = gidx(&gr, i, j);
                double ql[MAXM], qr[MAXM], al[NAUX], ar[NAUX], alo[NAUX], aown[NAUX], ahi[NAUX];
                double bm[MAXM], bp[MAXM];
                load_cell(&gr, q, m, i - 1, j, ql); load_cell(&gr, q, m, i, j, qr);
                load_cell(&gr, aux, NAUX, i - 1, j, al); load_cell(&gr, aux, NAUX, i, j, ar);
                for (int side = 0; side < 2; side++) {
                    int ic = side == 0 ? i : i - 1; /* cell the fluctuation lives in */
                    if (ic < 0 || ic >= nx) continue;
                    const double *d = side == 0 ? apx + e * MAXM : amx + e * MAXM;
                    load_cell(&gr, aux, NAUX, ic, j - 1, alo);
                    load_cell(&gr, aux, NAUX, ic, j, aown);
                    load_cell(&gr, aux, NAUX, ic, j + 1, ahi);
                    S->tsplit(1, d, alo, aown, ahi, ql, qr, al, ar, bm, bp, g);
                    if (j + 1 >= 0 && j + 1 <= ny) {
                        double *Gu = G + gidx(&gr, ic, j + 1) * MAXM;
                        for (int k = 0; k < m; k++) Gu[k] -= 0.5 * dtdx * bp[k];
                    }
                    if (j >= 0 && j <= ny) {
                        double *Gd = G + gidx(&gr, ic, j) * MAXM;
                        for (int k = 0; k < m; k++) Gd[k] -= 0.5 * dtdx * bm[k];
                    }
                }
            }
        }
        /* y-edge fluctuations into F.  B+dQ_{i,j-1/2} lives in cell (i,j),
         * B-dQ_{i,j-1/2} in cell (i,j-1). */
        for (int j = 0; j <= ny; j++) {
            for (int i = -1; i <= nx; i++) {
                long e = gidx(&gr, i, j);
                double ql[MAXM], qr[MAXM], al[NAUX], ar[NAUX], alo[NAUX], aown[NAUX], ahi[NAUX];
                double bm[MAXM], bp[MAXM];
                load_cell(&gr, q, m, i, j - 1, ql); load_cell(&gr, q, m, i, j, qr);
                load_cell(&gr, aux, NAUX, i, j - 1, al); load_cell(&gr, aux, NAUX, i, j, ar);
                for (int side = 0; side < 2; side++) {
                    int jc = side == 0 ? j : j - 1;
                    if (jc < 0 || jc >= ny) continue;
                    const double *d = side == 0 ? apy + e * MAXM : amy + e * MAXM;
                    load_cell(&gr, aux, NAUX, i - 1, jc, alo);
                    load_cell(&gr, aux, NAUX, i, jc, aown);
                    load_cell(&gr, aux, NAUX, i + 1, jc, ahi);
                    S->tsplit(0, d, alo, aown, ahi, ql, qr, al, ar, bm, bp, g);
                    if (i + 1 >= 0 && i + 1 <= nx) {
                        double *Fr = F + gidx(&gr, i + 1, jc) * MAXM;
                        for (int k = 0; k < m; k++) Fr[k] -= 0.5 * dtdy * bp[k];
                    }
                    if (i >= 0 && i <= nx) {
                        double *Fl = F + gidx(&gr, i, jc) * MAXM;
                        for (int k = 0; k < m; k++) Fl[k] -= 0.5 * dtdy * bm[k];
                    }
                }
            }
        }
    }

    /* cell update */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; j++) {
        for (int i = 0; i < nx; i++) {
            long c = gidx(&gr, i, j);
            long exl = c, exr = gidx(&gr, i + 1, j), eyb = c, eyt = gidx(&gr, i, j + 1);
            for (int k = 0; k < m; k++) {
                double v = q[k * ncell + c];
                v = v - dtdx * (apx[exl * MAXM + k] + amx[exr * MAXM + k]);
                v = v - dtdy * (apy[eyb * MAXM + k] + amy[eyt * MAXM + k]);
                v = v - dtdx * (F[exr * MAXM + k] - F[exl * MAXM + k]);
                v = v - dtdy * (G[eyt * MAXM + k] - G[eyb * MAXM + k]);
                qn[k * ncell + c] = v;
            }
        }
    }
    return cfl;
}

/* ------------------------------------------------------------------------ */
/* 1D step (acoustics forward or adjoint), Sec. 5.1.                        */
/* q: 2 fields of length nx+4; aux: NAUX fields of length nx+4.             */
/* ------------------------------------------------------------------------ */
double or_step1d(int which, int nx, double dtdx, const double *aux, const double *q, double *qn,
                 int order, int limiter)
{
    const int NXG = nx + 2 * NG;
    double *w = malloc(sizeof(double) * NXG * 2 * 2), *s = malloc(sizeof(double) * NXG * 2);
    double *am = malloc(sizeof(double) * NXG * 2), *ap = malloc(sizeof(double) * NXG * 2);
    double *F = malloc(sizeof(double) * NXG * 2);
    double cfl = 0.0;
    /* edge i (between cells i-1 and i) for i in [-1, nx+1] */
    for (int i = -1; i <= nx + 1; i++) {
        int l = i - 1 + NG, r = i + NG, e = i + NG;
        double Zl = aux[0 * NXG + l], Zr = aux[0 * NXG + r];
        double cl = aux[1 * NXG + l], cr = aux[1 * NXG + r];
        double w1[2], w2[2];
        if (which == 0) {
            double dp = q[r] - q[l], du = q[NXG + r] - q[NXG + l];
            double a1 = (-dp + Zr * du) / (Zl + Zr), a2 = (dp + Zl * du) / (Zl + Zr);
            w1[0] = -a1 * Zl; w1[1] = a1;
            w2[0] = a2 * Zr;  w2[1] = a2;
            am[e * 2 + 0] = -cl * w1[0]; am[e * 2 + 1] = -cl * w1[1];
            ap[e * 2 + 0] = cr * w2[0];  ap[e * 2 + 1] = cr * w2[1];
        } else {
            double rl = aux[2 * NXG + l], rr = aux[2 * NXG + r], Kl = aux[3 * NXG + l], Kr = aux[3 * NXG + r];
            double df1 = (-q[NXG + r] / rr) - (-q[NXG + l] / rl);
            double df2 = (-Kr * q[r]) - (-Kl * q[l]);
            double b1 = (Zr * df1 + df2) / (Zl + Zr), b2 = (Zl * df1 - df2) / (Zl + Zr);
            w1[0] = b1; w1[1] = b1 * Zl;
            w2[0] = b2; w2[1] = -b2 * Zr;
            am[e * 2 + 0] = w1[0]; am[e * 2 + 1] = w1[1];
            ap[e * 2 + 0] = w2[0]; ap[e * 2 + 1] = w2[1];
        }
        w[(e * 2 + 0) * 2 + 0] = w1[0]; w[(e * 2 + 0) * 2 + 1] = w1[1];
        w[(e * 2 + 1) * 2 + 0] = w2[0]; w[(e * 2 + 1) * 2 + 1] = w2[1];
        s[e * 2 + 0] = -cl;
        s[e * 2 + 1] = cr;
    }
    for (int i = 0; i <= nx; i++) {
        int e = i + NG;
        cfl = fmax(cfl, fmax(fabs(s[e * 2]), fabs(s[e * 2 + 1])) * dtdx);
        F[e * 2 + 0] = 0.0; F[e * 2 + 1] = 0.0;
        if (order < 2) continue;
        for (int p = 0; p < 2; p++) {
            double sp = s[e * 2 + p];
            int eu = sp > 0.0 ? e - 1 : e + 1;
            double phi = limiter_factor(2, w + (e * 2 + p) * 2, w + (eu * 2 + p) * 2, limiter);
            double as = fabs(sp);
            double coef = which == 1 ? (sp > 0.0 ? 1.0 : -1.0) : as;
            for (int k = 0; k < 2; k++) F[e * 2 + k] += 0.5 * coef * (1.0 - dtdx * as) * (phi * w[(e * 2 + p) * 2 + k]);
        }
    }
    for (int i = 0; i < nx; i++) {
        int c = i + NG;
        for (int k = 0; k < 2; k++) {
            double v = q[k * NXG + c];
            v = v - dtdx * (ap[c * 2 + k] + am[(c + 1) * 2 + k]);
            v = v - dtdx * (F[(c + 1) * 2 + k] - F[c * 2 + k]);
            qn[k * NXG + c] = v;
        }
    }
    free(w); free(s); free(am); free(ap); free(F);
    return cfl;
}

/* ------------------------------------------------------------------------ */
/* Uniform-grid driver: advance `nsteps` steps of size dt, filling ghosts    */
/* before every step; optionally store the interior every `snap_every`      */
/* steps (including step 0) into snaps[nsnap][m][ny][nx].                   */
/*   which: 0 fwd acoustics, 1 adj acoustics, 2 swe, 3 lswe adjoint          */
/*   c1, c2: acoustics rho, K; swe B (c2 unused); lswe B (hbar = -B)         */
/*   q: interior state [m][ny][nx], advanced in place                        */
/* Returns the largest Courant number seen, or -1 on a non-finite value.     */
/* ------------------------------------------------------------------------ */
double or_run(int which, int dim, int nx, int ny, double dx, double dy, double dt, int nsteps,
              const int *bc, int order, int limiter, int transverse, double g,
              const double *c1, const double *c2, double *q, int snap_every, double *snaps)
{
    int m = dim == 1 ? 2 : 3;
    int NX = nx + 2 * NG, NY = dim == 1 ? 1 : ny + 2 * NG;
    long ncell = (long)NX * NY;
    double *aux = calloc((size_t)NAUX * ncell, sizeof(double));
    double *qa = calloc((size_t)m * ncell, sizeof(double));
    double *qb = calloc((size_t)m * ncell, sizeof(double));
    grid_t gr = {nx, dim == 1 ? 1 : ny, NX, NY};
    int jofs = dim == 1 ? 0 : NG;
    for (int j = 0; j < (dim == 1 ? 1 : ny); j++)
        for (int i = 0; i < nx; i++) {
            long id = (long)(i + NG) + (long)(j + jofs) * NX, src = (long)j * nx + i;
            if (which <= 1) {
                double rho = c1[src], K = c2[src];
                aux[0 * ncell + id] = sqrt(rho * K);
                aux[1 * ncell + id] = sqrt(K / rho);
                aux[2 * ncell + id] = rho;
                aux[3 * ncell + id] = K;
            } else if (which == 2) {
                aux[id] = c1[src];
            } else {
                aux[0 * ncell + id] = -c1[src];
                aux[1 * ncell + id] = sqrt(g * -c1[src]);
            }
            for (int k = 0; k < m; k++) qa[k * ncell + id] = q[(long)k * nx * (dim == 1 ? 1 : ny) + src];
        }
    int ucomp = 1, vcomp = dim == 1 ? -1 : 2;
    if (dim == 1) {
        for (int k = 0; k < NAUX; k++) fill_ghosts_1d(nx, aux + k * ncell, bc[0], bc[1], 1.0);
    } else {
        for (int k = 0; k < NAUX; k++) fill_ghosts_field(&gr, aux + k * ncell, bc, 1.0, 1.0);
    }
    double cflmax = 0.0;
    int nsnap = 0;
    long nint = (long)nx * (dim == 1 ? 1 : ny);
    for (int step = 0; step <= nsteps; step++) {
        if (snaps && snap_every > 0 && step % snap_every == 0) {
            for (int k = 0; k < m; k++)
                for (int j = 0; j < (dim == 1 ? 1 : ny); j++)
                    for (int i = 0; i < nx; i++)
                        snaps[(long)nsnap * m * nint + k * nint + (long)j * nx + i] =
                            qa[k * ncell + (long)(i + NG) + (long)(j + jofs) * NX];
            nsnap++;
        }
        if (step == nsteps) break;
        if (dim == 1) {
            for (int k = 0; k < m; k++)
                fill_ghosts_1d(nx, qa + k * ncell, bc[0], bc[1], k == ucomp ? -1.0 : 1.0);
            double c = or_step1d(which, nx, dt / dx, aux, qa, qb, order, limiter);
            cflmax = fmax(cflmax, c);
        } else {
            or_fill_ghosts(m, nx, ny, qa, bc, ucomp, vcomp);
            double c = or_step2d(which, nx, ny, dt / dx, dt / dy, g, aux, qa, qb, order, limiter, transverse);
            cflmax = fmax(cflmax, c);
        }
        double *t = qa; qa = qb; qb = t;
    }
    int bad = 0;
    for (int k = 0; k < m; k++)
        for (int j = 0; j < (dim == 1 ? 1 : ny); j++)
            for (int i = 0; i < nx; i++) {
                double v = qa[k * ncell + (long)(i + NG) + (long)(j + jofs) * NX];
                if (!isfinite(v)) bad = 1;
                q[k * nint + (long)j * nx + i] = v;
            }
    free(aux); free(qa); free(qb);
    return bad ? -1.0 : cflmax;
}

/* Single 2D step on caller-provided ghosted arrays (used by the AMR driver
 * of the oracle, which fills the ghost cells itself). */
double or_patch_step(int which, int nx, int ny, double dtdx, double dtdy, double g,
                     const double *aux, const double *q, double *qn, int order, int limiter, int transverse)
{
    return or_step2d(which, nx, ny, dtdx, dtdy, g, aux, q, qn, order, limiter, transverse);
}

/* The same step, also returning the quantities each cell edge contributes to
 * its two cells, for the flux bookkeeping at coarse-fine edges (refluxing):
 *   xe [3][m][ny][nx+1]: A-dQ, A+dQ and the correction flux F (transverse
 *      terms included) at x-edge (i-1/2, j), i = 0..nx, j = 0..ny-1;
 *   ye [3][m][ny+1][nx]: B-dQ, B+dQ and G at y-edge (i, j-1/2), j = 0..ny.
 * The cell left of (below) an edge receives -dt/dx (A-dQ + F) (-dt/dy (B-dQ
 * + G)) from it, the cell right of (above) it -dt/dx (A+dQ - F). */
double or_patch_step_edges(int which, int nx, int ny, double dtdx, double dtdy, double g, const double *aux,
                           const double *q, double *qn, int order, int limiter, int transverse, double *xe,
                           double *ye)
{
    double cfl = or_step2d(which, nx, ny, dtdx, dtdy, g, aux, q, qn, order, limiter, transverse);
    grid_t gr = {nx, ny, nx + 2 * NG, ny + 2 * NG};
    const int m = SOLVERS[which].m;
    const long xs = (long)ny * (nx + 1), ys = (long)(ny + 1) * nx;
    for (int k = 0; k < m; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i <= nx; i++) {
                long e = gidx(&gr, i, j), o = (long)k * xs + (long)j * (nx + 1) + i;
                xe[o] = WORK.amx[e * MAXM + k];
                xe[(long)m * xs + o] = WORK.apx[e * MAXM + k];
                xe[2L * m * xs + o] = WORK.F[e * MAXM + k];
            }
    for (int k = 0; k < m; k++)
        for (int j = 0; j <= ny; j++)
            for (int i = 0; i < nx; i++) {
                long e = gidx(&gr, i, j), o = (long)k * ys + (long)j * nx + i;
                ye[o] = WORK.amy[e * MAXM + k];
                ye[(long)m * ys + o] = WORK.apy[e * MAXM + k];
                ye[2L * m * ys + o] = WORK.G[e * MAXM + k];
            }
    return cfl;
}

/* aux fields of a ghosted patch from interior coefficients: acoustics (rho,K)
 * -> {Z, c, rho, K}; swe B -> {B}; lswe B -> {-B, sqrt(-g B)}. */
void or_make_aux(int which, int nx, int ny, const double *c1, const double *c2, double g, double *aux)
{
    int NX = nx + 2 * NG, NY = ny + 2 * NG;
    long ncell = (long)NX * NY;
    for (int j = -NG; j < ny + NG; j++)
        for (int i = -NG; i < nx + NG; i++) {
            long id = (long)(i + NG) + (long)(j + NG) * NX, src = id;
            if (which <= 1) {
                double rho = c1[src], K = c2[src];
                aux[0 * ncell + id] = sqrt(rho * K);
                aux[1 * ncell + id] = sqrt(K / rho);
                aux[2 * ncell + id] = rho;
                aux[3 * ncell + id] = K;
            } else if (which == 2) {
                aux[id] = c1[src];
            } else {
                aux[0 * ncell + id] = -c1[src];
                aux[1 * ncell + id] = sqrt(g * -c1[src]);
            }
        }
}

/* Single-edge access for the oracle's own tests: the normal solve and the
 * transverse split of solver `which`, with the same argument meaning as the
 * solver table.  wave is [MAXW][MAXM], s is [MAXW]. */
void or_rp(int which, int dir, const double *ql, const double *qr, const double *al, const double *ar,
           double *wave, double *s, double *amdq, double *apdq, double g)
{
    double w[MAXW][MAXM] = {{0}};
    double sp[MAXW] = {0};
    SOLVERS[which].rp(dir, ql, qr, al, ar, w, sp, amdq, apdq, g);
    for (int p = 0; p < MAXW; p++) {
        s[p] = sp[p];
        for (int k = 0; k < MAXM; k++) wave[p * MAXM + k] = w[p][k];
    }
}

void or_tsplit(int which, int tdir, const double *d, const double *alo, const double *aown, const double *ahi,
               const double *ql, const double *qr, const double *al, const double *ar,
               double *bm, double *bp, double g)
{
    SOLVERS[which].tsplit(tdir, d, alo, aown, ahi, ql, qr, al, ar, bm, bp, g);
}
