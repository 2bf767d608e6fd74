/*
 * Plain CPU FP64 oracle for the two-step Lax-Wendroff shallow-water step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header, table or helper with the
 * HIP path.
 *
 * It follows the paper's "Shallow Water Model" section step by step, with
 * whole temporary face arrays exactly as the data-parallel formulation
 * describes them (Hx, Ux, Vx on x-faces; Hy, Uy, Vy on y-faces), and no
 * blocking, fusion or reordering:
 *   - conservation laws for (h, hu, hv) with fluxes
 *       F(U) = (hu, hu^2/h + g h^2/2, hu hv/h)
 *       G(U) = (hv, hu hv/h,          hv^2/h + g h^2/2)        (SWE equations)
 *   - CFL bound dt <= dx / (sqrt(g h) + |u|)                     (CFL remark)
 *   - step 1: half-step states on every face (first LW equation pair), in the
 *     sign of the paper's Fortran face statement: the flux difference enters
 *     as (lt - rt), i.e. minus (F_{i+1} - F_i); the y half-step uses G.
 *   - step 2: dimensionally unsplit conservative update (second LW equation),
 *     written as the paper's Fortran update: U + (dt/dx)(X_lt - X_rt)
 *     + (dt/dy)(Y_dn - Y_up) with the face ranges of its face halos.
 * Readings where the paper is silent: boundary conditions (reflective walls
 * negate the wall-normal momentum; periodic wraps), the per-step CFL dt
 * (dt = cfl * min(dx, dy) / max over cells of (max(|u|, |v|) + sqrt(g h))),
 * and an optional transverse term in the half-step (standard 2-D
 * Lax-Wendroff), which the paper does not have.
 *
 * Layout: every array is (ny + 2) x (nx + 2) doubles, row-major, x fastest,
 * with a one-cell halo; interior cells are i = 1..nx, j = 1..ny.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

enum { OR_REFLECT = 0, OR_PERIODIC = 1 };
enum { OR_SCHEME_PAPER = 0, OR_SCHEME_TRANSVERSE = 1 };
enum { OR_OK = 0, OR_EINVAL = -1, OR_ENOMEM = -3, OR_EUNSTABLE = -5 };

#define AT(a, i, j) (a)[(size_t)(j) * (size_t)(nx + 2) + (size_t)(i)]

/* Boundary conditions, applied outside the step as the paper prescribes.
 * x walls first (rows 1..ny), then y walls over the full width including the
 * x ghosts, so corner ghosts are "x then y". */
void or_fill_halo(int nx, int ny, int bcx, int bcy, double *H, double *U, double *V)
{
    for (int j = 1; j <= ny; ++j) {
        if (bcx == OR_PERIODIC) {
            AT(H, 0, j) = AT(H, nx, j);  AT(U, 0, j) = AT(U, nx, j);  AT(V, 0, j) = AT(V, nx, j);
            AT(H, nx + 1, j) = AT(H, 1, j);  AT(U, nx + 1, j) = AT(U, 1, j);  AT(V, nx + 1, j) = AT(V, 1, j);
        } else {
            AT(H, 0, j) = AT(H, 1, j);  AT(U, 0, j) = -AT(U, 1, j);  AT(V, 0, j) = AT(V, 1, j);
            AT(H, nx + 1, j) = AT(H, nx, j);  AT(U, nx + 1, j) = -AT(U, nx, j);  AT(V, nx + 1, j) = AT(V, nx, j);
        }
    }
    for (int i = 0; i <= nx + 1; ++i) {
        if (bcy == OR_PERIODIC) {
            AT(H, i, 0) = AT(H, i, ny);  AT(U, i, 0) = AT(U, i, ny);  AT(V, i, 0) = AT(V, i, ny);
            AT(H, i, ny + 1) = AT(H, i, 1);  AT(U, i, ny + 1) = AT(U, i, 1);  AT(V, i, ny + 1) = AT(V, i, 1);
        } else {
            AT(H, i, 0) = AT(H, i, 1);  AT(U, i, 0) = AT(U, i, 1);  AT(V, i, 0) = -AT(V, i, 1);
            AT(H, i, ny + 1) = AT(H, i, ny);  AT(U, i, ny + 1) = AT(U, i, ny);  AT(V, i, ny + 1) = -AT(V, i, ny);
        }
    }
}

/* Largest signal speed over the interior: max(|u|, |v|) + sqrt(g h). */
double or_max_speed(int nx, int ny, double g, const double *H, const double *U, const double *V)
{
    double s = 0.0;
    for (int j = 1; j <= ny; ++j)
        for (int i = 1; i <= nx; ++i) {
            double h = AT(H, i, j);
            double u = fabs(AT(U, i, j) / h);
            double v = fabs(AT(V, i, j) / h);
            double c = sqrt(g * h);
            double si = (u > v ? u : v) + c;
            if (si > s) s = si;
        }
    return s;
}

/* x-direction flux components of the momenta, F = (U, U^2/H + g H^2/2, U V/H). */
static double flux_fu(double g, double h, double u, double v) { (void)v; return u * u / h + 0.5 * g * h * h; }
static double flux_fv(double g, double h, double u, double v) { (void)g; return u * v / h; }
/* y-direction flux components of the momenta, G = (V, U V/H, V^2/H + g H^2/2). */
static double flux_gu(double g, double h, double u, double v) { (void)g; return u * v / h; }
static double flux_gv(double g, double h, double u, double v) { (void)u; return v * v / h + 0.5 * g * h * h; }

/*
 * One time step U^n -> U^{n+1} with a given dt.  The input halo must already
 * hold the boundary values.  Face arrays:
 *   x faces: Hx, Ux, Vx of (nx + 1) x ny, face f = 0..nx sits between halo
 *            cells f ("lt") and f + 1 ("rt") on row j = 1..ny;
 *   y faces: Hy, Uy, Vy of nx x (ny + 1), face f = 0..ny sits between rows
 *            f ("dn") and f + 1 ("up") on column i = 1..nx.
 * Only the interior of the outputs is written.
 */
int or_step(int nx, int ny, double g, double dx, double dy, double dt, int scheme,
            const double *H, const double *U, const double *V,
            double *oH, double *oU, double *oV)
{
    if (nx < 1 || ny < 1) return OR_EINVAL;
    size_t nxf = (size_t)(nx + 1) * (size_t)ny, nyf = (size_t)nx * (size_t)(ny + 1);
    double *Hx = malloc(nxf * sizeof(double)), *Ux = malloc(nxf * sizeof(double)), *Vx = malloc(nxf * sizeof(double));
    double *Hy = malloc(nyf * sizeof(double)), *Uy = malloc(nyf * sizeof(double)), *Vy = malloc(nyf * sizeof(double));
    if (!Hx || !Ux || !Vx || !Hy || !Uy || !Vy) {
        free(Hx); free(Ux); free(Vx); free(Hy); free(Uy); free(Vy);
        return OR_ENOMEM;
    }
#define XF(a, f, j) (a)[(size_t)((j) - 1) * (size_t)(nx + 1) + (size_t)(f)]
#define YF(a, i, f) (a)[(size_t)(f) * (size_t)nx + (size_t)((i) - 1)]
    const double hx = 0.5 * dt / dx, hy = 0.5 * dt / dy;

    /* Step 1, x faces. */
    for (int j = 1; j <= ny; ++j)
        for (int f = 0; f <= nx; ++f) {
            int lt = f, rt = f + 1;
            double hl = AT(H, lt, j), ul = AT(U, lt, j), vl = AT(V, lt, j);
            double hr = AT(H, rt, j), ur = AT(U, rt, j), vr = AT(V, rt, j);
            double h = 0.5 * (hl + hr) + hx * (ul - ur);
            double u = 0.5 * (ul + ur) + hx * (flux_fu(g, hl, ul, vl) - flux_fu(g, hr, ur, vr));
            double v = 0.5 * (vl + vr) + hx * (flux_fv(g, hl, ul, vl) - flux_fv(g, hr, ur, vr));
            if (scheme == OR_SCHEME_TRANSVERSE) {
                /* + (dt/2dy) * 1/4 [(G_{lt,dn} + G_{rt,dn}) - (G_{lt,up} + G_{rt,up})] */
                double hd0 = AT(H, lt, j - 1), ud0 = AT(U, lt, j - 1), vd0 = AT(V, lt, j - 1);
                double hd1 = AT(H, rt, j - 1), ud1 = AT(U, rt, j - 1), vd1 = AT(V, rt, j - 1);
                double hu0 = AT(H, lt, j + 1), uu0 = AT(U, lt, j + 1), vu0 = AT(V, lt, j + 1);
                double hu1 = AT(H, rt, j + 1), uu1 = AT(U, rt, j + 1), vu1 = AT(V, rt, j + 1);
                h += hy * 0.25 * ((vd0 + vd1) - (vu0 + vu1));
                u += hy * 0.25 * ((flux_gu(g, hd0, ud0, vd0) + flux_gu(g, hd1, ud1, vd1))
                                - (flux_gu(g, hu0, uu0, vu0) + flux_gu(g, hu1, uu1, vu1)));
                v += hy * 0.25 * ((flux_gv(g, hd0, ud0, vd0) + flux_gv(g, hd1, ud1, vd1))
                                - (flux_gv(g, hu0, uu0, vu0) + flux_gv(g, hu1, uu1, vu1)));
            }
            XF(Hx, f, j) = h;  XF(Ux, f, j) = u;  XF(Vx, f, j) = v;
        }

    /* Step 1, y faces. */
    for (int f = 0; f <= ny; ++f)
        for (int i = 1; i <= nx; ++i) {
            int dn = f, up = f + 1;
            double hd = AT(H, i, dn), ud = AT(U, i, dn), vd = AT(V, i, dn);
            double hu = AT(H, i, up), uu = AT(U, i, up), vu = AT(V, i, up);
            double h = 0.5 * (hd + hu) + hy * (vd - vu);
            double u = 0.5 * (ud + uu) + hy * (flux_gu(g, hd, ud, vd) - flux_gu(g, hu, uu, vu));
            double v = 0.5 * (vd + vu) + hy * (flux_gv(g, hd, ud, vd) - flux_gv(g, hu, uu, vu));
            if (scheme == OR_SCHEME_TRANSVERSE) {
                /* + (dt/2dx) * 1/4 [(F_{lt,dn} + F_{lt,up}) - (F_{rt,dn} + F_{rt,up})] */
                double hl0 = AT(H, i - 1, dn), ul0 = AT(U, i - 1, dn), vl0 = AT(V, i - 1, dn);
                double hl1 = AT(H, i - 1, up), ul1 = AT(U, i - 1, up), vl1 = AT(V, i - 1, up);
                double hr0 = AT(H, i + 1, dn), ur0 = AT(U, i + 1, dn), vr0 = AT(V, i + 1, dn);
                double hr1 = AT(H, i + 1, up), ur1 = AT(U, i + 1, up), vr1 = AT(V, i + 1, up);
                h += hx * 0.25 * ((ul0 + ul1) - (ur0 + ur1));
                u += hx * 0.25 * ((flux_fu(g, hl0, ul0, vl0) + flux_fu(g, hl1, ul1, vl1))
                                - (flux_fu(g, hr0, ur0, vr0) + flux_fu(g, hr1, ur1, vr1)));
                v += hx * 0.25 * ((flux_fv(g, hl0, ul0, vl0) + flux_fv(g, hl1, ul1, vl1))
                                - (flux_fv(g, hr0, ur0, vr0) + flux_fv(g, hr1, ur1, vr1)));
            }
            YF(Hy, i, f) = h;  YF(Uy, i, f) = u;  YF(Vy, i, f) = v;
        }

    /* Step 2: conservative update from the face states' fluxes. */
    const double mx = dt / dx, my = dt / dy;
    for (int j = 1; j <= ny; ++j)
        for (int i = 1; i <= nx; ++i) {
            int lt = i - 1, rt = i;   /* x faces i-1/2 and i+1/2 */
            int dn = j - 1, up = j;   /* y faces j-1/2 and j+1/2 */
            double hl = XF(Hx, lt, j), ul = XF(Ux, lt, j), vl = XF(Vx, lt, j);
            double hr = XF(Hx, rt, j), ur = XF(Ux, rt, j), vr = XF(Vx, rt, j);
            double hd = YF(Hy, i, dn), ud = YF(Uy, i, dn), vd = YF(Vy, i, dn);
            double hu = YF(Hy, i, up), uu = YF(Uy, i, up), vu = YF(Vy, i, up);
            AT(oH, i, j) = AT(H, i, j) + mx * (ul - ur) + my * (vd - vu);
            AT(oU, i, j) = AT(U, i, j) + mx * (flux_fu(g, hl, ul, vl) - flux_fu(g, hr, ur, vr))
                                       + my * (flux_gu(g, hd, ud, vd) - flux_gu(g, hu, uu, vu));
            AT(oV, i, j) = AT(V, i, j) + mx * (flux_fv(g, hl, ul, vl) - flux_fv(g, hr, ur, vr))
                                       + my * (flux_gv(g, hd, ud, vd) - flux_gv(g, hu, uu, vu));
        }
#undef XF
#undef YF
    free(Hx); free(Ux); free(Vx); free(Hy); free(Uy); free(Vy);
    return OR_OK;
}

/* Dry or broken state: any interior h <= 0 or any non-finite value. */
static int unstable(int nx, int ny, const double *H, const double *U, const double *V)
{
    for (int j = 1; j <= ny; ++j)
        for (int i = 1; i <= nx; ++i) {
            double h = AT(H, i, j);
            if (!(h > 0.0) || !isfinite(h) || !isfinite(AT(U, i, j)) || !isfinite(AT(V, i, j)))
                return 1;
        }
    return 0;
}

/*
 * The time loop: nsteps x (fill halo; dt; step 1; step 2; swap).
 * dt_fixed > 0 uses that dt (the paper's fixed step); otherwise
 * dt = cfl * min(dx, dy) / max_speed(U^n) is recomputed from every U^n.
 * H, U, V hold U^0 on entry and U^nsteps (with its halo filled) on exit.
 * t_out receives the simulated time; dts (optional, nsteps entries) each dt.
 * Returns OR_EUNSTABLE as soon as a step produces h <= 0 or a non-finite
 * value; *steps_done then counts the completed steps.
 */
int or_run(int nx, int ny, double g, double dx, double dy, double cfl, double dt_fixed,
           int scheme, int bcx, int bcy, int nsteps,
           double *H, double *U, double *V, double *t_out, double *dts, int *steps_done)
{
    if (nx < 1 || ny < 1 || nsteps < 0 || !(g > 0) || !(dx > 0) || !(dy > 0)) return OR_EINVAL;
    if (!(dt_fixed > 0) && !(cfl > 0)) return OR_EINVAL;
    size_t n = (size_t)(nx + 2) * (size_t)(ny + 2);
    double *bH = malloc(n * sizeof(double)), *bU = malloc(n * sizeof(double)), *bV = malloc(n * sizeof(double));
    if (!bH || !bU || !bV) { free(bH); free(bU); free(bV); return OR_ENOMEM; }
    memcpy(bH, H, n * sizeof(double)); memcpy(bU, U, n * sizeof(double)); memcpy(bV, V, n * sizeof(double));
    double *cH = H, *cU = U, *cV = V, *nH = bH, *nU = bU, *nV = bV;
    double t = 0.0;
    int rc = OR_OK, done = 0;
    for (int s = 0; s < nsteps; ++s) {
        or_fill_halo(nx, ny, bcx, bcy, cH, cU, cV);
        double dt = dt_fixed > 0 ? dt_fixed
                                 : cfl * (dx < dy ? dx : dy) / or_max_speed(nx, ny, g, cH, cU, cV);
        if (dts) dts[s] = dt;
        rc = or_step(nx, ny, g, dx, dy, dt, scheme, cH, cU, cV, nH, nU, nV);
        if (rc != OR_OK) break;
        t += dt;
        double *tmp;
        tmp = cH; cH = nH; nH = tmp;  tmp = cU; cU = nU; nU = tmp;  tmp = cV; cV = nV; nV = tmp;
        ++done;
        if (unstable(nx, ny, cH, cU, cV)) { rc = OR_EUNSTABLE; break; }
    }
    or_fill_halo(nx, ny, bcx, bcy, cH, cU, cV);
    if (cH != H) {
        memcpy(H, cH, n * sizeof(double)); memcpy(U, cU, n * sizeof(double)); memcpy(V, cV, n * sizeof(double));
    }
    free(bH); free(bU); free(bV);
    if (t_out) *t_out = t;
    if (steps_done) *steps_done = done;
    return rc;
}
