/*
 * FP64 CPU oracle of the immersed-boundary lattice Boltzmann (IB-LB) wetting
 * model.  TEST INFRASTRUCTURE ONLY: nothing in the product path links,
 * loads or calls this file; only the tests, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code, header, table or
 * helper with the HIP library.
 *
 * Everything is plain loops in double precision, written to be checked by
 * eye against the paper ("Immersed boundary - lattice Boltzmann method for
 * wetting problems"):
 *
 *   velocity set            Table I (D3Q19); D2Q9 is its 2D analogue
 *   LB update               eq. (LBE): stream + BGK collision + Guo source
 *   equilibrium             second-order Maxwell-Boltzmann expansion
 *   Guo source term         S_i(U, F) with the (1 - dt/2tau) prefactor
 *   moments                 eqs. (hydro_var1), (hydro_var2) (half-force U)
 *   delta kernel            Peskin 4-point Psi, Delta = Psi Psi Psi / dx^3
 *   spreading               eq. (force_spread)
 *   interpolation           eq. (vel_interpolation)
 *   advection               forward Euler q <- q + qdot dt
 *   surface tension         phi_sigma = -dW/dq with W = sigma e^a summed
 *                           over the reference area (Sec. "Modelling surface
 *                           tension forces"); e^a is the area ratio, so W is
 *                           sigma times the current area (perimeter in 2D)
 *   wetting                 eq. (disjoin-p) for Pi(h); nodal force
 *                           -(chi_j/3) Pi n_j; strength A from eq. (A_choice)
 *   boundaries              periodic sides, bounce-back walls (Sec. "Numerical
 *                           results", set-up paragraph)
 *   elastic interface       w(a, b) = sigma e^a + mu_s (b + 1 - e^a) with the
 *                           strain invariants a, b of eq. strain_inv measured
 *                           from a stress-free reference mesh (a different
 *                           strain energy in eq. force_bb, as the outlook
 *                           proposes); mu_s = 0 is the droplet of eq.
 *                           energy_drop
 *   two viscosities         tau = tau_in at cells enclosed by the interface,
 *                           tau_out elsewhere, reclassified every step (Sec.
 *                           IB-LB, last paragraph; eq. def_lambda)
 *
 * Conventions shared with every other implementation of the model (an
 * interface, not code): populations are stored [i][z][y][x] with x fastest;
 * cell (x,y,z) is centred at (x+1/2, y+1/2, z+1/2); walls sit at coordinate 0
 * and n of a wall axis; velocities are ordered rest, then opposite pairs
 * adjacent, so opp(i) = i+1 for odd i and i-1 for even i > 0.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PERIODIC 0
#define ORC_WALL 1

/* ------------------------------------------------------------------------ */
/* Velocity sets                                                             */
/* ------------------------------------------------------------------------ */

/* D2Q9: rest; +x,-x; +y,-y; (+1,+1),(-1,-1); (-1,+1),(+1,-1) */
static const int C2[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, -1, 0}, {-1, 1, 0}, {1, -1, 0}};
static const double W2[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

/* D3Q19 (Table I): rest w = 1/3; six axis velocities w = 1/18; twelve
 * face diagonals w = 1/36 */
static const int C3[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double W3[19] = {
    1.0 / 3.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

static const double CS2 = 1.0 / 3.0; /* c_s^2 = dx^2 / (3 dt^2) */
static const double PI = 3.14159265358979323846;

static int nq(int dim) { return dim == 2 ? 9 : 19; }
static const int *cvec(int dim, int i) { return dim == 2 ? C2[i] : C3[i]; }
static double wgt(int dim, int i) { return dim == 2 ? W2[i] : W3[i]; }

/* index of -c_i, found by search so it does not rely on the ordering */
static int opposite(int dim, int i)
{
    const int *c = cvec(dim, i);
    for (int k = 0; k < nq(dim); ++k) {
        const int *d = cvec(dim, k);
        if (d[0] == -c[0] && d[1] == -c[1] && d[2] == -c[2]) return k;
    }
    return -1;
}

void orc_lattice(int dim, int *c_out /* Q*3 */, double *w_out /* Q */)
{
    for (int i = 0; i < nq(dim); ++i) {
        for (int a = 0; a < 3; ++a) c_out[3 * i + a] = cvec(dim, i)[a];
        w_out[i] = wgt(dim, i);
    }
}

/* ------------------------------------------------------------------------ */
/* Collision ingredients                                                     */
/* ------------------------------------------------------------------------ */

/* second-order equilibrium f_i^eq(rho, U) */
void orc_equilibrium(int dim, double rho, const double *U, double *feq)
{
    double uu = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
    for (int i = 0; i < nq(dim); ++i) {
        const int *c = cvec(dim, i);
        double cu = c[0] * U[0] + c[1] * U[1] + c[2] * U[2];
        feq[i] = wgt(dim, i) * rho *
                 (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
    }
}

/* Guo source S_i(U, F) = (1 - dt/(2 tau)) w_i [ (c_i - U)/cs^2
 *                                             + (c_i.U) c_i / cs^4 ] . F  */
void orc_guo_source(int dim, double tau, const double *U, const double *F, double *S)
{
    double pre = 1.0 - 1.0 / (2.0 * tau);
    for (int i = 0; i < nq(dim); ++i) {
        const int *c = cvec(dim, i);
        double cu = c[0] * U[0] + c[1] * U[1] + c[2] * U[2];
        double s = 0.0;
        for (int a = 0; a < 3; ++a)
            s += ((c[a] - U[a]) / CS2 + cu * c[a] / (CS2 * CS2)) * F[a];
        S[i] = pre * wgt(dim, i) * s;
    }
}

/* ------------------------------------------------------------------------ */
/* One LB time step, pull form:                                              */
/*   f_i(x, t)   = f*_i(x - c_i, t - 1)  (streaming, left side of eq. LBE)   */
/*   rho, U      from eqs. (hydro_var1), (hydro_var2) with F(x, t)           */
/*   f*_i(x, t)  = f_i - (f_i - f_i^eq)/tau + S_i   (right side of eq. LBE)  */
/* A population whose source cell lies beyond a wall was reflected there     */
/* half a step earlier: it is the opposite population of the same cell       */
/* (half-way bounce-back, resting wall).                                     */
/* fin, fout: [Q][ncell]; F, U: [3][ncell] (unused components zero);        */
/* rho: [ncell].  F may be NULL (no force).  tau_cell: [ncell] relaxation     */
/* time of every cell, or NULL for tau everywhere; a cell's own tau enters   */
/* both the BGK term and the Guo prefactor.                                  */
/* ------------------------------------------------------------------------ */
void orc_lb_step(int dim, int nx, int ny, int nz, const int *bc, double tau,
                 const double *tau_cell, const double *fin, const double *F, double *fout,
                 double *rho_out, double *U_out)
{
    const int Q = nq(dim);
    const long ncell = (long)nx * ny * nz;
    const int n[3] = {nx, ny, nz};
    /* cells are independent: the rows may be shared among threads without
       changing any result */
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                double f[19], feq[19], S[19];
                const long cell = ((long)z * ny + y) * nx + x;
                const int pos[3] = {x, y, z};
                for (int i = 0; i < Q; ++i) {
                    const int *c = cvec(dim, i);
                    int src[3];
                    int bounced = 0;
                    for (int a = 0; a < 3; ++a) {
                        src[a] = pos[a] - c[a];
                        if (src[a] < 0 || src[a] >= n[a]) {
                            if (bc[a] == ORC_PERIODIC)
                                src[a] = (src[a] + n[a]) % n[a];
                            else
                                bounced = 1;
                        }
                    }
                    if (bounced) {
                        f[i] = fin[(long)opposite(dim, i) * ncell + cell];
                    } else {
                        long sc = ((long)src[2] * ny + src[1]) * nx + src[0];
                        f[i] = fin[(long)i * ncell + sc];
                    }
                }
                double Fx[3] = {0.0, 0.0, 0.0};
                if (F)
                    for (int a = 0; a < dim; ++a) Fx[a] = F[(long)a * ncell + cell];
                double rho = 0.0, mom[3] = {0.0, 0.0, 0.0};
                for (int i = 0; i < Q; ++i) {
                    rho += f[i];
                    for (int a = 0; a < 3; ++a) mom[a] += cvec(dim, i)[a] * f[i];
                }
                double U[3];
                for (int a = 0; a < 3; ++a) U[a] = (mom[a] + 0.5 * Fx[a]) / rho;
                const double t = tau_cell ? tau_cell[cell] : tau;
                orc_equilibrium(dim, rho, U, feq);
                orc_guo_source(dim, t, U, Fx, S);
                for (int i = 0; i < Q; ++i)
                    fout[(long)i * ncell + cell] = f[i] - (f[i] - feq[i]) / t + S[i];
                if (rho_out) rho_out[cell] = rho;
                if (U_out)
                    for (int a = 0; a < 3; ++a) U_out[(long)a * ncell + cell] = U[a];
            }
}

/* ------------------------------------------------------------------------ */
/* Peskin 4-point kernel Psi(x) (dx = 1), evaluated from its piecewise      */
/* definition.                                                               */
/* ------------------------------------------------------------------------ */
double orc_psi(double x)
{
    double r = fabs(x);
    if (r <= 1.0) return 3.0 / 8.0 - r / 4.0 + sqrt(r - r * r + 0.25) / 4.0;
    if (r <= 2.0) return 5.0 / 8.0 - r / 4.0 - sqrt(3.0 * r - r * r - 1.75) / 4.0;
    return 0.0;
}

/* Visit every lattice cell within the support of Delta(q - x): cells whose
 * centre lies within 2 of q along every axis.  Along a periodic axis the
 * cell index wraps; along a wall axis a cell beyond the wall is reported as
 * solid (index -1). */
typedef void (*tap_fn)(void *ctx, long cell, double weight);

static void for_each_tap(int dim, const int *n, const int *bc, const double *q,
                         tap_fn fn, void *ctx)
{
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        if (a < dim) {
            lo[a] = (int)floor(q[a]) - 3;
            hi[a] = (int)floor(q[a]) + 3;
        } else {
            lo[a] = hi[a] = 0;
        }
    }
    for (int k = lo[2]; k <= hi[2]; ++k)
        for (int j = lo[1]; j <= hi[1]; ++j)
            for (int i = lo[0]; i <= hi[0]; ++i) {
                const int idx[3] = {i, j, k};
                double wgt_ = 1.0;
                for (int a = 0; a < dim; ++a) wgt_ *= orc_psi(idx[a] + 0.5 - q[a]);
                if (wgt_ == 0.0) continue;
                int w[3];
                int solid = 0;
                for (int a = 0; a < 3; ++a) {
                    w[a] = idx[a];
                    if (a >= dim) { w[a] = 0; continue; }
                    if (w[a] < 0 || w[a] >= n[a]) {
                        if (bc[a] == ORC_PERIODIC)
                            w[a] = ((w[a] % n[a]) + n[a]) % n[a];
                        else
                            solid = 1;
                    }
                }
                long cell = solid ? -1 : ((long)w[2] * n[1] + w[1]) * n[0] + w[0];
                fn(ctx, cell, wgt_);
            }
}

struct spread_ctx {
    int dim;
    long ncell;
    const double *phi; /* this node's force */
    double *F;
    double *dropped;
};

static void spread_tap(void *vctx, long cell, double weight)
{
    struct spread_ctx *s = (struct spread_ctx *)vctx;
    for (int a = 0; a < s->dim; ++a) {
        if (cell >= 0)
            s->F[(long)a * s->ncell + cell] += s->phi[a] * weight;
        else
            s->dropped[a] += s->phi[a] * weight;
    }
}

/* eq. (force_spread): F(x) = sum_j phi_j Delta(q_j - x), dx = 1.
 * q, phi: [dim][N].  F: [3][ncell], overwritten.  dropped[3]: the part of
 * the nodal forces whose taps fall beyond a wall (not spread). */
void orc_spread(int dim, int nx, int ny, int nz, const int *bc, int N,
                const double *q, const double *phi, double *F, double *dropped)
{
    const int n[3] = {nx, ny, nz};
    const long ncell = (long)nx * ny * nz;
    memset(F, 0, sizeof(double) * 3 * ncell);
    dropped[0] = dropped[1] = dropped[2] = 0.0;
    for (int j = 0; j < N; ++j) {
        double qj[3] = {0, 0, 0}, pj[3] = {0, 0, 0};
        for (int a = 0; a < dim; ++a) {
            qj[a] = q[(long)a * N + j];
            pj[a] = phi[(long)a * N + j];
        }
        struct spread_ctx s = {dim, ncell, pj, F, dropped};
        for_each_tap(dim, n, bc, qj, spread_tap, &s);
    }
}

struct interp_ctx {
    int dim;
    long ncell;
    const double *U;
    double acc[3];
};

static void interp_tap(void *vctx, long cell, double weight)
{
    struct interp_ctx *s = (struct interp_ctx *)vctx;
    if (cell < 0) return; /* wall: the fluid velocity there is zero */
    for (int a = 0; a < s->dim; ++a) s->acc[a] += s->U[(long)a * s->ncell + cell] * weight;
}

/* eq. (vel_interpolation): qdot_j = sum_x U(x) Delta(q_j - x) dx^3 */
void orc_interp(int dim, int nx, int ny, int nz, const int *bc, const double *U,
                int N, const double *q, double *qdot)
{
    const int n[3] = {nx, ny, nz};
    const long ncell = (long)nx * ny * nz;
    for (int j = 0; j < N; ++j) {
        double qj[3] = {0, 0, 0};
        for (int a = 0; a < dim; ++a) qj[a] = q[(long)a * N + j];
        struct interp_ctx s = {dim, ncell, U, {0, 0, 0}};
        for_each_tap(dim, n, bc, qj, interp_tap, &s);
        for (int a = 0; a < dim; ++a) qdot[(long)a * N + j] = s.acc[a];
    }
}

/* ------------------------------------------------------------------------ */
/* Interface forces                                                          */
/* ------------------------------------------------------------------------ */

/* eq. (A_choice) */
double orc_wetting_strength(double sigma, double theta, double xi, int n, int m)
{
    return sigma * (double)((m - 1) * (n - 1)) / ((double)(n - m) * xi) * (1.0 + cos(theta));
}

/* eq. (disjoin-p) */
double orc_pi(double h, double A, double xi, int n, int m)
{
    return A * (pow(xi / h, n) - pow(xi / h, m));
}

/* 2D closed polygon, nodes counter-clockwise.  The membrane energy is sigma
 * times the perimeter (line tension), so the nodal surface-tension force is
 *   phi_sigma_j = -sigma d|Gamma|/dq_j = sigma (t_j - t_{j-1}),
 * t_j the unit tangent of edge j -> j+1.  The wetting force uses the node
 * normal (mean of the two adjacent edge normals, renormalised), the length
 * associated with the node chi_j = l_{j-1} + l_j, shared by the two nodes of
 * each edge (factor 1/2, the 2D counterpart of 1/3), and h_j = q_j,y.
 * q, phi: [2][N].  Outputs: phi (total), and optional normals [2][N]. */
void orc_forces_2d(int N, const double *q, double sigma, double A, double xi,
                   int n, int m, int wetting, double *phi, double *normal_out)
{
    const double *x = q, *y = q + N;
    for (int j = 0; j < N; ++j) {
        int jp = (j + 1) % N, jm = (j - 1 + N) % N;
        double ex = x[jp] - x[j], ey = y[jp] - y[j];           /* edge j */
        double fx = x[j] - x[jm], fy = y[j] - y[jm];           /* edge j-1 */
        double le = sqrt(ex * ex + ey * ey), lf = sqrt(fx * fx + fy * fy);
        double px = sigma * (ex / le - fx / lf);
        double py = sigma * (ey / le - fy / lf);
        /* outward unit normals of the two edges */
        double nex = ey / le, ney = -ex / le;
        double nfx = fy / lf, nfy = -fx / lf;
        double nx_ = nex + nfx, ny_ = ney + nfy;
        double nn = sqrt(nx_ * nx_ + ny_ * ny_);
        nx_ /= nn;
        ny_ /= nn;
        if (wetting) {
            double chi = le + lf;
            double P = orc_pi(y[j], A, xi, n, m);
            px += -(chi / 2.0) * P * nx_;
            py += -(chi / 2.0) * P * ny_;
        }
        phi[j] = px;
        phi[N + j] = py;
        if (normal_out) {
            normal_out[j] = nx_;
            normal_out[N + j] = ny_;
        }
    }
}

static double norm3(const double *a) { return sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]); }
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* 3D closed triangle mesh, triangles counter-clockwise seen from outside.
 * The membrane energy is sigma times the total area, so for triangle
 * (a, b, c) with unit normal n_t
 *   phi_sigma_a += -sigma d(area)/dq_a = -(sigma/2) n_t x (q_c - q_b)
 * and cyclically for b and c.  Wetting: n_j is the mean of the unit normals
 * of the faces sharing node j (renormalised), chi_j the sum of their areas,
 * phi_Pi_j = -(chi_j / 3) Pi(h_j) n_j with h_j = q_j,z.
 * q, phi: [3][N]; tri: [T][3]. */
void orc_forces_3d(int N, const double *q, int T, const int *tri, double sigma,
                   double A, double xi, int n, int m, int wetting, double *phi,
                   double *normal_out)
{
    double *nsum = (double *)calloc((size_t)3 * N, sizeof(double));
    double *chi = (double *)calloc((size_t)N, sizeof(double));
    for (long k = 0; k < 3L * N; ++k) phi[k] = 0.0;
    for (int t = 0; t < T; ++t) {
        int v[3] = {tri[3 * t], tri[3 * t + 1], tri[3 * t + 2]};
        double P[3][3];
        for (int s = 0; s < 3; ++s)
            for (int a = 0; a < 3; ++a) P[s][a] = q[(long)a * N + v[s]];
        double e1[3], e2[3], nt[3];
        for (int a = 0; a < 3; ++a) {
            e1[a] = P[1][a] - P[0][a];
            e2[a] = P[2][a] - P[0][a];
        }
        cross3(e1, e2, nt);
        double len = sqrt(nt[0] * nt[0] + nt[1] * nt[1] + nt[2] * nt[2]);
        double area = 0.5 * len;
        for (int a = 0; a < 3; ++a) nt[a] /= len;
        for (int s = 0; s < 3; ++s) {
            int sb = (s + 1) % 3, sc = (s + 2) % 3;
            double d[3], g[3];
            for (int a = 0; a < 3; ++a) d[a] = P[sc][a] - P[sb][a];
            cross3(nt, d, g);
            for (int a = 0; a < 3; ++a) {
                phi[(long)a * N + v[s]] += -0.5 * sigma * g[a];
                nsum[(long)a * N + v[s]] += nt[a];
            }
            chi[v[s]] += area;
        }
    }
    for (int j = 0; j < N; ++j) {
        double nv[3];
        for (int a = 0; a < 3; ++a) nv[a] = nsum[(long)a * N + j];
        double nn = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
        for (int a = 0; a < 3; ++a) nv[a] /= nn;
        if (wetting) {
            double Pi = orc_pi(q[2L * N + j], A, xi, n, m);
            for (int a = 0; a < 3; ++a) phi[(long)a * N + j] += -(chi[j] / 3.0) * Pi * nv[a];
        }
        if (normal_out)
            for (int a = 0; a < 3; ++a) normal_out[(long)a * N + j] = nv[a];
    }
    free(nsum);
    free(chi);
}

/* ------------------------------------------------------------------------ */
/* Elastic interface: shear part of the strain energy                        */
/* ------------------------------------------------------------------------ */
/* On a linear triangle the map from the reference triangle (vertices Q_k)  */
/* to the current one (q_k) has a constant in-plane deformation gradient.   */
/* With the reference edges written in an orthonormal frame of their own    */
/* plane, E0 = [Q1 - Q0, Q2 - Q0] (2 x 2), and the current edges            */
/* E = [q1 - q0, q2 - q0] (3 x 2), the gradient is F = E E0^-1 (3 x 2).     */
/* G = F^T F has the nonzero eigenvalues of D D^T, so the invariants of eq.  */
/* strain_inv are a = (1/2) log det G and b = (1/2) tr G - 1.  For           */
/*   w_s(a, b) = mu_s (b + 1 - e^a) = mu_s (l1 - l2)^2 / 2                   */
/* (l1, l2 the principal stretches) the triangle's energy is A0 w_s, A0 the  */
/* reference area, and with d(a)/dF = F G^-1, d(b)/dF = F:                   */
/*   dW/dF = A0 mu_s (F - e^a F G^-1),  dW/dE = dW/dF E0^-T,                 */
/* whose columns are dW/dq1 and dW/dq2; dW/dq0 = -(dW/dq1 + dW/dq2).         */
/* The force is phi = -dW/dq.  Added to phi (q, qref: [3][N]; tri [T][3]).  */
static void add_shear_forces(int N, const double *q, const double *qref, int T, const int *tri,
                             double mu_s, double *phi)
{
    for (int t = 0; t < T; ++t) {
        int v[3] = {tri[3 * t], tri[3 * t + 1], tri[3 * t + 2]};
        double R[3][3], P[3][3];
        for (int s = 0; s < 3; ++s)
            for (int k = 0; k < 3; ++k) {
                R[s][k] = qref[(long)k * N + v[s]];
                P[s][k] = q[(long)k * N + v[s]];
            }
        double r1[3], r2[3], e1[3], e2[3];
        for (int k = 0; k < 3; ++k) {
            r1[k] = R[1][k] - R[0][k];
            r2[k] = R[2][k] - R[0][k];
            e1[k] = P[1][k] - P[0][k];
            e2[k] = P[2][k] - P[0][k];
        }
        /* reference frame: t1 along r1, t2 in the plane, orthogonal to t1 */
        double l1 = sqrt(dot3(r1, r1)), nr[3], t1[3], t2[3];
        for (int k = 0; k < 3; ++k) t1[k] = r1[k] / l1;
        cross3(r1, r2, nr);
        double A0 = 0.5 * sqrt(dot3(nr, nr));
        cross3(nr, t1, t2);
        double ln = sqrt(dot3(t2, t2));
        for (int k = 0; k < 3; ++k) t2[k] /= ln;
        /* E0 = [[r1.t1, r2.t1], [r1.t2, r2.t2]] and its inverse */
        double E0[2][2] = {{dot3(r1, t1), dot3(r2, t1)}, {dot3(r1, t2), dot3(r2, t2)}};
        double det0 = E0[0][0] * E0[1][1] - E0[0][1] * E0[1][0];
        double Ei[2][2] = {{E0[1][1] / det0, -E0[0][1] / det0}, {-E0[1][0] / det0, E0[0][0] / det0}};
        /* F = E Ei (3 x 2) */
        double F[3][2];
        for (int k = 0; k < 3; ++k)
            for (int c = 0; c < 2; ++c) F[k][c] = e1[k] * Ei[0][c] + e2[k] * Ei[1][c];
        /* G = F^T F */
        double G[2][2];
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c) {
                G[r][c] = 0.0;
                for (int k = 0; k < 3; ++k) G[r][c] += F[k][r] * F[k][c];
            }
        double detG = G[0][0] * G[1][1] - G[0][1] * G[1][0];
        double ea = sqrt(detG); /* e^a */
        double Gi[2][2] = {{G[1][1] / detG, -G[0][1] / detG}, {-G[1][0] / detG, G[0][0] / detG}};
        /* dW/dF = A0 mu_s (F - e^a F G^-1) */
        double dF[3][2];
        for (int k = 0; k < 3; ++k)
            for (int c = 0; c < 2; ++c) {
                double fg = F[k][0] * Gi[0][c] + F[k][1] * Gi[1][c];
                dF[k][c] = A0 * mu_s * (F[k][c] - ea * fg);
            }
        /* dW/dE = dW/dF Ei^T: columns for q1 and q2 */
        for (int k = 0; k < 3; ++k) {
            double g1 = dF[k][0] * Ei[0][0] + dF[k][1] * Ei[0][1];
            double g2 = dF[k][0] * Ei[1][0] + dF[k][1] * Ei[1][1];
            phi[(long)k * N + v[1]] -= g1;
            phi[(long)k * N + v[2]] -= g2;
            phi[(long)k * N + v[0]] += g1 + g2;
        }
    }
}

/* Forces of eq. force_split with the elastic interface: orc_forces_3d plus
 * the shear part measured from the reference positions qref ([3][N]). */
void orc_forces_3d_elastic(int N, const double *q, const double *qref, int T, const int *tri,
                           double sigma, double mu_s, double A, double xi, int n, int m,
                           int wetting, double *phi, double *normal_out)
{
    orc_forces_3d(N, q, T, tri, sigma, A, xi, n, m, wetting, phi, normal_out);
    if (mu_s != 0.0) add_shear_forces(N, q, qref, T, tri, mu_s, phi);
}

/* ------------------------------------------------------------------------ */
/* Cells enclosed by the interface (Sec. IB-LB, last paragraph)              */
/* ------------------------------------------------------------------------ */
/* The paper finds the cells inside the closed interface by ray tracing.     */
/* Here the plain definition of "enclosed" is used instead: the winding      */
/* number of the interface around the cell centre, which is +-1 inside a    */
/* closed, non-self-intersecting interface and 0 outside.                    */
/*   2D: the sum over the polygon's edges of the signed angle under which    */
/*       the edge is seen from the point, over 2 pi;                         */
/*   3D: the sum over the triangles of the signed solid angle under which    */
/*       the triangle is seen from the point (van Oosterom and Strackee,     */
/*       IEEE Trans. Biomed. Eng. 30 (1983) 125), over 4 pi.                */
/* The interface is never wrapped across a periodic boundary; a cell centre  */
/* is taken at its periodic image in the window [ref - n/2, ref + n/2) of    */
/* each periodic axis, ref a point of the droplet.  The image the interface  */
/* can enclose is that one as long as the droplet stays inside the window.   */
static double image_in_window(double c, double ref, int n, int periodic)
{
    if (!periodic) return c;
    double lo = ref - 0.5 * n;
    return c + n * ceil((lo - c) / n);
}

static double winding_2d(int N, const double *q, const double *p)
{
    const double *x = q, *y = q + N;
    double w = 0.0;
    for (int j = 0; j < N; ++j) {
        int jp = (j + 1) % N;
        double ax = x[j] - p[0], ay = y[j] - p[1];
        double bx = x[jp] - p[0], by = y[jp] - p[1];
        w += atan2(ax * by - ay * bx, ax * bx + ay * by);
    }
    return w / (2.0 * PI);
}


static double winding_3d(int N, const double *q, int T, const int *tri, const double *p)
{
    double w = 0.0;
    for (int t = 0; t < T; ++t) {
        double a[3], b[3], c[3], bc_[3];
        for (int k = 0; k < 3; ++k) {
            a[k] = q[(long)k * N + tri[3 * t]] - p[k];
            b[k] = q[(long)k * N + tri[3 * t + 1]] - p[k];
            c[k] = q[(long)k * N + tri[3 * t + 2]] - p[k];
        }
        cross3(b, c, bc_);
        double la = norm3(a), lb = norm3(b), lc = norm3(c);
        double num = dot3(a, bc_);
        double den = la * lb * lc + dot3(a, b) * lc + dot3(a, c) * lb + dot3(b, c) * la;
        w += 2.0 * atan2(num, den);
    }
    return w / (4.0 * PI);
}

/* inside[cell] = 1 for cells enclosed by the interface (q: [dim][N]; tri:
 * [T][3], 3D only), 0 otherwise.  ref: [3] window centre (see above). */
void orc_inside(int dim, int nx, int ny, int nz, const int *bc, int N, const double *q,
                int T, const int *tri, const double *ref, int *inside)
{
    const int n[3] = {nx, ny, nz};
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int pos[3] = {x, y, z};
                double p[3] = {0.0, 0.0, 0.0};
                for (int a = 0; a < dim; ++a)
                    p[a] = image_in_window(pos[a] + 0.5, ref[a], n[a], bc[a] == ORC_PERIODIC);
                double w = dim == 2 ? winding_2d(N, q, p) : winding_3d(N, q, T, tri, p);
                inside[((long)z * ny + y) * nx + x] = fabs(w) > 0.5;
            }
}

/* orc_inside for the listed cells only (cells: flat indices [z][y][x]). */
void orc_inside_cells(int dim, int nx, int ny, int nz, const int *bc, int N, const double *q,
                      int T, const int *tri, const double *ref, long ncells, const long *cells,
                      int *inside)
{
    const int n[3] = {nx, ny, nz};
    for (long k = 0; k < ncells; ++k) {
        const long cell = cells[k];
        const int pos[3] = {(int)(cell % nx), (int)((cell / nx) % ny), (int)(cell / ((long)nx * ny))};
        double p[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < dim; ++a)
            p[a] = image_in_window(pos[a] + 0.5, ref[a], n[a], bc[a] == ORC_PERIODIC);
        double w = dim == 2 ? winding_2d(N, q, p) : winding_3d(N, q, T, tri, p);
        inside[k] = fabs(w) > 0.5;
    }
}

/* Tangential re-spacing of a closed 2D outline: an addition to the method,
 * not part of the paper.  Node j moves along the chord of its neighbours,
 *   dq_j = (beta / 2) (l_j+ - l_j-) (q_{j+1} - q_{j-1}) / |q_{j+1} - q_{j-1}|,
 * with l_j- = |q_j - q_{j-1}| and l_j+ = |q_{j+1} - q_j| (ring indices).
 * Uniformly spaced nodes do not move; along a straight run of nodes this is
 * an explicit diffusion of the node positions along the line (stable for
 * beta < 1) that keeps them on it, so the outline's shape changes only at
 * second order where it is curved.  q, dq: [2][N]. */
void orc_respace_2d(int N, const double *q, double beta, double *dq)
{
    for (int j = 0; j < N; ++j) {
        const int a = j == 0 ? N - 1 : j - 1, b = j == N - 1 ? 0 : j + 1;
        const double xa = q[a], ya = q[N + a], xj = q[j], yj = q[N + j], xb = q[b], yb = q[N + b];
        const double lm = sqrt((xj - xa) * (xj - xa) + (yj - ya) * (yj - ya));
        const double lp = sqrt((xb - xj) * (xb - xj) + (yb - yj) * (yb - yj));
        const double cx = xb - xa, cy = yb - ya;
        const double c = sqrt(cx * cx + cy * cy);
        const double s = c > 0.0 ? 0.5 * beta * (lp - lm) / c : 0.0;
        dq[j] = s * cx;
        dq[N + j] = s * cy;
    }
}

/* ------------------------------------------------------------------------ */
/* Time loop                                                                 */
/* ------------------------------------------------------------------------ */

/* Run nsteps of the coupled method.  Order inside a step: nodal forces at
 * q(t) -> spread to F(t) -> LB step with F(t) (in the Guo source and the
 * half-force velocity alike) -> interpolate U(t) at q(t) -> q(t+1).
 * mu_s != 0 (3D) adds the shear part of the elastic interface measured from
 * the reference positions qref ([3][N]).
 * respace > 0 (2D) adds orc_respace_2d's tangential re-spacing, computed
 * from q(t), to the advected positions: q(t+1) = (q(t) + qdot) + dq.
 * With tau_in != tau the cells enclosed by the interface at q(t) relax with
 * tau_in in the LB step of step t and the others with tau (classification
 * window centred on ref[3]; see orc_inside).
 *
 * f: [Q][ncell] post-collision populations, updated in place.
 * q: [dim][N] node positions, updated in place.
 * rho, U, F: outputs of the last step ([ncell], [3][ncell], [3][ncell]).
 * phi, qdot: outputs of the last step ([dim][N]).  dropped: [3].
 * N = 0 runs the fluid alone with the prescribed force field F_fixed
 * (may be NULL).  Returns 0, or -4 if a node reached h <= 0 (wetting on). */
int orc_run(int dim, int nx, int ny, int nz, const int *bc, double tau, double tau_in,
            const double *ref, double sigma, double mu_s, const double *qref, double theta,
            double xi, int n_exp, int m_exp, int wetting, double respace,
            int N, double *q, int T, const int *tri, int nsteps,
            double *f, double *rho, double *U, double *F, const double *F_fixed,
            double *phi, double *qdot, double *dropped)
{
    const int Q = nq(dim);
    const long ncell = (long)nx * ny * nz;
    double *g = (double *)malloc(sizeof(double) * Q * ncell);
    double A = orc_wetting_strength(sigma, theta, xi, n_exp, m_exp);
    const int two_tau = N > 0 && tau_in != tau;
    double *tau_cell = two_tau ? (double *)malloc(sizeof(double) * ncell) : NULL;
    int *inside = two_tau ? (int *)malloc(sizeof(int) * ncell) : NULL;
    double *dq = (dim == 2 && N > 0 && respace > 0.0) ? (double *)malloc(sizeof(double) * 2 * N) : NULL;
    int status = 0;
    for (int t = 0; t < nsteps; ++t) {
        if (N > 0) {
            if (wetting)
                for (int j = 0; j < N; ++j)
                    if (q[(long)(dim - 1) * N + j] <= 0.0) status = -4;
            if (status) break;
            if (dim == 2)
                orc_forces_2d(N, q, sigma, A, xi, n_exp, m_exp, wetting, phi, NULL);
            else
                orc_forces_3d_elastic(N, q, qref, T, tri, sigma, mu_s, A, xi, n_exp, m_exp,
                                      wetting, phi, NULL);
            orc_spread(dim, nx, ny, nz, bc, N, q, phi, F, dropped);
            if (two_tau) {
                orc_inside(dim, nx, ny, nz, bc, N, q, T, tri, ref, inside);
                for (long k = 0; k < ncell; ++k) tau_cell[k] = inside[k] ? tau_in : tau;
            }
        } else if (F_fixed) {
            memcpy(F, F_fixed, sizeof(double) * 3 * ncell);
        } else {
            memset(F, 0, sizeof(double) * 3 * ncell);
        }
        orc_lb_step(dim, nx, ny, nz, bc, tau, tau_cell, f, F, g, rho, U);
        memcpy(f, g, sizeof(double) * Q * ncell);
        if (N > 0) {
            orc_interp(dim, nx, ny, nz, bc, U, N, q, qdot);
            if (dq) {
                orc_respace_2d(N, q, respace, dq);
                for (long k = 0; k < 2L * N; ++k) q[k] = (q[k] + qdot[k]) + dq[k];
            } else {
                for (long k = 0; k < (long)dim * N; ++k) q[k] += qdot[k];
            }
        }
    }
    free(g);
    free(dq);
    free(tau_cell);
    free(inside);
    return status;
}

/* Threads used by the lattice update (OpenMP over rows; 1 without OpenMP).
 * n <= 0 leaves the count unchanged.  Returns the count in force. */
int orc_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
