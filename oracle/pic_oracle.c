/*
 * pic_oracle.c -- the FP64 CPU oracle for the particle-in-cell step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, obviously correct
 * transcription of the method of "YUNIC: A Multi-Dimensional Particle-In-Cell
 * Code for Laser-Plasma Interaction" (Song, Wang, Li; arXiv:2104.00642), used
 * to check the HIP path.  Only the test-suite, the smoke entry and the
 * benchmark's CPU-baseline leg may load it.  It shares no code with the HIP
 * library and never calls it.
 *
 * Everything is in the normalized units of Sec. II.A (Eq. 8): time in 1/w_r,
 * length in c/w_r, E and B in m_e c w_r / e, u = p/m in units of c, charge in
 * e, mass in m_e, density (and macro-particle weight) in n_r, current in
 * c e n_r.  In these units Eq. 4 reads dE/dt = curl B - J and Eq. 1 reads
 * div E = rho.
 *
 * Positions are ABSOLUTE FP64 coordinates x (not cell + offset).  The grid
 * node i of an unstaggered quantity sits at x = i*dx; a quantity staggered by
 * one half cell along an axis has its array index i at x = (i + 1/2)*dx
 * (the Yee cell of Sec. II.B, Fig. 1):
 *   E_x, J_x : (1/2, 0, 0)    B_x : (0, 1/2, 1/2)
 *   E_y, J_y : (0, 1/2, 0)    B_y : (1/2, 0, 1/2)
 *   E_z, J_z : (0, 0, 1/2)    B_z : (1/2, 1/2, 0)
 * In 2D3V the z offsets are dropped and d/dz = 0.
 *
 * Field arrays are one FP64 plane per component, index i + n0*(j + n1*k),
 * periodic in every axis.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t dim;     /* 2 (2D3V) or 3 (3D3V)                          */
    int32_t order;   /* 1 = linear (CIC), 2 = quadratic, 4 = quartic      */
    int64_t n[3];    /* cells per axis; n[2] = 1 in 2D                   */
    double d[3];     /* cell sizes dx, dy, dz                            */
    double dt;       /* time step                                        */
    int32_t pusher;  /* 0 Boris (Sec. II.C), 1 Vay                       */
    int32_t absorb_x;  /* absorbing faces at x = 0 and x = (n-1) dx: 1 first-, 2 second-order Mur */
    double laser[4];   /* a0, waist, duration, t0 of the pulse injected
                          through x = 0 (a0 = 0: none)                   */
    int32_t laser_circular;
} orc_grid;

/* Component stagger in half cells, indexed [component][axis];
 * components 0..2 = E_x,E_y,E_z (also J), 3..5 = B_x,B_y,B_z. */
#define ORC_PI 3.14159265358979323846

static const double STAG3[6][3] = {
    {0.5, 0.0, 0.0}, {0.0, 0.5, 0.0}, {0.0, 0.0, 0.5},
    {0.0, 0.5, 0.5}, {0.5, 0.0, 0.5}, {0.5, 0.5, 0.0}};

static int64_t wrap(int64_t i, int64_t n) {
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

static int64_t idx3(const orc_grid *g, int64_t i, int64_t j, int64_t k) {
    return wrap(i, g->n[0]) + g->n[0] * (wrap(j, g->n[1]) + g->n[1] * wrap(k, g->n[2]));
}

/*
 * Cell-integrated shape weights W_n of Sec. II.D: W(i) is the integral over
 * the cell [i-1/2, i+1/2] of the particle shape centred on the particle
 * (Eqs. 17-18).  `xi` is the particle position in cell units, already shifted
 * by the component stagger.  Writes the first node to *i0 and the weights of
 * the consecutive support nodes to w[]; returns the number of nodes.
 *   order 1: shape = unit top-hat; weights (1-delta, delta) on
 *            floor(xi), floor(xi)+1 (the order-1 member of the family).
 *   order 2: shape = S_2 (triangle, Eq. 17); i_c is the node nearest to xi,
 *            delta = xi - i_c in [-1/2, 1/2), weights
 *            ((1/2 - delta)^2 / 2, 3/4 - delta^2, (1/2 + delta)^2 / 2).
 *   order 4: shape = S_4 (cubic spline, Eq. 18); same i_c and delta, five
 *            weights on i_c-2 .. i_c+2, the cell integrals of S_4 worked out
 *            piece by piece (a quartic spline):
 *            (1-2d)^4/384, (19-44d+24d^2+16d^3-16d^4)/96,
 *            (115-120d^2+48d^4)/192, (19+44d+24d^2-16d^3-16d^4)/96,
 *            (1+2d)^4/384.
 */
int orc_shape(int order, double xi, int64_t *i0, double *w) {
    if (order == 1) {
        double f = floor(xi);
        double delta = xi - f;
        *i0 = (int64_t)f;
        w[0] = 1.0 - delta;
        w[1] = delta;
        return 2;
    }
    if (order == 2) {
        double ic = floor(xi + 0.5);
        double delta = xi - ic;
        *i0 = (int64_t)ic - 1;
        w[0] = 0.5 * (0.5 - delta) * (0.5 - delta);
        w[1] = 0.75 - delta * delta;
        w[2] = 0.5 * (0.5 + delta) * (0.5 + delta);
        return 3;
    }
    if (order == 4) {
        double ic = floor(xi + 0.5);
        double d = xi - ic;
        *i0 = (int64_t)ic - 2;
        w[0] = pow(1.0 - 2.0 * d, 4) / 384.0;
        w[1] = (19.0 - 44.0 * d + 24.0 * d * d + 16.0 * d * d * d - 16.0 * d * d * d * d) / 96.0;
        w[2] = (115.0 - 120.0 * d * d + 48.0 * d * d * d * d) / 192.0;
        w[3] = (19.0 + 44.0 * d + 24.0 * d * d - 16.0 * d * d * d - 16.0 * d * d * d * d) / 96.0;
        w[4] = pow(1.0 + 2.0 * d, 4) / 384.0;
        return 5;
    }
    return 0;
}

/*
 * Field interpolation, Eq. 19: each of the six components is the sum over its
 * own staggered nodes of the product of per-axis weights times the node value.
 * F[c] points at the plane of component c (E_x..E_z, B_x..B_z); x is the
 * absolute position.  Result in EB[6].
 */
/* With absorbing x faces, nodes with x index outside [0, n) lie beyond the
 * faces: no field there, and current deposited there leaves the domain. */
static int beyond_x(const orc_grid *g, int64_t i) { return g->absorb_x && (i < 0 || i >= g->n[0]); }

static void jadd(const orc_grid *g, double *J, int64_t i, int64_t j, int64_t k, double v) {
    if (!beyond_x(g, i)) J[idx3(g, i, j, k)] += v;
}

void orc_gather(const orc_grid *g, const double *const *F, const double *x, double *EB) {
    for (int c = 0; c < 6; ++c) {
        int64_t i0[3] = {0, 0, 0};
        double w[3][5];
        int nw[3] = {1, 1, 1};
        w[2][0] = 1.0;
        for (int a = 0; a < g->dim; ++a) {
            /* 2D3V: the staggers of B_x, B_y (z half offsets) are dropped. */
            double s = STAG3[c][a];
            nw[a] = orc_shape(g->order, x[a] / g->d[a] - s, &i0[a], w[a]);
        }
        double acc = 0.0;
        for (int kk = 0; kk < nw[2]; ++kk)
            for (int jj = 0; jj < nw[1]; ++jj)
                for (int ii = 0; ii < nw[0]; ++ii)
                    if (!beyond_x(g, i0[0] + ii))
                        acc += w[0][ii] * w[1][jj] * w[2][kk] *
                               F[c][idx3(g, i0[0] + ii, i0[1] + jj, i0[2] + kk)];
        EB[c] = acc;
    }
}

/*
 * Boris pusher, Sec. II.C Eqs. 13-16: half electric kick, rotation about B by
 * t = q_m dt B / (2 gamma), second half electric kick.  gamma^{n+1/2} is taken
 * from u^- (the rotation keeps |u| so u^+ gives the same value).  In place on u.
 */
void orc_boris(double qm, double dt, const double *E, const double *B, double *u) {
    double um[3], up[3], t[3], s[3], uprime[3];
    for (int a = 0; a < 3; ++a) um[a] = u[a] + 0.5 * qm * dt * E[a];
    double gh = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
    for (int a = 0; a < 3; ++a) t[a] = 0.5 * qm * dt * B[a] / gh;
    double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    for (int a = 0; a < 3; ++a) s[a] = 2.0 * t[a] / (1.0 + t2);
    uprime[0] = um[0] + (um[1] * t[2] - um[2] * t[1]);
    uprime[1] = um[1] + (um[2] * t[0] - um[0] * t[2]);
    uprime[2] = um[2] + (um[0] * t[1] - um[1] * t[0]);
    up[0] = um[0] + (uprime[1] * s[2] - uprime[2] * s[1]);
    up[1] = um[1] + (uprime[2] * s[0] - uprime[0] * s[2]);
    up[2] = um[2] + (uprime[0] * s[1] - uprime[1] * s[0]);
    for (int a = 0; a < 3; ++a) u[a] = up[a] + 0.5 * qm * dt * E[a];
}

/*
 * Vay pusher, the alternative Sec. II.C names for fields whose electric and
 * magnetic forces nearly cancel (J.-L. Vay, Phys. Plasmas 15, 056701 (2008)).
 * It advances u by the implicit equation
 *   u^{n+1} - u^n = q_m dt (E + (v^n + v^{n+1})/2 x B),   v = u / gamma,
 * which it solves in closed form: with h = q_m dt / 2,
 *   u' = u^n + 2 h E + h v^n x B,   tau = h B,   u* = u'.tau,
 *   sigma = 1 + |u'|^2 - |tau|^2,
 *   gamma^{n+1} = sqrt((sigma + sqrt(sigma^2 + 4 (|tau|^2 + u*^2))) / 2),
 *   t = tau / gamma^{n+1},
 *   u^{n+1} = (u' + (u'.t) t + u' x t) / (1 + |t|^2).
 * In place on u.
 */
void orc_vay(double qm, double dt, const double *E, const double *B, double *u) {
    double h = 0.5 * qm * dt;
    double g0 = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    double v[3] = {u[0] / g0, u[1] / g0, u[2] / g0};
    double tau[3] = {h * B[0], h * B[1], h * B[2]};
    double up[3];
    up[0] = u[0] + 2.0 * h * E[0] + (v[1] * tau[2] - v[2] * tau[1]);
    up[1] = u[1] + 2.0 * h * E[1] + (v[2] * tau[0] - v[0] * tau[2]);
    up[2] = u[2] + 2.0 * h * E[2] + (v[0] * tau[1] - v[1] * tau[0]);
    double tau2 = tau[0] * tau[0] + tau[1] * tau[1] + tau[2] * tau[2];
    double ustar = up[0] * tau[0] + up[1] * tau[1] + up[2] * tau[2];
    double sigma = 1.0 + up[0] * up[0] + up[1] * up[1] + up[2] * up[2] - tau2;
    double gn = sqrt(0.5 * (sigma + sqrt(sigma * sigma + 4.0 * (tau2 + ustar * ustar))));
    double t[3] = {tau[0] / gn, tau[1] / gn, tau[2] / gn};
    double s = 1.0 / (1.0 + t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    double ut = up[0] * t[0] + up[1] * t[1] + up[2] * t[2];
    u[0] = s * (up[0] + ut * t[0] + (up[1] * t[2] - up[2] * t[1]));
    u[1] = s * (up[1] + ut * t[1] + (up[2] * t[0] - up[0] * t[2]));
    u[2] = s * (up[2] + ut * t[2] + (up[0] * t[1] - up[1] * t[0]));
}

/*
 * Node weights of the particle charge along one axis on a stencil of `len`
 * nodes starting at `base` (integer nodes, no stagger).  Zero outside the
 * shape support.
 */
static void stencil_weights(int order, double xi, int64_t base, int len, double *S) {
    int64_t i0;
    double w[5];
    int nw = orc_shape(order, xi, &i0, w);
    for (int k = 0; k < len; ++k) S[k] = 0.0;
    for (int k = 0; k < nw; ++k) {
        int64_t pos = i0 + k - base;
        if (pos >= 0 && pos < len) S[pos] = w[k];
    }
}

/*
 * Esirkepov charge-conserving current deposit, Sec. II.E Eqs. 20-22, with the
 * decomposition W_x, W_y, W_z of the cited method (straight trajectory over
 * one step, shapes varying linearly in time along it).  The particle moves
 * from xh to xe (absolute positions, |xe - xh| < one cell per axis).  On a
 * stencil of order+2 nodes per axis starting at the lower of the two support
 * starts, S0/S1 are the node weights at the start/end and DS = S1 - S0.
 * Running sums from the low stencil edge give the current:
 *   J_x(i+1/2) = J_x(i-1/2) - q w (dx/dt) W_x(i)   (same for y, z).
 * In 2D3V J_z = q w v_z * [S0x S0y + DSx S0y/2 + S0x DSy/2 + DSx DSy/3].
 * J[a] is the plane of component a; `qw` = q * weight.
 */
void orc_deposit(const orc_grid *g, double qw, const double *xh, const double *xe, double vz,
                 double *const *J) {
    const int len = g->order + 2;
    double S0[3][6], DS[3][6];
    int64_t base[3] = {0, 0, 0};
    for (int a = 0; a < g->dim; ++a) {
        double w[5];
        int64_t ih, ie;
        orc_shape(g->order, xh[a] / g->d[a], &ih, w);
        orc_shape(g->order, xe[a] / g->d[a], &ie, w);
        base[a] = ih < ie ? ih : ie;
        double S1[6];
        stencil_weights(g->order, xh[a] / g->d[a], base[a], len, S0[a]);
        stencil_weights(g->order, xe[a] / g->d[a], base[a], len, S1);
        for (int k = 0; k < len; ++k) DS[a][k] = S1[k] - S0[a][k];
    }
    const double cx = qw * g->d[0] / g->dt, cy = qw * g->d[1] / g->dt;
    if (g->dim == 2) {
        /* J_x: running sum along x for each y row. */
        for (int jj = 0; jj < len; ++jj) {
            double acc = 0.0;
            for (int ii = 0; ii < len - 1; ++ii) {
                double Wx = DS[0][ii] * (S0[1][jj] + 0.5 * DS[1][jj]);
                acc -= cx * Wx;
                jadd(g, J[0], base[0] + ii, base[1] + jj, 0, acc);
            }
        }
        /* J_y: running sum along y for each x column. */
        for (int ii = 0; ii < len; ++ii) {
            double acc = 0.0;
            for (int jj = 0; jj < len - 1; ++jj) {
                double Wy = (S0[0][ii] + 0.5 * DS[0][ii]) * DS[1][jj];
                acc -= cy * Wy;
                jadd(g, J[1], base[0] + ii, base[1] + jj, 0, acc);
            }
        }
        /* J_z from the out-of-plane velocity. */
        for (int jj = 0; jj < len; ++jj)
            for (int ii = 0; ii < len; ++ii) {
                double Wz = S0[0][ii] * S0[1][jj] + 0.5 * DS[0][ii] * S0[1][jj] +
                            0.5 * S0[0][ii] * DS[1][jj] +
                            (1.0 / 3.0) * DS[0][ii] * DS[1][jj];
                jadd(g, J[2], base[0] + ii, base[1] + jj, 0, qw * vz * Wz);
            }
        return;
    }
    const double cz = qw * g->d[2] / g->dt;
    for (int kk = 0; kk < len; ++kk)
        for (int jj = 0; jj < len; ++jj) {
            double acc = 0.0;
            for (int ii = 0; ii < len - 1; ++ii) {
                double Wx = DS[0][ii] * (S0[1][jj] * S0[2][kk] + 0.5 * DS[1][jj] * S0[2][kk] +
                                         0.5 * S0[1][jj] * DS[2][kk] +
                                         (1.0 / 3.0) * DS[1][jj] * DS[2][kk]);
                acc -= cx * Wx;
                jadd(g, J[0], base[0] + ii, base[1] + jj, base[2] + kk, acc);
            }
        }
    for (int kk = 0; kk < len; ++kk)
        for (int ii = 0; ii < len; ++ii) {
            double acc = 0.0;
            for (int jj = 0; jj < len - 1; ++jj) {
                double Wy = DS[1][jj] * (S0[0][ii] * S0[2][kk] + 0.5 * DS[0][ii] * S0[2][kk] +
                                         0.5 * S0[0][ii] * DS[2][kk] +
                                         (1.0 / 3.0) * DS[0][ii] * DS[2][kk]);
                acc -= cy * Wy;
                jadd(g, J[1], base[0] + ii, base[1] + jj, base[2] + kk, acc);
            }
        }
    for (int jj = 0; jj < len; ++jj)
        for (int ii = 0; ii < len; ++ii) {
            double acc = 0.0;
            for (int kk = 0; kk < len - 1; ++kk) {
                double Wz = DS[2][kk] * (S0[0][ii] * S0[1][jj] + 0.5 * DS[0][ii] * S0[1][jj] +
                                         0.5 * S0[0][ii] * DS[1][jj] +
                                         (1.0 / 3.0) * DS[0][ii] * DS[1][jj]);
                acc -= cz * Wz;
                jadd(g, J[2], base[0] + ii, base[1] + jj, base[2] + kk, acc);
            }
        }
}

/*
 * One particle step of one species (gather, Boris or Vay, move, deposit) with fields
 * at time n+1/2, Sec. II.C-E in the full/half-step arrangement of Sec. II.F:
 *   1. gamma = sqrt(1+|u|^2); xh = x + dt u / (2 gamma)     (position n+1/2)
 *   2. gather E, B at xh (Eq. 19)
 *   3. Boris (Eqs. 13-16), or Vay (g->pusher = 1) -> u^{n+1}
 *   4. v = u^{n+1}/gamma^{n+1}; x^{n+1} = xh + dt v / 2; xe = xh + dt v  (Eq. 12)
 *   5. Esirkepov deposit of the move xh -> xe into J; periodic wrap of x
 *      (absorbing x faces: nothing is gathered from or deposited beyond
 *      them, and a particle leaving [0, (n-1) dx] gets weight 0).
 * x[a], u[a]: per-axis arrays of np particles (absolute FP64 positions);
 * w: per-particle weights or NULL (then w0); F: 6 field planes; J: 3 planes,
 * accumulated into.  diag (nullable) += {sum w m (gamma^{n+1}-1) dV,
 * sum q w dV}.
 */
void orc_push(const orc_grid *g, double q, double m, int64_t np, double *const *x,
              double *const *u, double *w, double w0, const double *const *F,
              double *const *J, double *diag) {
    const double qm = q / m, dt = g->dt;
    double dV = g->d[0] * g->d[1] * (g->dim == 3 ? g->d[2] : 1.0);
    double L[3];
    for (int a = 0; a < 3; ++a) L[a] = (double)g->n[a] * g->d[a];
    for (int64_t p = 0; p < np; ++p) {
        double up[3] = {u[0][p], u[1][p], u[2][p]};
        double xp[3] = {x[0][p], x[1][p], g->dim == 3 ? x[2][p] : 0.0};
        double wp = w ? w[p] : w0;
        double gam = sqrt(1.0 + up[0] * up[0] + up[1] * up[1] + up[2] * up[2]);
        double xh[3], xe[3], xn[3];
        for (int a = 0; a < 3; ++a) xh[a] = xp[a] + 0.5 * dt * up[a] / gam;
        double EB[6];
        orc_gather(g, F, xh, EB);
        if (g->pusher == 1) orc_vay(qm, dt, EB, EB + 3, up);
        else orc_boris(qm, dt, EB, EB + 3, up);
        double gn = sqrt(1.0 + up[0] * up[0] + up[1] * up[1] + up[2] * up[2]);
        for (int a = 0; a < 3; ++a) {
            double v = up[a] / gn;
            xn[a] = xh[a] + 0.5 * dt * v;
            xe[a] = xh[a] + dt * v;
        }
        orc_deposit(g, q * wp, xh, xe, up[2] / gn, J);
        /* absorbing x faces: a particle whose position leaves [0, (n-1) dx]
         * is absorbed (weight 0; its last move's current inside counted) */
        if (g->absorb_x && w && (xn[0] < 0.0 || xn[0] >= (double)(g->n[0] - 1) * g->d[0])) w[p] = 0.0;
        for (int a = 0; a < g->dim; ++a) {
            double r = fmod(xn[a], L[a]);
            if (r < 0) r += L[a];
            if (r >= L[a]) r -= L[a];
            x[a][p] = r;
        }
        for (int a = 0; a < 3; ++a) u[a][p] = up[a];
        if (diag) {
            diag[0] += wp * m * (gn - 1.0) * dV;
            diag[1] += q * wp * dV;
        }
    }
}

/*
 * Field of the pulse injected through x = 0, component 1 (E_y) or 2 (E_z),
 * at (x, y, z) and time t in laser units (w = k = c = 1):
 *   a0 exp(-r^2/w^2) S((t - t0 - x)/tau) sin(x - t  [+ pi/2 for E_z]),
 * S(s) = sin^2(pi s) on [0, 1] and 0 outside, r measured from the box axis;
 * E_z only for circular polarisation.
 */
static double orc_incident(const orc_grid *g, int comp, double x, double y, double z, double t) {
    double a0 = g->laser[0], w = g->laser[1], tau = g->laser[2], t0 = g->laser[3];
    if (a0 == 0.0 || (comp == 2 && !g->laser_circular)) return 0.0;
    double s = (t - t0 - x) / tau;
    if (s <= 0.0 || s >= 1.0) return 0.0;
    double yc = 0.5 * g->n[1] * g->d[1], zc = 0.5 * g->n[2] * g->d[2];
    double r2 = (y - yc) * (y - yc) + (g->dim == 3 ? (z - zc) * (z - zc) : 0.0);
    double env = sin(ORC_PI * s);
    return a0 * exp(-r2 / (w * w)) * env * env * sin(x - t + (comp == 2 ? 0.5 * ORC_PI : 0.0));
}

/*
 * Half field updates, Sec. II.B Eqs. 9-10 split in two halves (Sec. II.F):
 *   orc_half_e:  E += (dt/2) (curl B - J)      (t: time of E on entry)
 *   orc_half_b:  B -= (dt/2) curl E
 * Central differences on the Yee stagger, periodic.  A full step is
 * half_e(J^n); half_b; [particles]; half_b; half_e(J^{n+1}).
 *
 * Absorbing x faces (absorb_x): the domain is x in [0, (n-1) dx].  E_y and
 * E_z on the faces x = 0 and x = (n-1) dx follow Mur's rule over the half
 * step h = dt/2 (G. Mur, IEEE Trans. EMC 23, 377 (1981)); at x = 0 it acts
 * on E - E_inc, so the injected pulse enters while outgoing waves leave.
 * With node 0 on the face, node 1 inside, levels m-1, m, m+1 a half step
 * apart and k = (h - dx)/(h + dx):
 *   absorb_x = 1, first order, from the one-way wave equation E_t = E_x
 *   centred between nodes 0 and 1:
 *     E_0^{m+1} = E_1^m + k (E_1^{m+1} - E_0^m);
 *   absorb_x = 2, second order, from E_xt - E_tt + (1/2)(E_yy + E_zz) = 0
 *   (Engquist-Majda) centred the same way:
 *     E_0^{m+1} = -E_1^{m-1} + k (E_1^{m+1} + E_0^{m-1})
 *                 + 2 dx/(h + dx) (E_0^m + E_1^m)
 *                 + h^2 dx / (2 (h + dx)) (D E_0^m + D E_1^m),
 *   D the periodic second difference over y (and z) on the face planes.
 *   Level m-1 comes from `mur` (the face values on entry to the previous
 *   half update, kept by the caller between calls); while *mur_valid is 0
 *   (the first call) the first-order rule runs instead.  Each call leaves its
 *   entry values in `mur` and sets *mur_valid.
 * The far face is the mirror, nodes n-1 and n-2.  E_x, B_y, B_z half a cell
 * beyond the far face lie outside and stay 0.
 */
void orc_half_e(const orc_grid *g, double *const *E, const double *const *B,
                const double *const *J, double t, double *mur, int32_t *mur_valid) {
    const double h = 0.5 * g->dt;
    const double ix = 1.0 / g->d[0], iy = 1.0 / g->d[1];
    const double iz = g->dim == 3 ? 1.0 / g->d[2] : 0.0;
    const int64_t nx = g->n[0], nyz = g->n[1] * g->n[2];
    const int ab = g->absorb_x;
    double *old = NULL; /* [face node 0, 1, nx-2, nx-1][E_y, E_z][j + ny k] */
    const int64_t fx[4] = {0, 1, nx - 2, nx - 1};
    if (ab) {
        old = (double *)malloc(sizeof(double) * 8 * (size_t)nyz);
        for (int f = 0; f < 4; ++f)
            for (int cmp = 0; cmp < 2; ++cmp)
                for (int64_t k = 0; k < g->n[2]; ++k)
                    for (int64_t j = 0; j < g->n[1]; ++j)
                        old[(f * 2 + cmp) * nyz + j + g->n[1] * k] = E[1 + cmp][idx3(g, fx[f], j, k)];
    }
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                int64_t c = idx3(g, i, j, k);
                /* E_x(i+1/2,j,k): dBz/dy - dBy/dz */
                double cbx = (B[2][c] - B[2][idx3(g, i, j - 1, k)]) * iy -
                             (B[1][c] - B[1][idx3(g, i, j, k - 1)]) * iz;
                /* E_y(i,j+1/2,k): dBx/dz - dBz/dx */
                double cby = (B[0][c] - B[0][idx3(g, i, j, k - 1)]) * iz -
                             (B[2][c] - B[2][idx3(g, i - 1, j, k)]) * ix;
                /* E_z(i,j,k+1/2): dBy/dx - dBx/dy */
                double cbz = (B[1][c] - B[1][idx3(g, i - 1, j, k)]) * ix -
                             (B[0][c] - B[0][idx3(g, i, j - 1, k)]) * iy;
                if (ab && i == nx - 1) {
                    E[0][c] = 0.0;
                } else {
                    E[0][c] += h * (cbx - J[0][c]);
                }
                if (!ab || (i != 0 && i != nx - 1)) {
                    E[1][c] += h * (cby - J[1][c]);
                    E[2][c] += h * (cbz - J[2][c]);
                }
            }
    if (ab) {
        const double dx = g->d[0];
        const double km = (h - dx) / (h + dx);
        const int second = ab == 2 && mur && mur_valid && *mur_valid;
        const int64_t ny = g->n[1], nz = g->n[2];
        /* scattered entry values s[f][cmp][q] (face nodes 0, 1, n-2, n-1): E - E_inc at x = 0, 1 */
        double *sc = (double *)malloc(sizeof(double) * 8 * (size_t)nyz);
        for (int f = 0; f < 4; ++f)
            for (int cmp = 0; cmp < 2; ++cmp)
                for (int64_t k = 0; k < nz; ++k)
                    for (int64_t j = 0; j < ny; ++j) {
                        const int comp = 1 + cmp;
                        const double y = (j + (comp == 1 ? 0.5 : 0.0)) * g->d[1];
                        const double z = g->dim == 3 ? (k + (comp == 2 ? 0.5 : 0.0)) * g->d[2] : 0.0;
                        const int64_t q = j + ny * k;
                        double v = old[(f * 2 + cmp) * nyz + q];
                        if (f < 2) v -= orc_incident(g, comp, f * dx, y, z, t);
                        sc[(f * 2 + cmp) * nyz + q] = v;
                    }
        for (int64_t k = 0; k < nz; ++k)
            for (int64_t j = 0; j < ny; ++j)
                for (int cmp = 0; cmp < 2; ++cmp) {
                    const int comp = 1 + cmp;
                    const int64_t q = j + ny * k;
                    /* stagger of the component: E_y at y + dy/2, E_z at z + dz/2 */
                    const double y = (j + (comp == 1 ? 0.5 : 0.0)) * g->d[1];
                    const double z = g->dim == 3 ? (k + (comp == 2 ? 0.5 : 0.0)) * g->d[2] : 0.0;
                    /* face f0 (on the face) and f1 (inside): x = 0 uses nodes 0, 1; the far face n-1, n-2 */
                    for (int side = 0; side < 2; ++side) {
                        const int f0 = side == 0 ? 0 : 3, f1 = side == 0 ? 1 : 2;
                        const int64_t i0 = side == 0 ? 0 : nx - 1, i1 = side == 0 ? 1 : nx - 2;
                        const double inc_new0 = side == 0 ? orc_incident(g, comp, 0.0, y, z, t + h) : 0.0;
                        const double inc_new1 = side == 0 ? orc_incident(g, comp, dx, y, z, t + h) : 0.0;
                        const double u0 = sc[(f0 * 2 + cmp) * nyz + q], u1 = sc[(f1 * 2 + cmp) * nyz + q];
                        const double u1n = E[comp][idx3(g, i1, j, k)] - inc_new1;
                        double u0n;
                        if (!second) {
                            u0n = u1 + km * (u1n - u0);
                        } else {
                            const double inc_old0 = side == 0 ? orc_incident(g, comp, 0.0, y, z, t - h) : 0.0;
                            const double inc_old1 = side == 0 ? orc_incident(g, comp, dx, y, z, t - h) : 0.0;
                            const double u0m = mur[(f0 * 2 + cmp) * nyz + q] - inc_old0;
                            const double u1m = mur[(f1 * 2 + cmp) * nyz + q] - inc_old1;
                            /* second differences along y (and z) of the entry values, both planes */
                            double lap = 0.0;
                            for (int f = 0; f < 2; ++f) {
                                const double *pl = sc + ((f == 0 ? f0 : f1) * 2 + cmp) * nyz;
                                const int64_t jp = (j + 1) % ny, jm = (j + ny - 1) % ny;
                                lap += (pl[jp + ny * k] - 2.0 * pl[q] + pl[jm + ny * k]) / (g->d[1] * g->d[1]);
                                if (g->dim == 3) {
                                    const int64_t kp = (k + 1) % nz, kmi = (k + nz - 1) % nz;
                                    lap += (pl[j + ny * kp] - 2.0 * pl[q] + pl[j + ny * kmi]) / (g->d[2] * g->d[2]);
                                }
                            }
                            u0n = -u1m + km * (u1n + u0m) + 2.0 * dx / (h + dx) * (u0 + u1) +
                                  h * h * dx / (2.0 * (h + dx)) * lap;
                        }
                        E[comp][idx3(g, i0, j, k)] = inc_new0 + u0n;
                    }
                }
        if (ab == 2 && mur) {
            memcpy(mur, old, sizeof(double) * 8 * (size_t)nyz);
            if (mur_valid) *mur_valid = 1;
        }
        free(sc);
        free(old);
    }
}

void orc_half_b(const orc_grid *g, const double *const *E, double *const *B) {
    const double h = 0.5 * g->dt;
    const double ix = 1.0 / g->d[0], iy = 1.0 / g->d[1];
    const double iz = g->dim == 3 ? 1.0 / g->d[2] : 0.0;
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t i = 0; i < g->n[0]; ++i) {
                int64_t c = idx3(g, i, j, k);
                /* B_x(i,j+1/2,k+1/2): -(dEz/dy - dEy/dz) */
                double cex = (E[2][idx3(g, i, j + 1, k)] - E[2][c]) * iy -
                             (E[1][idx3(g, i, j, k + 1)] - E[1][c]) * iz;
                /* B_y(i+1/2,j,k+1/2): -(dEx/dz - dEz/dx) */
                double cey = (E[0][idx3(g, i, j, k + 1)] - E[0][c]) * iz -
                             (E[2][idx3(g, i + 1, j, k)] - E[2][c]) * ix;
                /* B_z(i+1/2,j+1/2,k): -(dEy/dx - dEx/dy) */
                double cez = (E[1][idx3(g, i + 1, j, k)] - E[1][c]) * ix -
                             (E[0][idx3(g, i, j + 1, k)] - E[0][c]) * iy;
                B[0][c] -= h * cex;
                if (g->absorb_x && i == g->n[0] - 1) {
                    B[1][c] = 0.0;
                    B[2][c] = 0.0;
                } else {
                    B[1][c] -= h * cey;
                    B[2][c] -= h * cez;
                }
            }
}

/* Field energy 1/2 sum (E^2 + B^2) dV (Gaussian energy density in the units
 * of Eq. 8), the field part of the total energy tracked in Fig. 6. */
double orc_field_energy(const orc_grid *g, const double *const *F) {
    double dV = g->d[0] * g->d[1] * (g->dim == 3 ? g->d[2] : 1.0);
    int64_t nc = g->n[0] * g->n[1] * g->n[2];
    double s = 0.0;
    for (int c = 0; c < 6; ++c)
        for (int64_t i = 0; i < nc; ++i) s += F[c][i] * F[c][i];
    return 0.5 * s * dV;
}

/* Charge density on the nodes, rho(i) += q w prod_a W(i_a - x_a/d_a)
 * (integer nodes, the shape of Sec. II.D). */
void orc_rho(const orc_grid *g, double q, int64_t np, const double *const *x, const double *w,
             double w0, double *rho) {
    for (int64_t p = 0; p < np; ++p) {
        int64_t i0[3] = {0, 0, 0};
        double wt[3][5] = {{0.0}};
        int nw[3] = {1, 1, 1};
        wt[2][0] = 1.0;
        for (int a = 0; a < g->dim; ++a) nw[a] = orc_shape(g->order, x[a][p] / g->d[a], &i0[a], wt[a]);
        double qw = q * (w ? w[p] : w0);
        for (int kk = 0; kk < nw[2]; ++kk)
            for (int jj = 0; jj < nw[1]; ++jj)
                for (int ii = 0; ii < nw[0]; ++ii)
                    rho[idx3(g, i0[0] + ii, i0[1] + jj, i0[2] + kk)] +=
                        qw * wt[0][ii] * wt[1][jj] * wt[2][kk];
    }
}

/* Discrete divergence on the nodes: div E(i) = sum_a (E_a(i+1/2) - E_a(i-1/2))/d_a
 * (for J the same stencil gives div J; Eqs. 1 and 5). */
void orc_div(const orc_grid *g, const double *const *V, double *out) {
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t i = 0; i < g->n[0]; ++i) {
                int64_t c = idx3(g, i, j, k);
                double s = (V[0][c] - V[0][idx3(g, i - 1, j, k)]) / g->d[0] +
                           (V[1][c] - V[1][idx3(g, i, j - 1, k)]) / g->d[1];
                if (g->dim == 3) s += (V[2][c] - V[2][idx3(g, i, j, k - 1)]) / g->d[2];
                out[c] = s;
            }
}

/* Discrete curl of E on the B stagger (the operator applied by orc_half_b),
 * exposed so the tests can check div(curl) = 0 and the dispersion relation. */
void orc_curl_e(const orc_grid *g, const double *const *E, double *const *out) {
    double *B[3] = {out[0], out[1], out[2]};
    int64_t nc = g->n[0] * g->n[1] * g->n[2];
    for (int c = 0; c < 3; ++c) memset(B[c], 0, sizeof(double) * nc);
    orc_grid g2 = *g;
    g2.dt = -2.0; /* B -= (dt/2) curl E with dt = -2 gives B = curl E */
    orc_half_b(&g2, E, B);
}

/*
 * Tile binning order (the particle sort).  Not a step of the paper's method:
 * it only reorders particles so that the GPU can stage one grid tile at a
 * time.  The order is fully defined on the integer cells, so any correct
 * implementation gives the same permutation:
 *   tile(p)  = (ix/Tx) + ntx*((iy/Ty) + nty*(iz/Tz))
 *   rank(p)  = number of particles q < p in the same cell
 *   local(p) = position of the cell inside the tile: cells are grouped by
 *              the parity class (lx&1) | (ly&1)<<1 | (lz&1)<<2 of their
 *              tile-local coordinates, classes taken in the order
 *              0 3 1 2 (2D) or 0 7 1 6 2 5 4 3 (3D), then ordered by
 *              (lz/2, ly/2, lx/2)
 * and particles are ordered by (tile, rank, local) ascending; these triples
 * are unique.  A particle whose cell lies off the grid has no tile: such
 * particles come after every tile, in their source order.  perm[new] = old;
 * tile_start[t] is the first new index of tile t, and tile_start[ntiles] the
 * number of particles on the grid (np when every cell is on it).
 */
static int64_t local_order(int dim, const int64_t *T, int64_t lx, int64_t ly, int64_t lz) {
    static const int order2[4] = {0, 3, 1, 2};
    static const int order3[8] = {0, 7, 1, 6, 2, 5, 4, 3};
    const int cls = (int)((lx & 1) | (ly & 1) << 1 | (lz & 1) << 2);
    int pos = 0;
    for (int q = 0; q < (dim == 3 ? 8 : 4); ++q)
        if ((dim == 3 ? order3[q] : order2[q]) == cls) pos = q;
    return ((pos * T[2] + lz / 2) * T[1] + ly / 2) * T[0] + lx / 2;
}

typedef struct {
    int64_t tile, rank, local, old;
} orc_sort_key;

static int cmp_key(const void *pa, const void *pb) {
    const orc_sort_key *a = (const orc_sort_key *)pa, *b = (const orc_sort_key *)pb;
    if (a->tile != b->tile) return a->tile < b->tile ? -1 : 1;
    if (a->rank != b->rank) return a->rank < b->rank ? -1 : 1;
    if (a->local != b->local) return a->local < b->local ? -1 : 1;
    return 0;
}

int orc_sort(const orc_grid *g, const int64_t *tile_size, int64_t np, const int32_t *const *cell,
             int64_t *perm, int64_t *tile_start) {
    int64_t nt[3] = {1, 1, 1}, T[3] = {1, 1, 1};
    for (int a = 0; a < g->dim; ++a) {
        T[a] = tile_size[a];
        nt[a] = g->n[a] / T[a];
    }
    int64_t ncell = g->n[0] * g->n[1] * g->n[2];
    int64_t ntiles = nt[0] * nt[1] * nt[2];
    int64_t *seen = (int64_t *)calloc((size_t)ncell, sizeof(int64_t));
    orc_sort_key *keys = (orc_sort_key *)malloc(sizeof(orc_sort_key) * (size_t)(np > 0 ? np : 1));
    if (!seen || !keys) {
        free(seen);
        free(keys);
        return -1;
    }
    for (int64_t p = 0; p < np; ++p) {
        int64_t c[3] = {cell[0][p], cell[1][p], cell[2][p]};
        int on_grid = 1;
        for (int a = 0; a < 3; ++a) on_grid &= c[a] >= 0 && c[a] < g->n[a];
        keys[p].old = p;
        if (!on_grid) {
            keys[p].tile = ntiles;
            keys[p].rank = p;
            keys[p].local = 0;
            continue;
        }
        int64_t lin = c[0] + g->n[0] * (c[1] + g->n[1] * c[2]);
        keys[p].tile = c[0] / T[0] + nt[0] * (c[1] / T[1] + nt[1] * (c[2] / T[2]));
        keys[p].local = local_order(g->dim, T, c[0] % T[0], c[1] % T[1], c[2] % T[2]);
        keys[p].rank = seen[lin]++;
    }
    qsort(keys, (size_t)np, sizeof(orc_sort_key), cmp_key);
    for (int64_t t = 0; t <= ntiles; ++t) tile_start[t] = 0;
    for (int64_t p = 0; p < np; ++p) {
        perm[p] = keys[p].old;
        if (keys[p].tile < ntiles) tile_start[keys[p].tile + 1]++;
    }
    for (int64_t t = 0; t < ntiles; ++t) tile_start[t + 1] += tile_start[t];
    free(seen);
    free(keys);
    return 0;
}
