/*
 * Plain FP64 CPU oracle of the volume-averaged lattice Boltzmann model of
 * Zhang, Wang & Ouyang, "Lattice Boltzmann Model for the Volume-Averaged
 * Navier-Stokes Equations" (arXiv:1406.6438).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * statement of what one time step of the method computes.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  The GPU library shares no code, header, table or constant with it.
 *
 * Conventions (the paper's lattice units, delta_t = delta_x = 1):
 *   populations f[i][y][x], i = 0..8, x fastest, stored as plain f_i;
 *   porosity eps[y][x];
 *   every floating point operation is IEEE binary64, round to nearest,
 *   built with -ffp-contract=off so that no fused multiply-add changes it.
 *
 * One step, in the paper's order (final lattice Boltzmann equation, Section
 * "Chapman-Enskog analysis", the equation following eq. VNS3):
 *   collide every cell:  f*_i = f_i - (f_i - f_i^eq)/tau + P_i + F_i
 *   stream (push):       f_i(x + e_i, t + 1) = f*_i(x, t)
 * with f^eq from eq. (d2q9eq), P_i from eq. (pi), F_i from eq. (Fi), the
 * density from eq. (0moment) and the velocity from eq. (1moment), and the
 * drag force of Section "Examples and discussions" (Darcy-Forchheimer law
 * with the Ergun closure for K and F_eps).
 *
 * Readings of points the paper leaves open (each one is listed in the design
 * notes of this repository):
 *   - the D2Q9 velocity set and weights are the textbook ones of Qian,
 *     d'Humieres & Lallemand (1992), c_s^2 = 1/3, with the ordering below;
 *   - "e . u" in eq. (d2q9eq) is e_i . u;
 *   - the force F of eqs. (Fi) and (1moment) is an external body-force
 *     density G plus the porous drag; the pressure correction P_i and F_i
 *     share the same Guo form and are applied together with
 *     T = c_s^2 rho grad(eps) + F;
 *   - rho in p = c_s^2 rho is the intrinsic density (eps rho) / eps;
 *   - grad(eps) is the isotropic lattice gradient 3 sum_i w_i e_i eps(x+e_i),
 *     with eps mirrored across a wall (the wall lies half way between the
 *     last fluid node and the next lattice node);
 *   - eq. (1moment) is implicit in u because F depends on u; it is solved
 *     exactly (the root is unique, see orc_velocity);
 *   - walls are half-way bounce-back: a population that would stream into a
 *     wall node returns to its own cell with the opposite velocity;
 *   - the plates of the Couette experiment (Section "Examples and
 *     discussions") slide along x: a y-wall moving with velocity (u_w, 0)
 *     returns the population with the momentum the moving wall imparts,
 *     f_j(x) = f*_i(x) + 6 w_j eps(x) rho0 (e_j . u_w) with j the opposite of
 *     i: the equilibrium's first-order term of eq. (d2q9eq) taken at the wall
 *     velocity (density rho0), twice, as in the moving-wall bounce-back rule
 *     for the plain lattice BGK model;
 *   - the initial state is f_i = f_i^eq(eps(x) rho0, u0);
 *   - open x-boundaries (inflow / outflow): the paper prescribes none for a
 *     through-flow channel; a population entering the domain across x = 0
 *     (x = Lx-1) is the equilibrium of eq. (d2q9eq) of a reservoir with the
 *     boundary node's porosity and the given density and x-velocity, and a
 *     population leaving across it is absorbed.  Where the source also lies
 *     behind a y-wall, bounce-back wins;
 *   - velocity inlet and pressure outlet (the second kind of open x ends):
 *     the reservoir beyond the inlet carries the given velocity (u_in, 0) and
 *     the inlet node's own density, the reservoir beyond the outlet the given
 *     density rho_out and the outlet node's own velocity (zero-gradient
 *     extrapolation of the free quantity), both taken from the state the step
 *     starts from: the populations entering at step n + 1 are
 *         inlet:  f_i^eq(eps rho of node (0, y) at step n, (u_in, 0)),
 *         outlet: f_i^eq(eps(Lx-1, y) rho_out, u of node (Lx-1, y) at step n).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* D2Q9 velocity set of Qian et al. (1992): rest, 4 axis links, 4 diagonals. */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                            1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
/* OPP[i] is the index of -e_i. */
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
/* Squared lattice sound speed of D2Q9. */
static const double CS2 = 1.0 / 3.0;

enum { ORC_PERIODIC = 0, ORC_WALL = 1, ORC_OPEN = 2, ORC_INOUT = 3 };
enum { ORC_DRAG_ERGUN = 0, ORC_DRAG_CONST = 1 };

/* Problem description (Section "Examples and discussions"). */
typedef struct {
    int32_t Lx, Ly;     /* lattice nodes along x and y                         */
    int32_t bc_x, bc_y; /* ORC_PERIODIC or ORC_WALL (both ends of the axis);    */
                        /* bc_x may be ORC_OPEN: inflow reservoir beyond x = 0, */
                        /* outflow reservoir beyond x = Lx-1; or ORC_INOUT:     */
                        /* velocity inlet at x = 0, pressure outlet at Lx-1      */
    int32_t drag;       /* ORC_DRAG_ERGUN: K, F_eps from d_p (Ergun closure)    */
                        /* ORC_DRAG_CONST: K and F_eps given, uniform            */
    int32_t pad_;
    double tau;         /* BGK relaxation time, > 1/2                          */
    double d_p;         /* particle diameter of the Ergun closure               */
    double K, F_eps;    /* permeability and geometric function (DRAG_CONST)     */
    double Gx, Gy;      /* external body-force density                         */
    double rho0, u0x, u0y; /* initial state                                    */
    double rho_in, u_in;   /* ORC_OPEN: density and x-velocity of the inflow reservoir  */
    double rho_out, u_out; /* ORC_OPEN: density and x-velocity of the outflow reservoir */
                           /* ORC_INOUT: u_in is the inlet velocity, rho_out the      */
                           /* outlet density (rho_in, u_out unused)                  */
    double uw_bot, uw_top; /* ORC_WALL in y: x-velocity of the wall below y = 0 and of the
                              wall above y = Ly-1 (sliding plates)                      */
} orc_params;

void orc_lattice(int32_t ex[9], int32_t ey[9], double w[9], int32_t opp[9], double *cs2)
{
    for (int i = 0; i < 9; i++) {
        ex[i] = EX[i];
        ey[i] = EY[i];
        w[i] = W[i];
        opp[i] = OPP[i];
    }
    *cs2 = CS2;
}

/* Porosity-modified equilibrium, eq. (d2q9eq):
 *   f_i^eq = w_i eps rho [1 + e_i.u/c_s^2 + (e_i.u)^2/(2 c_s^4) - u.u/(2 c_s^2)]
 * eps_rho is the product eps*rho. */
void orc_feq(double eps_rho, double ux, double uy, double feq[9])
{
    double uu = ux * ux + uy * uy;
    for (int i = 0; i < 9; i++) {
        double eu = EX[i] * ux + EY[i] * uy;
        feq[i] = W[i] * eps_rho *
                 (1.0 + eu / CS2 + (eu * eu) / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
    }
}

/* Discrete forcing term of Guo, Zheng & Shi (2002), the form shared by
 * eq. (pi) (with the vector p grad eps) and eq. (Fi) (with the force F):
 *   (1 - 1/(2 tau)) w_i [ (e_i - u)/c_s^2 + (e_i.u) e_i / c_s^4 ] . T
 * Because the expression is linear in T, P_i + F_i is this term applied to
 * T = p grad(eps) + F. */
void orc_guo_source(double tau, double ux, double uy, double Tx, double Ty, double s[9])
{
    double pre = 1.0 - 1.0 / (2.0 * tau);
    for (int i = 0; i < 9; i++) {
        double eu = EX[i] * ux + EY[i] * uy;
        double cx = (EX[i] - ux) / CS2 + eu * EX[i] / (CS2 * CS2);
        double cy = (EY[i] - uy) / CS2 + eu * EY[i] / (CS2 * CS2);
        s[i] = pre * W[i] * (cx * Tx + cy * Ty);
    }
}

/* Drag coefficients of the Darcy-Forchheimer force of Section "Examples and
 * discussions":  F_drag = -(eps^2 nu / K) u - (eps^3 F_eps / sqrt(K)) |u| u,
 * returned as a = eps^2 nu / K and b = eps^3 F_eps / sqrt(K).
 * Ergun closure: K = eps^3 d_p^2 / (150 (1 - eps)^2),
 *                F_eps = 1.75 / sqrt(150 eps^3).
 * nu = c_s^2 (tau - 1/2) (the viscosity of eq. (VNS2)).  At eps = 1 the
 * Ergun permeability is infinite and both coefficients are zero; an infinite
 * d_p likewise gives no drag. */
void orc_drag_coeffs(const orc_params *p, double eps, double *a, double *b)
{
    double nu = CS2 * (p->tau - 0.5);
    double K, Feps;
    if (p->drag == ORC_DRAG_CONST) {
        K = p->K;
        Feps = p->F_eps;
    } else {
        if (eps >= 1.0 || isinf(p->d_p)) {
            *a = 0.0;
            *b = 0.0;
            return;
        }
        K = eps * eps * eps * p->d_p * p->d_p / (150.0 * (1.0 - eps) * (1.0 - eps));
        Feps = 1.75 / sqrt(150.0 * eps * eps * eps);
    }
    if (isinf(K)) {
        *a = 0.0;
        *b = 0.0;
        return;
    }
    *a = eps * eps * nu / K;
    *b = eps * eps * eps * Feps / sqrt(K);
}

/* Velocity from eq. (1moment):
 *   eps rho u = m + (1/2) c_s^2 rho grad(eps) + (1/2) F(u),
 *   F(u) = G - a u - b |u| u,
 * with S = eps rho = sum f_i (eq. (0moment)) and m = sum e_i f_i.
 * Collecting the u terms:  (S + a/2) u + (b/2) |u| u = V,
 *   V = m + (1/2) (c_s^2 rho grad(eps) + G).
 * u is parallel to V; its length s >= 0 solves (b/2) s^2 + (S + a/2) s = |V|,
 * whose only non-negative root is s = 2|V| / (A + sqrt(A^2 + 4 B |V|)) with
 * A = S + a/2, B = b/2 (the form without cancellation; it reduces to
 * |V| / A when b = 0).  Outputs u and rho = S / eps. */
void orc_velocity(const orc_params *p, double S, double mx, double my, double eps,
                  double gex, double gey, double *ux, double *uy, double *rho)
{
    double a, b;
    orc_drag_coeffs(p, eps, &a, &b);
    double r = S / eps;
    double Qx = CS2 * r * gex, Qy = CS2 * r * gey;
    double Vx = mx + 0.5 * (Qx + p->Gx);
    double Vy = my + 0.5 * (Qy + p->Gy);
    double Vn = sqrt(Vx * Vx + Vy * Vy);
    double A = S + 0.5 * a;
    double B = 0.5 * b;
    double den = A + sqrt(A * A + 4.0 * B * Vn);
    *ux = 2.0 * Vx / den;
    *uy = 2.0 * Vy / den;
    *rho = r;
}

/* Lattice gradient of the porosity, 3 sum_i w_i e_i eps(x + e_i), which is
 * exact for a linear field because sum_i w_i e_i e_i = c_s^2 I.  A neighbour
 * beyond a wall takes the value of its mirror image across the wall (the
 * wall sits half way, so node -1 mirrors to node 0 and node L to L-1). */
static int nb_index(int v, int L, int bc)
{
    if (bc == ORC_PERIODIC) {
        if (v < 0) return v + L;
        if (v >= L) return v - L;
        return v;
    }
    if (v < 0) return 0;
    if (v >= L) return L - 1;
    return v;
}

void orc_grad_eps(const orc_params *p, const double *eps, double *gx, double *gy)
{
    int Lx = p->Lx, Ly = p->Ly;
    for (int y = 0; y < Ly; y++)
        for (int x = 0; x < Lx; x++) {
            double sx = 0.0, sy = 0.0;
            for (int i = 0; i < 9; i++) {
                int xn = nb_index(x + EX[i], Lx, p->bc_x);
                int yn = nb_index(y + EY[i], Ly, p->bc_y);
                double en = eps[(size_t)yn * Lx + xn];
                sx += W[i] * EX[i] * en;
                sy += W[i] * EY[i] * en;
            }
            gx[(size_t)y * Lx + x] = sx / CS2;
            gy[(size_t)y * Lx + x] = sy / CS2;
        }
}

/* Initial state (Section "Examples and discussions": density and velocity
 * start at given values):  f_i(x, 0) = f_i^eq(eps(x) rho0, u0). */
void orc_init(const orc_params *p, const double *eps, double *f)
{
    size_t N = (size_t)p->Lx * p->Ly;
    double feq[9];
    for (size_t c = 0; c < N; c++) {
        orc_feq(eps[c] * p->rho0, p->u0x, p->u0y, feq);
        for (int i = 0; i < 9; i++) f[i * N + c] = feq[i];
    }
}

/* Per-cell macroscopic state of f: eps rho (eq. (0moment)), rho, u
 * (eq. (1moment)) and the total vector T = c_s^2 rho grad(eps) + F(u) that
 * drives P_i + F_i.  Any output pointer may be NULL. */
static void cell_state(const orc_params *p, const double *f, size_t N, size_t c,
                       double eps, double gex, double gey, double *S_out,
                       double *mx_out, double *my_out, double *rho_out,
                       double *ux_out, double *uy_out, double *Tx_out, double *Ty_out)
{
    double S = 0.0, mx = 0.0, my = 0.0;
    for (int i = 0; i < 9; i++) {
        double fi = f[i * N + c];
        S += fi;
        mx += EX[i] * fi;
        my += EY[i] * fi;
    }
    double ux, uy, rho;
    orc_velocity(p, S, mx, my, eps, gex, gey, &ux, &uy, &rho);
    double a, b;
    orc_drag_coeffs(p, eps, &a, &b);
    double un = sqrt(ux * ux + uy * uy);
    double Fx = p->Gx - a * ux - b * un * ux;
    double Fy = p->Gy - a * uy - b * un * uy;
    double Tx = CS2 * rho * gex + Fx;
    double Ty = CS2 * rho * gey + Fy;
    if (S_out) *S_out = S;
    if (mx_out) *mx_out = mx;
    if (my_out) *my_out = my;
    if (rho_out) *rho_out = rho;
    if (ux_out) *ux_out = ux;
    if (uy_out) *uy_out = uy;
    if (Tx_out) *Tx_out = Tx;
    if (Ty_out) *Ty_out = Ty;
}

/* Collision of one node with incoming f[9], porosity eps and its gradient
 * (gex, gey): fpost_i = f_i - (f_i - f_i^eq)/tau + P_i + F_i. */
void orc_node_collide(const orc_params *p, const double f[9], double eps, double gex,
                      double gey, double fpost[9])
{
    double S, rho, ux, uy, Tx, Ty, feq[9], src[9];
    cell_state(p, f, 1, 0, eps, gex, gey, &S, NULL, NULL, &rho, &ux, &uy, &Tx, &Ty);
    orc_feq(S, ux, uy, feq);
    orc_guo_source(p->tau, ux, uy, Tx, Ty, src);
    for (int i = 0; i < 9; i++) fpost[i] = f[i] - (f[i] - feq[i]) / p->tau + src[i];
}

/* Collision of every cell (the right-hand side of the final lattice
 * Boltzmann equation):  f*_i = f_i - (f_i - f_i^eq)/tau + P_i + F_i.
 * gx, gy hold grad(eps) from orc_grad_eps.  fpost may not alias f. */
void orc_collide(const orc_params *p, const double *eps, const double *gx,
                 const double *gy, const double *f, double *fpost, int nthreads)
{
    long Ly = p->Ly;
    size_t Lx = (size_t)p->Lx;
    size_t N = Lx * (size_t)Ly;
    (void)nthreads;
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
    for (long y = 0; y < Ly; y++) {
        for (size_t x = 0; x < Lx; x++) {
            size_t c = (size_t)y * Lx + x;
            double S, rho, ux, uy, Tx, Ty, feq[9], src[9];
            cell_state(p, f, N, c, eps[c], gx[c], gy[c], &S, NULL, NULL, &rho, &ux,
                       &uy, &Tx, &Ty);
            orc_feq(S, ux, uy, feq);
            orc_guo_source(p->tau, ux, uy, Tx, Ty, src);
            for (int i = 0; i < 9; i++) {
                double fi = f[i * N + c];
                fpost[i * N + c] = fi - (fi - feq[i]) / p->tau + src[i];
            }
        }
    }
}

/* Populations entering across an open x-boundary: the equilibrium of
 * eq. (d2q9eq) of the reservoir (porosity of the boundary node, density rho_b,
 * velocity (u_b, 0)). */
static double reservoir(int i, double eps, double rho_b, double u_b)
{
    double feq[9];
    orc_feq(eps * rho_b, u_b, 0.0, feq);
    return feq[i];
}

/* Whether the source x - e_i of node (x, y) lies behind a y-wall. */
static int source_behind_ywall(const orc_params *p, int y, int i)
{
    int ys = y - EY[i];
    return p->bc_y == ORC_WALL && (ys < 0 || ys >= p->Ly);
}

/* Momentum gain per unit porosity of population j when it leaves a y-wall
 * that slides with x-velocity u_w: 6 w_j rho0 (e_j . u_w). */
static double wall_gain(const orc_params *p, int j, int top)
{
    double uw = top ? p->uw_top : p->uw_bot;
    return 6.0 * W[j] * p->rho0 * (EX[j] * uw);
}

/* Velocity inlet / pressure outlet: what the populations entering at the next
 * step are built from, taken from the state f (eqs. (0moment), (1moment)):
 * for each row y, ends[3 y] = eps rho of the inlet node (0, y) and
 * ends[3 y + 1], ends[3 y + 2] = the velocity of the outlet node (Lx-1, y). */
void orc_open_ends(const orc_params *p, const double *eps, const double *gx, const double *gy,
                   const double *f, double *ends)
{
    size_t N = (size_t)p->Lx * p->Ly;
    for (int y = 0; y < p->Ly; y++) {
        size_t c0 = (size_t)y * p->Lx, c1 = (size_t)y * p->Lx + (p->Lx - 1);
        double S, ux, uy;
        cell_state(p, f, N, c0, eps[c0], gx[c0], gy[c0], &S, NULL, NULL, NULL, NULL, NULL,
                   NULL, NULL);
        ends[3 * y] = S;
        cell_state(p, f, N, c1, eps[c1], gx[c1], gy[c1], NULL, NULL, NULL, NULL, &ux, &uy,
                   NULL, NULL);
        ends[3 * y + 1] = ux;
        ends[3 * y + 2] = uy;
    }
}

/* Streaming (push):  f_i(x + e_i) = f*_i(x).  Along a periodic axis the
 * target wraps around; a target beyond a wall sends the population back to
 * its own cell as the opposite direction (half-way bounce-back), plus the
 * gain of a sliding y-wall; a target beyond an open x-boundary leaves the
 * domain.  Beyond a y-wall bounce-back takes precedence.  Then the
 * populations that enter across an open x-boundary are set from the
 * reservoirs: fixed ones (ORC_OPEN), or for ORC_INOUT the inlet and outlet
 * reservoirs built from ends (orc_open_ends of the state the step starts
 * from; NULL for the other boundary kinds).  Every slot of f is written once. */
void orc_stream(const orc_params *p, const double *eps, const double *fpost,
                const double *ends, double *f, int nthreads)
{
    long Ly = p->Ly;
    int Lx = p->Lx;
    size_t N = (size_t)Lx * (size_t)Ly;
    (void)nthreads;
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
    for (long y = 0; y < Ly; y++) {
        for (int x = 0; x < Lx; x++) {
            size_t c = (size_t)y * Lx + x;
            for (int i = 0; i < 9; i++) {
                int xt = x + EX[i], yt = (int)y + EY[i];
                int wall = 0, gone = 0, ywall = 0;
                if (yt < 0 || yt >= Ly) {
                    if (p->bc_y == ORC_PERIODIC) yt = (int)((yt + Ly) % Ly);
                    else wall = ywall = 1;
                }
                if (!wall && (xt < 0 || xt >= Lx)) {
                    if (p->bc_x == ORC_PERIODIC) xt = (xt + Lx) % Lx;
                    else if (p->bc_x == ORC_WALL) wall = 1;
                    else gone = 1;
                }
                if (gone) continue;
                if (ywall)
                    f[OPP[i] * N + c] = fpost[i * N + c] +
                                        wall_gain(p, OPP[i], yt >= Ly) * eps[c];
                else if (wall)
                    f[OPP[i] * N + c] = fpost[i * N + c];
                else
                    f[i * N + (size_t)yt * Lx + xt] = fpost[i * N + c];
            }
        }
    }
    if (p->bc_x != ORC_OPEN && p->bc_x != ORC_INOUT) return;
    for (long y = 0; y < Ly; y++) {
        size_t c0 = (size_t)y * Lx, c1 = (size_t)y * Lx + (Lx - 1);
        double feq_in[9], feq_out[9];
        if (p->bc_x == ORC_INOUT) {
            orc_feq(ends[3 * y], p->u_in, 0.0, feq_in);
            orc_feq(eps[c1] * p->rho_out, ends[3 * y + 1], ends[3 * y + 2], feq_out);
        }
        for (int i = 0; i < 9; i++) {
            if (source_behind_ywall(p, (int)y, i)) continue;
            if (p->bc_x == ORC_INOUT) {
                if (EX[i] > 0) f[i * N + c0] = feq_in[i];
                if (EX[i] < 0) f[i * N + c1] = feq_out[i];
            } else {
                if (EX[i] > 0) f[i * N + c0] = reservoir(i, eps[c0], p->rho_in, p->u_in);
                if (EX[i] < 0) f[i * N + c1] = reservoir(i, eps[c1], p->rho_out, p->u_out);
            }
        }
    }
}

/* nsteps full time steps in place on f (collide, then stream).  scratch must
 * hold 9*Lx*Ly doubles; gx, gy from orc_grad_eps.  Returns 0, or -1 if memory
 * runs out. */
int orc_steps(const orc_params *p, const double *eps, const double *gx, const double *gy,
              double *f, double *scratch, int64_t nsteps, int nthreads)
{
    double *ends = NULL;
    if (p->bc_x == ORC_INOUT) {
        ends = malloc(sizeof(double) * 3 * (size_t)p->Ly);
        if (!ends) return -1;
    }
    for (int64_t n = 0; n < nsteps; n++) {
        orc_collide(p, eps, gx, gy, f, scratch, nthreads);
        if (ends) orc_open_ends(p, eps, gx, gy, f, ends);
        orc_stream(p, eps, scratch, ends, f, nthreads);
    }
    free(ends);
    return 0;
}

/* Macroscopic fields of the state f (eqs. (0moment), (1moment)):
 * eps rho, rho, u, the raw first moment m = sum e_i f_i and the total
 * vector T of P_i + F_i.  Any output may be NULL. */
void orc_moments(const orc_params *p, const double *eps, const double *gx,
                 const double *gy, const double *f, double *eps_rho, double *rho,
                 double *ux, double *uy, double *mx, double *my, double *Tx, double *Ty)
{
    size_t N = (size_t)p->Lx * p->Ly;
    for (size_t c = 0; c < N; c++) {
        double S, m_x, m_y, r, vx, vy, tx, ty;
        cell_state(p, f, N, c, eps[c], gx[c], gy[c], &S, &m_x, &m_y, &r, &vx, &vy, &tx,
                   &ty);
        if (eps_rho) eps_rho[c] = S;
        if (rho) rho[c] = r;
        if (ux) ux[c] = vx;
        if (uy) uy[c] = vy;
        if (mx) mx[c] = m_x;
        if (my) my[c] = m_y;
        if (Tx) Tx[c] = tx;
        if (Ty) Ty[c] = ty;
    }
}

/* ------------------------------------------------------------------------
 * Outlet mass flux and its gradient with respect to the porosity.
 *
 * Objective: J = sum over the last column x = Lx-1 of eps rho u_x of the state
 * f(., N) (eqs. (0moment), (1moment)), the superficial mass flux through the
 * outflow section per unit depth.
 *
 * dJ/deps(x) is the exact derivative of the discrete map N steps of
 * (collide, stream) from the initial state, taken in reverse mode: the
 * adjoint of each step is the transpose of the stream (a pull) followed by the
 * transposed Jacobian of each node's collision; porosity enters through
 * eps(x) itself (density, drag coefficients), through grad(eps) (the lattice
 * stencil, transposed once at the end), through the reservoir populations of
 * open boundaries (and, at a velocity inlet / pressure outlet, through the
 * boundary nodes' density and velocity those reservoirs carry) and through the
 * initial state.  All states are kept.
 * ------------------------------------------------------------------------ */

/* Derivatives of the drag coefficients a(eps), b(eps) of orc_drag_coeffs.
 * Ergun: a = eps^2 nu / K with dK/deps = K (3/eps + 2/(1-eps)), so
 * da/deps = -a (1/eps + 2/(1-eps)); b = eps^3 F_eps / sqrt(K) with
 * dF_eps/deps = -3 F_eps / (2 eps), so db/deps = -b / (1 - eps), whose limit at
 * eps = 1 is -1.75/d_p.  Constant K, F_eps: da/deps = 2a/eps, db/deps = 3b/eps. */
void orc_drag_derivs(const orc_params *p, double eps, double *da, double *db)
{
    double a, b;
    orc_drag_coeffs(p, eps, &a, &b);
    if (p->drag == ORC_DRAG_CONST) {
        *da = 2.0 * a / eps;
        *db = 3.0 * b / eps;
        return;
    }
    if (isinf(p->d_p)) {
        *da = 0.0;
        *db = 0.0;
        return;
    }
    if (eps >= 1.0) {
        *da = 0.0;
        *db = -1.75 / p->d_p;
        return;
    }
    *da = -a * (1.0 / eps + 2.0 / (1.0 - eps));
    *db = -b / (1.0 - eps);
}

/* Reverse-mode derivative of one node.  Forward: from the incoming f[9],
 * eps and grad(eps) = (gex, gey) the node forms S = eps rho, m, rho, u
 * (eq. (1moment)), F, T and the post-collision fpost_i = f_i - (f_i - feq_i)/tau
 * + src_i.  Given the adjoints fpost_bar[9] of the outputs and extra adjoints
 * S_bar0, ux_bar0, uy_bar0 of S and u, it adds the adjoints of the inputs to
 * f_bar[9], eps_bar, gex_bar, gey_bar. */
void orc_node_vjp(const orc_params *p, const double f[9], double eps, double gex, double gey,
                  const double fpost_bar[9], double S_bar0, double ux_bar0, double uy_bar0,
                  double f_bar[9], double *eps_bar, double *gex_bar, double *gey_bar)
{
    /* forward, as cell_state / orc_feq / orc_guo_source compute it */
    double S = 0.0, mx = 0.0, my = 0.0;
    for (int i = 0; i < 9; i++) {
        S += f[i];
        mx += EX[i] * f[i];
        my += EY[i] * f[i];
    }
    double a, b, da, db;
    orc_drag_coeffs(p, eps, &a, &b);
    orc_drag_derivs(p, eps, &da, &db);
    double rho = S / eps;
    double Qx = CS2 * rho * gex, Qy = CS2 * rho * gey;
    double Vx = mx + 0.5 * (Qx + p->Gx);
    double Vy = my + 0.5 * (Qy + p->Gy);
    double Vn = sqrt(Vx * Vx + Vy * Vy);
    double A = S + 0.5 * a;
    double B = 0.5 * b;
    double R = sqrt(A * A + 4.0 * B * Vn);
    double den = A + R;
    double ux = 2.0 * Vx / den, uy = 2.0 * Vy / den;
    double un = sqrt(ux * ux + uy * uy);
    double Fx = p->Gx - a * ux - b * un * ux;
    double Fy = p->Gy - a * uy - b * un * uy;
    double Tx = Qx + Fx, Ty = Qy + Fy;
    double uu = ux * ux + uy * uy;
    double pre = 1.0 - 1.0 / (2.0 * p->tau);

    /* reverse */
    double S_bar = S_bar0, ux_bar = ux_bar0, uy_bar = uy_bar0;
    double Tx_bar = 0.0, Ty_bar = 0.0, uu_bar = 0.0;
    for (int i = 0; i < 9; i++) {
        /* fpost_i = f_i - (f_i - feq_i)/tau + src_i */
        f_bar[i] += fpost_bar[i] * (1.0 - 1.0 / p->tau);
        double feq_bar = fpost_bar[i] / p->tau;
        double src_bar = fpost_bar[i];
        double eu = EX[i] * ux + EY[i] * uy;
        /* feq_i = w_i S (1 + eu/c2 + eu^2/(2 c2^2) - uu/(2 c2)) */
        double poly = 1.0 + eu / CS2 + (eu * eu) / (2.0 * CS2 * CS2) - uu / (2.0 * CS2);
        S_bar += feq_bar * W[i] * poly;
        double eu_bar = feq_bar * W[i] * S * (1.0 / CS2 + eu / (CS2 * CS2));
        uu_bar += -feq_bar * W[i] * S / (2.0 * CS2);
        /* src_i = pre w_i (cx Tx + cy Ty), cx = (ex - ux)/c2 + eu ex/c2^2 */
        double cx = (EX[i] - ux) / CS2 + eu * EX[i] / (CS2 * CS2);
        double cy = (EY[i] - uy) / CS2 + eu * EY[i] / (CS2 * CS2);
        Tx_bar += src_bar * pre * W[i] * cx;
        Ty_bar += src_bar * pre * W[i] * cy;
        double cx_bar = src_bar * pre * W[i] * Tx;
        double cy_bar = src_bar * pre * W[i] * Ty;
        ux_bar += -cx_bar / CS2;
        uy_bar += -cy_bar / CS2;
        eu_bar += (cx_bar * EX[i] + cy_bar * EY[i]) / (CS2 * CS2);
        /* eu = ex ux + ey uy */
        ux_bar += eu_bar * EX[i];
        uy_bar += eu_bar * EY[i];
    }
    ux_bar += 2.0 * ux * uu_bar;
    uy_bar += 2.0 * uy * uu_bar;
    /* T = Q + F,  F = G - a u - b |u| u */
    double Qx_bar = Tx_bar, Qy_bar = Ty_bar;
    double a_bar = -(Tx_bar * ux + Ty_bar * uy);
    double b_bar = -(Tx_bar * ux + Ty_bar * uy) * un;
    double un_bar = -b * (Tx_bar * ux + Ty_bar * uy);
    ux_bar += -(a + b * un) * Tx_bar;
    uy_bar += -(a + b * un) * Ty_bar;
    if (un > 0.0) {
        ux_bar += un_bar * ux / un;
        uy_bar += un_bar * uy / un;
    }
    /* u = 2 V / den,  den = A + R,  R = sqrt(A^2 + 4 B Vn) */
    double Vx_bar = ux_bar * 2.0 / den;
    double Vy_bar = uy_bar * 2.0 / den;
    double den_bar = -(ux_bar * ux + uy_bar * uy) / den;
    double A_bar = den_bar * (1.0 + A / R);
    double B_bar = den_bar * 2.0 * Vn / R;
    double Vn_bar = den_bar * 2.0 * B / R;
    if (Vn > 0.0) {
        Vx_bar += Vn_bar * Vx / Vn;
        Vy_bar += Vn_bar * Vy / Vn;
    }
    /* A = S + a/2, B = b/2 */
    S_bar += A_bar;
    a_bar += 0.5 * A_bar;
    b_bar += 0.5 * B_bar;
    /* V = m + (Q + G)/2 */
    double mx_bar = Vx_bar, my_bar = Vy_bar;
    Qx_bar += 0.5 * Vx_bar;
    Qy_bar += 0.5 * Vy_bar;
    /* Q = c2 rho grad(eps) */
    double rho_bar = CS2 * (Qx_bar * gex + Qy_bar * gey);
    *gex_bar += CS2 * rho * Qx_bar;
    *gey_bar += CS2 * rho * Qy_bar;
    /* rho = S / eps; a(eps), b(eps) */
    S_bar += rho_bar / eps;
    *eps_bar += -rho_bar * S / (eps * eps) + a_bar * da + b_bar * db;
    /* S = sum f, m = sum e f */
    for (int i = 0; i < 9; i++) f_bar[i] += S_bar + EX[i] * mx_bar + EY[i] * my_bar;
}

/* J = sum over x = Lx-1 of eps rho u_x of the state f. */
double orc_outlet_flux(const orc_params *p, const double *eps, const double *gx,
                       const double *gy, const double *f)
{
    size_t N = (size_t)p->Lx * p->Ly;
    double J = 0.0;
    for (int y = 0; y < p->Ly; y++) {
        size_t c = (size_t)y * p->Lx + (p->Lx - 1);
        double S, ux;
        cell_state(p, f, N, c, eps[c], gx[c], gy[c], &S, NULL, NULL, NULL, &ux, NULL, NULL,
                   NULL);
        J += S * ux;
    }
    return J;
}

/* J after nsteps steps from the initial state, and dJ/deps (Lx*Ly values).
 * Returns 0, or -1 if memory runs out. */
int orc_grad_outlet_flux(const orc_params *p, const double *eps, int64_t nsteps,
                         double *dJdeps, double *J_out, int nthreads)
{
    int Lx = p->Lx, Ly = p->Ly;
    size_t N = (size_t)Lx * Ly, S9 = 9 * N;
    double *fs = malloc(sizeof(double) * S9 * (size_t)(nsteps + 1));
    double *post = malloc(sizeof(double) * S9);
    double *fbar = malloc(sizeof(double) * S9);
    double *pbar = malloc(sizeof(double) * S9);
    double *gx = malloc(sizeof(double) * N), *gy = malloc(sizeof(double) * N);
    double *gxb = calloc(N, sizeof(double)), *gyb = calloc(N, sizeof(double));
    /* velocity inlet / pressure outlet: the boundary state of each step and the
     * adjoints it passes back to the boundary nodes (eps rho at the inlet, u at
     * the outlet) */
    int inout = p->bc_x == ORC_INOUT;
    double *ends = inout ? malloc(sizeof(double) * 3 * (size_t)Ly) : NULL;
    double *Sb = inout ? calloc(N, sizeof(double)) : NULL;
    double *uxb = inout ? calloc(N, sizeof(double)) : NULL;
    double *uyb = inout ? calloc(N, sizeof(double)) : NULL;
    if (!fs || !post || !fbar || !pbar || !gx || !gy || !gxb || !gyb ||
        (inout && (!ends || !Sb || !uxb || !uyb))) {
        free(fs); free(post); free(fbar); free(pbar); free(gx); free(gy); free(gxb); free(gyb);
        free(ends); free(Sb); free(uxb); free(uyb);
        return -1;
    }
    orc_grad_eps(p, eps, gx, gy);
    /* forward, keeping f(., n) for n = 0..nsteps */
    orc_init(p, eps, fs);
    for (int64_t n = 0; n < nsteps; n++) {
        orc_collide(p, eps, gx, gy, fs + S9 * n, post, nthreads);
        if (ends) orc_open_ends(p, eps, gx, gy, fs + S9 * n, ends);
        orc_stream(p, eps, post, ends, fs + S9 * (n + 1), nthreads);
    }
    const double *fN = fs + S9 * nsteps;
    *J_out = orc_outlet_flux(p, eps, gx, gy, fN);

    for (size_t k = 0; k < N; k++) dJdeps[k] = 0.0;
    for (size_t k = 0; k < S9; k++) fbar[k] = 0.0;
    /* seed: J = sum S ux over the outlet column */
    const double zero9[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int y = 0; y < Ly; y++) {
        size_t c = (size_t)y * Lx + (Lx - 1);
        double fc[9], fb[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, S, ux;
        for (int i = 0; i < 9; i++) fc[i] = fN[i * N + c];
        cell_state(p, fN, N, c, eps[c], gx[c], gy[c], &S, NULL, NULL, NULL, &ux, NULL, NULL,
                   NULL);
        orc_node_vjp(p, fc, eps[c], gx[c], gy[c], zero9, ux, S, 0.0, fb, &dJdeps[c], &gxb[c],
                     &gyb[c]);
        for (int i = 0; i < 9; i++) fbar[i * N + c] += fb[i];
    }
    for (int64_t n = nsteps - 1; n >= 0; n--) {
        /* velocity inlet: f_i(0, y; n+1) = f_i^eq(S, (u_in, 0)) with S = eps rho of
         * node (0, y) at step n; pressure outlet: f_i(Lx-1, y; n+1) =
         * f_i^eq(eps rho_out, u) with u the velocity of node (Lx-1, y) at step n */
        if (inout) {
            orc_open_ends(p, eps, gx, gy, fs + S9 * n, ends);
            for (int y = 0; y < Ly; y++) {
                size_t c0 = (size_t)y * Lx, c1 = (size_t)y * Lx + (Lx - 1);
                double feq_in1[9], feq_out1[9];
                double ux = ends[3 * y + 1], uy = ends[3 * y + 2];
                orc_feq(1.0, p->u_in, 0.0, feq_in1);
                orc_feq(p->rho_out, ux, uy, feq_out1);
                for (int i = 0; i < 9; i++) {
                    if (source_behind_ywall(p, y, i)) continue;
                    if (EX[i] > 0) Sb[c0] += fbar[i * N + c0] * feq_in1[i];
                    if (EX[i] < 0) {
                        double fb = fbar[i * N + c1];
                        /* d/d eps, and d/du of w_i S (1 + eu/c2 + eu^2/(2 c2^2) - uu/(2 c2)) */
                        dJdeps[c1] += fb * feq_out1[i];
                        double S = eps[c1] * p->rho_out;
                        double eu = EX[i] * ux + EY[i] * uy;
                        uxb[c1] += fb * W[i] * S *
                                   (EX[i] / CS2 + eu * EX[i] / (CS2 * CS2) - ux / CS2);
                        uyb[c1] += fb * W[i] * S *
                                   (EY[i] / CS2 + eu * EY[i] / (CS2 * CS2) - uy / CS2);
                    }
                }
            }
        }
        /* reservoir populations of f(., n+1) depend on the boundary porosity */
        if (p->bc_x == ORC_OPEN) {
            for (int y = 0; y < Ly; y++) {
                size_t c0 = (size_t)y * Lx, c1 = (size_t)y * Lx + (Lx - 1);
                for (int i = 0; i < 9; i++) {
                    if (source_behind_ywall(p, y, i)) continue;
                    if (EX[i] > 0)
                        dJdeps[c0] += fbar[i * N + c0] * reservoir(i, 1.0, p->rho_in, p->u_in);
                    if (EX[i] < 0)
                        dJdeps[c1] += fbar[i * N + c1] * reservoir(i, 1.0, p->rho_out, p->u_out);
                }
            }
        }
        /* transpose of the stream: post_bar_i(x) = f_bar at the slot x's f*_i went to */
        for (int y = 0; y < Ly; y++) {
            for (int x = 0; x < Lx; x++) {
                size_t c = (size_t)y * Lx + x;
                for (int i = 0; i < 9; i++) {
                    int xt = x + EX[i], yt = y + EY[i];
                    int wall = 0, gone = 0;
                    if (yt < 0 || yt >= Ly) {
                        if (p->bc_y == ORC_PERIODIC) {
                            yt = (yt + Ly) % Ly;
                        } else {
                            wall = 1;
                            /* the sliding wall's gain is eps(x) times a constant */
                            dJdeps[c] += fbar[OPP[i] * N + c] * wall_gain(p, OPP[i], yt >= Ly);
                        }
                    }
                    if (!wall && (xt < 0 || xt >= Lx)) {
                        if (p->bc_x == ORC_PERIODIC) xt = (xt + Lx) % Lx;
                        else if (p->bc_x == ORC_WALL) wall = 1;
                        else gone = 1;
                    }
                    if (gone) pbar[i * N + c] = 0.0;
                    else if (wall) pbar[i * N + c] = fbar[OPP[i] * N + c];
                    else pbar[i * N + c] = fbar[i * N + (size_t)yt * Lx + xt];
                }
            }
        }
        /* transposed collision Jacobian at every node, on the state f(., n) */
        const double *fn = fs + S9 * n;
        for (size_t c = 0; c < N; c++) {
            double fc[9], pb[9], fb[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            for (int i = 0; i < 9; i++) {
                fc[i] = fn[i * N + c];
                pb[i] = pbar[i * N + c];
            }
            double sb = 0.0, xb = 0.0, yb = 0.0;
            if (inout) {
                sb = Sb[c];
                xb = uxb[c];
                yb = uyb[c];
                Sb[c] = uxb[c] = uyb[c] = 0.0;
            }
            orc_node_vjp(p, fc, eps[c], gx[c], gy[c], pb, sb, xb, yb, fb, &dJdeps[c], &gxb[c],
                         &gyb[c]);
            for (int i = 0; i < 9; i++) fbar[i * N + c] = fb[i];
        }
    }
    /* initial state f_i = w_i eps rho0 (1 + ...) */
    {
        double feq1[9];
        orc_feq(p->rho0, p->u0x, p->u0y, feq1);
        for (size_t c = 0; c < N; c++)
            for (int i = 0; i < 9; i++) dJdeps[c] += fbar[i * N + c] * feq1[i];
    }
    /* grad(eps)(x) = (1/c2) sum_i W_i e_i eps(nb(x + e_i)): transpose the stencil */
    for (int y = 0; y < Ly; y++)
        for (int x = 0; x < Lx; x++) {
            size_t c = (size_t)y * Lx + x;
            for (int i = 0; i < 9; i++) {
                int xn = nb_index(x + EX[i], Lx, p->bc_x);
                int yn = nb_index(y + EY[i], Ly, p->bc_y);
                size_t cn = (size_t)yn * Lx + xn;
                dJdeps[cn] += (gxb[c] * W[i] * EX[i] + gyb[c] * W[i] * EY[i]) / CS2;
            }
        }
    free(fs); free(post); free(fbar); free(pbar); free(gx); free(gy); free(gxb); free(gyb);
    free(ends); free(Sb); free(uxb); free(uyb);
    return 0;
}
