// lbm_vans.hip -- gfx950 kernels and C-ABI of the volume-averaged lattice
// Boltzmann solver (Zhang, Wang & Ouyang, arXiv:1406.6438).
//
// Hot path: one fused pull sweep per time step.  Each lane owns a run of 4
// (FP32, FP16) or 2 (FP64) consecutive nodes of one row and, for each node x,
// in a single pass,
//   1. gathers f_i(x, n) from the post-collision populations of step n-1 at
//      x - e_i (periodic wrap, or the node's own opposite population behind a
//      half-way bounce-back wall);
//   2. forms eps rho (eq. (0moment)) and m = sum_i e_i f_i;
//   3. takes grad(eps) from an LDS tile of the porosity with a one-node halo,
//      the drag coefficients of the Ergun law from eps, and solves the
//      implicit velocity of eq. (1moment) in closed form;
//   4. relaxes toward the equilibrium of eq. (d2q9eq) and adds P_i + F_i
//      (eqs. (pi), (Fi)) in their common Guo form;
//   5. writes the 9 post-collision populations to its own nodes of the other
//      buffer (aligned, coalesced vector stores).
// Ensembles of independent problems run the same sweep over one list of the
// tiles of all members, one launch per step.
// The sweep moves 9 population loads, 9 population stores and one porosity
// load per node from HBM, so it is bandwidth-bound; there is no dense
// contraction and no MFMA.
//
// Storage.  Populations live in two SoA buffers [9][Ly][pitch] (x fastest,
// pitch a multiple of 256 nodes).  Slot (i, s) holds the post-collision value
// f*_i(s) minus the rest state at the middle of the link it travels next,
// w_i rho0 (eps(s) + eps(r)) / 2, where r = s + e_i is the node that pulls it
// (r = s when s + e_i lies behind a wall).  A post-collision population sits
// close to that midpoint rest state (about w_i rho0 (eps + e_i.grad(eps)/2)),
// so the stored numbers carry only the flow: FP32 and FP16 keep its
// significant digits.  The node that pulls a value adds back half the
// porosity difference to its source, and the one that stores it subtracts
// half the difference to its destination; both come from the porosity tile.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "lbm_vans.h"

namespace {

// ---------------------------------------------------------------------------
// Error reporting
// ---------------------------------------------------------------------------

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(LBM_VANS_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));  \
    } while (0)

// ---------------------------------------------------------------------------
// Library-held gradient workspace (lbm_vans_grad_static)
// ---------------------------------------------------------------------------
// For callers that cannot allocate device memory, lbm_vans_grad_static runs the
// gradient in this fixed array instead of a caller's buffer.  Every GPU the
// library runs on holds its own copy until the process ends.  In host code the
// name is not a device address: the address is looked up once per device
// (scratch_address) and only that address is passed to kernels and copies.
static __device__ __align__(256) char scratch[LBM_VANS_GRAD_STATIC_BYTES];

std::mutex g_scratch_mu;
std::vector<void *> g_scratch_addr;   // per device id; nullptr until looked up

// Device address of `scratch` on the current device (looked up on the first call
// for that device).
int scratch_address(void **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (static_cast<size_t>(dev) >= g_scratch_addr.size()) g_scratch_addr.resize(dev + 1, nullptr);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(LBM_VANS_EHIP, "no device address for the gradient workspace");
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return LBM_VANS_OK;
}

// ---------------------------------------------------------------------------
// Launch geometry
// ---------------------------------------------------------------------------

// Tile shape (compile-time).  Defaults: the fastest of the shapes timed on
// MI355X for the 4096^2 FP32 box (4 waves per block, non-temporal population
// loads, XCD-banded tile order).  The vector sweep takes its rows per thread
// from the storage type (sweep_rows): 1 for FP32 and FP64, 2 for FP16, whose
// narrower loads leave room for a second row in flight.
#ifndef LBM_VANS_NW
#define LBM_VANS_NW 4
#endif
#ifndef LBM_VANS_ROWS
#define LBM_VANS_ROWS 1
#endif
// rows each wave of the reverse step walks (k_adjoint_rows)
#ifndef LBM_VANS_ADJ_ROWS
#define LBM_VANS_ADJ_ROWS 4
#endif
#ifndef LBM_VANS_NT_LOADS
#define LBM_VANS_NT_LOADS 1
#endif
#ifndef LBM_VANS_XCD_BANDS
#define LBM_VANS_XCD_BANDS 1
#endif
#ifndef LBM_VANS_TB_AHEAD
#define LBM_VANS_TB_AHEAD 2
#endif
#ifndef LBM_VANS_TB_ROWS32
#define LBM_VANS_TB_ROWS32 8
#endif
#ifndef LBM_VANS_TB_ROWS16
#define LBM_VANS_TB_ROWS16 16
#endif
#ifndef LBM_VANS_TB3_ROWS32
#define LBM_VANS_TB3_ROWS32 24
#endif
#ifndef LBM_VANS_TB3_TALL32
#define LBM_VANS_TB3_TALL32 28
#endif
#ifndef LBM_VANS_TB3_SHORT32
#define LBM_VANS_TB3_SHORT32 12
#endif
#ifndef LBM_VANS_TB3_TINY32
#define LBM_VANS_TB3_TINY32 6
#endif
#ifndef LBM_VANS_TB4_ROWS32
#define LBM_VANS_TB4_ROWS32 24
#endif
#ifndef LBM_VANS_TB3_ROWS16
#define LBM_VANS_TB3_ROWS16 24
#endif
#ifndef LBM_VANS_TB_REUSE
#define LBM_VANS_TB_REUSE 3
#endif

constexpr int TX = 64;      // nodes per row segment: one wavefront
constexpr int NW = LBM_VANS_NW;      // wavefronts per block
constexpr int ROWS = LBM_VANS_ROWS;  // rows per thread of the one-node-per-lane kernels
constexpr int TY = NW * ROWS;
constexpr int ADJ_ROWS = LBM_VANS_ADJ_ROWS;

// Rows per thread of the vector sweep for a storage type.
template <typename S>
constexpr int sweep_rows()
{
    return std::is_same_v<S, _Float16> ? 2 : 1;
}
constexpr int NTHREADS = TX * NW;
constexpr int NRED = 8;     // doubles per block partial of the diagnostics
constexpr int NXCD = 8;     // accelerator complex dies of the MI355X
constexpr int PITCH_ALIGN = 256;  // row pitch in nodes: a multiple of 64 lanes x 4 nodes

struct Geo {
    int Lx, Ly, pitch;
    int wall_x, wall_y;     // the axis is not periodic (walls, or open for x)
    int open_x;             // x ends are open (inflow at x = 0, outflow at x = Lx-1)
    int nbx, ntiles;
    long long plane;        // Ly * pitch
};

// Workgroups are handed to the 8 XCDs round-robin by block id; renumber them
// so that each XCD walks one contiguous band of tiles (row-major), which keeps
// the porosity halo rows and the lines shared by neighbouring tiles in that
// XCD's L2.  The map is a bijection of [0, ntiles) for any ntiles.
__device__ __forceinline__ int xcd_tile(int bid, int ntiles)
{
    if (!LBM_VANS_XCD_BANDS) return bid;
    int q = ntiles / NXCD, r = ntiles % NXCD;
    int xcd = bid % NXCD, k = bid / NXCD;
    return xcd * q + min(xcd, r) + k;
}

// Index of a halo node along an axis: wrap-around when periodic, the mirror
// image across the half-way wall otherwise (node -1 -> 0, node L -> L-1).
__device__ __forceinline__ int halo_index(int v, int L, int wall)
{
    if (wall) return v < 0 ? 0 : (v >= L ? L - 1 : v);
    if (v < 0) v += L;
    else if (v >= L) v -= L;
    if (static_cast<unsigned>(v) >= static_cast<unsigned>(L)) {  // only for L below a tile width
        v %= L;
        if (v < 0) v += L;
    }
    return v;
}

// ---------------------------------------------------------------------------
// Storage codecs
// ---------------------------------------------------------------------------

// Every population, porosity and adjoint access goes through the global address
// space: the batched kernels take their pointers from member descriptors in memory,
// which the compiler cannot place, and would otherwise use flat instructions (64-bit
// addresses per lane, and a second counter to wait on).  For pointers passed as
// kernel arguments nothing changes.
template <typename T>
using gptr = __attribute__((address_space(1))) T *;

template <typename T>
__device__ __forceinline__ gptr<T> to_global(T *p)
{
    return (gptr<T>)p;
}

template <typename T>
__device__ __forceinline__ T load_global(const T *p)
{
    return *to_global(p);
}

template <typename S>
__device__ __forceinline__ S load_raw(const S *p)
{
    if constexpr (LBM_VANS_NT_LOADS)
        return __builtin_nontemporal_load(to_global(p));
    else
        return *to_global(p);
}

template <typename S, typename R>
__device__ __forceinline__ R decode_pop(S v, R inv_scale)
{
    if constexpr (std::is_same_v<S, _Float16>)
        return static_cast<R>(v) * inv_scale;
    else
        return static_cast<R>(v);
}

template <typename S, typename R>
__device__ __forceinline__ R load_pop(const S *p, R inv_scale)
{
    return decode_pop<S, R>(load_raw(p), inv_scale);
}

template <typename S, typename R>
__device__ __forceinline__ void store_pop(S *p, R v, R scale)
{
    if constexpr (std::is_same_v<S, _Float16>)
        __builtin_nontemporal_store(static_cast<_Float16>(v * scale), to_global(p));
    else
        __builtin_nontemporal_store(static_cast<S>(v), to_global(p));
}

// ---------------------------------------------------------------------------
// Physics of one node
// ---------------------------------------------------------------------------

template <typename R>
struct Phys {
    R omega;        // 1 / tau
    R pre;          // 1 - 1 / (2 tau)
    R rho0;         // shift reference density
    R Gx, Gy;       // body-force density
    R ca, cb;       // Ergun drag prefactors (0 under the constant law; see drag_coeffs)
    R ka, kb;       // constant-K drag prefactors (0 under the Ergun law)
    R scale, inv_scale;  // FP16 storage scale 2^s and 2^-s (1 otherwise)
    // Open x ends: a population entering across x = 0 (x = Lx-1) is the
    // equilibrium of a reservoir with the node's porosity, density rho_in
    // (rho_out) and velocity (u_in, 0) ((u_out, 0)); as a deviation from the
    // node's rest state it is eps * rin[i] (eps * rout[i]).  Applied from the
    // second state on (the initial state is the equilibrium everywhere).
    int reservoir;
    R rin[9], rout[9];
    // Velocity inlet / pressure outlet (inout): the reservoirs carry the inlet
    // node's own density with (u_in, 0) and rho_out with the outlet node's own
    // velocity, both of the state the step starts from.  The node at an end
    // writes them into its slots whose populations leave the domain (the
    // reader there pulls its own opposite slot, as behind a wall), so the
    // stored state stays the whole state.  rin[i] = w_i (P_i(u_in) - 1) for
    // the entering i (P_i the bracket of eq. (d2q9eq)); dro = rho_out - rho0.
    int inout;
    R dro, rho_out;
    // Sliding y-walls: a population leaving the wall below y = 0 (above
    // y = Ly-1) gains eps * 6 w_j rho0 (e_j . u_w); for the diagonals that is
    // +-eps * wb (+-eps * wt) with wb = rho0 u_bottom / 6, wt = rho0 u_top / 6.
    R wb, wt;
};

// Reciprocal and square root of the compute type: the hardware instructions
// (about 1 ulp) in FP32, correctly rounded operations in FP64.
template <typename R>
__device__ __forceinline__ R rcp(R x)
{
    if constexpr (std::is_same_v<R, float>)
        return __builtin_amdgcn_rcpf(x);
    else
        return R(1) / x;
}

template <typename R>
__device__ __forceinline__ R sqroot(R x)
{
    if constexpr (std::is_same_v<R, float>)
        return __builtin_amdgcn_sqrtf(x);
    else
        return sqrt(x);
}

// Darcy and Forchheimer coefficients a = eps^2 nu / K, b = eps^3 F_eps / sqrt(K)
// of the drag law, one branch-free form for both closures:
//   a = ca (1-eps)^2 / eps + ka eps^2,   b = cb (1-eps) + kb eps^3.
// Ergun closure: ca = 150 nu / d_p^2, cb = 1.75 / d_p, ka = kb = 0 (a = b = 0 at
// eps = 1); constant K, F_eps: ka = nu / K, kb = F_eps / sqrt(K), ca = cb = 0; all
// four 0 without drag.  inv_eps = 1 / eps.
template <typename R>
__device__ __forceinline__ void drag_coeffs(const Phys<R> &ph, R eps, R inv_eps, R &a, R &b)
{
    const R s = R(1) - eps, e2 = eps * eps;
    a = ph.ca * s * s * inv_eps + ph.ka * e2;
    b = ph.cb * s + ph.kb * e2 * eps;
}

template <typename R>
struct Node {
    R dS;           // eps rho - eps rho0  (sum of deviations)
    R S;            // eps rho             (eq. (0moment))
    R mx, my;       // sum_i e_i f_i
    R rho;          // intrinsic density S / eps
    R ux, uy;       // velocity of eq. (1moment)
    R Tx, Ty;       // c_s^2 rho grad(eps) + F(u): the vector of P_i + F_i
};

// Moments and velocity from the deviations d_i = f_i - w_i rho0 eps.
// eq. (1moment): eps rho u = m + (c_s^2 rho grad eps + F(u))/2 with
// F(u) = G - a u - b |u| u.  Writing A = eps rho + a/2, B = b/2 and
// V = m + (c_s^2 rho grad eps + G)/2, u is parallel to V and its length is
// the non-negative root of B s^2 + A s = |V|: u = k V with
// k = 2 / (A + sqrt(A^2 + 4 B |V|)), and |u| = k |V|.
template <typename R>
struct NodeFwd {  // the node's forward quantities (the reverse pass needs them all)
    Node<R> N;
    R ie, a, b, Vx, Vy, Vn, A, Rr, k, un, drag;
};

// The porosity-only terms of a node's update (the same at every step): eps,
// 1/eps, the lattice gradient of eps and the drag coefficients.
template <typename R>
struct EpsTerms {
    R e, ie, gex, gey, a, b;
};

template <typename R>
__device__ __forceinline__ EpsTerms<R> eps_terms(R eps, R gex, R gey, const Phys<R> &ph)
{
    EpsTerms<R> q;
    q.e = eps;
    q.ie = rcp(eps);
    q.gex = gex;
    q.gey = gey;
    drag_coeffs(ph, eps, q.ie, q.a, q.b);
    return q;
}

template <typename R>
__device__ __forceinline__ NodeFwd<R> node_forward_q(const R d[9], const EpsTerms<R> &q,
                                                     const Phys<R> &ph)
{
    NodeFwd<R> F;
    Node<R> &N = F.N;
    N.dS = ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8];
    N.S = q.e * ph.rho0 + N.dS;
    N.mx = (d[1] - d[3]) + (d[5] - d[6]) + (d[8] - d[7]);
    N.my = (d[2] - d[4]) + (d[5] + d[6]) - (d[7] + d[8]);
    F.ie = q.ie;
    N.rho = N.S * F.ie;
    const R third = R(1) / R(3);
    const R Qx = third * N.rho * q.gex, Qy = third * N.rho * q.gey;
    F.a = q.a;
    F.b = q.b;
    F.Vx = N.mx + R(0.5) * (Qx + ph.Gx);
    F.Vy = N.my + R(0.5) * (Qy + ph.Gy);
    F.A = N.S + R(0.5) * F.a;
    F.Vn = sqroot(F.Vx * F.Vx + F.Vy * F.Vy);
    F.Rr = sqroot(F.A * F.A + R(2) * F.b * F.Vn);
    F.k = R(2) * rcp(F.A + F.Rr);
    N.ux = F.k * F.Vx;
    N.uy = F.k * F.Vy;
    F.un = F.k * F.Vn;
    F.drag = F.a + F.b * F.un;
    N.Tx = Qx + ph.Gx - F.drag * N.ux;
    N.Ty = Qy + ph.Gy - F.drag * N.uy;
    return F;
}

template <typename R>
__device__ __forceinline__ NodeFwd<R> node_forward(const R d[9], R eps, R gex, R gey,
                                                   const Phys<R> &ph)
{
    return node_forward_q<R>(d, eps_terms<R>(eps, gex, gey, ph), ph);
}

template <typename R>
__device__ __forceinline__ Node<R> node_moments(const R d[9], R eps, R gex, R gey,
                                                const Phys<R> &ph)
{
    return node_forward<R>(d, eps, gex, gey, ph).N;
}

// D2Q9 velocities in the library's ordering.
__device__ constexpr int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

// Collision plus storage shift, in place on the deviations d_i = f_i - w_i rho0 eps:
//   f*_i = f_i - (f_i - f^eq_i)/tau + (1 - 1/(2 tau)) w_i [3 (e_i - u).T + 9 (e_i.u)(e_i.T)]
// with f^eq_i = w_i eps rho [1 + 3 e_i.u + 9/2 (e_i.u)^2 - 3/2 u.u].  With
// A_i = 3 e_i.u, B_i = 3 e_i.T, omega = 1/tau and P = 1 - 1/(2 tau):
//   d*_i = (1 - omega) d_i + w_i [K0 + A_i (omega S A_i / 2 + P B_i) + (omega S A_i + P B_i)]
//   K0   = omega (dS - 3/2 S u.u) - 3 P u.T.
// The middle term is even and the last one odd under e_i -> -e_i, so each pair of
// opposite directions shares them.  The stored value is d*_i - w_i de_i with
// de_i = (rho0/2) (eps(x + e_i) - eps(x)), the link-midpoint shift (0 when the
// value bounces back).
template <typename R>
__device__ __forceinline__ void collide(R d[9], const Node<R> &N, const Phys<R> &ph,
                                        const R de[9])
{
    const R om = ph.omega, omc = R(1) - ph.omega, P = ph.pre;
    const R uu = N.ux * N.ux + N.uy * N.uy;
    const R uT = N.ux * N.Tx + N.uy * N.Ty;
    const R oS = om * N.S, hS = R(0.5) * oS;
    const R K0 = om * (N.dS - R(1.5) * N.S * uu) - R(3) * P * uT;
    const R Ax = R(3) * N.ux, Ay = R(3) * N.uy;
    const R pBx = R(3) * P * N.Tx, pBy = R(3) * P * N.Ty;
    const R w0 = R(4) / R(9), w1 = R(1) / R(9), w2 = R(1) / R(36);
    auto pair = [&](R &di, R &dj, R A, R pB, R w, R dei, R dej) {
        const R base = K0 + A * (hS * A + pB);
        const R anti = oS * A + pB;
        di = omc * di + w * ((base + anti) - dei);
        dj = omc * dj + w * ((base - anti) - dej);
    };
    d[0] = omc * d[0] + w0 * K0;
    pair(d[1], d[3], Ax, pBx, w1, de[1], de[3]);
    pair(d[2], d[4], Ay, pBy, w1, de[2], de[4]);
    pair(d[5], d[7], Ax + Ay, pBx + pBy, w2, de[5], de[7]);
    pair(d[6], d[8], Ay - Ax, pBy - pBx, w2, de[6], de[8]);
}

// Neighbour coordinates of node (x, y) along both axes with wall flags.
struct Nbr {
    int xm, xp, ym, yp;
    bool wxm, wxp, wym, wyp;
};

__device__ __forceinline__ Nbr neighbours(int x, int y, const Geo &g)
{
    Nbr n;
    n.xm = x - 1; n.xp = x + 1; n.ym = y - 1; n.yp = y + 1;
    n.wxm = n.wxp = n.wym = n.wyp = false;
    if (n.xm < 0) { if (g.wall_x) { n.wxm = true; n.xm = x; } else n.xm = g.Lx - 1; }
    if (n.xp >= g.Lx) { if (g.wall_x) { n.wxp = true; n.xp = x; } else n.xp = 0; }
    if (n.ym < 0) { if (g.wall_y) { n.wym = true; n.ym = y; } else n.ym = g.Ly - 1; }
    if (n.yp >= g.Ly) { if (g.wall_y) { n.wyp = true; n.yp = y; } else n.yp = 0; }
    return n;
}

// Pull-gather of the deviations d_i(x, y) (gather_src: the addresses of the nine
// stored values).  A population whose source node x - e_i lies behind a wall is the
// node's own opposite post-collision value (half-way bounce-back).
template <typename S>
__device__ __forceinline__ void gather_src(const S *p[9], const S *__restrict__ f,
                                           long long plane, int pitch, int x, int y,
                                           const Nbr &n)
{
    const int c = y * pitch + x;
    const int rm = n.ym * pitch, r0 = y * pitch, rp = n.yp * pitch;
    const S *f1 = f + plane, *f2 = f + 2 * plane, *f3 = f + 3 * plane, *f4 = f + 4 * plane,
            *f5 = f + 5 * plane, *f6 = f + 6 * plane, *f7 = f + 7 * plane, *f8 = f + 8 * plane;
    p[0] = f + c;
    p[1] = n.wxm ? f3 + c : f1 + r0 + n.xm;
    p[2] = n.wym ? f4 + c : f2 + rm + x;
    p[3] = n.wxp ? f1 + c : f3 + r0 + n.xp;
    p[4] = n.wyp ? f2 + c : f4 + rp + x;
    p[5] = (n.wxm || n.wym) ? f7 + c : f5 + rm + n.xm;
    p[6] = (n.wxp || n.wym) ? f8 + c : f6 + rm + n.xp;
    p[7] = (n.wxp || n.wyp) ? f5 + c : f7 + rp + n.xp;
    p[8] = (n.wxm || n.wyp) ? f6 + c : f8 + rp + n.xm;
}

template <typename S, typename R>
__device__ __forceinline__ void gather(R d[9], const S *__restrict__ f, long long plane,
                                       int pitch, int x, int y, const Nbr &n, R inv_scale)
{
    const S *p[9];
    gather_src<S>(p, f, plane, pitch, x, y, n);
#pragma unroll
    for (int i = 0; i < 9; i++) d[i] = load_pop<S, R>(p[i], inv_scale);
}

// Porosity tile with a one-node halo, filled with the halo rule (wrap or
// mirror) so that every neighbour of an in-domain node is correct.
template <typename R, int W>
__device__ __forceinline__ void load_eps_tile(R (*tile)[W], const R *__restrict__ eps,
                                              const Geo &g, int x0, int y0)
{
    for (int k = threadIdx.x; k < (TY + 2) * W; k += NTHREADS) {
        int ly = k / W, lx = k - ly * W;
        int gx = halo_index(x0 + lx - 1, g.Lx, g.wall_x);
        int gy = halo_index(y0 + ly - 1, g.Ly, g.wall_y);
        tile[ly][lx] = load_global(eps + (long long)gy * g.pitch + gx);
    }
}

// The same tile fill split in two: issue() starts the global loads into
// registers, commit() writes them to LDS.  Population loads issued in between
// stay in flight while the tile is committed (memory counters retire in order,
// so waiting for the tile does not wait for loads issued after it).
template <typename R, int W, int TYV = TY>
struct EpsTile {
    static constexpr int N = (TYV + 2) * W;
    static constexpr int NE = (N + NTHREADS - 1) / NTHREADS;
    R v[NE];

    __device__ __forceinline__ void issue(const R *__restrict__ eps, const Geo &g, int x0, int y0)
    {
#pragma unroll
        for (int j = 0; j < NE; j++) {
            const int k = threadIdx.x + j * NTHREADS;
            if (k < N) {
                const int ly = k / W, lx = k - ly * W;
                // columns beyond the right halo only feed the nodes past the row end
                if (x0 + lx - 1 <= g.Lx) {
                    const int gx = halo_index(x0 + lx - 1, g.Lx, g.wall_x);
                    const int gy = halo_index(y0 + ly - 1, g.Ly, g.wall_y);
                    v[j] = load_global(eps + (long long)gy * g.pitch + gx);
                } else {
                    v[j] = R(1);
                }
            }
        }
    }

    __device__ __forceinline__ void commit(R (*tile)[W]) const
    {
#pragma unroll
        for (int j = 0; j < NE; j++) {
            const int k = threadIdx.x + j * NTHREADS;
            if (k < N) tile[k / W][k % W] = v[j];
        }
    }
};

// ---------------------------------------------------------------------------
// FP64 block reduction of the diagnostics
// ---------------------------------------------------------------------------
// v[0] = eps rho - eps rho0, v[1..2] = m, v[3..4] = eps rho u, v[5] = |u| (max),
// v[6] = non-finite count, v[7] unused.  One partial of NRED doubles per tile.

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ void block_partial(double acc[NRED], double *__restrict__ part,
                                              int tile)
{
    __shared__ double red[NW][NRED];
    const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
#pragma unroll
    for (int k = 0; k < NRED; k++) {
        double v = (k == 5) ? wave_max(acc[k]) : wave_sum(acc[k]);
        if (lane == 0) red[wv][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < NRED) {
        int k = threadIdx.x;
        double v = red[0][k];
        for (int w = 1; w < NW; w++) v = (k == 5) ? fmax(v, red[w][k]) : v + red[w][k];
        part[(long long)tile * NRED + k] = v;
    }
}

template <typename R>
__device__ __forceinline__ void accumulate(double acc[NRED], const Node<R> &N)
{
    bool ok = isfinite(static_cast<double>(N.S)) && isfinite(static_cast<double>(N.ux)) &&
              isfinite(static_cast<double>(N.uy));
    if (!ok) {
        acc[6] += 1.0;
        return;
    }
    acc[0] += static_cast<double>(N.dS);
    acc[1] += static_cast<double>(N.mx);
    acc[2] += static_cast<double>(N.my);
    acc[3] += static_cast<double>(N.S) * static_cast<double>(N.ux);
    acc[4] += static_cast<double>(N.S) * static_cast<double>(N.uy);
    double un = sqrt(static_cast<double>(N.ux) * N.ux + static_cast<double>(N.uy) * N.uy);
    acc[5] = fmax(acc[5], un);
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Porosity around one node from the tile: eps(x), the isotropic lattice
// gradient 3 sum_i w_i e_i eps(x + e_i) (the tile holds mirror images behind a
// wall), and the differences D[i] = eps(x + e_i) - eps(x), set to zero when
// x + e_i lies behind a wall (a bounced value never leaves its node).
template <typename R>
struct PorNb {
    R e0, gex, gey;
    R D[9];
};

template <typename R, int W>
__device__ __forceinline__ PorNb<R> porosity_nb(const R (*t)[W], int lyy, int lx, bool wxm,
                                                bool wxp, bool wym, bool wyp)
{
    PorNb<R> P;
    const R e0 = t[lyy][lx];
    const R eE = t[lyy][lx + 1], eW = t[lyy][lx - 1], eN = t[lyy + 1][lx], eS = t[lyy - 1][lx];
    const R eNE = t[lyy + 1][lx + 1], eNW = t[lyy + 1][lx - 1];
    const R eSW = t[lyy - 1][lx - 1], eSE = t[lyy - 1][lx + 1];
    const R c1 = R(1) / R(3), c2 = R(1) / R(12);
    P.e0 = e0;
    P.gex = c1 * (eE - eW) + c2 * ((eNE - eSW) + (eSE - eNW));
    P.gey = c1 * (eN - eS) + c2 * ((eNE - eSW) + (eNW - eSE));
    P.D[0] = R(0);
    P.D[1] = wxp ? R(0) : eE - e0;
    P.D[2] = wyp ? R(0) : eN - e0;
    P.D[3] = wxm ? R(0) : eW - e0;
    P.D[4] = wym ? R(0) : eS - e0;
    P.D[5] = (wxp || wyp) ? R(0) : eNE - e0;
    P.D[6] = (wxm || wyp) ? R(0) : eNW - e0;
    P.D[7] = (wxm || wym) ? R(0) : eSW - e0;
    P.D[8] = (wxp || wym) ? R(0) : eSE - e0;
    return P;
}

// Stored slots are shifted by the rest state at the link midpoint,
// w_i rho0 (eps(source) + eps(destination)) / 2.  The incoming value of
// direction i at x came from x - e_i, so the deviation from x's own rest state
// is the stored value plus (rho0/2) w_i (eps(x - e_i) - eps(x)).  FULL: the
// incoming values are the source's own deviations (post-collision values a
// multi-step pass hands over in registers, never shifted), which take the whole
// difference rho0 w_i (eps(x - e_i) - eps(x)).
template <typename R, bool FULL = false>
__device__ __forceinline__ void unshift_incoming(R d[9], const PorNb<R> &P, R rho0)
{
    const R hf = FULL ? R(1) : R(0.5);
    const R h1 = hf * rho0 * (R(1) / R(9)), h2 = hf * rho0 * (R(1) / R(36));
    d[1] += h1 * P.D[3];
    d[2] += h1 * P.D[4];
    d[3] += h1 * P.D[1];
    d[4] += h1 * P.D[2];
    d[5] += h2 * P.D[7];
    d[6] += h2 * P.D[8];
    d[7] += h2 * P.D[5];
    d[8] += h2 * P.D[6];
}

// Incoming values set by the boundaries rather than by a stored slot: the
// reservoir equilibria when the node is the first / last of an open x axis and
// reservoirs are active (a y-wall wins at the corners), and the momentum a
// sliding y-wall adds to the diagonals it returns.
template <typename R>
__device__ __forceinline__ void boundary_inflow(R d[9], R e0, bool open_l, bool open_r,
                                                bool wym, bool wyp, const Phys<R> &ph)
{
    if (ph.inout) open_l = open_r = false;   // their values are in the stored slots
    if (open_l) {
        d[1] = e0 * ph.rin[1];
        if (!wym) d[5] = e0 * ph.rin[5];
        if (!wyp) d[8] = e0 * ph.rin[8];
    }
    if (open_r) {
        d[3] = e0 * ph.rout[3];
        if (!wym) d[6] = e0 * ph.rout[6];
        if (!wyp) d[7] = e0 * ph.rout[7];
    }
    if (wym) {
        d[5] += e0 * ph.wb;
        d[6] -= e0 * ph.wb;
    }
    if (wyp) {
        d[8] += e0 * ph.wt;
        d[7] -= e0 * ph.wt;
    }
}

// Velocity inlet / pressure outlet: the populations that enter at the next step,
// as deviations from this node's rest state, written over the outgoing values
// that leave the domain (the slot of the opposite direction; behind a y-wall
// bounce-back keeps it).  Inlet (x = 0): w_i S P_i(u_in) - w_i rho0 eps =
// w_i dS + S rin[i] for i = 1, 5, 8 into slots 3, 7, 6.  Outlet (x = Lx-1):
// w_i eps (rho_out P_i(u) - rho0) = w_i eps (dro + rho_out (P_i(u) - 1)) for
// i = 3, 6, 7 into slots 1, 8, 5, u the node's velocity N of this step.
template <typename R>
__device__ __forceinline__ void inout_ends(R d[9], const Node<R> &N, R e0, bool open_l,
                                           bool open_r, bool wym, bool wyp, const Phys<R> &ph)
{
    const R w1 = R(1) / R(9), w2 = R(1) / R(36);
    if (open_l) {
        d[3] = w1 * N.dS + N.S * ph.rin[1];
        if (!wym) d[7] = w2 * N.dS + N.S * ph.rin[5];
        if (!wyp) d[6] = w2 * N.dS + N.S * ph.rin[8];
    }
    if (open_r) {
        const R uu = N.ux * N.ux + N.uy * N.uy;
        auto q = [&](R eu) {   // P(u) - 1 for e.u = eu
            return R(3) * eu + R(4.5) * eu * eu - R(1.5) * uu;
        };
        const R a = e0 * ph.rho_out, b = e0 * ph.dro;
        d[1] = w1 * (b + a * q(-N.ux));
        if (!wym) d[8] = w2 * (b + a * q(N.uy - N.ux));
        if (!wyp) d[5] = w2 * (b + a * q(-N.ux - N.uy));
    }
}

// Everything a node does after its gather: porosity neighbourhood from the
// tile, deviations from the node's rest state, moments and velocity,
// collision, and the shift of each outgoing value to its link midpoint (no
// shift when the value bounces back from a wall).  d holds the stored values
// of the incoming populations on entry and the values to store on exit.
// (lyy, lx) is the node's position in the tile.
// The same with the node's porosity-only terms given (q; P supplies its link
// differences).  IN_FULL: the incoming values are unshifted deviations of their
// sources (see unshift_incoming); OUT_SHIFT: shift the outgoing values to their
// link midpoints (values that go to memory), else leave them as this node's own
// deviations (values a multi-step pass keeps in registers for its next step).
template <typename R, bool DIAG, bool IN_FULL = false, bool OUT_SHIFT = true>
__device__ __forceinline__ void update_node_q(R d[9], const PorNb<R> &P, const EpsTerms<R> &q,
                                              bool wym, bool wyp, bool open_l, bool open_r,
                                              const Phys<R> &ph, double *acc, bool count)
{
    boundary_inflow<R>(d, P.e0, open_l, open_r, wym, wyp, ph);
    unshift_incoming<R, IN_FULL>(d, P, ph.rho0);
    Node<R> N = node_forward_q<R>(d, q, ph).N;
    if constexpr (DIAG) {
        if (count) accumulate<R>(acc, N);
    }
    const R hr = OUT_SHIFT ? R(0.5) * ph.rho0 : R(0);
    R de[9];
#pragma unroll
    for (int i = 0; i < 9; i++) de[i] = OUT_SHIFT ? hr * P.D[i] : R(0);
    collide<R>(d, N, ph, de);
    if (ph.inout && (open_l || open_r)) inout_ends<R>(d, N, P.e0, open_l, open_r, wym, wyp, ph);
}

template <typename R, int W, bool DIAG, bool IN_FULL = false, bool OUT_SHIFT = true>
__device__ __forceinline__ void update_node(R d[9], const R (*t)[W], int lyy, int lx, bool wxm,
                                            bool wxp, bool wym, bool wyp, bool open_l,
                                            bool open_r, const Phys<R> &ph, double *acc,
                                            bool count)
{
    const PorNb<R> P = porosity_nb<R, W>(t, lyy, lx, wxm, wxp, wym, wyp);
    update_node_q<R, DIAG, IN_FULL, OUT_SHIFT>(d, P, eps_terms<R>(P.e0, P.gex, P.gey, ph), wym,
                                               wyp, open_l, open_r, ph, acc, count);
}

// ---- vector sweep: V consecutive nodes per lane, full-width loads and stores

template <typename S, int V>
struct VecT {
    typedef S type __attribute__((ext_vector_type(V)));
};

template <typename S, typename R, int V>
__device__ __forceinline__ void ldv(R (&o)[V], const S *p, R inv_scale)
{
    using vt = typename VecT<S, V>::type;
    vt v = load_raw(reinterpret_cast<const vt *>(p));
#pragma unroll
    for (int k = 0; k < V; k++) {
        if constexpr (std::is_same_v<S, _Float16>)
            o[k] = static_cast<R>(v[k]) * inv_scale;
        else
            o[k] = static_cast<R>(v[k]);
    }
}

template <typename S, typename R, int V>
__device__ __forceinline__ void stv(S *p, const R (&o)[V], R scale)
{
    using vt = typename VecT<S, V>::type;
    vt v;
#pragma unroll
    for (int k = 0; k < V; k++) {
        if constexpr (std::is_same_v<S, _Float16>)
            v[k] = static_cast<S>(o[k] * scale);
        else
            v[k] = static_cast<S>(o[k]);
    }
    __builtin_nontemporal_store(v, to_global(reinterpret_cast<vt *>(p)));
}

// Lane geometry of the vector sweep: the run [x, x + V), of which the first n
// nodes lie in the domain (n < V only for the last lane of a row when Lx is not
// a multiple of V: a ragged run), its last node, its left / right neighbours
// (wrapped, or flagged as walls), and whether the lane must load the neighbour
// itself (wave edge, periodic seam or ragged end) instead of taking it from the
// adjacent lane.
struct LaneX {
    int x, n, last, xl, xr;
    bool wl, wr, need_l, need_r;
};

template <int V, bool WX, bool RG>
__device__ __forceinline__ LaneX lane_x(int x0, int lane, const Geo &g)  // WX: x not periodic
{
    LaneX L;
    L.x = x0 + lane * V;
    L.n = RG ? min(V, g.Lx - L.x) : V;
    L.last = L.x + L.n - 1;
    L.xl = L.x - 1;
    L.xr = L.last + 1;
    L.wl = L.wr = false;
    bool nl = lane == 0, nr = lane == TX - 1;
    if (L.xl < 0) {
        if (WX) { L.wl = true; L.xl = L.x; }
        else { L.xl = g.Lx - 1; nl = true; }
    }
    if (L.xr >= g.Lx) {
        if (WX) { L.wr = true; L.xr = L.last; }
        else { L.xr = L.xr % g.Lx; nr = true; }
    }
    L.need_l = nl && !L.wl;
    L.need_r = nr && !L.wr;
    return L;
}

// Pull-gather of the V nodes of one lane in row y: d[i][k] = f_i(x + k, y).
// Returns the wall flags of the rows above / below and the row offset.
// Phase 1 issues every load (nine aligned vectors, and for the lanes at a wave
// edge or periodic seam the single values beyond their run); phase 2 waits and
// rebuilds the x-shifted populations with cross-lane shuffles.  Keeping all
// loads ahead of the first shuffle keeps them in flight together.
template <typename S, typename R, int V, bool WY, bool RG>
__device__ __forceinline__ void gather_vec(R (&d)[9][V], const S *const F[9], int y,
                                           const Geo &g, const LaneX &L, R inv_scale,
                                           bool &wym, bool &wyp, unsigned &r0)
{
    using vt = typename VecT<S, V>::type;
    int ym = y - 1, yp = y + 1;
    wym = false;
    wyp = false;
    if (ym < 0) { if (WY) { wym = true; ym = y; } else ym = g.Ly - 1; }
    if (yp >= g.Ly) { if (WY) { wyp = true; yp = y; } else yp = 0; }
    r0 = y * g.pitch;
    const unsigned rm = ym * g.pitch, rp = yp * g.pitch;
    const int x = L.x;
    // Source rows of the nine vectors.  Behind a y wall a population is the
    // node's own opposite one (no shift then).
    // e_0 (0,0); e_2 (0,1) from y-1; e_4 (0,-1) from y+1; e_1 (1,0) from x-1;
    // e_3 (-1,0) from x+1; e_5 (1,1) from (x-1,y-1); e_6 (-1,1) from (x+1,y-1);
    // e_7 (-1,-1) from (x+1,y+1); e_8 (1,-1) from (x-1,y+1).
    const S *src[9] = {
        F[0] + r0 + x,
        F[1] + r0 + x,
        wym ? F[4] + r0 + x : F[2] + rm + x,
        F[3] + r0 + x,
        wyp ? F[2] + r0 + x : F[4] + rp + x,
        wym ? F[7] + r0 + x : F[5] + rm + x,
        wym ? F[8] + r0 + x : F[6] + rm + x,
        wyp ? F[5] + r0 + x : F[7] + rp + x,
        wyp ? F[6] + r0 + x : F[8] + rp + x,
    };
    // Lanes past the end of the row (last tile column) all read the row's
    // first vector instead (one shared line, no traffic of their own).
    const bool live = x < g.Lx;
    vt raw[9];
#pragma unroll
    for (int i = 0; i < 9; i++)
        raw[i] = load_raw(reinterpret_cast<const vt *>(live ? src[i] : F[i] + r0));
    // Values entering from the left (e_1, e_5, e_8) for the first node and from
    // the right (e_3, e_6, e_7) for the last node, where the adjacent lane does
    // not hold them: beyond a wall, the edge node's own opposite population.
    S el[3] = {S(0), S(0), S(0)}, er[3] = {S(0), S(0), S(0)};
    if (!live) {
    } else if (L.wl) {
        el[0] = load_raw(F[3] + r0 + x);
        el[1] = load_raw(F[7] + r0 + x);
        el[2] = load_raw(F[6] + r0 + x);
    } else if (L.need_l) {
        el[0] = load_raw(F[1] + r0 + L.xl);
        el[1] = load_raw(F[5] + rm + L.xl);
        el[2] = load_raw(F[8] + rp + L.xl);
    }
    if (!live) {
    } else if (L.wr) {
        er[0] = load_raw(F[1] + r0 + L.last);
        er[1] = load_raw(F[8] + r0 + L.last);
        er[2] = load_raw(F[5] + r0 + L.last);
    } else if (L.need_r) {
        er[0] = load_raw(F[3] + r0 + L.xr);
        er[1] = load_raw(F[6] + rm + L.xr);
        er[2] = load_raw(F[7] + rp + L.xr);
    }
    const bool own_l = L.wl || L.need_l, own_r = L.wr || L.need_r;
    auto cvt = [&](S v) {
        if constexpr (std::is_same_v<S, _Float16>)
            return static_cast<R>(v) * inv_scale;
        else
            return static_cast<R>(v);
    };
    // unshifted populations
#pragma unroll
    for (int k = 0; k < V; k++) {
        d[0][k] = cvt(raw[0][k]);
        d[2][k] = cvt(raw[2][k]);
        d[4][k] = cvt(raw[4][k]);
    }
    // from the left: node k takes element k-1; node 0 the previous lane's last
    auto left = [&](R (&o)[V], const vt &a, S edge, bool shifted) {
        R prev = cvt(a[V - 1]);
        prev = __shfl_up(prev, 1, 64);
        if (!shifted) {
#pragma unroll
            for (int k = 0; k < V; k++) o[k] = cvt(a[k]);
            return;
        }
        o[0] = own_l ? cvt(edge) : prev;
#pragma unroll
        for (int k = 1; k < V; k++) o[k] = cvt(a[k - 1]);
    };
    auto right = [&](R (&o)[V], const vt &a, S edge, bool shifted) {
        R next = cvt(a[0]);
        next = __shfl_down(next, 1, 64);
        if (!shifted) {
#pragma unroll
            for (int k = 0; k < V; k++) o[k] = cvt(a[k]);
            return;
        }
#pragma unroll
        for (int k = 0; k < V - 1; k++) o[k] = cvt(a[k + 1]);
        o[V - 1] = own_r ? cvt(edge) : next;
        if constexpr (RG) {
            // a ragged run ends at node n-1: its right neighbour is the edge value
#pragma unroll
            for (int k = 0; k < V - 1; k++)
                if (k == L.n - 1) o[k] = cvt(edge);
        }
    };
    left(d[1], raw[1], el[0], true);
    right(d[3], raw[3], er[0], true);
    left(d[5], raw[5], el[1], !wym);
    right(d[6], raw[6], er[1], !wym);
    right(d[7], raw[7], er[2], !wyp);
    left(d[8], raw[8], el[2], !wyp);
}

// The fused sweep with V consecutive nodes per lane (a pitch that is a
// multiple of 64 V); BX: x ends periodic (0), walls (1) or open (2); WY: walls
// across y; RG: Lx need not be a multiple of V (the last lane of a row may
// hold a ragged run; its nodes beyond Lx are computed from padding and stored
// into the padding, where nothing reads them).  Each
// population is one aligned vector load per lane; the x-shifted ones are
// rebuilt with one cross-lane shuffle and a masked scalar load for the lane at
// the wave's edge.  The first row's populations are requested before the
// porosity tile is filled, so their latency overlaps the tile load and the
// barrier.  The node update (moments, velocity, collision) then runs per node, and
// the 9 results leave as aligned vector stores.
template <typename S, typename R, int V, int BX, bool WY, bool DIAG, bool RG>
__device__ __forceinline__ void sweep_vec_tile(const S *__restrict__ fin, S *__restrict__ fout,
                                               const R *__restrict__ eps, const Geo &g,
                                               const Phys<R> &ph, double *__restrict__ part,
                                               int t)
{
    constexpr int W = TX * V + 2;
    constexpr int RW = sweep_rows<S>();
    constexpr int TYS = NW * RW;
    __shared__ R tile[TYS + 2][W];
    const int bx = t % g.nbx, by = t / g.nbx;
    const int x0 = bx * TX * V, y0 = by * TYS;
    const int lane = threadIdx.x % TX, ty = threadIdx.x / TX;
    constexpr bool WX = BX != 0;
    const LaneX L = lane_x<V, WX, RG>(x0, lane, g);
    const bool valid = L.x < g.Lx;
    const S *F[9];
#pragma unroll
    for (int i = 0; i < 9; i++) F[i] = fin + i * g.plane;

    EpsTile<R, W, TYS> et;
    et.issue(eps, g, x0, y0);
    R d[9][V];
    bool wym, wyp;
    unsigned r0;
    if (y0 + ty < g.Ly)
        gather_vec<S, R, V, WY, RG>(d, F, y0 + ty, g, L, ph.inv_scale, wym, wyp, r0);
    et.commit(tile);
    __syncthreads();

    double acc[NRED];
#pragma unroll
    for (int k = 0; k < NRED; k++) acc[k] = 0.0;
#pragma unroll
    for (int r = 0; r < RW; r++) {
        const int ly = ty + NW * r;
        const int y = y0 + ly;
        if (y >= g.Ly) break;
        if (r > 0) gather_vec<S, R, V, WY, RG>(d, F, y, g, L, ph.inv_scale, wym, wyp, r0);
#pragma unroll
        for (int k = 0; k < V; k++) {
            R dk[9];
#pragma unroll
            for (int i = 0; i < 9; i++) dk[i] = d[i][k];
            const bool wxm = WX && L.x + k == 0;
            const bool wxp = WX && L.x + k == g.Lx - 1;
            const bool ores = BX == 2 && ph.reservoir;
            update_node<R, W, DIAG>(dk, tile, ly + 1, lane * V + k + 1, wxm, wxp, wym, wyp,
                                    ores && wxm, ores && wxp, ph, acc, valid && k < L.n);
#pragma unroll
            for (int i = 0; i < 9; i++) d[i][k] = dk[i];
        }
        if (valid) {
#pragma unroll
            for (int i = 0; i < 9; i++)
                stv<S, R, V>(fout + i * g.plane + r0 + L.x, d[i], ph.scale);
        }
    }
    if constexpr (DIAG) block_partial(acc, part, t);
}

template <typename S, typename R, int V, int BX, bool WY, bool DIAG, bool RG>
__global__ __launch_bounds__(NTHREADS) void k_sweep_vec(const S *__restrict__ fin,
                                                        S *__restrict__ fout,
                                                        const R *__restrict__ eps, Geo g,
                                                        Phys<R> ph, double *__restrict__ part)
{
    sweep_vec_tile<S, R, V, BX, WY, DIAG, RG>(fin, fout, eps, g, ph, part,
                                              xcd_tile(blockIdx.x, g.ntiles));
}

// ---- two time steps per pass (periodic x) ----------------------------------
// Each wave walks a strip of 62 output columns down a chunk of tb_rows output
// rows, one node per lane: lane l holds column c0 + l - 1, so lanes 0 and 63
// are the strip's halo.  Per row it (A) gathers and collides step n -> n+1
// for the row below the output row from the input buffer, keeping the last
// three post-collision rows of step n+1 in registers, and (B) pulls step
// n+1 -> n+2 for the output row from those rows (x-shifts by DPP wave shifts,
// bounce-back behind y-walls from the node's own row) and stores it.  The
// state of step n+1 never leaves the registers: the pass moves the bytes of
// one step for two.  The node update is the sweep's own (update_node on a 3x3
// porosity window held per lane).  The row loop is unrolled by three so that
// the register window rotates by renaming.
// Output columns per strip of the NS-step pass: 64 lanes less NS-1 halo lanes
// on each side.
template <int NS>
constexpr int tb_cols()
{
    return TX - 2 * (NS - 1);
}

// Output rows per chunk: shorter chunks recompute more halo rows (2 (NS-1) per
// chunk) but give more waves to overlap; measured best for two steps: 8 rows
// in FP32, 16 in FP16; for three steps 24 in FP16, and in FP32 two heights:
// 28 rows where the lattice still has waves to fill the chip with them, else
// 24 (FP32 three-step pass, GLUPS at 16 / 24 / 28 / 32 rows: 4096^2 158.5 /
// 160.7 / 163.0 / 160.3; 2048^2 144.9 / 149.9 / 139.0 / 127.4; 64-member
// ensemble 144.1 / 144.2 / 146.3 / 146.4).
// The batched kernels tell the two FP32 heights apart by their row count.
static_assert(LBM_VANS_TB3_SHORT32 < LBM_VANS_TB3_ROWS32,
              "the short chunks of the FP32 three-step pass must be shorter than the default");
static_assert(LBM_VANS_TB3_TINY32 < LBM_VANS_TB3_SHORT32,
              "the tiny chunks of the FP32 three-step pass must be shorter than the short ones");
static_assert(LBM_VANS_TB3_TALL32 > LBM_VANS_TB3_ROWS32,
              "the tall chunks of the FP32 three-step pass must be taller than the short ones");

template <typename S, int NS = 2>
constexpr int tb_rows()
{
    if constexpr (NS == 4)
        return LBM_VANS_TB4_ROWS32;
    else if constexpr (NS == 3)
        return std::is_same_v<S, _Float16> ? LBM_VANS_TB3_ROWS16 : LBM_VANS_TB3_ROWS32;
    else
        return std::is_same_v<S, _Float16> ? LBM_VANS_TB_ROWS16 : LBM_VANS_TB_ROWS32;
}

// Value of the lane below (wave_shr: lane l reads lane l-1) and above
// (wave_shl: lane l reads lane l+1); the wave's end lanes read 0.
__device__ __forceinline__ float lane_from_below(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
                                         0, __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, false));
}

__device__ __forceinline__ float lane_from_above(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
                                         0, __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, false));
}

// Cached loads and stores of the multi-step passes: a strip's columns start
// off a cache line, so the lines at strip seams are shared by two waves;
// through the cache their halves meet in L2 instead of going to HBM separately
// (non-temporal accesses measured 20-30% slower here).
template <typename S, typename R>
__device__ __forceinline__ R load_cached(const S *p, R inv_scale)
{
    if constexpr (std::is_same_v<S, _Float16>)
        return static_cast<R>(load_global(p)) * inv_scale;
    else
        return static_cast<R>(load_global(p));
}

// Store through a buffer resource of one plane: a byte offset at or beyond the
// resource's size (TB_NO_STORE) makes the hardware drop the store, so lanes that
// must not write need no branch (a branch around the stores would make every
// later wait for data also wait for the loads issued ahead).
constexpr unsigned TB_NO_STORE = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(char *base, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(base, 0, static_cast<int>(bytes), 0x00020000);
}

template <typename S, typename R>
__device__ __forceinline__ void store_plane(__amdgpu_buffer_rsrc_t r, unsigned off, R v, R scale)
{
    if constexpr (std::is_same_v<S, _Float16>)
        __builtin_amdgcn_raw_buffer_store_b16(
            __builtin_bit_cast(unsigned short, static_cast<_Float16>(v * scale)), r,
            static_cast<int>(off), 0, 0);
    else
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, static_cast<float>(v)),
                                              r, static_cast<int>(off), 0, 0);
}

// BX: x ends periodic (0), walls (1) or open (2); WY: walls across y.  res_a:
// the reservoirs of open x ends are active in the first step of the pass (the
// pass starts from a state n >= 1); they are in the later ones.  With x ends,
// the lanes beside the domain compute on clamped columns and are never read.
// The work of one wave: strip `strip`, chunk `chunk` of the lattice g; both
// are uniform over the wave, so rows, row offsets and the y-wall tests live in
// scalar registers.  Addresses are a uniform per-plane base plus a 32-bit byte
// offset within the plane (the host runs this pass only when a plane's bytes
// fit in 31 bits and a row's in 24); only a value bounced at an x end, whose
// plane differs from lane to lane, takes a full per-lane address.
//
// The rows of the chunk are unrolled at compile time: the first step at row
// y0 + a (a = -(NS-1) .. n+NS-2), the middle step of three at y0 + b (b = -1
// .. n) and the last at y0 + j (j = 0 .. n-1) are straight-line code whose
// windows are plain values.  The gather loads of the
// first step run TB_AHEAD rows ahead of their use and, like the porosity loads
// and the stores, are issued with no branch around them: a row outside the
// lattice (behind a y wall, past the last chunk's end) loads a row inside it
// and its result goes unused.
constexpr int TB_AHEAD = LBM_VANS_TB_AHEAD;

// Whether the three-step pass computes the porosity-only terms of a row once and
// carries them to the row's later steps (six values for each of three rows in
// flight; LBM_VANS_TB_REUSE 0: never, 1: FP16 storage, 2: both, 3: FP32).
// Measured (GLUPS, 4096^2 FP32 / open-walls / ensemble, 8192^2 FP16 / open-walls):
// without 156.1 / 147.0 / 129.7, 209.3 / 169.6; with 156.7 / 150.3 / 133.6,
// 184.8 / 176.7 -- the FP16 periodic pass loses, so FP32 only.
template <typename S, int NS>
constexpr bool tb_reuse()
{
    constexpr bool f16 = std::is_same_v<S, _Float16>;
    return NS >= 3 && (LBM_VANS_TB_REUSE == 2 || (LBM_VANS_TB_REUSE == 1 && f16) ||
                       (LBM_VANS_TB_REUSE == 3 && !f16));
}

// Rows the gathers run ahead: TB_AHEAD, except one for the three-step passes in
// FP16 and for those with x ends or y walls, whose windows and boundary rules take
// the registers (GLUPS, two rows ahead / one: FP16 8192^2 box 211 / 191 in an older
// layout, 241.6 / 241.4 now; FP32 4096^2 channel with walls and open ends, 28-row
// chunks, 155.5 / 160.1; FP32 4096^2 box 156.7 / 149.8).
template <typename S, int NS, int BX = 0, bool WY = false>
constexpr int tb_ahead()
{
    return (NS >= 3 && (std::is_same_v<S, _Float16> || BX != 0 || WY)) ? 1 : TB_AHEAD;
}

// Most waves per SIMD the compiler schedules the three-step kernel for: 2 for the
// periodic FP32 pass (its schedule for 2 waves keeps the gathers of a row together
// and beats the 3 waves its registers would allow: 4096^2 box 163.4 against 156.7
// GLUPS), else no bound (the FP16 pass at 2: 197 against 242).
template <typename S, int BX, bool WY>
constexpr int tb3_max_waves()
{
    return (std::is_same_v<S, float> && BX == 0 && !WY) ? 2 : 8;
}

// f(integral_constant<int, J>) for J = 0, 1, ... while it returns true: code
// unrolled at compile time whatever its size.
template <typename F, int... J>
__device__ __forceinline__ void static_while_impl(F &&f, std::integer_sequence<int, J...>)
{
    (void)(f(std::integral_constant<int, J>{}) && ...);
}

template <int N, typename F>
__device__ __forceinline__ void static_while(F &&f)
{
    static_while_impl(f, std::make_integer_sequence<int, N>{});
}

// BXA: the x ends whose gather lookahead the pass takes (the kernel's own, also when a
// wave of it runs without x-end rules, so that both paths fit its registers).
template <typename S, typename R, int BX, bool WY, int NS, int NR, int BXA = BX>
__device__ __forceinline__ void tb_wave(const S *__restrict__ fin, S *__restrict__ fout,
                                        const R *__restrict__ eps, const Geo &g,
                                        const Phys<R> &ph, int strip, int chunk, int res_a)
{
    static_assert(std::is_same_v<R, float>, "the multi-step pass computes in FP32");
    static_assert(NS >= 2 && NS <= 4, "two to four steps per pass");
    constexpr bool WX = BX != 0;
    constexpr int H = NS - 1;                 // halo lanes per side, halo rows per chunk end
    constexpr int PD = tb_ahead<S, NS, BXA, WY>();
    constexpr int NA = NR + 2 * H;            // first-step rows y0-H .. y0+NR+H-1
    constexpr int NE = NA + 2;                // porosity rows y0-H-1 .. y0+NR+H
    constexpr unsigned SB = sizeof(S), EB = sizeof(R);
    const int lane = threadIdx.x % TX;
    const int xu = strip * tb_cols<NS>() + lane - H;  // unwrapped column
    int xi;
    if constexpr (WX) {
        xi = min(max(xu, 0), g.Lx - 1);
    } else {
        xi = xu % g.Lx;
        if (xi < 0) xi += g.Lx;
    }
    // x neighbours: wrapped, or the node itself behind an x wall / open end (the
    // gather then takes its own opposite population, the porosity its mirror)
    const bool wxm = WX && xu == 0, wxp = WX && xu == g.Lx - 1;
    const unsigned x = static_cast<unsigned>(xi);
    unsigned xm, xp;
    if constexpr (WX) {
        xm = xi == 0 ? 0 : xi - 1;
        xp = xi == g.Lx - 1 ? g.Lx - 1 : xi + 1;
    } else {
        xm = xi == 0 ? g.Lx - 1 : xi - 1;
        xp = xi == g.Lx - 1 ? 0 : xi + 1;
    }
    const bool out_ok = lane >= H && lane < TX - H && xu >= 0 && xu < g.Lx;
    const int y0 = chunk * NR;
    const unsigned pb = static_cast<unsigned>(g.pitch) * SB;   // bytes per state row
    const unsigned pe = static_cast<unsigned>(g.pitch) * EB;   // bytes per porosity row
    const unsigned xb = x * SB, xmb = xm * SB, xpb = xp * SB;
    const unsigned xe = x * EB, xme = xm * EB, xpe = xp * EB;
    const char *Fb[9];
    __amdgpu_buffer_rsrc_t Gr[9];
    const unsigned plane_b = static_cast<unsigned>(g.plane) * SB;
#pragma unroll
    for (int i = 0; i < 9; i++) {
        Fb[i] = reinterpret_cast<const char *>(fin + i * g.plane);
        Gr[i] = plane_rsrc(reinterpret_cast<char *>(fout + i * g.plane), plane_b);
    }
    const char *Eb = reinterpret_cast<const char *>(eps);
    auto ld = [&](const char *base, unsigned off) -> R {
        return load_cached<S, R>(reinterpret_cast<const S *>(base + off), ph.inv_scale);
    };
    // Row index of the lattice for window row v = y0 + a (a = -H-1 .. NR+H): clamped
    // behind y walls (such rows are never read), else wrapped once: the host runs the
    // pass with periodic y only when Ly >= NR + 2H + 2, so one wrap reaches every
    // window row.  Uniform over the wave: scalar selects, no branch.
    auto row_of = [&](int v) {
        if constexpr (WY) {
            return min(max(v, 0), g.Ly - 1);
        } else {
            v += v < 0 ? g.Ly : 0;
            return v - (v >= g.Ly ? g.Ly : 0);
        }
    };

    // porosity rows y0-H-1+k (k = 0 .. NE-1), columns x-1 .. x+1
    R E[NE][3];
    auto eps_row = [&](int k) {
        const unsigned o = __umul24(static_cast<unsigned>(row_of(y0 - H - 1 + k)), pe);
        E[k][0] = load_global(reinterpret_cast<const R *>(Eb + (o + xme)));
        E[k][1] = load_global(reinterpret_cast<const R *>(Eb + (o + xe)));
        E[k][2] = load_global(reinterpret_cast<const R *>(Eb + (o + xpe)));
    };
    // first step at row y0+a (a = -H .. NR+H-1): gather into Q[a+H], update into P1[a+H]
    R Q[NA][9], P1[NA][9];
    bool qm[NA], qp[NA];
    // Every row of the chunk's window is computed, also those behind a y wall or
    // past the lattice's last row (the last chunk): they take a row inside the
    // lattice, their results are never read, and the output rows past the last
    // row are not stored.  The chunk's code thus has no branch on its rows.
    auto issue = [&](int a) {
        const int yy = row_of(y0 + a);
        bool wym = false, wyp = false;
        int ym = yy - 1, yp = yy + 1;
        if (ym < 0) { if (WY) { wym = true; ym = yy; } else ym = g.Ly - 1; }
        if (yp >= g.Ly) { if (WY) { wyp = true; yp = yy; } else yp = 0; }
        qm[a + H] = wym;
        qp[a + H] = wyp;
        const unsigned r0 = __umul24(static_cast<unsigned>(yy), pb);
        const unsigned rm = __umul24(static_cast<unsigned>(ym), pb);
        const unsigned rp = __umul24(static_cast<unsigned>(yp), pb);
        const unsigned c = r0 + xb;
        R *q = Q[a + H];
        // a y wall is uniform over the wave: it picks the plane and the offset
        q[0] = ld(Fb[0], c);
        q[2] = ld(wym ? Fb[4] : Fb[2], wym ? c : rm + xb);
        q[4] = ld(wyp ? Fb[2] : Fb[4], wyp ? c : rp + xb);
        const char *b5 = wym ? Fb[7] : Fb[5], *b6 = wym ? Fb[8] : Fb[6];
        const char *b7 = wyp ? Fb[5] : Fb[7], *b8 = wyp ? Fb[6] : Fb[8];
        const unsigned o5 = wym ? c : rm + xmb, o6 = wym ? c : rm + xpb;
        const unsigned o7 = wyp ? c : rp + xpb, o8 = wyp ? c : rp + xmb;
        if constexpr (WX) {
            // a lane at an x end takes its own opposite populations
            auto lx = [&](bool own, const char *ob, const char *base, unsigned off) -> R {
                const S *p = own ? reinterpret_cast<const S *>(ob + c)
                                 : reinterpret_cast<const S *>(base + off);
                return load_cached<S, R>(p, ph.inv_scale);
            };
            q[1] = lx(wxm, Fb[3], Fb[1], r0 + xmb);
            q[3] = lx(wxp, Fb[1], Fb[3], r0 + xpb);
            q[5] = lx(wxm, Fb[7], b5, o5);
            q[6] = lx(wxp, Fb[8], b6, o6);
            q[7] = lx(wxp, Fb[5], b7, o7);
            q[8] = lx(wxm, Fb[6], b8, o8);
        } else {
            q[1] = ld(Fb[1], r0 + xmb);
            q[3] = ld(Fb[3], r0 + xpb);
            q[5] = ld(b5, o5);
            q[6] = ld(b6, o6);
            q[7] = ld(b7, o7);
            q[8] = ld(b8, o8);
        }
    };
    const bool oa = BX == 2 && res_a;        // reservoirs in the first step
    // the porosity-only terms of the row whose porosity tile starts at E[k]
    constexpr bool REUSE = tb_reuse<S, NS>();
    EpsTerms<R> T[REUSE ? NE : 1];
    auto finish = [&](int a) {
        const int k = a + H;                  // porosity rows of row y0+a: E[k .. k+2]
        const R t[3][3] = {{E[k][0], E[k][1], E[k][2]},
                           {E[k + 1][0], E[k + 1][1], E[k + 1][2]},
                           {E[k + 2][0], E[k + 2][1], E[k + 2][2]}};
#pragma unroll
        for (int i = 0; i < 9; i++) P1[k][i] = Q[k][i];
        if constexpr (REUSE) {
            const PorNb<R> P = porosity_nb<R, 3>(t, 1, 1, wxm, wxp, qm[k], qp[k]);
            T[k] = eps_terms<R>(P.e0, P.gex, P.gey, ph);
            update_node_q<R, false, false, false>(P1[k], P, T[k], qm[k], qp[k], oa && wxm,
                                                  oa && wxp, ph, nullptr, false);
        } else {
            update_node<R, 3, false, false, false>(P1[k], t, 1, 1, wxm, wxp, qm[k], qp[k],
                                                   oa && wxm, oa && wxp, ph, nullptr, false);
        }
    };
    // a later step at row y from the previous step's rows y-1 (A0), y (A1), y+1
    // (A2) of this wave (unshifted deviations), porosity rows E[k .. k+2]; a row
    // behind a y wall is never read, and the reservoirs are active (the step starts
    // from n + 1 >= 1).  LAST: the step's values go to memory (shifted to their
    // link midpoints); else they stay in registers for the next step.
    auto pull = [&](auto last_c, R (&d)[9], const R *A0, const R *A1, const R *A2, int y,
                    int k) {
        constexpr bool LAST = decltype(last_c)::value;
        const bool wym = WY && y == 0, wyp = WY && y == g.Ly - 1;
        const R s1 = lane_from_below(A1[1]), s3 = lane_from_above(A1[3]);
        d[0] = A1[0];
        d[1] = wxm ? A1[3] : s1;
        d[3] = wxp ? A1[1] : s3;
        if (wym) {
            d[2] = A1[4];
            d[5] = A1[7];
            d[6] = A1[8];
        } else {
            const R s5 = lane_from_below(A0[5]), s6 = lane_from_above(A0[6]);
            d[2] = A0[2];
            d[5] = wxm ? A1[7] : s5;
            d[6] = wxp ? A1[8] : s6;
        }
        if (wyp) {
            d[4] = A1[2];
            d[7] = A1[5];
            d[8] = A1[6];
        } else {
            const R s7 = lane_from_above(A2[7]), s8 = lane_from_below(A2[8]);
            d[4] = A2[4];
            d[7] = wxp ? A1[5] : s7;
            d[8] = wxm ? A1[6] : s8;
        }
        const R t[3][3] = {{E[k][0], E[k][1], E[k][2]},
                           {E[k + 1][0], E[k + 1][1], E[k + 1][2]},
                           {E[k + 2][0], E[k + 2][1], E[k + 2][2]}};
        if constexpr (REUSE) {
            // the row's first step computed its porosity-only terms
            const PorNb<R> P = porosity_nb<R, 3>(t, 1, 1, wxm, wxp, wym, wyp);
            update_node_q<R, false, true, LAST>(d, P, T[k], wym, wyp, BX == 2 && wxm,
                                                BX == 2 && wxp, ph, nullptr, false);
        } else {
            update_node<R, 3, false, true, LAST>(d, t, 1, 1, wxm, wxp, wym, wyp, BX == 2 && wxm,
                                                 BX == 2 && wxp, ph, nullptr, false);
        }
    };
    // second step of a three- or four-step pass at row y0+b (b = -(NS-2) .. NR+NS-3)
    // into P2[b+O2]; third step of a four-step pass at row y0+c (c = -1 .. NR) into
    // P3[c+1]
    constexpr int O2 = NS - 2;
    R P2[NS >= 3 ? NR + 2 * (NS - 2) : 1][9];
    R P3[NS == 4 ? NR + 2 : 1][9];
    auto middle = [&](int b) {
        if constexpr (NS >= 3) {
            pull(std::false_type{}, P2[b + O2], P1[b - 1 + H], P1[b + H], P1[b + 1 + H], y0 + b,
                 b + H);
        }
    };
    auto middle2 = [&](int c) {
        if constexpr (NS == 4) {
            pull(std::false_type{}, P3[c + 1], P2[c - 1 + O2], P2[c + O2], P2[c + 1 + O2],
                 y0 + c, c + H);
        }
    };
    // last step at output row y0+j, stored
    auto last = [&](int j) {
        R d[9];
        if constexpr (NS == 4)
            pull(std::true_type{}, d, P3[j], P3[j + 1], P3[j + 2], y0 + j, j + H);
        else if constexpr (NS == 3)
            pull(std::true_type{}, d, P2[j], P2[j + 1], P2[j + 2], y0 + j, j + H);
        else
            pull(std::true_type{}, d, P1[j - 1 + H], P1[j + H], P1[j + 1 + H], y0 + j, j + H);
        const bool row_ok = y0 + j < g.Ly;   // uniform: the last chunk's rows past the end
        const unsigned c = (out_ok && row_ok) ? __umul24(static_cast<unsigned>(y0 + j), pb) + xb
                                              : TB_NO_STORE;
#pragma unroll
        for (int i = 0; i < 9; i++) store_plane<S, R>(Gr[i], c, d[i], ph.scale);
    };

    // prologue: the porosity rows of the first PD iterations, the gathers of the
    // first-step rows -H .. H-1+PD, the first-step rows -H .. H-1, the second-step
    // rows -(NS-2) .. NS-3 and, for four steps, the third-step rows -1 and 0
#pragma unroll
    for (int k = 0; k < 2 * H + 2 + PD && k < NE; k++) eps_row(k);
#pragma unroll
    for (int a = -H; a <= H - 1 + PD && a <= NR + H - 1; a++) issue(a);
#pragma unroll
    for (int a = -H; a <= H - 1; a++) finish(a);
#pragma unroll
    for (int b = -(NS - 2); b <= NS - 3; b++) middle(b);
    middle2(-1);
    middle2(0);
    static_while<NR>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        finish(j + H);
        if constexpr (j + H + PD <= NR + H - 1) issue(j + H + PD);
        if constexpr (j + 2 * H + 2 + PD < NE) eps_row(j + 2 * H + 2 + PD);
        middle(j + NS - 2);
        middle2(j + 1);
        last(j);
        return true;
    });
}

// Whether the wave of strip `strip` has no lane, its halo lanes included, at an x
// end of a lattice Lx wide or beyond it: such a wave meets none of the x-end rules
// (walls, reservoirs, inlet / outlet), so the pass built without them (x periodic,
// whose wrap it never reaches) computes the same values with fewer instructions.
template <int NS>
__device__ __forceinline__ bool strip_clear_of_x_ends(int strip, int Lx)
{
    const int xlo = strip * tb_cols<NS>() - (NS - 1);
    return xlo >= 1 && xlo + TX - 1 <= Lx - 2;
}

// Whether the chunk `chunk` of NR rows, with the halo rows its first step computes and
// their porosity rows, keeps off the first and the last row of a lattice Ly tall: its
// waves meet no y-wall rule.
template <int NS, int NR>
__device__ __forceinline__ bool chunk_clear_of_y_walls(int chunk, int Ly)
{
    const int y0 = chunk * NR;
    return y0 - (NS - 1) >= 1 && y0 + NR + (NS - 1) - 1 <= Ly - 2;
}

// The multi-step pass of one wave: with open x ends (BX == 2: reservoirs, or an inlet
// and an outlet), the waves clear of them take the pass without x-end rules, and those
// also clear of the y walls (WY) the pass without any boundary rule (branches uniform
// over the wave).  Not for x walls: there the second path costs the four-step kernel
// half its waves per SIMD (256 VGPRs), the lattices are closed boxes, and their wall
// rules are cheap selects.
template <typename S, typename R, int BX, bool WY, int NS, int NR, bool BATCH = false>
__device__ __forceinline__ void tb_wave_x(const S *__restrict__ fin, S *__restrict__ fout,
                                          const R *__restrict__ eps, const Geo &g,
                                          const Phys<R> &ph, int strip, int chunk, int res_a)
{
    // the wall-free third path only where it leaves the kernel's waves per SIMD as
    // they are (the lone four-step and FP16 kernels drop to one wave with it)
    constexpr bool YCLEAR = WY && (BATCH || (NS == 3 && std::is_same_v<S, float>));
    // the batched three-step kernel keeps one path (with the others it measured 142
    // against 154 GLUPS)
    constexpr bool XCLEAR = BX == 2 && !(BATCH && NS == 3);
    if constexpr (XCLEAR) {
        if (strip_clear_of_x_ends<NS>(strip, g.Lx)) {
            if constexpr (YCLEAR) {
                if (chunk_clear_of_y_walls<NS, NR>(chunk, g.Ly)) {
                    tb_wave<S, R, 0, false, NS, NR, BX>(fin, fout, eps, g, ph, strip, chunk,
                                                        res_a);
                    return;
                }
            }
            tb_wave<S, R, 0, WY, NS, NR, BX>(fin, fout, eps, g, ph, strip, chunk, res_a);
            return;
        }
    }
    tb_wave<S, R, BX, WY, NS, NR>(fin, fout, eps, g, ph, strip, chunk, res_a);
}

template <typename S, typename R, int BX, bool WY, int NS, int NR>
__device__ __forceinline__ void sweep_multi(const S *__restrict__ fin, S *__restrict__ fout,
                                            const R *__restrict__ eps, const Geo &g,
                                            const Phys<R> &ph, int nstrips, int nchunks,
                                            int res_a)
{
    // the wave's id is uniform: keep it (and all row logic) in scalar registers
    const int wid = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * NW +
                                                   threadIdx.x / TX);
    const int strip = wid % nstrips, chunk = wid / nstrips;
    if (chunk >= nchunks) return;              // whole waves only; no barrier below
    tb_wave_x<S, R, BX, WY, NS, NR>(fin, fout, eps, g, ph, strip, chunk, res_a);
}

// Two steps per launch (one wave per strip and chunk).
template <typename S, typename R, int BX, bool WY>
__global__ __launch_bounds__(NTHREADS) void k_sweep_tb2(const S *__restrict__ fin,
                                                        S *__restrict__ fout,
                                                        const R *__restrict__ eps, Geo g,
                                                        Phys<R> ph, int nstrips, int nchunks,
                                                        int res_a)
{
    sweep_multi<S, R, BX, WY, 2, tb_rows<S, 2>()>(fin, fout, eps, g, ph, nstrips, nchunks,
                                                  res_a);
}

// Three steps per launch, in chunks of NR rows.
template <typename S, typename R, int BX, bool WY, int NR>
__global__ __launch_bounds__(NTHREADS)
__attribute__((amdgpu_waves_per_eu(1, tb3_max_waves<S, BX, WY>()))) void k_sweep_tb3(const S *__restrict__ fin,
                                                        S *__restrict__ fout,
                                                        const R *__restrict__ eps, Geo g,
                                                        Phys<R> ph, int nstrips, int nchunks,
                                                        int res_a)
{
    sweep_multi<S, R, BX, WY, 3, NR>(fin, fout, eps, g, ph, nstrips, nchunks, res_a);
}

// Four steps per launch (FP32 storage), in chunks of NR rows.
template <typename S, typename R, int BX, bool WY, int NR>
__global__ __launch_bounds__(NTHREADS)
__attribute__((amdgpu_waves_per_eu(1, tb3_max_waves<S, BX, WY>()))) void k_sweep_tb4(const S *__restrict__ fin,
                                                        S *__restrict__ fout,
                                                        const R *__restrict__ eps, Geo g,
                                                        Phys<R> ph, int nstrips, int nchunks,
                                                        int res_a)
{
    sweep_multi<S, R, BX, WY, 4, NR>(fin, fout, eps, g, ph, nstrips, nchunks, res_a);
}

// Macroscopic fields of the current state (no collision, no store of
// populations) plus the FP64 diagnostics partials.
template <typename S, typename R>
__global__ __launch_bounds__(NTHREADS) void k_moments(const S *__restrict__ fin,
                                                      const R *__restrict__ eps, Geo g,
                                                      Phys<R> ph, R *__restrict__ o_epsrho,
                                                      R *__restrict__ o_rho,
                                                      R *__restrict__ o_ux, R *__restrict__ o_uy,
                                                      double *__restrict__ part)
{
    constexpr int W = TX + 2;
    __shared__ R tile[TY + 2][W];
    const int t = xcd_tile(blockIdx.x, g.ntiles);
    const int bx = t % g.nbx, by = t / g.nbx;
    const int x0 = bx * TX, y0 = by * TY;
    load_eps_tile<R, W>(tile, eps, g, x0, y0);
    __syncthreads();
    double acc[NRED];
#pragma unroll
    for (int k = 0; k < NRED; k++) acc[k] = 0.0;
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int x = x0 + tx;
    for (int r = 0; r < ROWS; r++) {
        const int ly = ty + NW * r;
        const int y = y0 + ly;
        if (x < g.Lx && y < g.Ly) {
            Nbr n = neighbours(x, y, g);
            R d[9];
            gather<S, R>(d, fin, g.plane, g.pitch, x, y, n, ph.inv_scale);
            const PorNb<R> P = porosity_nb<R, W>(tile, ly + 1, tx + 1, n.wxm, n.wxp, n.wym, n.wyp);
            const bool ores = g.open_x && ph.reservoir;
            boundary_inflow<R>(d, P.e0, ores && x == 0, ores && x == g.Lx - 1, n.wym, n.wyp, ph);
            unshift_incoming<R>(d, P, ph.rho0);
            Node<R> N = node_moments<R>(d, P.e0, P.gex, P.gey, ph);
            accumulate<R>(acc, N);
            const long long o = (long long)y * g.Lx + x;
            if (o_epsrho) o_epsrho[o] = N.S;
            if (o_rho) o_rho[o] = N.rho;
            if (o_ux) o_ux[o] = N.ux;
            if (o_uy) o_uy[o] = N.uy;
        }
    }
    block_partial(acc, part, t);
}

// The outlet mass flux J = sum over x = Lx-1 of eps rho u_x of the current state
// (eqs. (0moment), (1moment)): one thread per row, FP64 partial of each block in
// part[block][0], summed by k_finalize.
template <typename S, typename R>
__global__ __launch_bounds__(NTHREADS) void k_outlet_flux(const S *__restrict__ fin,
                                                          const R *__restrict__ eps, Geo g,
                                                          Phys<R> ph, double *__restrict__ part)
{
    double acc[NRED];
#pragma unroll
    for (int k = 0; k < NRED; k++) acc[k] = 0.0;
    const int y = blockIdx.x * NTHREADS + threadIdx.x;
    if (y < g.Ly) {
        const int x = g.Lx - 1;
        const Nbr n = neighbours(x, y, g);
        R d[9];
        gather<S, R>(d, fin, g.plane, g.pitch, x, y, n, ph.inv_scale);
        // the porosity around the node, from the padded field with the halo rule
        R t[3][3];
        for (int j = 0; j < 3; j++)
            for (int i = 0; i < 3; i++)
                t[j][i] = eps[(long long)halo_index(y + j - 1, g.Ly, g.wall_y) * g.pitch +
                              halo_index(x + i - 1, g.Lx, g.wall_x)];
        const PorNb<R> P = porosity_nb<R, 3>(t, 1, 1, n.wxm, n.wxp, n.wym, n.wyp);
        const bool ores = g.open_x && ph.reservoir;
        boundary_inflow<R>(d, P.e0, ores && x == 0, ores, n.wym, n.wyp, ph);
        unshift_incoming<R>(d, P, ph.rho0);
        const Node<R> N = node_moments<R>(d, P.e0, P.gex, P.gey, ph);
        acc[0] = static_cast<double>(N.S) * static_cast<double>(N.ux);
    }
    block_partial(acc, part, blockIdx.x);
}

// Deterministic second pass: one block sums the tile partials in a fixed
// order and writes one diagnostics record (slot 0 gets rho0 * sum eps added,
// slot 7 the step index).
__global__ __launch_bounds__(1024) void k_finalize(const double *__restrict__ part, int nparts,
                                                   const double *__restrict__ mass0,
                                                   double step, double *__restrict__ out)
{
    __shared__ double red[1024];
    for (int k = 0; k < 7; k++) {
        double v = 0.0;
        for (int j = threadIdx.x; j < nparts; j += 1024) {
            double p = part[(long long)j * NRED + k];
            v = (k == 5) ? fmax(v, p) : v + p;
        }
        red[threadIdx.x] = v;
        __syncthreads();
        for (int s = 512; s > 0; s >>= 1) {
            if (threadIdx.x < s) {
                double a = red[threadIdx.x], b = red[threadIdx.x + s];
                red[threadIdx.x] = (k == 5) ? fmax(a, b) : a + b;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) out[k] = (k == 0 && mass0) ? red[0] + *mass0 : red[0];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[7] = step;
}

// Porosity copy into the padded layout, with the (0, 1] check and FP64 sum:
// partial slot 0 = sum eps, slot 6 = count of values outside (0, 1].
template <typename R>
__global__ __launch_bounds__(NTHREADS) void k_eps_copy(const R *__restrict__ src,
                                                       R *__restrict__ dst, Geo g,
                                                       double *__restrict__ part)
{
    double acc[NRED];
#pragma unroll
    for (int k = 0; k < NRED; k++) acc[k] = 0.0;
    const int t = blockIdx.x;
    const int bx = t % g.nbx, by = t / g.nbx;
    const int x = bx * TX + threadIdx.x % TX;
    for (int r = 0; r < ROWS; r++) {
        const int y = by * TY + threadIdx.x / TX + NW * r;
        if (x < g.Lx && y < g.Ly) {
            R e = src[(long long)y * g.Lx + x];
            dst[(long long)y * g.pitch + x] = e;
            if (e > R(0) && e <= R(1)) acc[0] += static_cast<double>(e);
            else acc[6] += 1.0;
        }
    }
    block_partial(acc, part, t);
}

// Rest-state reference w_i rho0 eps for a stored slot and the deviation of
// a plain population from it, in FP64 (used by init and set_state only).
__device__ __forceinline__ double wgt(int i)
{
    return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
}

__device__ constexpr int OPPI[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

// Node that pulls slot (i, x, y) next, and the direction it pulls it as;
// ywall: the slot returns from a y-wall (-1 below, +1 above, 0 otherwise).
__device__ __forceinline__ void reader(int i, int x, int y, const Geo &g, int &rx, int &ry,
                                       int &ri, int &ywall)
{
    int tx = x + CX[i], ty = y + CY[i];
    bool wall = false;
    ywall = 0;
    if (tx < 0 || tx >= g.Lx) {
        if (g.wall_x) wall = true;
        else tx = tx < 0 ? tx + g.Lx : tx - g.Lx;
    }
    if (ty < 0 || ty >= g.Ly) {
        if (g.wall_y) {
            wall = true;
            ywall = ty < 0 ? -1 : 1;
        } else {
            ty = ty < 0 ? ty + g.Ly : ty - g.Ly;
        }
    }
    if (wall) { rx = x; ry = y; ri = OPPI[i]; }
    else { rx = tx; ry = ty; ri = i; }
}

// Gain per unit porosity of population j returned by a sliding y-wall
// (ywall -1: the wall below, +1: above), 6 w_j rho0 (e_j . u_w), in FP64.
__device__ __forceinline__ double wall_gain(int j, int ywall, double wb6, double wt6)
{
    if (ywall == 0 || CX[j] == 0) return 0.0;
    return CX[j] * (ywall < 0 ? wb6 : wt6);
}

// Writes the storage of a plain state f(., n): fplain == nullptr means the
// equilibrium f_i = f_i^eq(eps rho0, u0) of eq. (d2q9eq) (the initial state).
// rho_ref is the shift reference rho0 as the sweep sees it (rounded to R), so
// that the stored deviations and the sweep's rest state agree exactly.
// wb6, wt6: rho0 u_w / 6 of the sliding y-walls (below, above): a slot that
// returns from such a wall is stored without the gain the reader adds.
template <typename S, typename R>
__global__ __launch_bounds__(NTHREADS) void k_set_state(S *__restrict__ fout,
                                                        const R *__restrict__ eps, Geo g,
                                                        double rho0, double rho_ref,
                                                        double u0x, double u0y,
                                                        const double *__restrict__ fplain,
                                                        R scale, double wb6, double wt6)
{
    const int t = blockIdx.x;
    const int bx = t % g.nbx, by = t / g.nbx;
    const int x = bx * TX + threadIdx.x % TX;
    for (int r = 0; r < ROWS; r++) {
        const int y = by * TY + threadIdx.x / TX + NW * r;
        if (x >= g.Lx || y >= g.Ly) continue;
        for (int i = 0; i < 9; i++) {
            int rx, ry, ri, yw;
            reader(i, x, y, g, rx, ry, ri, yw);
            // stored = f_ri(reader) - w rho_ref (eps(x) + eps(reader)) / 2
            double er = static_cast<double>(eps[(long long)ry * g.pitch + rx]);
            double es = static_cast<double>(eps[(long long)y * g.pitch + x]);
            double w = wgt(ri);
            double dev;
            if (fplain) {
                long long N = (long long)g.Lx * g.Ly;
                dev = fplain[ri * N + (long long)ry * g.Lx + rx] - w * rho_ref * 0.5 * (es + er);
            } else {
                double eu = CX[ri] * u0x + CY[ri] * u0y;
                double uu = u0x * u0x + u0y * u0y;
                dev = w * (er * ((rho0 - rho_ref) + rho0 * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu)) +
                           0.5 * rho_ref * (er - es));
            }
            dev -= wall_gain(ri, yw, wb6, wt6) * er;
            S *p = fout + i * g.plane + (long long)y * g.pitch + x;
            if constexpr (std::is_same_v<S, _Float16>)
                *p = static_cast<_Float16>(static_cast<R>(dev) * scale);
            else
                *p = static_cast<S>(dev);
        }
    }
}

// Plain populations f_i(x, n) = d_i + w_i rho0 eps(x) of the current state.
template <typename S, typename R>
__global__ __launch_bounds__(NTHREADS) void k_get_state(const S *__restrict__ fin,
                                                        const R *__restrict__ eps, Geo g,
                                                        Phys<R> ph, double *__restrict__ out)
{
    constexpr int W = TX + 2;
    __shared__ R tile[TY + 2][W];
    const int t = blockIdx.x;
    const int bx = t % g.nbx, by = t / g.nbx;
    const int x0 = bx * TX, y0 = by * TY;
    load_eps_tile<R, W>(tile, eps, g, x0, y0);
    __syncthreads();
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int x = x0 + tx;
    const long long N = (long long)g.Lx * g.Ly;
    for (int r = 0; r < ROWS; r++) {
        const int ly = ty + NW * r;
        const int y = y0 + ly;
        if (x >= g.Lx || y >= g.Ly) continue;
        Nbr n = neighbours(x, y, g);
        R d[9];
        gather<S, R>(d, fin, g.plane, g.pitch, x, y, n, ph.inv_scale);
        const PorNb<R> P = porosity_nb<R, W>(tile, ly + 1, tx + 1, n.wxm, n.wxp, n.wym, n.wyp);
        const bool ores = g.open_x && ph.reservoir;
        boundary_inflow<R>(d, P.e0, ores && x == 0, ores && x == g.Lx - 1, n.wym, n.wyp, ph);
        unshift_incoming<R>(d, P, ph.rho0);
        const double e0 = static_cast<double>(P.e0);
        for (int i = 0; i < 9; i++)
            out[i * N + (long long)y * g.Lx + x] =
                static_cast<double>(d[i]) + wgt(i) * static_cast<double>(ph.rho0) * e0;
    }
}

// ---------------------------------------------------------------------------
// Adjoint (reverse) sweep: gradient of the outlet mass flux with respect to eps
// ---------------------------------------------------------------------------
// The forward map of one step takes the stored post-collision values F^n to
// F^{n+1}: every node pulls its incoming populations (streaming, bounce-back,
// reservoirs) and collides them.  Its adjoint takes lambda^{n+1} (the
// adjoint of F^{n+1}, i.e. of each node's 9 outgoing values) to lambda^n:
// every node applies the transposed Jacobian of its collision to its 9
// outgoing adjoints and pushes each incoming adjoint back into the slot it
// was pulled from (the same bijection as the gather, run backwards).  Porosity
// enters a node through eps (density, drag coefficients), through grad(eps)
// (accumulated per node, transposed through the lattice stencil at the end),
// through the reservoir populations and through the initial state.  Adjoints
// are of the plain populations; the storage shifts are decoded as in the
// forward.

// d(a)/d(eps), d(b)/d(eps) of drag_coeffs.
template <typename R>
__device__ __forceinline__ void drag_derivs(const Phys<R> &ph, R eps, R inv_eps, R &da, R &db)
{
    da = -ph.ca * (R(1) - eps) * (R(1) + eps) * inv_eps * inv_eps + R(2) * ph.ka * eps;
    db = -ph.cb + R(3) * ph.kb * eps * eps;
}

// Reverse of one node.  d: the node's incoming deviations (as update_node
// sees them before the collision); mu: adjoints of its 9 post-collision
// values; S_bar0, ux_bar0, uy_bar0: adjoints of eps rho and u (the objective).
// Returns the adjoints of the 9 incoming plain populations in nu and adds the
// direct porosity and porosity-gradient adjoints to eb, gxb, gyb.
template <typename R>
__device__ __forceinline__ void node_vjp(const R d[9], R e0, R gex, R gey, const Phys<R> &ph,
                                         const R mu[9], R S_bar0, R ux_bar0, R uy_bar0,
                                         R nu[9], R &eb, R &gxb, R &gyb)
{
    const NodeFwd<R> F = node_forward<R>(d, e0, gex, gey, ph);
    const Node<R> &N = F.N;
    const R om = ph.omega, P = ph.pre, S = N.S, ux = N.ux, uy = N.uy;
    const R uu = ux * ux + uy * uy;
    R S_bar = S_bar0, ux_bar = ux_bar0, uy_bar = uy_bar0;
    R Tx_bar = R(0), Ty_bar = R(0), uu_bar = R(0), uT_bar = R(0);
    // out_i = (1 - omega) f_i + omega feq_i + src_i,
    // feq_i = w_i S (1 + A_i + A_i^2/2 - 3/2 u.u), src_i = P w_i (B_i (1 + A_i) - 3 u.T),
    // A_i = 3 e_i.u, B_i = 3 e_i.T
#pragma unroll
    for (int i = 0; i < 9; i++) {
        const R cx = R(CX[i]), cy = R(CY[i]);
        const R w = i == 0 ? R(4) / R(9) : (i < 5 ? R(1) / R(9) : R(1) / R(36));
        const R Ai = R(3) * (cx * ux + cy * uy);
        const R Bi = R(3) * (cx * N.Tx + cy * N.Ty);
        const R m = mu[i];
        nu[i] = (R(1) - om) * m;
        S_bar += om * m * w * (R(1) + Ai + R(0.5) * Ai * Ai - R(1.5) * uu);
        const R A_bar = om * m * w * S * (R(1) + Ai) + m * P * w * Bi;
        const R B_bar = m * P * w * (R(1) + Ai);
        uu_bar -= R(1.5) * om * S * m * w;
        uT_bar -= R(3) * P * m * w;
        ux_bar += R(3) * cx * A_bar;
        uy_bar += R(3) * cy * A_bar;
        Tx_bar += R(3) * cx * B_bar;
        Ty_bar += R(3) * cy * B_bar;
    }
    ux_bar += R(2) * ux * uu_bar + N.Tx * uT_bar;
    uy_bar += R(2) * uy * uu_bar + N.Ty * uT_bar;
    Tx_bar += ux * uT_bar;
    Ty_bar += uy * uT_bar;
    // T = Q + G - drag u, drag = a + b |u|
    R Qx_bar = Tx_bar, Qy_bar = Ty_bar;
    const R drag_bar = -(Tx_bar * ux + Ty_bar * uy);
    ux_bar -= F.drag * Tx_bar;
    uy_bar -= F.drag * Ty_bar;
    R a_bar = drag_bar, b_bar = drag_bar * F.un;
    const R un_bar = drag_bar * F.b;
    // u = k V, |u| = k |V|, k = 2 / (A + Rr), Rr = sqrt(A^2 + 2 b |V|)
    const R k_bar = ux_bar * F.Vx + uy_bar * F.Vy + un_bar * F.Vn;
    R Vx_bar = F.k * ux_bar, Vy_bar = F.k * uy_bar, Vn_bar = F.k * un_bar;
    const R den_bar = -k_bar * F.k * F.k * R(0.5);
    R A_bar = den_bar;
    const R Rr_bar = den_bar * rcp(F.Rr);
    A_bar += Rr_bar * F.A;
    b_bar += Rr_bar * F.Vn;
    Vn_bar += Rr_bar * F.b;
    if (F.Vn > R(0)) {
        const R iv = rcp(F.Vn);
        Vx_bar += Vn_bar * F.Vx * iv;
        Vy_bar += Vn_bar * F.Vy * iv;
    }
    // A = S + a/2;  V = m + (Q + G)/2;  Q = rho grad(eps)/3;  rho = S/eps
    S_bar += A_bar;
    a_bar += R(0.5) * A_bar;
    Qx_bar += R(0.5) * Vx_bar;
    Qy_bar += R(0.5) * Vy_bar;
    const R third = R(1) / R(3);
    const R rho_bar = third * (Qx_bar * gex + Qy_bar * gey);
    gxb += third * N.rho * Qx_bar;
    gyb += third * N.rho * Qy_bar;
    S_bar += rho_bar * F.ie;
    R da, db;
    drag_derivs(ph, e0, F.ie, da, db);
    eb += -rho_bar * S * F.ie * F.ie + a_bar * da + b_bar * db;
    // S = sum f, m = sum e f
#pragma unroll
    for (int i = 0; i < 9; i++) nu[i] += S_bar + R(CX[i]) * Vx_bar + R(CY[i]) * Vy_bar;
}

// The reverse of one node at one step.  d: the node's incoming deviations of the
// state the step starts from (gathered, with the boundary rules applied and the
// storage shift removed); mu: adjoints of its 9 outgoing values (SEED: unused, the
// objective seeds the node instead).  At a velocity inlet / pressure outlet end the
// slots that leave the domain hold the next step's reservoir populations: their
// adjoints go to the end node's eps rho, velocity and porosity, not to the collision.
// Returns the adjoints of the 9 incoming values in nu, the directions whose incoming
// value came from an equilibrium reservoir (res: nothing to push) and the node's
// porosity sensitivities; SEED adds J's share of the node to acc[0].
template <typename R, bool SEED>
__device__ __forceinline__ void adjoint_node(const R d[9], const PorNb<R> &P, const Nbr &n,
                                             bool ol, bool orr, bool last_col, const Phys<R> &ph,
                                             R mu[9], R nu[9], bool res[9], R &e_b, R &gx_b,
                                             R &gy_b, double *acc)
{
    R S_bar0 = R(0), ux_bar0 = R(0), uy_bar0 = R(0), e_end = R(0);
    const R w1 = R(1) / R(9), w2 = R(1) / R(36);
    if constexpr (SEED) {
#pragma unroll
        for (int i = 0; i < 9; i++) mu[i] = R(0);
        if (last_col) {
            const Node<R> N = node_moments<R>(d, P.e0, P.gex, P.gey, ph);
            S_bar0 = N.ux;
            ux_bar0 = N.S;
            acc[0] += static_cast<double>(N.S) * static_cast<double>(N.ux);
        }
    } else {
        if (ph.inout && (ol || orr)) {
            if (ol) {
                S_bar0 += mu[3] * (w1 + ph.rin[1]);
                mu[3] = R(0);
                if (!n.wym) { S_bar0 += mu[7] * (w2 + ph.rin[5]); mu[7] = R(0); }
                if (!n.wyp) { S_bar0 += mu[6] * (w2 + ph.rin[8]); mu[6] = R(0); }
            }
            if (orr) {
                const Node<R> N = node_moments<R>(d, P.e0, P.gex, P.gey, ph);
                const R uu = N.ux * N.ux + N.uy * N.uy;
                const R er = P.e0 * ph.rho_out;
                // plain value w (eps rho_out) P(u): d/d eps = w rho_out P(u),
                // d/du = w eps rho_out (3 e + 9 (e.u) e - 3 u)
                auto link = [&](int slot, R w, R ex, R ey) {
                    const R m = mu[slot], eu = ex * N.ux + ey * N.uy;
                    e_end += m * w * ph.rho_out *
                             (R(1) + R(3) * eu + R(4.5) * eu * eu - R(1.5) * uu);
                    ux_bar0 += m * w * er * (R(3) * ex + R(9) * eu * ex - R(3) * N.ux);
                    uy_bar0 += m * w * er * (R(3) * ey + R(9) * eu * ey - R(3) * N.uy);
                    mu[slot] = R(0);
                };
                link(1, w1, R(-1), R(0));
                if (!n.wym) link(8, w2, R(-1), R(1));
                if (!n.wyp) link(5, w2, R(-1), R(-1));
            }
        }
    }
    e_b = e_end;
    gx_b = R(0);
    gy_b = R(0);
    node_vjp<R>(d, P.e0, P.gex, P.gey, ph, mu, S_bar0, ux_bar0, uy_bar0, nu, e_b, gx_b, gy_b);
    // reservoir links: the incoming value is eps0 * (rin_i + w_i rho0)
#pragma unroll
    for (int i = 0; i < 9; i++) res[i] = false;
    if (ol && !ph.inout) {
        res[1] = true; res[5] = !n.wym; res[8] = !n.wyp;
        e_b += nu[1] * (ph.rin[1] + w1 * ph.rho0);
        if (res[5]) e_b += nu[5] * (ph.rin[5] + w2 * ph.rho0);
        if (res[8]) e_b += nu[8] * (ph.rin[8] + w2 * ph.rho0);
    }
    if (orr && !ph.inout) {
        res[3] = true; res[6] = !n.wym; res[7] = !n.wyp;
        e_b += nu[3] * (ph.rout[3] + w1 * ph.rho0);
        if (res[6]) e_b += nu[6] * (ph.rout[6] + w2 * ph.rho0);
        if (res[7]) e_b += nu[7] * (ph.rout[7] + w2 * ph.rho0);
    }
    // sliding y-walls: the returned diagonals carry +-eps * wb (wt)
    if (n.wym) e_b += (nu[5] - nu[6]) * ph.wb;
    if (n.wyp) e_b += (nu[8] - nu[7]) * ph.wt;
}

// Push of a node's incoming adjoints into the adjoint slots of the state the
// step started from (the gather run backwards; every slot receives exactly one
// value, a reservoir link a zero).
template <typename R, typename A>
__device__ __forceinline__ void push_global(A *__restrict__ lam, const Geo &g, int x, int y,
                                            const Nbr &n, const R nu[9], const bool res[9])
{
    const int c = y * g.pitch + x;
    const int rm = n.ym * g.pitch, r0 = y * g.pitch, rp = n.yp * g.pitch;
    const long long pl = g.plane;
    const gptr<A> lg = to_global(lam);
    gptr<A> L0 = lg, L1 = lg + pl, L2 = lg + 2 * pl, L3 = lg + 3 * pl, L4 = lg + 4 * pl,
            L5 = lg + 5 * pl, L6 = lg + 6 * pl, L7 = lg + 7 * pl, L8 = lg + 8 * pl;
    auto v = [&](int i) { return res[i] ? A(0) : static_cast<A>(nu[i]); };
    L0[c] = static_cast<A>(nu[0]);
    *(n.wxm ? L3 + c : L1 + r0 + n.xm) = v(1);
    *(n.wym ? L4 + c : L2 + rm + x) = static_cast<A>(nu[2]);
    *(n.wxp ? L1 + c : L3 + r0 + n.xp) = v(3);
    *(n.wyp ? L2 + c : L4 + rp + x) = static_cast<A>(nu[4]);
    *((n.wxm || n.wym) ? L7 + c : L5 + rm + n.xm) = v(5);
    *((n.wxp || n.wym) ? L8 + c : L6 + rm + n.xp) = v(6);
    *((n.wxp || n.wyp) ? L5 + c : L7 + rp + n.xp) = v(7);
    *((n.wxm || n.wyp) ? L6 + c : L8 + rp + n.xm) = v(8);
}

// Storage type of the adjoints between reverse steps: FP64 for FP64 storage, FP32
// for FP32 and FP16 storage (the reverse step computes in FP64 either way).
template <typename S>
using AdjT = std::conditional_t<std::is_same_v<S, double>, double, float>;

// The objective's seed over one tile of TX x TY nodes: J = sum over x = Lx-1 of
// eps rho u_x of the stored state N in fin (tile partials in part) and the adjoint
// of that state from it into lam, with the state's porosity sensitivities added to
// the FP64 accumulators eb, gxb, gyb [Ly][pitch].  R is the compute type of the
// reverse pass (FP64 for every storage: the states of FP32 / FP16 storage are
// decoded into FP64, and eps is an FP64 copy of the forward's porosity).  It runs
// once per gradient; the reverse steps are the row-walking waves below.
template <typename S, typename R>
__device__ __forceinline__ void adjoint_seed_tile(const S *__restrict__ fin,
                                                  AdjT<S> *__restrict__ lam,
                                                  const R *__restrict__ eps, const Geo &g,
                                                  const Phys<R> &ph, double *__restrict__ eb,
                                                  double *__restrict__ gxb,
                                                  double *__restrict__ gyb,
                                                  double *__restrict__ part, int t)
{
    constexpr int W = TX + 2;
    __shared__ R tile[TY + 2][W];
    const int bx = t % g.nbx, by = t / g.nbx;
    const int x0 = bx * TX, y0 = by * TY;
    double acc[NRED];
#pragma unroll
    for (int k = 0; k < NRED; k++) acc[k] = 0.0;
    const gptr<double> ebg = to_global(eb), gxg = to_global(gxb), gyg = to_global(gyb);
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int x = x0 + tx;
    // The porosity tile's loads go first, then every node's own loads (its gather and
    // its accumulators), and only then the tile to LDS and the barrier: memory
    // counters retire in order, so waiting for the tile does not wait for the node's
    // loads, whose latency runs under the tile's.
    EpsTile<R, W> et;
    et.issue(eps, g, x0, y0);
    bool ok[ROWS];
    Nbr nb[ROWS];
    R d[ROWS][9];
    double ae[ROWS], ax[ROWS], ay[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; r++) {
        const int y = y0 + ty + NW * r;
        ok[r] = x < g.Lx && y < g.Ly;
        if (!ok[r]) continue;
        nb[r] = neighbours(x, y, g);
        gather<S, R>(d[r], fin, g.plane, g.pitch, x, y, nb[r], ph.inv_scale);
        const int c = y * g.pitch + x;
        ae[r] = ebg[c];
        ax[r] = gxg[c];
        ay[r] = gyg[c];
    }
    et.commit(tile);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ROWS; r++) {
        if (!ok[r]) continue;
        const int ly = ty + NW * r;
        const int y = y0 + ly;
        const Nbr &n = nb[r];
        const int c = y * g.pitch + x;
        const PorNb<R> P = porosity_nb<R, W>(tile, ly + 1, tx + 1, n.wxm, n.wxp, n.wym, n.wyp);
        const bool ores = g.open_x && ph.reservoir;
        const bool ol = ores && x == 0, orr = ores && x == g.Lx - 1;
        boundary_inflow<R>(d[r], P.e0, ol, orr, n.wym, n.wyp, ph);
        unshift_incoming<R>(d[r], P, ph.rho0);
        R mu[9], nu[9], e_b, gx_b, gy_b;     // the seed sets mu (no later step)
        bool res[9];
        adjoint_node<R, true>(d[r], P, n, ol, orr, x == g.Lx - 1, ph, mu, nu, res, e_b, gx_b,
                              gy_b, acc);
        push_global<R, AdjT<S>>(lam, g, x, y, n, nu, res);
        ebg[c] = ae[r] + static_cast<double>(e_b);
        gxg[c] = ax[r] + static_cast<double>(gx_b);
        gyg[c] = ay[r] + static_cast<double>(gy_b);
    }
    block_partial(acc, part, t);
}

template <typename S, typename R>
__global__ __launch_bounds__(NTHREADS) void k_adjoint_seed(const S *__restrict__ fin,
                                                           AdjT<S> *__restrict__ lam,
                                                           const R *__restrict__ eps, Geo g,
                                                           Phys<R> ph, double *__restrict__ eb,
                                                           double *__restrict__ gxb,
                                                           double *__restrict__ gyb,
                                                           double *__restrict__ part)
{
    adjoint_seed_tile<S, R>(fin, lam, eps, g, ph, eb, gxb, gyb, part, blockIdx.x);
}

// One reverse step (no seed) with each wave walking K consecutive rows of a
// 64-column strip, top to bottom.  The loads of row r + 1 (its adjoints, its
// gather, its accumulators and the porosity row above it) are issued before the
// arithmetic of row r, so that a row's FP64 arithmetic runs under the memory
// latency of the next one instead of after it.  A node's porosity window is
// three rows of three columns in registers, wrapped or mirrored as in the tile,
// so waves share no LDS and wait at no barrier.  The porosity is the forward's
// own array (FP32 for FP32 / FP16 storage, widened exactly on load).  The
// arithmetic of a node is the seed's (adjoint_node) given the adjoints of its
// outgoing values.  A lane past the row end computes on
// the last column and stores nothing.
template <typename S, typename R, int K>
__device__ __forceinline__ void adjoint_rows_wave(
    const S *__restrict__ fin, const AdjT<S> *__restrict__ lam_next, AdjT<S> *__restrict__ lam,
    const AdjT<S> *__restrict__ eps, const Geo &g, const Phys<R> &ph, double *__restrict__ eb,
    double *__restrict__ gxb, double *__restrict__ gyb, int strip, int chunk)
{
    using A = AdjT<S>;
    const int xr = strip * TX + static_cast<int>(threadIdx.x % TX);
    const bool act = xr < g.Lx;
    const int x = act ? xr : g.Lx - 1;
    const int y0 = chunk * K;
    const int cm = halo_index(x - 1, g.Lx, g.wall_x), cp = halo_index(x + 1, g.Lx, g.wall_x);
    const gptr<double> ebg = to_global(eb), gxg = to_global(gxb), gyg = to_global(gyb);
    // Every load below is issued with no branch around it and keeps its raw value
    // until the row that uses it converts it: a conversion next to its load would make
    // the wave wait for the next row's loads before the current row's arithmetic.  The
    // rows of the last chunk past the lattice's end take its last row (their results
    // are not stored).
    // porosity rows y0 - 1 + k (k = 0 .. K + 1), columns x - 1 .. x + 1
    A E[K + 2][3];
    auto eps_row = [&](int k) __attribute__((always_inline)) {
        const int yy = halo_index(min(y0 - 1 + k, g.Ly), g.Ly, g.wall_y);
        const A *row = eps + static_cast<long long>(yy) * g.pitch;
        E[k][0] = load_global(row + cm);
        E[k][1] = load_global(row + x);
        E[k][2] = load_global(row + cp);
    };
    A mu[K][9];
    S q[K][9];
    double ae[K], ax[K], ay[K];
    Nbr nb[K];
    auto issue = [&](int r) __attribute__((always_inline)) {
        const int y = min(y0 + r, g.Ly - 1);
        nb[r] = neighbours(x, y, g);
        const int c = y * g.pitch + x;
        const S *p[9];
        gather_src<S>(p, fin, g.plane, g.pitch, x, y, nb[r]);
#pragma unroll
        for (int i = 0; i < 9; i++) {
            mu[r][i] = load_global(lam_next + i * g.plane + c);
            q[r][i] = load_raw(p[i]);
        }
        ae[r] = ebg[c];
        ax[r] = gxg[c];
        ay[r] = gyg[c];
    };
    auto compute = [&](int r) __attribute__((always_inline)) {
        const int y = min(y0 + r, g.Ly - 1);
        const bool row_ok = y0 + r < g.Ly;     // uniform
        const Nbr &n = nb[r];
        R d[9], m[9];
#pragma unroll
        for (int i = 0; i < 9; i++) {
            d[i] = decode_pop<S, R>(q[r][i], ph.inv_scale);
            m[i] = static_cast<R>(mu[r][i]);
        }
        const R t[3][3] = {{R(E[r][0]), R(E[r][1]), R(E[r][2])},
                           {R(E[r + 1][0]), R(E[r + 1][1]), R(E[r + 1][2])},
                           {R(E[r + 2][0]), R(E[r + 2][1]), R(E[r + 2][2])}};
        const PorNb<R> P = porosity_nb<R, 3>(t, 1, 1, n.wxm, n.wxp, n.wym, n.wyp);
        const bool ores = g.open_x && ph.reservoir;
        const bool ol = ores && x == 0, orr = ores && x == g.Lx - 1;
        boundary_inflow<R>(d, P.e0, ol, orr, n.wym, n.wyp, ph);
        unshift_incoming<R>(d, P, ph.rho0);
        R nu[9], e_b, gx_b, gy_b;
        bool res[9];
        adjoint_node<R, false>(d, P, n, ol, orr, x == g.Lx - 1, ph, m, nu, res, e_b, gx_b,
                               gy_b, nullptr);
        if (act && row_ok) {
            push_global<R, A>(lam, g, x, y, n, nu, res);
            const int c = y * g.pitch + x;
            ebg[c] = ae[r] + static_cast<double>(e_b);
            gxg[c] = ax[r] + static_cast<double>(gx_b);
            gyg[c] = ay[r] + static_cast<double>(gy_b);
        }
    };
    eps_row(0);
    eps_row(1);
    eps_row(2);
    issue(0);
    static_while<K>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        if constexpr (r + 1 < K) {
            eps_row(r + 3);
            issue(r + 1);
        }
        compute(r);
        return true;
    });
}

template <typename S, typename R, int K>
__global__ __launch_bounds__(NTHREADS) void k_adjoint_rows(
    const S *__restrict__ fin, const AdjT<S> *__restrict__ lam_next, AdjT<S> *__restrict__ lam,
    const AdjT<S> *__restrict__ eps, Geo g, Phys<R> ph, double *__restrict__ eb,
    double *__restrict__ gxb, double *__restrict__ gyb, int nstrips, int nchunks)
{
    const int wid = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * NW +
                                                   threadIdx.x / TX);
    const int strip = wid % nstrips, chunk = wid / nstrips;
    if (chunk >= nchunks) return;              // whole waves only; no barrier below
    adjoint_rows_wave<S, R, K>(fin, lam_next, lam, eps, g, ph, eb, gxb, gyb, strip, chunk);
}

// Initial state: f_i(r, 0) = w_i eps(r) rho0 (1 + 3 e_i.u0 + 9/2 (e_i.u0)^2 -
// 3/2 u0.u0); its porosity derivative, weighted by the adjoint of the slot the
// first gather pulls it from.
template <typename R>
__global__ __launch_bounds__(NTHREADS) void k_adjoint_init(const R *__restrict__ lam, Geo g,
                                                           double rho0, double u0x, double u0y,
                                                           double wb6, double wt6,
                                                           double *__restrict__ eb)
{
    const int t = blockIdx.x;
    const int bx = t % g.nbx, by = t / g.nbx;
    const int x = bx * TX + threadIdx.x % TX;
    for (int r = 0; r < ROWS; r++) {
        const int y = by * TY + threadIdx.x / TX + NW * r;
        if (x >= g.Lx || y >= g.Ly) continue;
        const Nbr n = neighbours(x, y, g);
        const long long pl = g.plane;
        const int c = y * g.pitch + x, rm = n.ym * g.pitch, r0 = y * g.pitch, rp = n.yp * g.pitch;
        const long long src[9] = {
            c,
            n.wxm ? 3 * pl + c : 1 * pl + r0 + n.xm,
            n.wym ? 4 * pl + c : 2 * pl + rm + x,
            n.wxp ? 1 * pl + c : 3 * pl + r0 + n.xp,
            n.wyp ? 2 * pl + c : 4 * pl + rp + x,
            (n.wxm || n.wym) ? 7 * pl + c : 5 * pl + rm + n.xm,
            (n.wxp || n.wym) ? 8 * pl + c : 6 * pl + rm + n.xp,
            (n.wxp || n.wyp) ? 5 * pl + c : 7 * pl + rp + n.xp,
            (n.wxm || n.wyp) ? 6 * pl + c : 8 * pl + rp + n.xm,
        };
        const double uu = u0x * u0x + u0y * u0y;
        double s = 0.0;
        for (int i = 0; i < 9; i++) {
            const double eu = CX[i] * u0x + CY[i] * u0y;
            s += static_cast<double>(lam[src[i]]) * wgt(i) * rho0 *
                 (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
        }
        // the initial slots behind a sliding wall are stored without the gain the
        // first gather adds (the initial state is the equilibrium): its porosity
        // term, which the reverse step of that gather counted, cancels here
        if (n.wym)
            s -= (static_cast<double>(lam[src[5]]) - static_cast<double>(lam[src[6]])) * wb6;
        if (n.wyp)
            s -= (static_cast<double>(lam[src[8]]) - static_cast<double>(lam[src[7]])) * wt6;
        eb[c] += s;
    }
}

// Nodes x0 along one axis whose halo neighbour x0 + e (wrapped, or mirrored
// behind a non-periodic end) is v: at most two.
__device__ __forceinline__ int halo_sources(int v, int e, int L, int wall, int out[2])
{
    int n = 0;
    if (!wall) {
        int s = v - e;
        if (s < 0) s += L;
        else if (s >= L) s -= L;
        out[n++] = s;
        return n;
    }
    const int s = v - e;
    if (s >= 0 && s < L) out[n++] = s;
    if (e == -1 && v == 0) out[n++] = 0;
    if (e == 1 && v == L - 1) out[n++] = L - 1;
    return n;
}

// dJ/deps(v) = direct adjoint + grad(eps) adjoint through the transposed
// stencil grad(eps)(x) = sum_i 3 w_i e_i eps(halo(x + e_i)), in gather form
// (deterministic).  out is [Ly][Lx].
__global__ __launch_bounds__(NTHREADS) void k_adjoint_finish(const double *__restrict__ eb,
                                                             const double *__restrict__ gxb,
                                                             const double *__restrict__ gyb,
                                                             Geo g, double *__restrict__ out)
{
    const int t = blockIdx.x;
    const int bx = t % g.nbx, by = t / g.nbx;
    const int x = bx * TX + threadIdx.x % TX;
    for (int r = 0; r < ROWS; r++) {
        const int y = by * TY + threadIdx.x / TX + NW * r;
        if (x >= g.Lx || y >= g.Ly) continue;
        double s = eb[y * g.pitch + x];
        for (int i = 1; i < 9; i++) {
            int sx[2], sy[2];
            const int nx = halo_sources(x, CX[i], g.Lx, g.wall_x, sx);
            const int ny = halo_sources(y, CY[i], g.Ly, g.wall_y, sy);
            const double c = 3.0 * wgt(i);
            for (int a = 0; a < nx; a++)
                for (int b = 0; b < ny; b++) {
                    const int k = sy[b] * g.pitch + sx[a];
                    s += c * (CX[i] * gxb[k] + CY[i] * gyb[k]);
                }
        }
        out[(long long)y * g.Lx + x] = s;
    }
}

// FP64 copy of an FP32 array of n elements.
__global__ __launch_bounds__(NTHREADS) void k_widen(const float *__restrict__ src,
                                                    double *__restrict__ dst, long long n)
{
    const long long i = static_cast<long long>(blockIdx.x) * NTHREADS + threadIdx.x;
    if (i < n) dst[i] = static_cast<double>(src[i]);
}

// Fill with zero (used for the FP64 accumulators; a kernel rather than a
// memset so the grad sequence stays capturable).
__global__ __launch_bounds__(NTHREADS) void k_zero(double *__restrict__ p, long long n)
{
    const long long i = static_cast<long long>(blockIdx.x) * NTHREADS + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// ---------------------------------------------------------------------------
// Ensembles: many independent problems in one launch
// ---------------------------------------------------------------------------
// The tiles of all members are numbered into one list (member by member, each
// in its own row-major tile order).  A device table maps a list position to
// its member, whose descriptor gives the geometry, physics and buffers.  The
// members share the storage type and the boundary kinds (one kernel template);
// everything else (size, tau, drag, forcing, reservoirs) is per member.

template <typename R>
struct Member {
    Geo gs;                 // tiling of the batched sweep (vec nodes per lane)
    Geo g;                  // one node per lane (adjoint)
    Phys<R> ph;
    Phys<double> pha;       // the FP64 reverse step's constants (shift reference as ph's)
    const double *eps_a;    // FP64 porosity of the reverse step (padded; the gradient
                            // workspace's copy for FP32 / FP16 storage)
    char *buf[2];           // the member's two population buffers (state slots 0, 1)
    const R *eps;           // padded porosity
    double *part;           // tile partials [g.ntiles][NRED]
    char *gw;               // gradient workspace: state slots 2.., adjoints, accumulators
    long long gpop, glam, gacc;
    int nslot;              // state slots in gw (checkpoints + recomputed segment)
    int vec;                // nodes per lane of this member's sweep
    int tile0;              // first position in the sweep tile list of its width
    int tile0_adj;          // first position in the adjoint tile list
    int tb_strips[3];       // strips of the two-, three- and four-step passes
    int tw0[4];             // first position in the wave lists of the two-step pass, of
                            // the three-step pass in short and in tall chunks, and of
                            // the four-step pass
};

template <typename R>
__device__ __forceinline__ char *state_slot(const Member<R> &d, int slot)
{
    return slot < 2 ? d.buf[slot] : d.gw + (long long)(slot - 2) * d.gpop;
}

template <typename A, typename R>
__device__ __forceinline__ A *adj_buf(const Member<R> &d, int a)
{
    return reinterpret_cast<A *>(d.gw + (long long)d.nslot * d.gpop + a * d.glam);
}

template <typename R>
__device__ __forceinline__ double *acc_buf(const Member<R> &d, int k)
{
    return reinterpret_cast<double *>(d.gw + (long long)d.nslot * d.gpop + 2 * d.glam +
                                      k * d.gacc);
}

// Positions of the tile list this block takes: one position when the grid
// covers the list (XCD-banded as in the single sweep), else a persistent walk
// in which the blocks of each XCD share that XCD's band of the list.
struct TileWalk {
    int first, end, stride;
};

__device__ __forceinline__ TileWalk tile_walk(int ntiles)
{
    TileWalk w;
    if ((int)gridDim.x >= ntiles) {
        w.first = xcd_tile(blockIdx.x, ntiles);
        w.end = w.first + 1;
        w.stride = 1;
        return w;
    }
    const int per = gridDim.x / NXCD;
    const int xcd = blockIdx.x % NXCD, k = blockIdx.x / NXCD;
    const int q = ntiles / NXCD, r = ntiles % NXCD;
    const int start = xcd * q + min(xcd, r);
    w.first = start + k;
    w.end = start + q + (xcd < r ? 1 : 0);
    w.stride = per;
    return w;
}

// One time step of every member, from state slot src to state slot dst, with
// V nodes per lane (ragged runs where a member's Lx is not a multiple of V).
template <typename S, typename R, int V, int BX, bool WY>
__global__ __launch_bounds__(NTHREADS) void k_batch_sweep(const Member<R> *__restrict__ M,
                                                          const int *__restrict__ tmap,
                                                          int ntiles, int src, int dst,
                                                          int reservoir)
{
    const TileWalk w = tile_walk(ntiles);
    for (int T = w.first; T < w.end; T += w.stride) {
        const Member<R> &d = M[tmap[T]];
        const Geo gs = d.gs;
        Phys<R> ph = d.ph;
        ph.reservoir = reservoir;
        sweep_vec_tile<S, R, V, BX, WY, false, true>(
            reinterpret_cast<const S *>(state_slot(d, src)),
            reinterpret_cast<S *>(state_slot(d, dst)), d.eps, gs, ph, nullptr, T - d.tile0);
        __syncthreads();  // a next tile of this block reuses the LDS porosity tile
    }
}

// NS steps of every member in one pass (the multi-step pass, one wave per
// strip and chunk of NR rows of a member, wave list Q), from state slot src to
// state slot dst.
template <typename S, typename R, int BX, bool WY, int NS, int NR, int Q>
__device__ __forceinline__ void batch_multi_wave(const Member<R> *__restrict__ M,
                                                 const int *__restrict__ wmap, int nwaves,
                                                 int src, int dst, int res_a)
{
    const int wid = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * NW +
                                                   threadIdx.x / TX);
    if (wid >= nwaves) return;                 // whole waves only; no barrier below
    const Member<R> &d = M[wmap[wid]];
    const Geo g = d.g;
    Phys<R> ph = d.ph;
    ph.reservoir = 1;
    const int local = wid - d.tw0[Q], ns = d.tb_strips[NS - 2];
    tb_wave_x<S, R, BX, WY, NS, NR, true>(reinterpret_cast<const S *>(state_slot(d, src)),
                                    reinterpret_cast<S *>(state_slot(d, dst)), d.eps, g, ph,
                                    local % ns, local / ns, res_a);
}

template <typename S, typename R, int BX, bool WY>
__global__ __launch_bounds__(NTHREADS) void k_batch_tb2(const Member<R> *__restrict__ M,
                                                        const int *__restrict__ wmap,
                                                        int nwaves, int src, int dst, int res_a)
{
    batch_multi_wave<S, R, BX, WY, 2, tb_rows<S, 2>(), 0>(M, wmap, nwaves, src, dst, res_a);
}

// Three steps of every member: chunks of NR rows (wave list 1: the short
// height, 2: the tall one).
template <typename S, typename R, int BX, bool WY, int NR>
__global__ __launch_bounds__(NTHREADS)
__attribute__((amdgpu_waves_per_eu(1, tb3_max_waves<S, BX, WY>()))) void k_batch_tb3(
    const Member<R> *__restrict__ M, const int *__restrict__ wmap, int nwaves, int src, int dst,
    int res_a)
{
    batch_multi_wave<S, R, BX, WY, 3, NR, NR == tb_rows<S, 3>() ? 1 : 2>(M, wmap, nwaves, src,
                                                                         dst, res_a);
}

// Four steps of every member (FP32 storage; wave list 3).
template <typename S, typename R, int BX, bool WY>
__global__ __launch_bounds__(NTHREADS)
__attribute__((amdgpu_waves_per_eu(1, tb3_max_waves<S, BX, WY>()))) void k_batch_tb4(
    const Member<R> *__restrict__ M, const int *__restrict__ wmap, int nwaves, int src, int dst,
    int res_a)
{
    batch_multi_wave<S, R, BX, WY, 4, tb_rows<float, 4>(), 3>(M, wmap, nwaves, src, dst, res_a);
}

// The seed of every member: the adjoint (slot a) of the state in state slot src
// from each member's objective (FP64 for every storage, as lbm_vans_grad).
template <typename S, typename R>
__global__ __launch_bounds__(NTHREADS) void k_batch_adjoint_seed(
    const Member<R> *__restrict__ M, const int *__restrict__ tmap, int ntiles, int src, int a,
    int reservoir)
{
    const int T = xcd_tile(blockIdx.x, ntiles);
    const Member<R> &d = M[tmap[T]];
    const Geo g = d.g;
    Phys<double> ph = d.pha;
    ph.reservoir = reservoir;
    adjoint_seed_tile<S, double>(reinterpret_cast<const S *>(state_slot(d, src)),
                                 adj_buf<AdjT<S>>(d, a), d.eps_a, g, ph, acc_buf(d, 0),
                                 acc_buf(d, 1), acc_buf(d, 2), d.part, T - d.tile0_adj);
}

// One reverse step (no seed) of every member, one wave per entry of the adjoint
// tile list: a tile of TX columns and TY rows is the strip and chunk one wave of
// the row-walking reverse step takes.
template <typename S, typename R>
__global__ __launch_bounds__(NTHREADS) void k_batch_adjoint_rows(const Member<R> *__restrict__ M,
                                                                 const int *__restrict__ tmap,
                                                                 int ntiles, int src,
                                                                 int a_next, int a,
                                                                 int reservoir)
{
    const int wid = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * NW +
                                                   threadIdx.x / TX);
    if (wid >= ntiles) return;                 // whole waves only; no barrier below
    const Member<R> &d = M[tmap[wid]];
    const Geo g = d.g;
    Phys<double> ph = d.pha;
    ph.reservoir = reservoir;
    const int t = wid - d.tile0_adj;
    adjoint_rows_wave<S, double, TY>(reinterpret_cast<const S *>(state_slot(d, src)),
                                     adj_buf<AdjT<S>>(d, a_next), adj_buf<AdjT<S>>(d, a),
                                     reinterpret_cast<const AdjT<S> *>(d.eps), g, ph,
                                     acc_buf(d, 0), acc_buf(d, 1), acc_buf(d, 2), t % g.nbx,
                                     t / g.nbx);
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

struct lbm_vans_handle {
    lbm_vans_params p;
    hipStream_t stream;
    Geo g;                  // one node per thread: moments, state copies, adjoint
    Geo gs;                 // geometry of the sweep actually launched (vec nodes per lane)
    int vec;                // nodes per lane of the sweep
    int ntiles;
    size_t pop_bytes;       // bytes of one population buffer
    char *buf[2];           // population buffers; buf[cur] holds the current state
    int cur;
    void *eps;              // padded porosity (double or float)
    double *part;           // tile partials [ntiles][NRED]
    double *mass0;          // rho0 * sum eps
    double *scratch_rec;    // one diagnostics record
    double *ring;           // [LBM_VANS_DIAG_RING][NRED]
    int64_t n;              // steps taken
    int64_t nrec;           // diagnostics records written
    int rows3;              // rows per chunk of the three-step pass
    int auto_pass;          // automatic most steps per pass
    void *scratch;          // device address of the library-held gradient workspace on the
                            // handle's device (lbm_vans_grad_static)
    // Step graphs of small lattices (launch-bound: fewer sweep tiles than twice the
    // compute units): lbm_vans_step replays GRAPH_STEPS steps from state slot 0 / 1
    // as one captured graph, captured on first use on a private stream.
    bool use_graphs;
    hipStream_t cap;
    hipGraphExec_t graph[2];
    // The gradient recomputes segment c - 1 on a second stream while the handle's
    // stream runs the reverse steps of segment c: events hand the checkpoints over
    // (ev_start), a recomputed segment set over (ev_rec[set]) and a set back once its
    // reverse steps have read it (ev_rev[set]).
    hipStream_t stream2;
    hipEvent_t ev_start, ev_rec[2], ev_rev[2];
};

namespace {

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

int elem_bytes(int storage)
{
    return storage == LBM_F64 ? 8 : (storage == LBM_F32_SHIFTED ? 4 : 2);
}

// Row pitch in nodes (Lx rounded up to PITCH_ALIGN) and plane stride.  (An
// odd multiple of PITCH_ALIGN for power-of-two widths, and a pad between the
// planes, were measured: no gain for the two-step pass, and the one-step
// sweep at 4096^2 FP32 fell from 82 to 65 GLUPS with the odd pitch.)
long long geo_pitch(int Lx) { return (Lx + PITCH_ALIGN - 1LL) / PITCH_ALIGN * PITCH_ALIGN; }

long long geo_plane(int Lx, int Ly) { return geo_pitch(Lx) * Ly; }

// Chunk rows of the three-step pass a caller may ask for: 0 (automatic), the
// short, default or tall height with FP32 storage, the one height with FP16 storage.
int check_pass_rows(int32_t rows, int32_t storage)
{
    if (rows == 0) return LBM_VANS_OK;
    if (storage == LBM_F32_SHIFTED &&
        (rows == LBM_VANS_TB3_TINY32 || rows == LBM_VANS_TB3_SHORT32 ||
         rows == tb_rows<float, 3>() || rows == LBM_VANS_TB3_TALL32))
        return LBM_VANS_OK;
    if (storage == LBM_F16_SHIFTED && rows == tb_rows<_Float16, 3>()) return LBM_VANS_OK;
    return fail(LBM_VANS_EINVAL,
                "pass_rows = %d: 0 (automatic); %d, %d, %d or %d with LBM_F32_SHIFTED storage; "
                "%d with LBM_F16_SHIFTED storage",
                rows, LBM_VANS_TB3_TINY32, LBM_VANS_TB3_SHORT32, tb_rows<float, 3>(),
                LBM_VANS_TB3_TALL32, tb_rows<_Float16, 3>());
}

int check_params(const lbm_vans_params *p)
{
    if (!p) return fail(LBM_VANS_EINVAL, "params is NULL");
    if (p->Lx < 1 || p->Ly < 1)
        return fail(LBM_VANS_EINVAL, "lattice size %d x %d must be at least 1 x 1", p->Lx, p->Ly);
    if (geo_plane(p->Lx, p->Ly) >= (1LL << 31))
        return fail(LBM_VANS_EINVAL, "lattice %d x %d too large (padded nodes must be < 2^31)",
                    p->Lx, p->Ly);
    if ((p->bc_x != LBM_BC_PERIODIC && p->bc_x != LBM_BC_BOUNCEBACK && p->bc_x != LBM_BC_OPEN &&
         p->bc_x != LBM_BC_INOUT) ||
        (p->bc_y != LBM_BC_PERIODIC && p->bc_y != LBM_BC_BOUNCEBACK))
        return fail(LBM_VANS_EINVAL, "boundary kinds (%d, %d) not supported", p->bc_x, p->bc_y);
    if (p->bc_x == LBM_BC_OPEN) {
        if (p->Lx < 2) return fail(LBM_VANS_EINVAL, "open x ends need Lx >= 2");
        if (!(p->rho_in > 0.0) || !std::isfinite(p->rho_in) || !(p->rho_out > 0.0) ||
            !std::isfinite(p->rho_out) || !std::isfinite(p->u_in) || !std::isfinite(p->u_out))
            return fail(LBM_VANS_EINVAL, "reservoir densities must be finite and > 0, velocities finite");
    }
    if (p->bc_x == LBM_BC_INOUT) {
        if (p->Lx < 2) return fail(LBM_VANS_EINVAL, "open x ends need Lx >= 2");
        if (!(p->rho_out > 0.0) || !std::isfinite(p->rho_out) || !std::isfinite(p->u_in))
            return fail(LBM_VANS_EINVAL, "outlet density must be finite and > 0, inlet velocity finite");
    }
    if (p->storage != LBM_F64 && p->storage != LBM_F32_SHIFTED && p->storage != LBM_F16_SHIFTED)
        return fail(LBM_VANS_EINVAL, "unknown storage %d", p->storage);
    if (!(p->tau > 0.5) || !std::isfinite(p->tau))
        return fail(LBM_VANS_EINVAL, "tau = %g must be finite and > 1/2", p->tau);
    if (p->drag == LBM_DRAG_ERGUN) {
        if (!(p->d_p > 0.0)) return fail(LBM_VANS_EINVAL, "d_p = %g must be > 0", p->d_p);
    } else if (p->drag == LBM_DRAG_CONST) {
        if (!(p->K > 0.0)) return fail(LBM_VANS_EINVAL, "K = %g must be > 0", p->K);
        if (!(p->F_eps >= 0.0) || !std::isfinite(p->F_eps))
            return fail(LBM_VANS_EINVAL, "F_eps = %g must be finite and >= 0", p->F_eps);
    } else {
        return fail(LBM_VANS_EINVAL, "unknown drag law %d", p->drag);
    }
    if (!std::isfinite(p->G[0]) || !std::isfinite(p->G[1]))
        return fail(LBM_VANS_EINVAL, "body force must be finite");
    if (!(p->rho0 > 0.0) || !std::isfinite(p->rho0))
        return fail(LBM_VANS_EINVAL, "rho0 = %g must be finite and > 0", p->rho0);
    if (!std::isfinite(p->u0[0]) || !std::isfinite(p->u0[1]))
        return fail(LBM_VANS_EINVAL, "u0 must be finite");
    if (p->storage == LBM_F16_SHIFTED && (p->fp16_scale_log2 < 0 || p->fp16_scale_log2 > 24))
        return fail(LBM_VANS_EINVAL, "fp16_scale_log2 = %d outside 0..24", p->fp16_scale_log2);
    if (p->diag_every < 0) return fail(LBM_VANS_EINVAL, "diag_every = %d < 0", p->diag_every);
    if (!std::isfinite(p->u_wall[0]) || !std::isfinite(p->u_wall[1]))
        return fail(LBM_VANS_EINVAL, "u_wall must be finite");
    if (p->bc_y != LBM_BC_BOUNCEBACK && (p->u_wall[0] != 0.0 || p->u_wall[1] != 0.0))
        return fail(LBM_VANS_EINVAL, "u_wall needs bounce-back walls in y (bc_y)");
    const int vmax = p->storage == LBM_F64 ? 2 : 4;
    if (p->sweep_vec != 0 && p->sweep_vec != 1 && p->sweep_vec != vmax)
        return fail(LBM_VANS_EINVAL, "sweep_vec = %d: 0 (automatic), 1 or %d", p->sweep_vec,
                    vmax);
    if (p->steps_per_pass < 0 || p->steps_per_pass > 4)
        return fail(LBM_VANS_EINVAL, "steps_per_pass = %d: 0 (automatic), 1, 2, 3 or 4",
                    p->steps_per_pass);
    if (p->steps_per_pass == 4 && p->storage != LBM_F32_SHIFTED)
        return fail(LBM_VANS_EINVAL, "steps_per_pass = 4 needs LBM_F32_SHIFTED storage");
    if (check_pass_rows(p->pass_rows, p->storage)) return LBM_VANS_EINVAL;
    return LBM_VANS_OK;
}


// Rows per thread of the vector sweep for a storage code (see sweep_rows).
int sweep_rows_of(int storage) { return storage == LBM_F16_SHIFTED ? 2 : 1; }

// Tiling for `vec` nodes per lane and `rows` rows per thread; the pitch is
// shared by all tilings.
Geo make_geo(const lbm_vans_params *p, int vec = 1, int rows = ROWS)
{
    Geo g;
    g.Lx = p->Lx;
    g.Ly = p->Ly;
    g.pitch = static_cast<int>(geo_pitch(p->Lx));
    g.wall_x = p->bc_x != LBM_BC_PERIODIC;
    g.wall_y = p->bc_y == LBM_BC_BOUNCEBACK;
    g.open_x = p->bc_x == LBM_BC_OPEN || p->bc_x == LBM_BC_INOUT;
    g.nbx = (p->Lx + TX * vec - 1) / (TX * vec);
    int nby = (p->Ly + NW * rows - 1) / (NW * rows);
    g.ntiles = g.nbx * nby;
    g.plane = geo_plane(p->Lx, p->Ly);
    return g;
}

// Widest vector width of the one-step sweep: 16-byte accesses per lane (4
// FP32, 2 FP64) and 8-byte ones for FP16 (ragged runs when Lx is not a
// multiple of it).
int sweep_vmax(int storage) { return storage == LBM_F64 ? 2 : 4; }

// Nodes per lane of the one-step sweep: as requested; automatically the widest,
// unless its tiles would leave compute units without a workgroup (fewer tiles
// than units), then one node per lane (four (FP64: two) times the tiles).
// Measured, FP32 open channel, microseconds per step at 4 / 1 nodes per lane:
// 512 x 256 (128 / 512 tiles) 6.16 / 4.49; 1024 x 512 (512 / 2048 tiles) 9.15 /
// 10.38.
int sweep_vec(const lbm_vans_params *p, int ncu)
{
    if (p->sweep_vec != 0) return p->sweep_vec;
    const int vmax = sweep_vmax(p->storage);
    return make_geo(p, vmax, sweep_rows_of(p->storage)).ntiles < ncu ? 1 : vmax;
}

struct Layout {
    size_t pop, eps, part, small, total;
};

Layout make_layout(const lbm_vans_params *p)
{
    Geo g = make_geo(p);
    Layout L;
    L.pop = align256((size_t)9 * g.plane * elem_bytes(p->storage));
    L.eps = align256((size_t)g.plane * (p->storage == LBM_F64 ? 8 : 4));
    L.part = align256((size_t)g.ntiles * NRED * sizeof(double));
    L.small = align256((size_t)(2 + NRED + (size_t)LBM_VANS_DIAG_RING * NRED) * sizeof(double));
    L.total = 2 * L.pop + L.eps + L.part + L.small;
    return L;
}

template <typename R>
Phys<R> make_phys(const lbm_vans_params *p)
{
    Phys<R> ph;
    double nu = (p->tau - 0.5) / 3.0;
    ph.omega = static_cast<R>(1.0 / p->tau);
    ph.pre = static_cast<R>(1.0 - 0.5 / p->tau);
    ph.rho0 = static_cast<R>(p->rho0);
    ph.Gx = static_cast<R>(p->G[0]);
    ph.Gy = static_cast<R>(p->G[1]);
    ph.ca = ph.cb = ph.ka = ph.kb = R(0);
    if (p->drag == LBM_DRAG_ERGUN) {
        bool none = std::isinf(p->d_p);
        ph.ca = none ? R(0) : static_cast<R>(150.0 * nu / (p->d_p * p->d_p));
        ph.cb = none ? R(0) : static_cast<R>(1.75 / p->d_p);
    } else {
        bool none = std::isinf(p->K);
        ph.ka = none ? R(0) : static_cast<R>(nu / p->K);
        ph.kb = none ? R(0) : static_cast<R>(p->F_eps / std::sqrt(p->K));
    }
    double s = p->storage == LBM_F16_SHIFTED ? std::ldexp(1.0, p->fp16_scale_log2) : 1.0;
    ph.scale = static_cast<R>(s);
    ph.inv_scale = static_cast<R>(1.0 / s);
    // reservoir deviations per unit porosity: w_i (rho_b (1 + 3 e.u + 9/2 (e.u)^2
    // - 3/2 u.u) - rho0) with u = (u_b, 0), for the directions entering the domain
    static const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static const double wt[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    const double rho_ref = static_cast<double>(ph.rho0);
    for (int i = 0; i < 9; i++) {
        double eui = cx[i] * p->u_in, euo = cx[i] * p->u_out;
        double pin = 1.0 + 3.0 * eui + 4.5 * eui * eui - 1.5 * p->u_in * p->u_in;
        double pout = 1.0 + 3.0 * euo + 4.5 * euo * euo - 1.5 * p->u_out * p->u_out;
        ph.rin[i] = cx[i] > 0 ? static_cast<R>(wt[i] * (p->rho_in * pin - rho_ref)) : R(0);
        ph.rout[i] = cx[i] < 0 ? static_cast<R>(wt[i] * (p->rho_out * pout - rho_ref)) : R(0);
    }
    ph.reservoir = 0;
    ph.inout = p->bc_x == LBM_BC_INOUT;
    ph.dro = R(0);
    ph.rho_out = R(0);
    if (ph.inout) {
        for (int i = 0; i < 9; i++) {
            const double eu = cx[i] * p->u_in;
            const double q = 3.0 * eu + 4.5 * eu * eu - 1.5 * p->u_in * p->u_in;
            ph.rin[i] = cx[i] > 0 ? static_cast<R>(wt[i] * q) : R(0);
            ph.rout[i] = R(0);
        }
        ph.dro = static_cast<R>(p->rho_out - rho_ref);
        ph.rho_out = static_cast<R>(p->rho_out);
    }
    ph.wb = static_cast<R>(p->rho0 * p->u_wall[0] / 6.0);
    ph.wt = static_cast<R>(p->rho0 * p->u_wall[1] / 6.0);
    return ph;
}

// LBM_VANS_WMACH (with a message) when the largest speed of a state leaves the
// low-Mach range of the lattice BGK model, max |u| / c_s > LBM_VANS_MACH_WARN.
int mach_check(double umax, double step)
{
    const double ma = umax * std::sqrt(3.0);
    if (ma > LBM_VANS_MACH_WARN) {
        fail(LBM_VANS_WMACH, "Mach number %.3f > %.2f at step %.0f (max |u| = %.4g)", ma,
             LBM_VANS_MACH_WARN, step, umax);
        return LBM_VANS_WMACH;
    }
    return LBM_VANS_OK;
}

// Whether the open-end rules apply to a step from state n: the fixed reservoirs
// from n = 1 on (the initial state is the equilibrium everywhere), the velocity
// inlet / pressure outlet from the start (its reservoirs live in the stored
// slots, which the initial state fills).
int res_on(const lbm_vans_params *p, int64_t n) { return n >= 1 || p->bc_x == LBM_BC_INOUT; }

// rho0 u_w / 6 of the sliding y-walls in FP64 (init, set_state, adjoint init).
double wall6(const lbm_vans_params *p, int top) { return p->rho0 * p->u_wall[top] / 6.0; }

int check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(LBM_VANS_EHIP, "launch of %s failed: %s", what, hipGetErrorString(e));
    return LBM_VANS_OK;
}

// Dispatch on the storage type: f(S, R) with S the stored and R the compute type.
template <typename Fn>
int with_types(int storage, Fn &&fn)
{
    switch (storage) {
    case LBM_F64: return fn((double *)nullptr, (double *)nullptr);
    case LBM_F32_SHIFTED: return fn((float *)nullptr, (float *)nullptr);
    default: return fn((_Float16 *)nullptr, (float *)nullptr);
    }
}

template <typename S, typename R, bool DIAG, bool RG, int V>
void launch_sweep_rg(lbm_vans_handle *h, const S *src, S *dst, const Phys<R> &ph,
                     hipStream_t st)
{
    const dim3 grid(h->gs.ntiles), block(NTHREADS);
    const R *eps = (const R *)h->eps;
    const int bx = h->gs.open_x ? 2 : (h->gs.wall_x ? 1 : 0);
    const bool wy = h->gs.wall_y;
#define LBM_VANS_VEC(BXV, WYV)                                                                  \
    hipLaunchKernelGGL((k_sweep_vec<S, R, V, BXV, WYV, DIAG, RG>), grid, block, 0, st,           \
                       src, dst, eps, h->gs, ph, h->part)
    if (bx == 0 && !wy) LBM_VANS_VEC(0, false);
    else if (bx == 0) LBM_VANS_VEC(0, true);
    else if (bx == 1 && !wy) LBM_VANS_VEC(1, false);
    else if (bx == 1) LBM_VANS_VEC(1, true);
    else if (!wy) LBM_VANS_VEC(2, false);
    else LBM_VANS_VEC(2, true);
#undef LBM_VANS_VEC
}

template <typename S, typename R, bool DIAG>
void launch_sweep_t(lbm_vans_handle *h, const S *src, S *dst, const Phys<R> &ph,
                    hipStream_t st)
{
    constexpr int VMAX = sizeof(S) == 8 ? 2 : 4;
    if (h->vec == 1) launch_sweep_rg<S, R, DIAG, false, 1>(h, src, dst, ph, st);
    else if (h->p.Lx % VMAX) launch_sweep_rg<S, R, DIAG, true, VMAX>(h, src, dst, ph, st);
    else launch_sweep_rg<S, R, DIAG, false, VMAX>(h, src, dst, ph, st);
}

// The multi-step passes address a plane (state or porosity, at most 4 bytes a
// node) with byte offsets below 2^31 (their stores mark a dropped store with
// 2^31) and rows with 24-bit products.
bool multi_fits(const Geo &g)
{
    return static_cast<unsigned long long>(g.pitch) * 4 < (1ull << 24) && g.Ly < (1 << 24) &&
           static_cast<unsigned long long>(g.plane) * 4 < (1ull << 31);
}

// Whether an ns-step pass (2 or 3) in chunks of `rows` may run a lattice of Ly rows:
// with periodic y the pass wraps each window row once, which needs Ly >= rows +
// 2 (ns - 1) + 2 (the chunk, its halo rows and their porosity neighbours); with
// walls in y it clamps.
bool multi_rows_ok(int Ly, bool wall_y, int ns, int rows)
{
    return wall_y || Ly >= rows + 2 * (ns - 1) + 2;
}

// Rows per chunk of the two-step pass for a storage code.
int tb2_rows_of(int storage)
{
    return storage == LBM_F16_SHIFTED ? tb_rows<_Float16, 2>() : tb_rows<float, 2>();
}

// Waves of the ns-step pass (2 or 3) over an Lx x Ly lattice in chunks of `rows`.
long long waves_of(int Lx, int Ly, int ns, int rows)
{
    const int cols = TX - 2 * (ns - 1);
    return static_cast<long long>((Lx + cols - 1) / cols) * ((Ly + rows - 1) / rows);
}

// f(integral_constant<int, BX>, integral_constant<bool, WY>) for the x ends (0
// periodic, 1 walls, 2 open) and the y walls of a lattice.
template <typename F>
void with_bxwy(int bx, bool wy, F &&f)
{
    using F0 = std::false_type;
    using T1 = std::true_type;
    using B0 = std::integral_constant<int, 0>;
    using B1 = std::integral_constant<int, 1>;
    using B2 = std::integral_constant<int, 2>;
    if (bx == 0 && !wy) f(B0{}, F0{});
    else if (bx == 0) f(B0{}, T1{});
    else if (bx == 1 && !wy) f(B1{}, F0{});
    else if (bx == 1) f(B1{}, T1{});
    else if (!wy) f(B2{}, F0{});
    else f(B2{}, T1{});
}

// Waves of the three-step kernel (lone, or batched) in chunks of `rows` that the
// chip holds at once: its workgroups per compute unit (registers decide: the
// periodic FP32 kernel holds two waves per SIMD, the kernels with walls four)
// times the waves per workgroup and the compute units.
int tb3_resident(int storage, int bx, bool wy, int rows, bool batch, long long *out)
{
    int nb = 0, dev = 0, ncu = 0;
    hipError_t e = hipSuccess;
    auto q = [&](auto ker) { e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ker, NTHREADS, 0); };
    with_bxwy(bx, wy, [&](auto bxc, auto wyc) {
        constexpr int BXV = decltype(bxc)::value;
        constexpr bool WYV = decltype(wyc)::value;
        if (storage == LBM_F16_SHIFTED) {
            constexpr int NR = tb_rows<_Float16, 3>();
            if (batch) q(k_batch_tb3<_Float16, float, BXV, WYV, NR>);
            else q(k_sweep_tb3<_Float16, float, BXV, WYV, NR>);
        } else if (rows == LBM_VANS_TB3_TALL32) {
            constexpr int NR = LBM_VANS_TB3_TALL32;
            if (batch) q(k_batch_tb3<float, float, BXV, WYV, NR>);
            else q(k_sweep_tb3<float, float, BXV, WYV, NR>);
        } else if (rows == LBM_VANS_TB3_SHORT32 && !batch) {
            q(k_sweep_tb3<float, float, BXV, WYV, LBM_VANS_TB3_SHORT32>);
        } else if (rows == LBM_VANS_TB3_TINY32 && !batch) {
            q(k_sweep_tb3<float, float, BXV, WYV, LBM_VANS_TB3_TINY32>);
        } else {
            constexpr int NR = tb_rows<float, 3>();
            if (batch) q(k_batch_tb3<float, float, BXV, WYV, NR>);
            else q(k_sweep_tb3<float, float, BXV, WYV, NR>);
        }
    });
    HIP_TRY(e);
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    *out = static_cast<long long>(nb) * NW * ncu;
    return LBM_VANS_OK;
}

// The same for the four-step kernel (FP32; lone, or batched).
int tb4_resident(int bx, bool wy, bool batch, long long *out)
{
    int nb = 0, dev = 0, ncu = 0;
    hipError_t e = hipSuccess;
    with_bxwy(bx, wy, [&](auto bxc, auto wyc) {
        constexpr int BXV = decltype(bxc)::value;
        constexpr bool WYV = decltype(wyc)::value;
        if (batch)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_tb4<float, float, BXV, WYV>,
                                                             NTHREADS, 0);
        else
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &nb, k_sweep_tb4<float, float, BXV, WYV, tb_rows<float, 4>()>, NTHREADS, 0);
    });
    HIP_TRY(e);
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    *out = static_cast<long long>(nb) * NW * ncu;
    return LBM_VANS_OK;
}

// Automatic choices of the multi-step passes, measured on MI355X.  A three-step
// wave walks its chunk's rows one after another, so the pass needs many waves in
// flight: FP32 GLUPS at pairs / three steps in 12-row / 24-row chunks, periodic box
// 1024^2 109 / 127 / 118, 1536 x 1024 124 / 139 / 123, 2048 x 1024 134 / 158 / 157,
// 2048^2 109 / 157 / 161, 4096^2 108 / 164 / 164 (28 rows 164); channel with walls
// and inlet / outlet 1024 x 512 57 / 64 / 37 (one step per pass 58), 1024^2 88 / 93
// / 72, 2048 x 1024 112 / 121 / 108.  Three steps in 12-row / 6-row chunks (one step
// per pass): box 512^2 53.0 / 76.3 (40.7), 1024 x 512 102.3 / 104.9, 768^2 115.5 /
// 117.0, 1024^2 137.1 / 120.7, 2048 x 1024 178.6 / 156.4; channel 512 x 256 16.9 /
// 27.0 (31.7), 1024 x 512 65.6 / 79.8, 1024^2 96.6 / 101.9, 2048 x 1024 147.4 / 137.1.
// FP32: 24-row chunks when the lattice has at least 0.9 times as many of their waves
// as the chip holds at once (28-row chunks, which recompute fewer halo rows, with four
// times as many), else 12-row chunks when those have at least half of what the chip
// holds, else 6-row chunks; three steps in the chosen height when its waves are at
// least a fifth of what the chip holds, else pairs when the two-step pass has >= 2048
// waves, else one step.
// FP16 (one height): three steps when the lattice has 0.7 times as many waves as
// the chip holds, else pairs or one step as above.  Four steps per pass (FP32, 24-row
// chunks, 58-column strips) when that pass has at least as many waves as the chip
// holds and the chunk height is automatic: GLUPS at three / four steps, periodic box
// 2048^2 160.8 / 163.5, 4096^2 162.8 / 198.0, 8192^2 164.9 / 208.5.
// Open x ends (channels), whose waves clear of the ends skip the x-end rules: GLUPS at
// three steps in 24 / 12 / 6-row chunks and four steps, 4096^2 159.6 / 151.8 / - /
// 175.6; 2048^2 127.3 / 146.5 / 144.7 / 124.4; 2048 x 1024 - / 146.2 / 150.0 / -;
// 1024^2 - / 91.0 / 109.4 / -; 1024 x 512 - / - / 78.7 / -: four steps with three
// times the resident waves, 24-row chunks with four times, 12-row chunks with 1.5
// times, else 6-row chunks.
constexpr int QUAD_FILL_10 = 10;            // four steps: waves >= resident
constexpr int TALL_FILL = 4;                // tall chunks: waves >= 4 x resident
constexpr int DEFAULT_FILL_10 = 9;          // FP32 24-row chunks: waves >= 0.9 x resident
constexpr int HALF_FILL_10 = 5;             // FP32 12-row chunks: waves >= 0.5 x resident,
constexpr int SHORT_FILL_10 = 2;            // else 6-row chunks: waves >= 0.2 x resident
constexpr int TRIPLE_FILL_10 = 7;           // FP16, or an explicit height: >= 0.7 x
// open x ends (the channels): their waves clear of the ends take the pass without
// x-end rules, and the heights and the fourth step pay off only with more waves
constexpr int OPEN_QUAD_FILL_10 = 30;
constexpr int OPEN_DEFAULT_FILL_10 = 40;
constexpr int OPEN_HALF_FILL_10 = 15;

bool tall_auto(long long tall_waves, long long resident)
{
    return tall_waves >= TALL_FILL * resident;
}

int choose_passes(lbm_vans_handle *h)
{
    const lbm_vans_params *p = &h->p;
    h->rows3 = tb_rows<float, 3>();
    h->auto_pass = 1;
    if (p->storage == LBM_F64 || !multi_fits(h->g)) return LBM_VANS_OK;
    const int bx = h->g.open_x ? 2 : (h->g.wall_x ? 1 : 0);
    const bool f16 = p->storage == LBM_F16_SHIFTED;
    const bool wy = h->g.wall_y;
    long long res = 0;
    int rc;
    // the fill a three-step pass in rows3-row chunks needs (tenths of the waves
    // the chip holds of its kernel)
    int fill10 = TRIPLE_FILL_10;
    if (f16) {
        h->rows3 = tb_rows<_Float16, 3>();
    } else if (p->pass_rows != 0) {
        h->rows3 = p->pass_rows;
    } else {
        rc = tb3_resident(p->storage, bx, wy, LBM_VANS_TB3_TALL32, false, &res);
        if (rc) return rc;
        long long res24 = 0;
        rc = tb3_resident(p->storage, bx, wy, tb_rows<float, 3>(), false, &res24);
        if (rc) return rc;
        long long res12 = 0;
        rc = tb3_resident(p->storage, bx, wy, LBM_VANS_TB3_SHORT32, false, &res12);
        if (rc) return rc;
        const int fill24 = bx == 2 ? OPEN_DEFAULT_FILL_10 : DEFAULT_FILL_10;
        const int fill12 = bx == 2 ? OPEN_HALF_FILL_10 : HALF_FILL_10;
        if (tall_auto(waves_of(p->Lx, p->Ly, 3, LBM_VANS_TB3_TALL32), res)) {
            h->rows3 = LBM_VANS_TB3_TALL32;
        } else if (10 * waves_of(p->Lx, p->Ly, 3, tb_rows<float, 3>()) >= fill24 * res24 ||
                   !multi_rows_ok(p->Ly, wy, 3, LBM_VANS_TB3_SHORT32)) {
            h->rows3 = tb_rows<float, 3>();
            fill10 = DEFAULT_FILL_10;
        } else if (10 * waves_of(p->Lx, p->Ly, 3, LBM_VANS_TB3_SHORT32) >= fill12 * res12) {
            h->rows3 = LBM_VANS_TB3_SHORT32;
            fill10 = SHORT_FILL_10;
        } else {
            h->rows3 = LBM_VANS_TB3_TINY32;
            fill10 = SHORT_FILL_10;
        }
    }
    rc = tb3_resident(p->storage, bx, wy, h->rows3, false, &res);
    if (rc) return rc;
    if (10 * waves_of(p->Lx, p->Ly, 3, h->rows3) >= fill10 * res)
        h->auto_pass = 3;
    else if (waves_of(p->Lx, p->Ly, 2, tb2_rows_of(p->storage)) >= 2048)
        h->auto_pass = 2;
    if (!f16 && p->pass_rows == 0 && multi_rows_ok(p->Ly, wy, 4, tb_rows<float, 4>())) {
        long long res4 = 0;
        rc = tb4_resident(bx, wy, false, &res4);
        if (rc) return rc;
        const int fill4 = bx == 2 ? OPEN_QUAD_FILL_10 : QUAD_FILL_10;
        if (10 * waves_of(p->Lx, p->Ly, 4, tb_rows<float, 4>()) >= fill4 * res4) h->auto_pass = 4;
    }
    return LBM_VANS_OK;
}

// Most time steps one pass may take: 2 or 3 with the multi-step passes (FP32 and
// FP16 storage, lattices they can run), else 1.
int max_pass(const lbm_vans_handle *h)
{
    if (h->p.storage == LBM_F64 || !multi_fits(h->g)) return 1;
    int m = h->p.steps_per_pass != 0 ? h->p.steps_per_pass : h->auto_pass;
    if (m == 4 && (h->p.storage != LBM_F32_SHIFTED ||
                   !multi_rows_ok(h->p.Ly, h->g.wall_y, 4, tb_rows<float, 4>())))
        m = 3;
    if (m == 3 && !multi_rows_ok(h->p.Ly, h->g.wall_y, 3, h->rows3)) m = 2;
    if (m == 2 && !multi_rows_ok(h->p.Ly, h->g.wall_y, 2, tb2_rows_of(h->p.storage))) m = 1;
    return m;
}

// NS (2 or 3) time steps in one pass, from the state n in src into dst.
int launch_multi(lbm_vans_handle *h, const void *src, void *dst, int ns)
{
    if (!multi_fits(h->g)) return fail(LBM_VANS_EINVAL, "lattice too large for the multi-step pass");
    if (ns == 4 && h->p.storage != LBM_F32_SHIFTED)
        return fail(LBM_VANS_EINVAL, "the four-step pass needs LBM_F32_SHIFTED storage");
    const int nsrows = ns == 4 ? tb_rows<float, 4>() : (ns == 3 ? h->rows3 : tb2_rows_of(h->p.storage));
    if (!multi_rows_ok(h->p.Ly, h->g.wall_y, ns, nsrows))
        return fail(LBM_VANS_EINVAL, "lattice too short in y for the multi-step pass");
    return with_types(h->p.storage, [&](auto *sp, auto *rp) -> int {
        using S = std::remove_pointer_t<decltype(sp)>;
        using R = std::remove_pointer_t<decltype(rp)>;
        if constexpr (std::is_same_v<S, double>) {
            return fail(LBM_VANS_EINVAL, "multi-step pass needs FP32 or FP16 storage");
        } else {
            const int cols = TX - 2 * (ns - 1);
            const int rows = nsrows;
            const int nstrips = (h->p.Lx + cols - 1) / cols;
            const int nchunks = (h->p.Ly + rows - 1) / rows;
            const long long waves = (long long)nstrips * nchunks;
            if (waves > (long long)INT32_MAX - NW)
                return fail(LBM_VANS_EINVAL, "lattice too large");
            const int grid = static_cast<int>((waves + NW - 1) / NW);
            Phys<R> ph = make_phys<R>(&h->p);
            ph.reservoir = 1;                     // the later steps start from n + 1 >= 1
            const int res_a = res_on(&h->p, h->n);
            const int bx = h->g.open_x ? 2 : (h->g.wall_x ? 1 : 0);
            with_bxwy(bx, h->g.wall_y, [&](auto bxc, auto wyc) {
                constexpr int BXV = decltype(bxc)::value;
                constexpr bool WYV = decltype(wyc)::value;
                auto run = [&](auto ker) {
                    hipLaunchKernelGGL(ker, dim3(grid), dim3(NTHREADS), 0, h->stream,
                                       (const S *)src, (S *)dst, (const R *)h->eps, h->g, ph,
                                       nstrips, nchunks, res_a);
                };
                if (ns == 2) {
                    run(k_sweep_tb2<S, R, BXV, WYV>);
                } else if constexpr (std::is_same_v<S, float>) {
                    if (ns == 4)
                        run(k_sweep_tb4<S, R, BXV, WYV, tb_rows<float, 4>()>);
                    else if (rows == LBM_VANS_TB3_TALL32)
                        run(k_sweep_tb3<S, R, BXV, WYV, LBM_VANS_TB3_TALL32>);
                    else if (rows == LBM_VANS_TB3_SHORT32)
                        run(k_sweep_tb3<S, R, BXV, WYV, LBM_VANS_TB3_SHORT32>);
                    else if (rows == LBM_VANS_TB3_TINY32)
                        run(k_sweep_tb3<S, R, BXV, WYV, LBM_VANS_TB3_TINY32>);
                    else
                        run(k_sweep_tb3<S, R, BXV, WYV, tb_rows<S, 3>()>);
                } else {
                    run(k_sweep_tb3<S, R, BXV, WYV, tb_rows<S, 3>()>);
                }
            });
            return check_launch(ns == 4 ? "k_sweep_tb4" : ns == 3 ? "k_sweep_tb3" : "k_sweep_tb2");
        }
    });
}

// One step n from the state stored in src into dst, on stream st (the handle's
// stream when st is null).
int launch_sweep_ptrs(lbm_vans_handle *h, const void *src, void *dst, int64_t n, bool diag,
                      hipStream_t st = nullptr)
{
    if (!st) st = h->stream;
    return with_types(h->p.storage, [&](auto *sp, auto *rp) {
        using S = std::remove_pointer_t<decltype(sp)>;
        using R = std::remove_pointer_t<decltype(rp)>;
        Phys<R> ph = make_phys<R>(&h->p);
        ph.reservoir = res_on(&h->p, n);
        if (diag) launch_sweep_t<S, R, true>(h, (const S *)src, (S *)dst, ph, st);
        else launch_sweep_t<S, R, false>(h, (const S *)src, (S *)dst, ph, st);
        return check_launch("sweep");
    });
}

int launch_sweep(lbm_vans_handle *h, bool diag)
{
    return launch_sweep_ptrs(h, h->buf[h->cur], h->buf[1 - h->cur], h->n, diag);
}

int launch_finalize(lbm_vans_handle *h, double *out, int nparts, bool add_mass0, double step)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, h->stream, (const double *)h->part,
                       nparts, add_mass0 ? (const double *)h->mass0 : nullptr, step, out);
    return check_launch("k_finalize");
}

}  // namespace

extern "C" {

int lbm_vans_abi_version(void) { return LBM_VANS_ABI_VERSION; }

const char *lbm_vans_last_error(void) { return g_last_error.c_str(); }

size_t lbm_vans_work_bytes(const lbm_vans_params *p)
{
    if (check_params(p) != LBM_VANS_OK) return 0;
    return make_layout(p).total;
}

int lbm_vans_init(const lbm_vans_params *p, const void *eps, void *work, size_t work_bytes,
                  void *stream, lbm_vans_handle **out)
{
    g_last_error.clear();
    int rc = check_params(p);
    if (rc) return rc;
    if (!out) return fail(LBM_VANS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!eps || !work) return fail(LBM_VANS_EINVAL, "eps and work must be device pointers");
    if (reinterpret_cast<uintptr_t>(work) % 256)
        return fail(LBM_VANS_EINVAL, "work buffer must be 256-byte aligned");
    Layout L = make_layout(p);
    if (work_bytes < L.total)
        return fail(LBM_VANS_EINVAL, "work buffer has %zu bytes, %zu needed", work_bytes, L.total);

    int dev = 0, ncu = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    void *scratch_dev = nullptr;
    rc = scratch_address(&scratch_dev);
    if (rc) return rc;
    lbm_vans_handle *h = new (std::nothrow) lbm_vans_handle();
    if (!h) return fail(LBM_VANS_EINVAL, "out of host memory");
    h->scratch = scratch_dev;
    h->p = *p;
    h->stream = static_cast<hipStream_t>(stream);
    h->g = make_geo(p);
    h->vec = sweep_vec(p, ncu);
    h->gs = make_geo(p, h->vec, sweep_rows_of(p->storage));
    h->ntiles = h->g.ntiles;
    h->pop_bytes = L.pop;
    char *w = static_cast<char *>(work);
    h->buf[0] = w;
    h->buf[1] = w + L.pop;
    h->eps = w + 2 * L.pop;
    h->part = reinterpret_cast<double *>(w + 2 * L.pop + L.eps);
    double *small = reinterpret_cast<double *>(w + 2 * L.pop + L.eps + L.part);
    h->mass0 = small;
    h->scratch_rec = small + 2;
    h->ring = small + 2 + NRED;
    h->cur = 0;
    h->n = 0;
    h->nrec = 0;

    rc = with_types(p->storage, [&](auto *sp, auto *rp) {
        using S = std::remove_pointer_t<decltype(sp)>;
        using R = std::remove_pointer_t<decltype(rp)>;
        hipLaunchKernelGGL((k_eps_copy<R>), dim3(h->ntiles), dim3(NTHREADS), 0, h->stream,
                           (const R *)eps, (R *)h->eps, h->g, h->part);
        int r = check_launch("k_eps_copy");
        if (r) return r;
        r = launch_finalize(h, h->scratch_rec, h->ntiles, false, 0.0);
        if (r) return r;
        double rec[NRED];
        HIP_TRY(hipMemcpyAsync(rec, h->scratch_rec, sizeof rec, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        if (rec[6] != 0.0)
            return fail(LBM_VANS_EINVAL, "%.0f porosity values outside (0, 1]", rec[6]);
        double m0 = p->rho0 * rec[0];
        HIP_TRY(hipMemcpyAsync(h->mass0, &m0, sizeof m0, hipMemcpyHostToDevice, h->stream));
        Phys<R> ph = make_phys<R>(p);
        hipLaunchKernelGGL((k_set_state<S, R>), dim3(h->ntiles), dim3(NTHREADS), 0, h->stream,
                           (S *)h->buf[0], (const R *)h->eps, h->g, p->rho0,
                           static_cast<double>(ph.rho0), p->u0[0], p->u0[1],
                           (const double *)nullptr, ph.scale, wall6(p, 0), wall6(p, 1));
        r = check_launch("k_set_state");
        if (r) return r;
        // The host value m0 must stay alive until the copy has run.
        HIP_TRY(hipStreamSynchronize(h->stream));
        return LBM_VANS_OK;
    });
    if (!rc) rc = choose_passes(h);
    if (rc) {
        delete h;
        return rc;
    }
    // launch-bound lattices replay their steps as graphs (measured on MI355X, FP64
    // 80 x 80: see the design notes)
    h->use_graphs = h->gs.ntiles < 2 * ncu;
    // the gradient's second stream (default priority) and its events
    hipError_t e = hipStreamCreateWithFlags(&h->stream2, hipStreamNonBlocking);
    hipEvent_t *evs[5] = {&h->ev_start, &h->ev_rec[0], &h->ev_rec[1], &h->ev_rev[0],
                          &h->ev_rev[1]};
    for (int k = 0; k < 5 && e == hipSuccess; k++)
        e = hipEventCreateWithFlags(evs[k], hipEventDisableTiming);
    if (e != hipSuccess) {
        rc = fail(LBM_VANS_EHIP, "stream / event creation failed: %s", hipGetErrorString(e));
        lbm_vans_destroy(h);
        return rc;
    }
    *out = h;
    return LBM_VANS_OK;
}

}  // extern "C"

namespace {

// Steps per replay of a handle's step graph.
constexpr int GRAPH_STEPS = 32;

// The launches of `steps` steps from the handle's current state, as lbm_vans_step
// issues them without diagnostics (up to max_pass steps per launch), on h->stream;
// the handle's state slot and step count advance.
int plain_steps(lbm_vans_handle *h, int64_t steps)
{
    for (int64_t k = 0; k < steps;) {
        const int m = static_cast<int>(std::min<int64_t>(max_pass(h), steps - k));
        const int rc = m >= 2 ? launch_multi(h, h->buf[h->cur], h->buf[1 - h->cur], m)
                              : launch_sweep(h, false);
        if (rc) return rc;
        h->cur = 1 - h->cur;
        h->n += m;
        k += m;
    }
    return LBM_VANS_OK;
}

// Capture GRAPH_STEPS steps from the current state slot (with the open-end rules of
// a state n >= 1) into graph[h->cur]; the handle's state and count are unchanged.
int capture_steps(lbm_vans_handle *h)
{
    if (!h->cap) HIP_TRY(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
    const int cur = h->cur;
    const int64_t n = h->n;
    hipStream_t st = h->stream;
    h->stream = h->cap;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal);
    int rc = e == hipSuccess ? plain_steps(h, GRAPH_STEPS) : LBM_VANS_OK;
    hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(h->cap, &graph) : e;
    h->stream = st;
    h->cur = cur;
    h->n = n;
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e2 != hipSuccess)
        return fail(LBM_VANS_EHIP, "step graph capture failed: %s", hipGetErrorString(e2));
    e = hipGraphInstantiate(&h->graph[cur], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        h->graph[cur] = nullptr;
        return fail(LBM_VANS_EHIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
    }
    return LBM_VANS_OK;
}

}  // namespace

extern "C" {

int lbm_vans_step(lbm_vans_handle *h, int64_t nsteps)
{
    if (!h) return fail(LBM_VANS_EINVAL, "handle is NULL");
    if (nsteps < 0) return fail(LBM_VANS_EINVAL, "nsteps = %lld < 0", (long long)nsteps);
    // small lattices without diagnostics: whole chunks of steps as graph replays (the
    // same launches, without a host launch per step); the rest one launch at a time
    if (h->use_graphs && h->p.diag_every == 0) {
        while (nsteps >= GRAPH_STEPS && res_on(&h->p, h->n)) {
            if (!h->graph[h->cur]) {
                const int rc = capture_steps(h);
                if (rc) return rc;
            }
            HIP_TRY(hipGraphLaunch(h->graph[h->cur], h->stream));
            const int64_t launches = (GRAPH_STEPS + max_pass(h) - 1) / max_pass(h);
            if (launches & 1) h->cur = 1 - h->cur;
            h->n += GRAPH_STEPS;
            nsteps -= GRAPH_STEPS;
        }
    }
    for (int64_t k = 0; k < nsteps; k++) {
        bool diag = h->p.diag_every > 0 && h->n % h->p.diag_every == 0;
        // up to three steps in one pass when they remain in this call and none
        // records diagnostics
        const int m = h->p.diag_every == 0
                          ? static_cast<int>(std::min<int64_t>(max_pass(h), nsteps - k))
                          : 1;
        if (m >= 2) {
            int rc = launch_multi(h, h->buf[h->cur], h->buf[1 - h->cur], m);
            if (rc) return rc;
            h->cur = 1 - h->cur;
            h->n += m;
            k += m - 1;
            continue;
        }
        int rc = launch_sweep(h, diag);
        if (rc) return rc;
        if (diag) {
            double *slot = h->ring + (h->nrec % LBM_VANS_DIAG_RING) * NRED;
            rc = launch_finalize(h, slot, h->gs.ntiles, true, static_cast<double>(h->n));
            if (rc) return rc;
            h->nrec++;
        }
        h->cur = 1 - h->cur;
        h->n++;
    }
    return LBM_VANS_OK;
}

int64_t lbm_vans_step_count(const lbm_vans_handle *h) { return h ? h->n : -1; }

int lbm_vans_pass_plan(const lbm_vans_handle *h, int32_t *steps_per_pass, int32_t *pass_rows)
{
    if (!h) return fail(LBM_VANS_EINVAL, "handle is NULL");
    const bool multi = h->p.storage != LBM_F64 && multi_fits(h->g);
    const int m = max_pass(h);
    if (steps_per_pass) *steps_per_pass = m;
    if (pass_rows) *pass_rows = multi ? (m == 4 ? tb_rows<float, 4>() : h->rows3) : 0;
    return LBM_VANS_OK;
}

int lbm_vans_moments(lbm_vans_handle *h, void *eps_rho, void *rho, void *ux, void *uy,
                     double *diag)
{
    if (!h) return fail(LBM_VANS_EINVAL, "handle is NULL");
    int rc = with_types(h->p.storage, [&](auto *sp, auto *rp) {
        using S = std::remove_pointer_t<decltype(sp)>;
        using R = std::remove_pointer_t<decltype(rp)>;
        Phys<R> ph = make_phys<R>(&h->p);
        ph.reservoir = res_on(&h->p, h->n);
        hipLaunchKernelGGL((k_moments<S, R>), dim3(h->ntiles), dim3(NTHREADS), 0, h->stream,
                           (const S *)h->buf[h->cur], (const R *)h->eps, h->g, ph, (R *)eps_rho,
                           (R *)rho, (R *)ux, (R *)uy, h->part);
        return check_launch("k_moments");
    });
    if (rc) return rc;
    if (!diag) return LBM_VANS_OK;
    rc = launch_finalize(h, h->scratch_rec, h->ntiles, true, static_cast<double>(h->n));
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(diag, h->scratch_rec, NRED * sizeof(double), hipMemcpyDeviceToHost,
                           h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (diag[6] != 0.0)
        return fail(LBM_VANS_ENONFINITE, "%.0f nodes have non-finite moments at step %lld",
                    diag[6], (long long)h->n);
    return mach_check(diag[5], static_cast<double>(h->n));
}

int lbm_vans_objective(lbm_vans_handle *h, int32_t objective, double *J)
{
    if (!h) return fail(LBM_VANS_EINVAL, "handle is NULL");
    if (objective != LBM_OBJ_OUTLET_FLUX)
        return fail(LBM_VANS_EINVAL, "unknown objective %d", objective);
    if (!J) return fail(LBM_VANS_EINVAL, "J is NULL");
    const int nblk = (h->p.Ly + NTHREADS - 1) / NTHREADS;
    int rc = with_types(h->p.storage, [&](auto *sp, auto *rp) {
        using S = std::remove_pointer_t<decltype(sp)>;
        using R = std::remove_pointer_t<decltype(rp)>;
        Phys<R> ph = make_phys<R>(&h->p);
        ph.reservoir = res_on(&h->p, h->n);
        hipLaunchKernelGGL((k_outlet_flux<S, R>), dim3(nblk), dim3(NTHREADS), 0, h->stream,
                           (const S *)h->buf[h->cur], (const R *)h->eps, h->g, ph, h->part);
        return check_launch("k_outlet_flux");
    });
    if (rc) return rc;
    rc = launch_finalize(h, h->scratch_rec, nblk, false, static_cast<double>(h->n));
    if (rc) return rc;
    double rec[NRED];
    HIP_TRY(hipMemcpyAsync(rec, h->scratch_rec, sizeof rec, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    *J = rec[0];
    if (!std::isfinite(rec[0])) return fail(LBM_VANS_ENONFINITE, "objective is not finite");
    return LBM_VANS_OK;
}

int lbm_vans_get_state(lbm_vans_handle *h, void *f)
{
    if (!h) return fail(LBM_VANS_EINVAL, "handle is NULL");
    if (!f) return fail(LBM_VANS_EINVAL, "f is NULL");
    return with_types(h->p.storage, [&](auto *sp, auto *rp) {
        using S = std::remove_pointer_t<decltype(sp)>;
        using R = std::remove_pointer_t<decltype(rp)>;
        Phys<R> ph = make_phys<R>(&h->p);
        ph.reservoir = res_on(&h->p, h->n);
        hipLaunchKernelGGL((k_get_state<S, R>), dim3(h->ntiles), dim3(NTHREADS), 0, h->stream,
                           (const S *)h->buf[h->cur], (const R *)h->eps, h->g, ph, (double *)f);
        return check_launch("k_get_state");
    });
}

int lbm_vans_set_state(lbm_vans_handle *h, const void *f)
{
    if (!h) return fail(LBM_VANS_EINVAL, "handle is NULL");
    if (!f) return fail(LBM_VANS_EINVAL, "f is NULL");
    return with_types(h->p.storage, [&](auto *sp, auto *rp) {
        using S = std::remove_pointer_t<decltype(sp)>;
        using R = std::remove_pointer_t<decltype(rp)>;
        Phys<R> ph = make_phys<R>(&h->p);
        hipLaunchKernelGGL((k_set_state<S, R>), dim3(h->ntiles), dim3(NTHREADS), 0, h->stream,
                           (S *)h->buf[h->cur], (const R *)h->eps, h->g, h->p.rho0,
                           static_cast<double>(ph.rho0), 0.0, 0.0, (const double *)f, ph.scale,
                           wall6(&h->p, 0), wall6(&h->p, 1));
        return check_launch("k_set_state");
    });
}

int lbm_vans_diag_read(lbm_vans_handle *h, double *records, int32_t max_records,
                       int32_t *n_records)
{
    if (!h) return fail(LBM_VANS_EINVAL, "handle is NULL");
    if (!n_records || (max_records > 0 && !records))
        return fail(LBM_VANS_EINVAL, "records / n_records is NULL");
    int64_t avail = h->nrec < LBM_VANS_DIAG_RING ? h->nrec : LBM_VANS_DIAG_RING;
    int64_t cnt = max_records < avail ? max_records : avail;
    *n_records = static_cast<int32_t>(cnt);
    // Oldest kept record first: the last cnt records written.
    for (int64_t k = 0; k < cnt; k++) {
        int64_t idx = (h->nrec - cnt + k) % LBM_VANS_DIAG_RING;
        HIP_TRY(hipMemcpyAsync(records + k * NRED, h->ring + idx * NRED, NRED * sizeof(double),
                               hipMemcpyDeviceToHost, h->stream));
    }
    HIP_TRY(hipStreamSynchronize(h->stream));
    for (int64_t k = 0; k < cnt; k++)
        if (records[k * NRED + 6] != 0.0)
            return fail(LBM_VANS_ENONFINITE, "non-finite moments recorded at step %.0f",
                        records[k * NRED + 7]);
    for (int64_t k = 0; k < cnt; k++)
        if (mach_check(records[k * NRED + 5], records[k * NRED + 7]) != LBM_VANS_OK)
            return LBM_VANS_WMACH;
    return LBM_VANS_OK;
}

namespace {

// Gradient workspace: nck checkpoints, nset sets of seg buffers for recomputed
// segments, two adjoint buffers, three accumulators and (FP32 / FP16 storage) an
// FP64 porosity copy.  Two segment sets (a lone handle with two or more segments)
// let the recompute of one segment run beside the reverse steps of the next.
struct GradLayout {
    size_t pop, lam, acc, eps64, total;
    int64_t nck, seg, nset;
    int64_t states() const { return nck + nset * seg; }
};

GradLayout grad_layout(const lbm_vans_params *p, int64_t nsteps, int32_t ckpt_every,
                       bool two_sets)
{
    Layout L = make_layout(p);
    Geo g = make_geo(p);
    GradLayout G;
    G.pop = L.pop;
    G.nck = (nsteps + ckpt_every - 1) / ckpt_every;
    if (G.nck < 1) G.nck = 1;
    G.seg = ckpt_every;
    G.nset = two_sets && G.nck >= 2 ? 2 : 1;
    // the reverse steps run in FP64 for every storage, with FP64 accumulators and,
    // for FP32 / FP16 storage, an FP64 copy of the porosity; the adjoints between
    // the steps are stored in FP64 for FP64 storage, else in FP32
    const size_t adj_bytes = p->storage == LBM_F64 ? sizeof(double) : sizeof(float);
    G.lam = align256((size_t)9 * g.plane * adj_bytes);
    G.acc = align256((size_t)g.plane * sizeof(double));
    G.eps64 = p->storage != LBM_F64 ? align256((size_t)g.plane * sizeof(double)) : 0;
    G.total = (size_t)G.states() * G.pop + 2 * G.lam + 3 * G.acc + G.eps64;
    return G;
}

int check_grad_args(const lbm_vans_params *p, int32_t objective, int64_t nsteps,
                    int32_t ckpt_every)
{
    int rc = check_params(p);
    if (rc) return rc;
    if (objective != LBM_OBJ_OUTLET_FLUX)
        return fail(LBM_VANS_EINVAL, "unknown objective %d", objective);
    if (nsteps < 0) return fail(LBM_VANS_EINVAL, "nsteps = %lld < 0", (long long)nsteps);
    if (ckpt_every < 1) return fail(LBM_VANS_EINVAL, "ckpt_every = %d < 1", ckpt_every);
    return LBM_VANS_OK;
}

}  // namespace

size_t lbm_vans_grad_work_bytes(const lbm_vans_params *p, int32_t objective, int64_t nsteps,
                                int32_t ckpt_every)
{
    if (check_grad_args(p, objective, nsteps, ckpt_every)) return 0;
    return grad_layout(p, nsteps, ckpt_every, true).total;
}

namespace {

// The gradient of lbm_vans_grad in the workspace grad_work (a caller's buffer, or
// the library-held array).
int grad_run(lbm_vans_handle *h, int32_t objective, int64_t nsteps, int32_t ckpt_every,
             void *grad_work, size_t grad_work_bytes, double *dJdeps, double *J)
{
    if (!h) return fail(LBM_VANS_EINVAL, "handle is NULL");
    int rc = check_grad_args(&h->p, objective, nsteps, ckpt_every);
    if (rc) return rc;
    if (!grad_work || !dJdeps) return fail(LBM_VANS_EINVAL, "grad_work and dJdeps are required");
    if (reinterpret_cast<uintptr_t>(grad_work) % 256)
        return fail(LBM_VANS_EINVAL, "grad_work must be 256-byte aligned");
    const GradLayout G = grad_layout(&h->p, nsteps, ckpt_every, true);
    if (grad_work_bytes < G.total)
        return fail(LBM_VANS_EINVAL, "grad_work has %zu bytes, %zu needed", grad_work_bytes,
                    G.total);
    char *w = static_cast<char *>(grad_work);
    auto ckpt = [&](int64_t c) { return w + c * G.pop; };
    auto seg = [&](int64_t set, int64_t j) { return w + (G.nck + set * G.seg + j) * G.pop; };
    char *lam[2] = {w + G.states() * G.pop, w + G.states() * G.pop + G.lam};
    double *eb = reinterpret_cast<double *>(w + G.states() * G.pop + 2 * G.lam);
    double *gxb = eb + G.acc / sizeof(double);
    double *gyb = gxb + G.acc / sizeof(double);
    double *eps64 = G.eps64 ? reinterpret_cast<double *>(w + G.states() * G.pop +
                                                         2 * G.lam + 3 * G.acc)
                            : nullptr;
    const Geo &g = h->g;
    const int K = ckpt_every;

    return with_types(h->p.storage, [&](auto *sp, auto *rp) -> int {
        using S = std::remove_pointer_t<decltype(sp)>;
        using R = std::remove_pointer_t<decltype(rp)>;
        const Phys<R> ph0 = make_phys<R>(&h->p);
        // 1. initial state, forward with a checkpoint every K steps
        hipLaunchKernelGGL((k_set_state<S, R>), dim3(h->ntiles), dim3(NTHREADS), 0, h->stream,
                           (S *)h->buf[0], (const R *)h->eps, g, h->p.rho0,
                           static_cast<double>(ph0.rho0), h->p.u0[0], h->p.u0[1],
                           (const double *)nullptr, ph0.scale, wall6(&h->p, 0),
                           wall6(&h->p, 1));
        int r = check_launch("k_set_state");
        if (r) return r;
        h->cur = 0;
        h->n = 0;
        for (int64_t s0 = 0; s0 < nsteps || s0 == 0; s0 += K) {
            HIP_TRY(hipMemcpyAsync(ckpt(s0 / K), h->buf[h->cur], G.pop, hipMemcpyDeviceToDevice,
                                   h->stream));
            // only the checkpoints are kept, so the steps in between may go up to
            // three per pass
            for (int64_t k = 0; k < K && s0 + k < nsteps; k++) {
                const int m = static_cast<int>(
                    std::min<int64_t>({(int64_t)max_pass(h), K - k, nsteps - s0 - k}));
                if (m >= 2) {
                    r = launch_multi(h, h->buf[h->cur], h->buf[1 - h->cur], m);
                    if (r) return r;
                    h->cur = 1 - h->cur;
                    h->n += m;
                    k += m - 1;
                    continue;
                }
                r = launch_sweep(h, false);
                if (r) return r;
                h->cur = 1 - h->cur;
                h->n++;
            }
            if (nsteps == 0) break;
        }
        // 2. seed: J of the state N and the adjoint of that state
        const long long nz = (long long)(3 * G.acc / sizeof(double));
        hipLaunchKernelGGL(k_zero, dim3((unsigned)((nz + NTHREADS - 1) / NTHREADS)),
                           dim3(NTHREADS), 0, h->stream, eb, nz);
        r = check_launch("k_zero");
        if (r) return r;
        // the reverse steps compute in FP64 for every storage: on an FP64 copy of the
        // porosity (FP32 / FP16 storage) and with the forward's shift reference rho0
        using RA = double;
        Phys<RA> ph = make_phys<RA>(&h->p);
        ph.rho0 = static_cast<RA>(ph0.rho0);
        const RA *eps_a = reinterpret_cast<const RA *>(h->eps);
        if constexpr (!std::is_same_v<RA, R>) {
            const long long npl = g.plane;
            hipLaunchKernelGGL(k_widen, dim3((unsigned)((npl + NTHREADS - 1) / NTHREADS)),
                               dim3(NTHREADS), 0, h->stream, (const float *)h->eps, eps64, npl);
            r = check_launch("k_widen");
            if (r) return r;
            eps_a = eps64;
        }
        ph.reservoir = res_on(&h->p, nsteps);
        int a = 0;
        hipLaunchKernelGGL((k_adjoint_seed<S, RA>), dim3(h->ntiles), dim3(NTHREADS), 0,
                           h->stream, (const S *)h->buf[h->cur], (AdjT<S> *)lam[a], eps_a, g,
                           ph, eb, gxb, gyb, h->part);
        r = check_launch("k_adjoint_seed");
        if (r) return r;
        r = launch_finalize(h, h->scratch_rec, h->ntiles, false, static_cast<double>(nsteps));
        if (r) return r;
        double rec[NRED];
        HIP_TRY(hipMemcpyAsync(rec, h->scratch_rec, sizeof rec, hipMemcpyDeviceToHost,
                               h->stream));
        // 3. reverse, one checkpoint segment at a time (states recomputed).  With two
        // segment sets, segment c is recomputed into set c % 2 on the second stream
        // while the handle's stream runs the reverse steps of segment c + 1: the
        // recompute is bound by HBM and the FP64 reverse steps by their arithmetic,
        // so the two share the GPU.
        const int64_t nck = nsteps == 0 ? 0 : (nsteps + K - 1) / K;
        const bool two = G.nset == 2;
        // reverse steps: one wave per strip of TX columns and chunk of ADJ_ROWS rows
        const int adj_strips = (g.Lx + TX - 1) / TX;
        const int adj_chunks = (g.Ly + ADJ_ROWS - 1) / ADJ_ROWS;
        const unsigned adj_blocks =
            static_cast<unsigned>(((long long)adj_strips * adj_chunks + NW - 1) / NW);
        hipStream_t rs = two ? h->stream2 : h->stream;
        auto recompute = [&](int64_t c) -> int {
            const int64_t s0 = c * K, s1 = std::min<int64_t>(s0 + K, nsteps);
            const int64_t set = two ? c % 2 : 0;
            for (int64_t j = 1; j < s1 - s0; j++) {
                const void *src = j == 1 ? (const void *)ckpt(c) : (const void *)seg(set, j - 1);
                int rr = launch_sweep_ptrs(h, src, seg(set, j), s0 + j - 1, false, rs);
                if (rr) return rr;
            }
            if (two) HIP_TRY(hipEventRecord(h->ev_rec[set], rs));
            return LBM_VANS_OK;
        };
        if (two) {
            // the checkpoints are written (and the seed has read the final state)
            HIP_TRY(hipEventRecord(h->ev_start, h->stream));
            HIP_TRY(hipStreamWaitEvent(rs, h->ev_start, 0));
        }
        if (nck > 0) {
            r = recompute(nck - 1);
            if (r) return r;
        }
        for (int64_t c = nck - 1; c >= 0; c--) {
            const int64_t s0 = c * K, s1 = std::min<int64_t>(s0 + K, nsteps);
            const int64_t set = two ? c % 2 : 0;
            if (two && c >= 1) {
                // set (c - 1) % 2 is free once the reverse steps of segment c + 1 ran
                if (c + 1 <= nck - 1) HIP_TRY(hipStreamWaitEvent(rs, h->ev_rev[(c + 1) % 2], 0));
                r = recompute(c - 1);
                if (r) return r;
            } else if (!two && c < nck - 1) {
                r = recompute(c);
                if (r) return r;
            }
            if (two) HIP_TRY(hipStreamWaitEvent(h->stream, h->ev_rec[set], 0));
            for (int64_t n = s1 - 1; n >= s0; n--) {
                const void *state =
                    n == s0 ? (const void *)ckpt(c) : (const void *)seg(set, n - s0);
                ph.reservoir = res_on(&h->p, n);
                hipLaunchKernelGGL((k_adjoint_rows<S, RA, ADJ_ROWS>), dim3(adj_blocks),
                                   dim3(NTHREADS), 0, h->stream, (const S *)state,
                                   (const AdjT<S> *)lam[a], (AdjT<S> *)lam[1 - a],
                                   (const AdjT<S> *)h->eps, g, ph, eb, gxb, gyb, adj_strips,
                                   adj_chunks);
                r = check_launch("k_adjoint_rows");
                if (r) return r;
                a = 1 - a;
            }
            if (two) HIP_TRY(hipEventRecord(h->ev_rev[set], h->stream));
        }
        // 4. initial state and the porosity stencil
        hipLaunchKernelGGL((k_adjoint_init<AdjT<S>>), dim3(h->ntiles), dim3(NTHREADS), 0,
                           h->stream, (const AdjT<S> *)lam[a], g, h->p.rho0, h->p.u0[0], h->p.u0[1],
                           wall6(&h->p, 0), wall6(&h->p, 1), eb);
        r = check_launch("k_adjoint_init");
        if (r) return r;
        hipLaunchKernelGGL(k_adjoint_finish, dim3(h->ntiles), dim3(NTHREADS), 0, h->stream,
                           (const double *)eb, (const double *)gxb, (const double *)gyb, g,
                           dJdeps);
        r = check_launch("k_adjoint_finish");
        if (r) return r;
        HIP_TRY(hipStreamSynchronize(h->stream));
        if (J) *J = rec[0];
        if (!std::isfinite(rec[0]))
            return fail(LBM_VANS_ENONFINITE, "objective is not finite");
        return LBM_VANS_OK;
    });
}

}  // namespace

int lbm_vans_grad(lbm_vans_handle *h, int32_t objective, int64_t nsteps, int32_t ckpt_every,
                  void *grad_work, size_t grad_work_bytes, double *dJdeps, double *J)
{
    return grad_run(h, objective, nsteps, ckpt_every, grad_work, grad_work_bytes, dJdeps, J);
}

int lbm_vans_grad_static(lbm_vans_handle *h, int32_t objective, int64_t nsteps,
                         int32_t ckpt_every, double *dJdeps, double *J)
{
    if (!h) return fail(LBM_VANS_EINVAL, "handle is NULL");
    const size_t need = lbm_vans_grad_work_bytes(&h->p, objective, nsteps, ckpt_every);
    if (need == 0) return LBM_VANS_EINVAL;   // the message is set
    if (need > LBM_VANS_GRAD_STATIC_BYTES)
        return fail(LBM_VANS_EINVAL,
                    "the gradient needs %zu bytes of workspace; the library-held workspace has "
                    "%zu (use lbm_vans_grad with a caller buffer, or a larger ckpt_every / "
                    "smaller lattice)",
                    need, static_cast<size_t>(LBM_VANS_GRAD_STATIC_BYTES));
    return grad_run(h, objective, nsteps, ckpt_every, h->scratch, LBM_VANS_GRAD_STATIC_BYTES,
                    dJdeps, J);
}

void lbm_vans_destroy(lbm_vans_handle *h)
{
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    for (auto &gx : h->graph)
        if (gx) (void)hipGraphExecDestroy(gx);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    if (h->stream2) {
        (void)hipStreamSynchronize(h->stream2);
        (void)hipStreamDestroy(h->stream2);
    }
    for (hipEvent_t ev : {h->ev_start, h->ev_rec[0], h->ev_rec[1], h->ev_rev[0], h->ev_rev[1]})
        if (ev) (void)hipEventDestroy(ev);
    delete h;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Ensembles (host side)
// ---------------------------------------------------------------------------

struct lbm_vans_batch {
    std::vector<lbm_vans_handle *> m;
    hipStream_t stream = nullptr;   // the caller's stream: every batched launch
    hipStream_t cap = nullptr;      // private stream used only to capture step graphs
    hipEvent_t ev[2] = {nullptr, nullptr};
    int storage = 0, bx = 0, wy = 0, vmax = 4;
    lbm_vans_batch_config cfg{};
    size_t desc_bytes = 0;          // bytes of one device descriptor
    std::vector<char> desc;         // host image of the descriptors
    std::vector<int> tmap, tmap_adj;  // tile lists of the sweep and of the adjoint
    std::vector<int> wmap[4];         // wave lists of the two-step pass, of the three-step
                                      // pass in short and in tall chunks (FP32 only) and of
                                      // the four-step pass (FP32 only)
    void *d_desc = nullptr;
    int *d_tmap = nullptr, *d_tmap_adj = nullptr,
        *d_wmap[4] = {nullptr, nullptr, nullptr, nullptr};
    int ntiles = 0, ntiles_adj = 0, nwaves[4] = {0, 0, 0, 0};
    bool multi_ok = true;           // every member fits the multi-step passes' addressing
    bool multi4_ok = false;         // ... and the four-step pass (FP32, rows)
    long long tall_resident = 0;    // waves of the tall batched three-step kernel the chip holds
    long long quad_resident = 0;    // waves of the batched four-step kernel the chip holds
    hipGraphExec_t graph[2] = {nullptr, nullptr};  // chunk of cfg.graph_steps steps from slot 0 / 1
};

namespace {

size_t batch_table_bytes(int storage, size_t nmembers, size_t ntiles_adj, const size_t *nwaves)
{
    const size_t d = storage == LBM_F64 ? sizeof(Member<double>) : sizeof(Member<float>);
    return align256(nmembers * d) + 2 * align256(ntiles_adj * sizeof(int)) +
           align256(nwaves[0] * sizeof(int)) + align256(nwaves[1] * sizeof(int)) +
           align256(nwaves[2] * sizeof(int)) + align256(nwaves[3] * sizeof(int));
}

// Waves of one member in wave list q: the two-step pass (0), the three-step pass
// in short (1) and in tall chunks (2; FP32 storage only), the four-step pass (3;
// FP32 storage only); none in FP64, which has no such pass.
size_t batch_waves(const lbm_vans_params *p, int q)
{
    if (p->storage == LBM_F64) return 0;
    const bool f16 = p->storage == LBM_F16_SHIFTED;
    if (q == 0) return waves_of(p->Lx, p->Ly, 2, f16 ? tb_rows<_Float16, 2>() : tb_rows<float, 2>());
    if (q == 1) return waves_of(p->Lx, p->Ly, 3, f16 ? tb_rows<_Float16, 3>() : tb_rows<float, 3>());
    if (q == 2) return f16 ? 0 : waves_of(p->Lx, p->Ly, 3, LBM_VANS_TB3_TALL32);
    return f16 ? 0 : waves_of(p->Lx, p->Ly, 4, tb_rows<float, 4>());
}

// The batched three-step pass runs in tall chunks (FP32 storage): as configured, or
// automatically as for a lone lattice (waves of the whole batch against what the
// chip holds of the batched kernel).
bool batch_tall(const lbm_vans_batch *b)
{
    if (b->storage != LBM_F32_SHIFTED) return false;
    if (b->cfg.pass_rows != 0) return b->cfg.pass_rows == LBM_VANS_TB3_TALL32;
    return tall_auto(b->nwaves[2], b->tall_resident);
}

void drop_graphs(lbm_vans_batch *b)
{
    for (auto &gx : b->graph)
        if (gx) {
            (void)hipGraphExecDestroy(gx);
            gx = nullptr;
        }
}

// Descriptors and tile lists for a sweep width of vec nodes per lane, plus the
// gradient workspace layout when gw is given; uploaded to the batch's table.
int batch_upload(lbm_vans_batch *b, int vec, char *gw, int64_t nsteps, int32_t ckpt_every)
{
    const size_t nm = b->m.size();
    b->tmap.clear();
    b->tmap_adj.clear();
    for (auto &wm : b->wmap) wm.clear();
    int rc = with_types(b->storage, [&](auto *sp, auto *rp) -> int {
        using R = std::remove_pointer_t<decltype(rp)>;
        (void)sp;
        b->desc_bytes = sizeof(Member<R>);
        b->desc.assign(nm * sizeof(Member<R>), 0);
        std::vector<Member<R>> D(nm);
        for (size_t k = 0; k < nm; k++) {
            lbm_vans_handle *h = b->m[k];
            Member<R> &d = D[k];
            std::memset(&d, 0, sizeof d);
            d.vec = vec;
            d.gs = make_geo(&h->p, d.vec, sweep_rows_of(h->p.storage));
            d.g = h->g;
            d.ph = make_phys<R>(&h->p);
            d.pha = make_phys<double>(&h->p);
            d.pha.rho0 = static_cast<double>(d.ph.rho0);
            d.eps_a = h->p.storage == LBM_F64 ? static_cast<const double *>(h->eps) : nullptr;
            d.buf[0] = h->buf[0];
            d.buf[1] = h->buf[1];
            d.eps = static_cast<const R *>(h->eps);
            d.part = h->part;
            d.tile0 = static_cast<int>(b->tmap.size());
            d.tile0_adj = static_cast<int>(b->tmap_adj.size());
            b->tmap.insert(b->tmap.end(), d.gs.ntiles, static_cast<int>(k));
            b->tmap_adj.insert(b->tmap_adj.end(), d.g.ntiles, static_cast<int>(k));
            for (int q = 0; q < 4; q++) {
                const int ns = q == 0 ? 2 : (q < 3 ? 3 : 4);
                const int cols = TX - 2 * (ns - 1);
                d.tb_strips[ns - 2] = (h->p.Lx + cols - 1) / cols;
                d.tw0[q] = static_cast<int>(b->wmap[q].size());
                b->wmap[q].insert(b->wmap[q].end(), batch_waves(&h->p, q), static_cast<int>(k));
            }
        }
        size_t off = 0;
        for (size_t k = 0; k < nm; k++) {
            lbm_vans_handle *h = b->m[k];
            Member<R> &d = D[k];
            if (gw) {
                const GradLayout G = grad_layout(&h->p, nsteps, ckpt_every, false);
                d.gw = gw + off;
                d.gpop = static_cast<long long>(G.pop);
                d.glam = static_cast<long long>(G.lam);
                d.gacc = static_cast<long long>(G.acc);
                d.nslot = static_cast<int>(G.states());
                if (G.eps64)
                    d.eps_a = reinterpret_cast<const double *>(
                        d.gw + G.states() * G.pop + 2 * G.lam + 3 * G.acc);
                off += align256(G.total);
            }
            std::memcpy(b->desc.data() + k * sizeof d, &d, sizeof d);
        }
        return LBM_VANS_OK;
    });
    if (rc) return rc;
    b->ntiles = static_cast<int>(b->tmap.size());
    b->ntiles_adj = static_cast<int>(b->tmap_adj.size());
    for (int q = 0; q < 4; q++) b->nwaves[q] = static_cast<int>(b->wmap[q].size());
    HIP_TRY(hipMemcpyAsync(b->d_desc, b->desc.data(), b->desc.size(), hipMemcpyHostToDevice,
                           b->stream));
    HIP_TRY(hipMemcpyAsync(b->d_tmap, b->tmap.data(), b->tmap.size() * sizeof(int),
                           hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipMemcpyAsync(b->d_tmap_adj, b->tmap_adj.data(), b->tmap_adj.size() * sizeof(int),
                           hipMemcpyHostToDevice, b->stream));
    for (int q = 0; q < 4; q++)
        if (!b->wmap[q].empty())
            HIP_TRY(hipMemcpyAsync(b->d_wmap[q], b->wmap[q].data(),
                                   b->wmap[q].size() * sizeof(int), hipMemcpyHostToDevice,
                                   b->stream));
    // the host images must outlive the copies; they also must not change under them
    HIP_TRY(hipStreamSynchronize(b->stream));
    return LBM_VANS_OK;
}

template <typename S, typename R, int V>
void batch_sweep_v(const lbm_vans_batch *b, hipStream_t st, int src, int dst, int reservoir)
{
    const int n = b->ntiles;
    const int grid = (b->cfg.grid > 0 && b->cfg.grid < n) ? b->cfg.grid : n;
    const Member<R> *M = static_cast<const Member<R> *>(b->d_desc);
    const int *tm = b->d_tmap;
#define LBM_VANS_BATCH(BXV, WYV)                                                             \
    hipLaunchKernelGGL((k_batch_sweep<S, R, V, BXV, WYV>), dim3(grid), dim3(NTHREADS), 0, st, \
                       M, tm, n, src, dst, reservoir)
    if (b->bx == 0 && !b->wy) LBM_VANS_BATCH(0, false);
    else if (b->bx == 0) LBM_VANS_BATCH(0, true);
    else if (b->bx == 1 && !b->wy) LBM_VANS_BATCH(1, false);
    else if (b->bx == 1) LBM_VANS_BATCH(1, true);
    else if (!b->wy) LBM_VANS_BATCH(2, false);
    else LBM_VANS_BATCH(2, true);
#undef LBM_VANS_BATCH
}

// One batched step on stream st: every member from state slot src to dst in
// one launch.
int batch_sweep(lbm_vans_batch *b, hipStream_t st, int src, int dst, int reservoir)
{
    return with_types(b->storage, [&](auto *sp, auto *rp) -> int {
        using S = std::remove_pointer_t<decltype(sp)>;
        using R = std::remove_pointer_t<decltype(rp)>;
        if constexpr (sizeof(S) != 8) {
            if (b->cfg.vec == 4) batch_sweep_v<S, R, 4>(b, st, src, dst, reservoir);
        }
        if (b->cfg.vec == 2) batch_sweep_v<S, R, 2>(b, st, src, dst, reservoir);
        if (b->cfg.vec == 1) batch_sweep_v<S, R, 1>(b, st, src, dst, reservoir);
        return check_launch("k_batch_sweep");
    });
}

// ns (2, 3 or 4) batched steps on stream st: every member from state slot src to
// dst in one launch of the multi-step pass; res_a: the first step starts from
// n >= 1.
int batch_multi(lbm_vans_batch *b, hipStream_t st, int src, int dst, int res_a, int ns)
{
    return with_types(b->storage, [&](auto *sp, auto *rp) -> int {
        using S = std::remove_pointer_t<decltype(sp)>;
        using R = std::remove_pointer_t<decltype(rp)>;
        if constexpr (std::is_same_v<S, double>) {
            return fail(LBM_VANS_EINVAL, "multi-step pass needs FP32 or FP16 storage");
        } else {
            if (!b->multi_ok)
                return fail(LBM_VANS_EINVAL, "a member is too large for the multi-step pass");
            if (ns == 4 && !b->multi4_ok)
                return fail(LBM_VANS_EINVAL, "the four-step pass needs FP32 storage and members "
                            "of at least 32 rows with periodic y");
            const bool tall = ns == 3 && batch_tall(b);
            const int q = ns == 4 ? 3 : ns == 3 ? (tall ? 2 : 1) : 0;
            const int n = b->nwaves[q];
            const int grid = (n + NW - 1) / NW;
            const Member<R> *M = static_cast<const Member<R> *>(b->d_desc);
            const int *wm = b->d_wmap[q];
            with_bxwy(b->bx, b->wy, [&](auto bxc, auto wyc) {
                constexpr int BXV = decltype(bxc)::value;
                constexpr bool WYV = decltype(wyc)::value;
                auto run = [&](auto ker) {
                    hipLaunchKernelGGL(ker, dim3(grid), dim3(NTHREADS), 0, st, M, wm, n, src, dst,
                                       res_a);
                };
                if (ns == 2) {
                    run(k_batch_tb2<S, R, BXV, WYV>);
                } else if constexpr (std::is_same_v<S, float>) {
                    if (ns == 4)
                        run(k_batch_tb4<S, R, BXV, WYV>);
                    else if (tall)
                        run(k_batch_tb3<S, R, BXV, WYV, LBM_VANS_TB3_TALL32>);
                    else
                        run(k_batch_tb3<S, R, BXV, WYV, tb_rows<S, 3>()>);
                } else {
                    run(k_batch_tb3<S, R, BXV, WYV, tb_rows<S, 3>()>);
                }
            });
            return check_launch(ns == 4 ? "k_batch_tb4" : ns == 3 ? "k_batch_tb3" : "k_batch_tb2");
        }
    });
}

// Most steps one batched launch may take (as max_pass for a lone problem):
// automatically four (FP32, with at least as many waves as the chip holds of the
// batched four-step kernel), else three.
int batch_max_pass(const lbm_vans_batch *b)
{
    if (b->storage == LBM_F64 || !b->multi_ok || b->nwaves[0] == 0) return 1;
    int m = b->cfg.steps_per_pass;
    if (m == 0)
        m = b->multi4_ok && b->cfg.pass_rows == 0 && 10LL * b->nwaves[3] >= QUAD_FILL_10 * b->quad_resident
                ? 4
                : 3;
    return m == 4 && !b->multi4_ok ? 3 : m;
}

// One batched launch of m steps (the one-step sweep for m = 1).
int batch_launch(lbm_vans_batch *b, hipStream_t st, int src, int res_a, int m)
{
    return m >= 2 ? batch_multi(b, st, src, 1 - src, res_a, m)
                  : batch_sweep(b, st, src, 1 - src, res_a);
}

// Launches of a run of `steps` steps, each as many as batch_max_pass allows.
int64_t batch_launch_count(const lbm_vans_batch *b, int64_t steps)
{
    const int mp = batch_max_pass(b);
    return (steps + mp - 1) / mp;
}

int batch_adjoint(lbm_vans_batch *b, bool seed, int src, int a_next, int a, int reservoir)
{
    return with_types(b->storage, [&](auto *sp, auto *rp) -> int {
        using S = std::remove_pointer_t<decltype(sp)>;
        using R = std::remove_pointer_t<decltype(rp)>;
        const Member<R> *M = static_cast<const Member<R> *>(b->d_desc);
        if (seed)
            hipLaunchKernelGGL((k_batch_adjoint_seed<S, R>), dim3(b->ntiles_adj),
                               dim3(NTHREADS), 0, b->stream, M, (const int *)b->d_tmap_adj,
                               b->ntiles_adj, src, a, reservoir);
        else
            hipLaunchKernelGGL((k_batch_adjoint_rows<S, R>),
                               dim3((unsigned)((b->ntiles_adj + NW - 1) / NW)), dim3(NTHREADS),
                               0, b->stream, M, (const int *)b->d_tmap_adj, b->ntiles_adj, src,
                               a_next, a, reservoir);
        return check_launch("k_batch_adjoint");
    });
}

// Capture cfg.graph_steps steps starting from slot s0 (all with the
// reservoirs active, i.e. from a state n >= 1) into an executable graph.
int batch_capture(lbm_vans_batch *b, int s0)
{
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    int rc = LBM_VANS_OK;
    const int mp = batch_max_pass(b);
    int src = s0;
    for (int j = 0; j < b->cfg.graph_steps && !rc; src = 1 - src) {
        const int m = std::min(mp, b->cfg.graph_steps - j);
        rc = batch_launch(b, b->cap, src, 1, m);
        j += m;
    }
    hipError_t e = hipStreamEndCapture(b->cap, &graph);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess)
        return fail(LBM_VANS_EHIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&b->graph[s0], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        b->graph[s0] = nullptr;
        return fail(LBM_VANS_EHIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
    }
    return LBM_VANS_OK;
}

int check_config(const lbm_vans_batch *b, const lbm_vans_batch_config *c)
{
    if (!c) return fail(LBM_VANS_EINVAL, "config is NULL");
    if (c->vec < 1 || c->vec > b->vmax || (c->vec & (c->vec - 1)))
        return fail(LBM_VANS_EINVAL, "vec = %d: a power of two up to %d", c->vec, b->vmax);
    if (c->grid < 0 || c->grid % NXCD)
        return fail(LBM_VANS_EINVAL, "grid = %d: 0 or a positive multiple of %d", c->grid, NXCD);
    if (c->graph_steps < 0 || c->graph_steps % 2)
        return fail(LBM_VANS_EINVAL, "graph_steps = %d: 0 or a positive even number",
                    c->graph_steps);
    if (c->steps_per_pass < 0 || c->steps_per_pass > 4)
        return fail(LBM_VANS_EINVAL, "steps_per_pass = %d: 0 (automatic), 1, 2, 3 or 4",
                    c->steps_per_pass);
    if (c->steps_per_pass == 4 && b->storage != LBM_F32_SHIFTED)
        return fail(LBM_VANS_EINVAL, "steps_per_pass = 4 needs LBM_F32_SHIFTED storage");
    if (c->pass_rows == LBM_VANS_TB3_SHORT32 || c->pass_rows == LBM_VANS_TB3_TINY32)
        return fail(LBM_VANS_EINVAL, "pass_rows = %d: batches take %d or %d (or 0)",
                    c->pass_rows, tb_rows<float, 3>(), LBM_VANS_TB3_TALL32);
    return check_pass_rows(c->pass_rows, b->storage);
}

// The members must still be in step with each other (a member may have been
// stepped on its own in between).
int batch_in_step(const lbm_vans_batch *b)
{
    for (lbm_vans_handle *h : b->m)
        if (h->n != b->m[0]->n || h->cur != b->m[0]->cur)
            return fail(LBM_VANS_EINVAL,
                        "batch members are at different steps (%lld and %lld)",
                        (long long)h->n, (long long)b->m[0]->n);
    return LBM_VANS_OK;
}

// Account for steps taken in launches that each swap the two state slots once.
void batch_advance(lbm_vans_batch *b, int64_t steps, int64_t launches)
{
    for (lbm_vans_handle *h : b->m) {
        h->n += steps;
        if (launches & 1) h->cur = 1 - h->cur;
    }
}


}  // namespace

extern "C" {

size_t lbm_vans_batch_work_bytes(lbm_vans_handle *const *members, int32_t nmembers)
{
    if (!members || nmembers < 1) return 0;
    size_t tiles = 0, waves[4] = {0, 0, 0, 0};
    for (int32_t k = 0; k < nmembers; k++) {
        if (!members[k]) return 0;
        tiles += static_cast<size_t>(members[k]->g.ntiles);
        for (int q = 0; q < 4; q++) waves[q] += batch_waves(&members[k]->p, q);
    }
    return batch_table_bytes(members[0]->p.storage, nmembers, tiles, waves);
}

int lbm_vans_batch_create(lbm_vans_handle *const *members, int32_t nmembers, void *work,
                          size_t work_bytes, void *stream, lbm_vans_batch **out)
{
    g_last_error.clear();
    if (!out) return fail(LBM_VANS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!members || nmembers < 1) return fail(LBM_VANS_EINVAL, "no members");
    const lbm_vans_handle *h0 = members[0];
    if (!h0) return fail(LBM_VANS_EINVAL, "member 0 is NULL");
    size_t tiles = 0, waves[4] = {0, 0, 0, 0};
    for (int32_t k = 0; k < nmembers; k++) {
        const lbm_vans_handle *h = members[k];
        if (!h) return fail(LBM_VANS_EINVAL, "member %d is NULL", k);
        for (int32_t j = 0; j < k; j++)
            if (members[j] == h) return fail(LBM_VANS_EINVAL, "member %d repeats member %d", k, j);
        if (h->p.storage != h0->p.storage || h->p.bc_x != h0->p.bc_x || h->p.bc_y != h0->p.bc_y)
            return fail(LBM_VANS_EINVAL,
                        "member %d differs from member 0 in storage or boundary kinds", k);
        if (h->p.diag_every != 0)
            return fail(LBM_VANS_EINVAL, "member %d records diagnostics (diag_every = %d); "
                        "batched steps do not", k, h->p.diag_every);
        if (h->n != h0->n || h->cur != h0->cur)
            return fail(LBM_VANS_EINVAL, "member %d is at step %lld, member 0 at %lld", k,
                        (long long)h->n, (long long)h0->n);
        tiles += static_cast<size_t>(h->g.ntiles);
        for (int q = 0; q < 4; q++) waves[q] += batch_waves(&h->p, q);
    }
    if (tiles > static_cast<size_t>(INT32_MAX))
        return fail(LBM_VANS_EINVAL, "%zu tiles: too many for one launch", tiles);
    const size_t wmax = std::max({waves[0], waves[1], waves[2], waves[3]});
    if (wmax > static_cast<size_t>(INT32_MAX - NW))
        return fail(LBM_VANS_EINVAL, "%zu waves: too many for one launch", wmax);
    if (!work || reinterpret_cast<uintptr_t>(work) % 256)
        return fail(LBM_VANS_EINVAL, "work must be a 256-byte aligned device buffer");
    const size_t need = batch_table_bytes(h0->p.storage, nmembers, tiles, waves);
    if (work_bytes < need)
        return fail(LBM_VANS_EINVAL, "work has %zu bytes, %zu needed", work_bytes, need);

    lbm_vans_batch *b = new (std::nothrow) lbm_vans_batch();
    if (!b) return fail(LBM_VANS_EINVAL, "out of host memory");
    b->m.assign(members, members + nmembers);
    b->stream = static_cast<hipStream_t>(stream);
    b->storage = h0->p.storage;
    b->bx = h0->g.open_x ? 2 : (h0->g.wall_x ? 1 : 0);
    b->wy = h0->g.wall_y;
    b->vmax = b->storage == LBM_F64 ? 2 : 4;
    // every member must fit the multi-step passes' addressing and rows (in the taller
    // chunks, which the batch may choose)
    for (int32_t k = 0; k < nmembers; k++)
        b->multi_ok = b->multi_ok && multi_fits(members[k]->g) &&
                      multi_rows_ok(members[k]->p.Ly, members[k]->g.wall_y, 3,
                                    LBM_VANS_TB3_TALL32) &&
                      multi_rows_ok(members[k]->p.Ly, members[k]->g.wall_y, 2,
                                    tb2_rows_of(members[k]->p.storage));
    b->multi4_ok = b->multi_ok && b->storage == LBM_F32_SHIFTED;
    for (int32_t k = 0; k < nmembers; k++)
        b->multi4_ok = b->multi4_ok && multi_rows_ok(members[k]->p.Ly, members[k]->g.wall_y, 4,
                                                     tb_rows<float, 4>());
    const size_t dsz = b->storage == LBM_F64 ? sizeof(Member<double>) : sizeof(Member<float>);
    char *w = static_cast<char *>(work);
    b->d_desc = w;
    b->d_tmap = reinterpret_cast<int *>(w + align256(nmembers * dsz));
    b->d_tmap_adj = reinterpret_cast<int *>(w + align256(nmembers * dsz) +
                                            align256(tiles * sizeof(int)));
    size_t off = align256(nmembers * dsz) + 2 * align256(tiles * sizeof(int));
    for (int q = 0; q < 4; q++) {
        b->d_wmap[q] = reinterpret_cast<int *>(w + off);
        off += align256(waves[q] * sizeof(int));
    }
    b->cfg.vec = b->vmax;
    b->cfg.grid = 0;
    b->cfg.graph_steps = 24;
    b->cfg.steps_per_pass = 0;
    b->cfg.pass_rows = 0;
    int rc = LBM_VANS_OK;
    hipError_t e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&b->ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&b->ev[1]);
    if (e != hipSuccess) rc = fail(LBM_VANS_EHIP, "stream / event creation failed: %s",
                                   hipGetErrorString(e));
    if (!rc && b->storage == LBM_F32_SHIFTED && b->multi_ok)
        rc = tb3_resident(b->storage, b->bx, b->wy, LBM_VANS_TB3_TALL32, true, &b->tall_resident);
    if (!rc && b->multi4_ok) rc = tb4_resident(b->bx, b->wy, true, &b->quad_resident);
    if (!rc) rc = batch_upload(b, b->cfg.vec, nullptr, 0, 1);
    if (rc) {
        lbm_vans_batch_destroy(b);
        return rc;
    }
    *out = b;
    return LBM_VANS_OK;
}

int lbm_vans_batch_configure(lbm_vans_batch *b, const lbm_vans_batch_config *cfg)
{
    if (!b) return fail(LBM_VANS_EINVAL, "batch is NULL");
    int rc = check_config(b, cfg);
    if (rc) return rc;
    drop_graphs(b);
    b->cfg = *cfg;
    b->cfg.us_per_step = 0.0;
    return batch_upload(b, b->cfg.vec, nullptr, 0, 1);
}

int lbm_vans_batch_pass_plan(const lbm_vans_batch *b, int32_t *steps_per_pass,
                             int32_t *pass_rows)
{
    if (!b) return fail(LBM_VANS_EINVAL, "batch is NULL");
    const bool multi = b->storage != LBM_F64 && b->multi_ok && b->nwaves[0] > 0;
    const int m = batch_max_pass(b);
    if (steps_per_pass) *steps_per_pass = m;
    if (pass_rows)
        *pass_rows = !multi ? 0
                     : b->storage == LBM_F16_SHIFTED ? tb_rows<_Float16, 3>()
                     : m == 4 ? tb_rows<float, 4>()
                     : batch_tall(b) ? LBM_VANS_TB3_TALL32
                                     : tb_rows<float, 3>();
    return LBM_VANS_OK;
}

int lbm_vans_batch_get_config(const lbm_vans_batch *b, lbm_vans_batch_config *cfg)
{
    if (!b || !cfg) return fail(LBM_VANS_EINVAL, "batch or cfg is NULL");
    *cfg = b->cfg;
    return LBM_VANS_OK;
}

int lbm_vans_batch_tune(lbm_vans_batch *b, int32_t reps, lbm_vans_batch_config *best,
                        lbm_vans_batch_config *trials, int32_t max_trials, int32_t *n_trials)
{
    if (!b) return fail(LBM_VANS_EINVAL, "batch is NULL");
    if (reps < 1) return fail(LBM_VANS_EINVAL, "reps = %d < 1", reps);
    if (max_trials > 0 && !trials) return fail(LBM_VANS_EINVAL, "trials is NULL");
    int rc = batch_in_step(b);
    if (rc) return rc;
    int dev = 0, ncu = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const int src = b->m[0]->cur, dst = 1 - src, res = res_on(&b->m[0]->p, b->m[0]->n);
    const lbm_vans_batch_config keep = b->cfg;
    lbm_vans_batch_config top = keep;
    top.us_per_step = INFINITY;
    int nt = 0;
    drop_graphs(b);
    for (int vec = b->vmax; vec >= 1; vec /= 2) {
        rc = batch_upload(b, vec, nullptr, 0, 1);
        if (rc) return rc;
        // one block per tile, then persistent grids of 1, 2, 4 and 8 blocks per CU
        const int grids[5] = {0, ncu, 2 * ncu, 4 * ncu, 8 * ncu};
        for (int gi = 0; gi < 5; gi++) {
            const int grid = grids[gi] / NXCD * NXCD;
            if (gi > 0 && (grid < NXCD || grid >= b->ntiles)) continue;
            b->cfg.vec = vec;
            b->cfg.grid = grid;
            b->cfg.steps_per_pass = 1;
            // the state in slot src is only read, so the trials leave it unchanged
            rc = batch_sweep(b, b->stream, src, dst, res);
            if (rc) return rc;
            HIP_TRY(hipEventRecord(b->ev[0], b->stream));
            for (int r = 0; r < reps && !rc; r++) rc = batch_sweep(b, b->stream, src, dst, res);
            if (rc) return rc;
            HIP_TRY(hipEventRecord(b->ev[1], b->stream));
            HIP_TRY(hipEventSynchronize(b->ev[1]));
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, b->ev[0], b->ev[1]));
            b->cfg.us_per_step = 1000.0 * ms / reps;
            if (nt < max_trials) trials[nt] = b->cfg;
            nt++;
            if (b->cfg.us_per_step < top.us_per_step) top = b->cfg;
        }
    }
    // the multi-step passes (independent of vec and grid; the single-step shape
    // found so far is kept for the steps they leave over), timed per step
    const lbm_vans_batch_config single = top;
    const int ns_max = b->multi4_ok ? 4 : 3;
    for (int ns = 2; ns <= ns_max && b->storage != LBM_F64 && b->nwaves[0] > 0 && b->multi_ok;
         ns++) {
        rc = batch_multi(b, b->stream, src, dst, res, ns);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(b->ev[0], b->stream));
        for (int r = 0; r < reps && !rc; r++) rc = batch_multi(b, b->stream, src, dst, res, ns);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(b->ev[1], b->stream));
        HIP_TRY(hipEventSynchronize(b->ev[1]));
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, b->ev[0], b->ev[1]));
        lbm_vans_batch_config pc = single;
        pc.steps_per_pass = ns;
        pc.us_per_step = 1000.0 * ms / (static_cast<double>(ns) * reps);
        if (nt < max_trials) trials[nt] = pc;
        nt++;
        if (pc.us_per_step < top.us_per_step) top = pc;
    }
    if (n_trials) *n_trials = nt;
    top.graph_steps = keep.graph_steps;
    b->cfg = top;
    if (best) *best = top;
    return batch_upload(b, top.vec, nullptr, 0, 1);
}

int lbm_vans_batch_step(lbm_vans_batch *b, int64_t nsteps)
{
    if (!b) return fail(LBM_VANS_EINVAL, "batch is NULL");
    if (nsteps < 0) return fail(LBM_VANS_EINVAL, "nsteps = %lld < 0", (long long)nsteps);
    int rc = batch_in_step(b);
    if (rc) return rc;
    const int C = b->cfg.graph_steps;
    int64_t k = 0;
    while (k < nsteps) {
        const int cur = b->m[0]->cur;
        const int64_t n = b->m[0]->n;
        if (C > 0 && n >= 1 && nsteps - k >= C) {
            if (!b->graph[cur]) {
                rc = batch_capture(b, cur);
                if (rc) return rc;
            }
            HIP_TRY(hipGraphLaunch(b->graph[cur], b->stream));
            batch_advance(b, C, batch_launch_count(b, C));
            k += C;
        } else {
            const int m = static_cast<int>(std::min<int64_t>(batch_max_pass(b), nsteps - k));
            rc = batch_launch(b, b->stream, cur, res_on(&b->m[0]->p, n), m);
            if (rc) return rc;
            batch_advance(b, m, 1);
            k += m;
        }
    }
    return LBM_VANS_OK;
}

size_t lbm_vans_batch_grad_work_bytes(const lbm_vans_batch *b, int32_t objective,
                                      int64_t nsteps, int32_t ckpt_every)
{
    if (!b) return 0;
    size_t total = 0;
    for (const lbm_vans_handle *h : b->m) {
        if (check_grad_args(&h->p, objective, nsteps, ckpt_every)) return 0;
        total += align256(grad_layout(&h->p, nsteps, ckpt_every, false).total);
    }
    return total;
}

int lbm_vans_batch_grad(lbm_vans_batch *b, int32_t objective, int64_t nsteps,
                        int32_t ckpt_every, void *grad_work, size_t grad_work_bytes,
                        double *const *dJdeps, double *J)
{
    if (!b) return fail(LBM_VANS_EINVAL, "batch is NULL");
    for (const lbm_vans_handle *h : b->m) {
        int rc = check_grad_args(&h->p, objective, nsteps, ckpt_every);
        if (rc) return rc;
    }
    if (!grad_work || !dJdeps) return fail(LBM_VANS_EINVAL, "grad_work and dJdeps are required");
    for (size_t k = 0; k < b->m.size(); k++)
        if (!dJdeps[k]) return fail(LBM_VANS_EINVAL, "dJdeps[%zu] is NULL", k);
    if (reinterpret_cast<uintptr_t>(grad_work) % 256)
        return fail(LBM_VANS_EINVAL, "grad_work must be 256-byte aligned");
    const size_t need = lbm_vans_batch_grad_work_bytes(b, objective, nsteps, ckpt_every);
    if (grad_work_bytes < need)
        return fail(LBM_VANS_EINVAL, "grad_work has %zu bytes, %zu needed", grad_work_bytes,
                    need);
    const int K = ckpt_every;
    const int64_t nck_slots = std::max<int64_t>(1, (nsteps + K - 1) / K);
    if (nck_slots + K + 2 > INT32_MAX) return fail(LBM_VANS_EINVAL, "too many state slots");
    auto ckpt_slot = [&](int64_t c) { return static_cast<int>(2 + c); };
    auto seg_slot = [&](int64_t j) { return static_cast<int>(2 + nck_slots + j); };
    drop_graphs(b);
    int rc = batch_upload(b, b->cfg.vec, static_cast<char *>(grad_work), nsteps, ckpt_every);
    if (rc) return rc;
    std::vector<GradLayout> G;
    std::vector<char *> gw;
    size_t off = 0;
    for (lbm_vans_handle *h : b->m) {
        G.push_back(grad_layout(&h->p, nsteps, ckpt_every, false));
        gw.push_back(static_cast<char *>(grad_work) + off);
        off += align256(G.back().total);
    }
    std::vector<double> rec(b->m.size() * NRED);
    rc = with_types(b->storage, [&](auto *sp, auto *rp) -> int {
        using S = std::remove_pointer_t<decltype(sp)>;
        using R = std::remove_pointer_t<decltype(rp)>;
        // 1. every member back to its initial state; forward with checkpoints
        for (lbm_vans_handle *h : b->m) {
            const Phys<R> ph0 = make_phys<R>(&h->p);
            hipLaunchKernelGGL((k_set_state<S, R>), dim3(h->ntiles), dim3(NTHREADS), 0,
                               b->stream, (S *)h->buf[0], (const R *)h->eps, h->g, h->p.rho0,
                               static_cast<double>(ph0.rho0), h->p.u0[0], h->p.u0[1],
                               (const double *)nullptr, ph0.scale, wall6(&h->p, 0),
                               wall6(&h->p, 1));
            int r = check_launch("k_set_state");
            if (r) return r;
            h->cur = 0;
            h->n = 0;
        }
        int r;
        for (int64_t s0 = 0; s0 < nsteps || s0 == 0; s0 += K) {
            for (size_t k = 0; k < b->m.size(); k++) {
                lbm_vans_handle *h = b->m[k];
                HIP_TRY(hipMemcpyAsync(gw[k] + (s0 / K) * G[k].pop, h->buf[h->cur], G[k].pop,
                                       hipMemcpyDeviceToDevice, b->stream));
            }
            // only the checkpoints are kept, so the steps in between may go up to
            // three per launch
            for (int64_t j = 0; j < K && s0 + j < nsteps;) {
                const int cur = b->m[0]->cur;
                const int m = static_cast<int>(
                    std::min<int64_t>({(int64_t)batch_max_pass(b), K - j, nsteps - s0 - j}));
                r = batch_launch(b, b->stream, cur, res_on(&b->m[0]->p, b->m[0]->n), m);
                if (r) return r;
                batch_advance(b, m, 1);
                j += m;
            }
            if (nsteps == 0) break;
        }
        // 2. seed: J of the state nsteps and the adjoint of that state
        for (size_t k = 0; k < b->m.size(); k++) {
            double *eb = reinterpret_cast<double *>(gw[k] + G[k].states() * G[k].pop +
                                                    2 * G[k].lam);
            const long long nz = (long long)(3 * G[k].acc / sizeof(double));
            hipLaunchKernelGGL(k_zero, dim3((unsigned)((nz + NTHREADS - 1) / NTHREADS)),
                               dim3(NTHREADS), 0, b->stream, eb, nz);
            r = check_launch("k_zero");
            if (r) return r;
            if (G[k].eps64) {   // the reverse steps' FP64 copy of the porosity
                const long long npl = b->m[k]->g.plane;
                hipLaunchKernelGGL(k_widen, dim3((unsigned)((npl + NTHREADS - 1) / NTHREADS)),
                                   dim3(NTHREADS), 0, b->stream, (const float *)b->m[k]->eps,
                                   reinterpret_cast<double *>(
                                       gw[k] + G[k].states() * G[k].pop + 2 * G[k].lam +
                                       3 * G[k].acc),
                                   npl);
                r = check_launch("k_widen");
                if (r) return r;
            }
        }
        int a = 0;
        r = batch_adjoint(b, true, b->m[0]->cur, 0, a, res_on(&b->m[0]->p, nsteps));
        if (r) return r;
        for (size_t k = 0; k < b->m.size(); k++) {
            lbm_vans_handle *h = b->m[k];
            hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, b->stream,
                               (const double *)h->part, h->ntiles, (const double *)nullptr,
                               static_cast<double>(nsteps), h->scratch_rec);
            r = check_launch("k_finalize");
            if (r) return r;
            HIP_TRY(hipMemcpyAsync(rec.data() + k * NRED, h->scratch_rec, NRED * sizeof(double),
                                   hipMemcpyDeviceToHost, b->stream));
        }
        // 3. reverse, one checkpoint segment at a time (states recomputed)
        const int64_t nck = nsteps == 0 ? 0 : (nsteps + K - 1) / K;
        for (int64_t c = nck - 1; c >= 0; c--) {
            const int64_t s0 = c * K, s1 = std::min<int64_t>(s0 + K, nsteps);
            for (int64_t j = 1; j < s1 - s0; j++) {
                const int src = j == 1 ? ckpt_slot(c) : seg_slot(j - 1);
                r = batch_sweep(b, b->stream, src, seg_slot(j), res_on(&b->m[0]->p, s0 + j - 1));
                if (r) return r;
            }
            for (int64_t n = s1 - 1; n >= s0; n--) {
                const int state = n == s0 ? ckpt_slot(c) : seg_slot(n - s0);
                r = batch_adjoint(b, false, state, a, 1 - a, res_on(&b->m[0]->p, n));
                if (r) return r;
                a = 1 - a;
            }
        }
        // 4. initial state and the porosity stencil, member by member
        for (size_t k = 0; k < b->m.size(); k++) {
            lbm_vans_handle *h = b->m[k];
            char *base = gw[k] + G[k].states() * G[k].pop;
            const AdjT<S> *lam = reinterpret_cast<const AdjT<S> *>(base + a * G[k].lam);
            double *eb = reinterpret_cast<double *>(base + 2 * G[k].lam);
            double *gxb = eb + G[k].acc / sizeof(double);
            double *gyb = gxb + G[k].acc / sizeof(double);
            hipLaunchKernelGGL((k_adjoint_init<AdjT<S>>), dim3(h->ntiles), dim3(NTHREADS), 0,
                               b->stream, lam, h->g, h->p.rho0, h->p.u0[0], h->p.u0[1],
                               wall6(&h->p, 0), wall6(&h->p, 1), eb);
            r = check_launch("k_adjoint_init");
            if (r) return r;
            hipLaunchKernelGGL(k_adjoint_finish, dim3(h->ntiles), dim3(NTHREADS), 0, b->stream,
                               (const double *)eb, (const double *)gxb, (const double *)gyb,
                               h->g, dJdeps[k]);
            r = check_launch("k_adjoint_finish");
            if (r) return r;
        }
        HIP_TRY(hipStreamSynchronize(b->stream));
        return LBM_VANS_OK;
    });
    if (rc) return rc;
    for (size_t k = 0; k < b->m.size(); k++) {
        if (J) J[k] = rec[k * NRED];
        if (!std::isfinite(rec[k * NRED]))
            return fail(LBM_VANS_ENONFINITE, "objective of member %zu is not finite", k);
    }
    return LBM_VANS_OK;
}

void lbm_vans_batch_destroy(lbm_vans_batch *b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    drop_graphs(b);
    for (auto &e : b->ev)
        if (e) (void)hipEventDestroy(e);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
}

}  // extern "C"
