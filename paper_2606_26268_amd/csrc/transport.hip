// transport.hip -- explicit M1 transport step on gfx950.
//
// One Euler stage of the hyperbolic part (Sect. 2.4-2.6): boundary values
// by index mapping in the loader (periodic wrap / outflow copy), PLM van
// Leer reconstruction of (E, F) on faces with the f-preserving fix, the
// Levermore closure and signal speeds of both face states, the HLL flux with
// the optical-depth limiter, and the conservative update with the geometric
// sources of the flux equation in cylindrical / spherical coordinates.
#include <mutex>

#include "m1_internal.h"
#include "m1_device.h"

namespace m1 {

template <typename R>
struct TArgs {
    const R *U[4];
    const R *tau;
    R *out[4];
    int n[3];
    int bc[3][2];
    int ign[3];
    Metric<R> m;
    R dt, c_hat, e_floor;
    int recon, riemann;
    int limo3;                 // LimO3 slopes instead of PLM van Leer
    int special;               // some side is reflective or fixed
    R bcs[3][2][4];            // ghost state of fixed sides
    long gs_in, gs_out, gs_tau; // element strides between frequency groups
    unsigned long long *cnt;
};

// Frequency group of this block (grid y): offset the group's arrays.
template <typename R>
__device__ __forceinline__ void select_group(TArgs<R> &a)
{
    const long g = blockIdx.y;
    if (g == 0) return;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        a.U[v] += g * a.gs_in;
        a.out[v] += g * a.gs_out;
    }
    a.tau += g * a.gs_tau;
}

// index along one direction after applying the boundary condition: periodic
// wrap, mirror image (reflective), or the edge cell (outflow and fixed,
// whose ghost state is replaced by ghost_fix).  Mirror indices past the
// interior (cells no face uses, in ragged tiles) are clamped.
__device__ __forceinline__ int map_index(int t, int n, int lo, int hi)
{
    if (t < 0) {
        if (lo == M1_BC_PERIODIC) { while (t < 0) t += n; return t; }
        if (lo == M1_BC_REFLECT) return min(-1 - t, n - 1);
        return 0;
    }
    if (t >= n) {
        if (hi == M1_BC_PERIODIC) { while (t >= n) t -= n; return t; }
        if (hi == M1_BC_REFLECT) return max(2 * n - 1 - t, 0);
        return n - 1;
    }
    return t;
}

// State of a ghost cell of direction d at index t (t outside [0, n)): a
// reflective side reverses the flux component normal to it, a fixed side
// supplies its given state.  Interior indices are left alone.
template <typename R>
__device__ __forceinline__ void ghost_fix(const TArgs<R> &a, int d, int t, int n, R q[4])
{
    if (t >= 0 && t < n) return;
    const int side = t < 0 ? 0 : 1;
    const int bc = a.bc[d][side];
    if (bc == M1_BC_REFLECT) {
        if (d == 0) q[1] = -q[1];
        else if (d == 1) q[2] = -q[2];
        else q[3] = -q[3];
    } else if (bc == M1_BC_FIXED) {
#pragma unroll
        for (int v = 0; v < 4; ++v) q[v] = a.bcs[d][side][v];
    }
}

template <typename R>
__device__ __forceinline__ void load4(const TArgs<R> &a, int lin, R q[4])
{
    q[0] = a.U[0][lin];
    q[1] = a.U[1][lin];
    q[2] = a.U[2][lin];
    q[3] = a.U[3][lin];
}

// Whether the two faces of a cell along D carry the same area factor A / V:
// every Cartesian direction, the azimuthal and axial directions of the
// cylindrical grid and the azimuthal direction of the spherical grid.
template <int GEOM, int D>
constexpr bool same_area = GEOM == M1_CARTESIAN || (GEOM == M1_CYLINDRICAL && D > 0) ||
                           (GEOM == M1_SPHERICAL && D == 2);

// A_hi/V Phi_hi - A_lo/V Phi_lo of one direction.  With equal area factors
// it is formed as a (Phi_hi - Phi_lo), so that equal face fluxes (a uniform
// state) cancel exactly: the contracted a Phi_hi - a Phi_lo would leave the
// rounding error of one product behind in every cell.
template <bool SAME, typename R>
__device__ __forceinline__ R face_diff(R al, R ah, R flo, R fhi)
{
    if constexpr (SAME)
        return ah * (fhi - flo);
    else
        return ah * fhi - al * flo;
}

// Contribution of direction D to the flux divergence of the cell at index t
// along D (row base `base`, stride `stride`): reconstruct cells t-1, t, t+1
// (stencil t-2 .. t+2), take HLL fluxes at both faces of cell t and add
// A_hi/V * Phi_hi - A_lo/V * Phi_lo to acc.
template <typename R, int D, int GEOM>
__device__ __forceinline__ void direction_div(const TArgs<R> &a, int base, int stride, int t,
                                              R tr, R acc[4])
{
    const int n = a.n[D], lo = a.bc[D][0], hi = a.bc[D][1];
    R q[5][4];
    int li[5];
#pragma unroll
    for (int s = 0; s < 5; ++s) {
        li[s] = base + map_index(t - 2 + s, n, lo, hi) * stride;
        load4(a, li[s], q[s]);
        if (a.special) ghost_fix(a, D, t - 2 + s, n, q[s]);
    }
    const R *winv = a.m.winv[D], *hp = a.m.hp[D], *hm = a.m.hm[D];
    // face states: cell t-1 upper, cell t lower and upper, cell t+1 lower
    R Lm[4], Rt[4], Lt[4], Rp[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const R dA = (q[1][v] - q[0][v]) * winv[t + 1];
        const R dB = (q[2][v] - q[1][v]) * winv[t + 2];
        const R dC = (q[3][v] - q[2][v]) * winv[t + 3];
        const R dD = (q[4][v] - q[3][v]) * winv[t + 4];
        if (a.limo3) {
            // each face takes its own slope: the difference on the face side
            // is the near one
            Lm[v] = q[1][v] + limo3(dA, dB) * hp[t + 1];
            Rt[v] = q[2][v] - limo3(dC, dB) * hm[t + 2];
            Lt[v] = q[2][v] + limo3(dB, dC) * hp[t + 2];
            Rp[v] = q[3][v] - limo3(dD, dC) * hm[t + 3];
        } else {
            const R sm = vanleer(dA, dB), s0 = vanleer(dB, dC), sp = vanleer(dC, dD);
            Lm[v] = q[1][v] + sm * hp[t + 1];
            Rt[v] = q[2][v] - s0 * hm[t + 2];
            Lt[v] = q[2][v] + s0 * hp[t + 2];
            Rp[v] = q[3][v] - sp * hm[t + 3];
        }
    }
    if (a.recon == M1_RECON_FPRESERVE) {
        ffix(Lm, q[1]);
        ffix(Rt, q[2]);
        ffix(Lt, q[2]);
        ffix(Rp, q[3]);
    } else {
        face_fix(a.recon, Lm, q[1]);
        face_fix(a.recon, Rt, q[2]);
        face_fix(a.recon, Lt, q[2]);
        face_fix(a.recon, Rp, q[3]);
    }
    const R tm = a.tau[li[1]], t0 = a.tau[li[2]], tp = a.tau[li[3]];
    R flo[4], fhi[4];
    hll_flux<R, D>(Lm, Rt, R(0.5) * (tm + t0), a.c_hat, flo, a.riemann);
    hll_flux<R, D>(Lt, Rp, R(0.5) * (t0 + tp), a.c_hat, fhi, a.riemann);
    const R al = a.m.alo[D][t] * tr, ah = a.m.ahi[D][t] * tr;
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] += face_diff<same_area<GEOM, D>>(al, ah, flo[v], fhi[v]);
}

template <typename R, int D>
__device__ __forceinline__ void ignorable_div(const TArgs<R> &a, const R U[4], R tr, R acc[4])
{
    const Wave<R> w = closure_wave<R, D>(U[0], U[1], U[2], U[3]);
    const R dA = (a.m.ahi[D][0] - a.m.alo[D][0]) * tr * a.c_hat;
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] += dA * w.phi[v];
}

// U* = U - dt div(Phi) + dt c_hat S_geo(U), then E >= floor and f <= 1
// (counted), stored to the transported state.
template <typename R, int GEOM>
__device__ __forceinline__ void finish_cell(const TArgs<R> &a, const R U[4], Centre<R> cu, const R acc[4], R ir, R ct,
                                            int id)
{
    R Us[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) Us[v] = U[v] - a.dt * acc[v];

    if (GEOM != M1_CARTESIAN) {
        // geometric sources from the cell-centre pressure tensor
        // P_ij = (2 - s) E F_i F_j / |F|^2 + delta_ij (s - 1) E / 3 (Levermore:
        // (3 xi - 1) / 2 = 2 - s, (1 - xi) / 2 = (s - 1) / 3), from the cell's
        // |F|^2 and 1 / E
        const R f2 = vmin(cu.f2 * cu.ie * cu.ie, R(1));
        const R s = Num<R>::sqrt_(R(4) - R(3) * f2);
        const R iF2 = cu.f2 >= Num<R>::tiny ? Num<R>::rcp(cu.f2) : R(0);
        const R iso = (s - R(1)) * (R(1) / R(3)) * U[0];
        const R an = (R(2) - s) * U[0] * iF2;
        const R k_ = a.dt * a.c_hat * ir;
        if (GEOM == M1_CYLINDRICAL) {           // (R, phi, z)
            const R Ppp = an * U[2] * U[2] + iso, PRp = an * U[1] * U[2];
            Us[1] += k_ * Ppp;
            Us[2] -= k_ * PRp;
        } else {                                 // (r, theta, phi)
            const R Ptt = an * U[2] * U[2] + iso, Ppp = an * U[3] * U[3] + iso;
            const R Prt = an * U[1] * U[2], Prp = an * U[1] * U[3], Ptp = an * U[2] * U[3];
            Us[1] += k_ * (Ptt + Ppp);
            Us[2] += k_ * (ct * Ppp - Prt);
            Us[3] -= k_ * (Prp + ct * Ptp);
        }
    }

    // positivity floor on E, then f <= 1 at the cell centre
    const bool floored = Us[0] < a.e_floor;
    if (floored) Us[0] = a.e_floor;
    count_hits(a.cnt, 0, floored);
    const R Fn = Num<R>::sqrt_(Us[1] * Us[1] + Us[2] * Us[2] + Us[3] * Us[3]);
    const bool clipped = Fn > Us[0];
    if (clipped) {
        const R sc = Us[0] * Num<R>::rcp(Fn);
        Us[1] *= sc;
        Us[2] *= sc;
        Us[3] *= sc;
    }
    count_hits(a.cnt, 1, clipped);
#pragma unroll
    for (int v = 0; v < 4; ++v) a.out[v][id] = Us[v];
}

template <typename R, int NDIM, int GEOM>
__global__ void __launch_bounds__(256) k_transport(TArgs<R> a)
{
    select_group(a);
    const int n0 = a.n[0], n1 = a.n[1], n2 = a.n[2];
    const int N = n0 * n1 * n2;
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= N) return;
    const int i = id % n0, j = (id / n0) % n1, k = id / (n0 * n1);
    R U[4];
    load4(a, id, U);
    R acc[4] = {R(0), R(0), R(0), R(0)};

    direction_div<R, 0, GEOM>(a, id - i, 1, i, R(1), acc);
    if (NDIM >= 2) {
        const R tr = a.m.trA[1][i];
        direction_div<R, 1, GEOM>(a, id - j * n0, n0, j, tr, acc);
    } else if (a.ign[1]) {
        ignorable_div<R, 1>(a, U, a.m.trA[1][i], acc);
    }
    if (NDIM >= 3) {
        const R tr = a.m.trA[2][i] * a.m.trB[2][j];
        direction_div<R, 2, GEOM>(a, id - k * n0 * n1, n0 * n1, k, tr, acc);
    } else if (a.ign[2]) {
        ignorable_div<R, 2>(a, U, a.m.trA[2][i] * a.m.trB[2][j], acc);
    }

    finish_cell<R, GEOM>(a, U, centre_of(U), acc, GEOM == M1_CARTESIAN ? R(0) : a.m.inv_reff[i],
                         GEOM == M1_SPHERICAL ? a.m.cot_eff[j] : R(0), id);
}

// ---------------------------------------------------------------------------
// 3D tiled kernel: a block owns a TX x TY column of cells (Tile below) and
// marches along z
// over a chunk of planes.  Per plane: (1) the state with a two-cell halo in
// x and y (cross-shaped, no corners) is staged in LDS; (2) van Leer slopes
// of every cell that donates to a face of the tile are computed once per
// direction (x: columns -1 .. TX, y: rows -1 .. TY) into LDS; (3) every x
// and y face of the tile is computed once from the two donor states and
// slopes (faces of both directions in one flat pass, direction chosen at run
// time), and the z face above the plane from a per-thread register window
// of four planes and the z slopes of planes k and k+1; (4) the update.
// Each thread's slope and face assignments are the same in every plane, so
// their metric factors are loaded once, before the march.
// ---------------------------------------------------------------------------
// Tile of a block: TX x TY cells, one thread per cell, TY = 8 (256 threads)
// or 16 (512 threads).  The taller tile computes 4 % fewer halo faces and
// slopes per cell; FP32 blocks of it take 55 KB of LDS (two per CU, four
// waves per SIMD), FP64 blocks 110 KB (one per CU, the two waves per SIMD
// their registers allow anyway).  The general FP32 kernel has only the
// 32 x 8 tile: its 150 VGPRs allow three waves per SIMD only in 256-thread
// blocks.
template <int TY_>
struct Tile {
    static constexpr int TX = 32, TY = TY_, HX = TX + 4, HY = TY + 4, NT = TX * TY;
    static constexpr int NXF = TY * (TX + 1), NYF = (TY + 1) * TX, NHALO = 2 * (2 * TY + 2 * TX);
    static constexpr int NXS = TY * (TX + 2), NYS = (TY + 2) * TX;
    // Task passes of the slope and face stages: pass 0 takes x tasks
    // 0 .. NT-1, pass 1 y tasks 0 .. NT-1, pass 2 the rest of both (x first),
    // so that the first two passes run with their direction fixed at compile
    // time.
    static_assert(NXF >= NT && NYF >= NT && NXS >= NT && NYS >= NT, "tile too small for the task passes");
    static_assert(NXF + NYF <= 3 * NT && NXS + NYS <= 3 * NT, "tile too large for three task passes");
    static_assert(NHALO <= NT, "one halo cell per thread at most");
};
constexpr int NSP = 3, NFP = 3;

// task of thread tid in pass p: direction (0 = x, 1 = y) and index within
// that direction's tasks, or -1 past the last (nx, ny: task counts)
template <int NT>
__device__ __forceinline__ int task_of(int p, int tid, int nx, int ny, int &dir)
{
    dir = p == 1 ? 1 : 0;
    if (p < 2) return tid;
    if (tid < nx - NT) return NT + tid;
    dir = 1;
    return tid - (nx - NT) < ny - NT ? NT + tid - (nx - NT) : -1;
}

// FP32 instantiations ask for at least four (default) and three (general)
// waves per SIMD (the second argument of the bound), i.e. at most 128 and
// 168 VGPRs: the general one just exceeds its bound otherwise, the default
// one fits exactly.
// LIMO3 (general kernel only): each donor cell keeps two slopes per
// direction, one for its lower and one for its upper face, and takes the
// 32 x 8 tile in FP64 (the 512-thread block spilled).  FP32 fits three
// waves per SIMD.  FP64 asks for two waves per SIMD: the compiler then
// keeps the kernel within 256 registers by spilling 14-22 of them to
// scratch, and it runs 31 % faster than unbounded at 256 VGPRs plus
// accumulation registers, one wave per SIMD (0.276 against 0.398 ms per
// launch on the 192x96x192 grid).
template <typename R, int GEOM, bool GENERAL, int TYB, bool LIMO3 = false>
__global__ void __launch_bounds__((Tile<TYB>::NT),
                                  (sizeof(R) == 4 ? (GENERAL ? 3 : 4) : (LIMO3 ? 2 : 1)))
    k_transport3d(TArgs<R> a, int nz_chunk, int tiles_x, int tiles_y, int nblocks, int cus)
{
    using T = Tile<TYB>;
    constexpr int TX = T::TX, TY = T::TY, HX = T::HX, HY = T::HY, NT = T::NT;
    constexpr int NXF = T::NXF, NYF = T::NYF, NHALO = T::NHALO, NXS = T::NXS, NYS = T::NYS;
    select_group(a);
    // the default scheme (f-preserving fix + HLL, periodic / outflow sides)
    // is compiled without the variant and ghost-state code
    const int recon = GENERAL ? a.recon : int(M1_RECON_FPRESERVE);
    const int riemann = GENERAL ? a.riemann : int(M1_RIEMANN_HLL);
    __shared__ R sq[4][HY][HX];
    __shared__ R st[HY][HX];
    __shared__ R scf[2][HY][HX];        // |F|^2 and 1 / E of the staged cells
    static_assert(GENERAL || !LIMO3, "LimO3 only in the general kernel");
    __shared__ R ss[4][NXS + NYS];      // slopes: x tasks, then y tasks (LimO3: upper-face slopes)
    __shared__ R ssl[LIMO3 ? 4 : 1][LIMO3 ? NXS + NYS : 1];   // LimO3: lower-face slopes
    __shared__ R sfx[4][TY][TX + 1];
    __shared__ R sfy[4][TY + 1][TX];
    R *const sqf = &sq[0][0][0];
    const R *const stf = &st[0][0];
    const R *const scf2 = &scf[0][0][0], *const scie = &scf[1][0][0];
    constexpr int QS = HY * HX;

    // consecutive logical tiles share an XCD (blocks are dealt to XCDs round-robin)
    const int per = (nblocks + 7) / 8;
    const int L = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (L >= nblocks) return;
    const int n0 = a.n[0], n1 = a.n[1], n2 = a.n[2];
    const int tx_i = L % tiles_x, rest = L / tiles_x;
    const int x0 = tx_i * TX, y0 = (rest % tiles_y) * TY, z0 = (rest / tiles_y) * nz_chunk;
    const int z1 = min(z0 + nz_chunk, n2);
    const int tid = threadIdx.x, lx = tid % TX, ly = tid / TX;
    const int i = x0 + lx, j = y0 + ly;
    const bool live = i < n0 && j < n1;
    const int mi = map_index(i, n0, a.bc[0][0], a.bc[0][1]);
    const int mj = map_index(j, n1, a.bc[1][0], a.bc[1][1]);
    const int plane = n0 * n1;
    const int col = mj * n0 + mi;

    // halo cell of this thread (tid < NHALO): cross-shaped, no corners
    int hx = 0, hy = 0, hcol = 0;
    if (tid < NHALO) {
        if (tid < 2 * TX) { hy = tid / TX; hx = 2 + tid % TX; }
        else if (tid < 4 * TX) { hy = TY + 2 + (tid - 2 * TX) / TX; hx = 2 + (tid - 2 * TX) % TX; }
        else if (tid < 4 * TX + 2 * TY) { hx = (tid - 4 * TX) / TY; hy = 2 + (tid - 4 * TX) % TY; }
        else { hx = TX + 2 + (tid - 4 * TX - 2 * TY) / TY; hy = 2 + (tid - 4 * TX - 2 * TY) % TY; }
        const int gi = map_index(x0 - 2 + hx, n0, a.bc[0][0], a.bc[0][1]);
        const int gj = map_index(y0 - 2 + hy, n1, a.bc[1][0], a.bc[1][1]);
        hcol = gj * n0 + gi;
    }
    // ghost transformation of a state in this thread's column (x, y ghosts)
    // and in plane kk (z ghosts); halo cells are ghosts in x or y only
    auto fix_col = [&](int kk, R q[4]) {
        if (!GENERAL || !a.special) return;
        ghost_fix(a, 0, i, n0, q);
        ghost_fix(a, 1, j, n1, q);
        ghost_fix(a, 2, kk, n2, q);
    };
    auto fix_halo = [&](R q[4]) {
        if (!GENERAL || !a.special) return;
        ghost_fix(a, 0, x0 - 2 + hx, n0, q);
        ghost_fix(a, 1, y0 - 2 + hy, n1, q);
    };

    // slope tasks: centre cell in sq (flat), neighbour stride, inverse spacings.
    // Cells past the last ghost (m > n) feed no face and are skipped.
    int s_ctr[NSP], s_str[NSP], s_slot[NSP];
    R s_wl[NSP], s_wr[NSP];
    bool s_on[NSP];
#pragma unroll
    for (int p = 0; p < NSP; ++p) {
        int dir;
        const int q = task_of<NT>(p, tid, NXS, NYS, dir);
        s_on[p] = false;
        s_ctr[p] = 2 * HX + 2;
        s_str[p] = 1;
        s_wl[p] = s_wr[p] = R(0);
        if (q >= 0 && dir == 0) {
            const int r = q / (TX + 2), c = q % (TX + 2), m = x0 + c - 1;
            if (m <= n0) {
                s_on[p] = true;
                s_ctr[p] = (r + 2) * HX + c + 1;
                s_wl[p] = a.m.winv[0][m + 2];
                s_wr[p] = a.m.winv[0][m + 3];
            }
        } else if (q >= 0) {
            const int qq = q, r = qq / TX, c = qq % TX, m = y0 + r - 1;
            if (m <= n1) {
                s_on[p] = true;
                s_ctr[p] = (r + 1) * HX + c + 2;
                s_str[p] = HX;
                s_wl[p] = a.m.winv[1][m + 2];
                s_wr[p] = a.m.winv[1][m + 3];
            }
        }
        s_slot[p] = dir == 0 ? q : NXS + q;
    }
    // face tasks: direction, left donor in sq, its slope in ss, flux slot,
    // centre-to-face offsets of the two donors
    int f_d[NFP], f_b[NFP], f_sb[NFP], f_o[NFP];
    R f_hp[NFP], f_hm[NFP];
    bool f_on[NFP];
#pragma unroll
    for (int p = 0; p < NFP; ++p) {
        int dir;
        const int q = task_of<NT>(p, tid, NXF, NYF, dir);
        f_on[p] = false;
        f_d[p] = 0;
        f_b[p] = f_sb[p] = f_o[p] = 0;
        f_hp[p] = f_hm[p] = R(0);
        if (q >= 0 && dir == 0) {
            const int row = q / (TX + 1), fo = q % (TX + 1), g = x0 + fo;
            if (g <= n0 && y0 + row < n1) {
                f_on[p] = true;
                f_b[p] = (row + 2) * HX + fo + 1;
                f_sb[p] = row * (TX + 2) + fo;
                f_o[p] = row * (TX + 1) + fo;
                f_hp[p] = a.m.hp[0][g + 1];
                f_hm[p] = a.m.hm[0][g + 2];
            }
        } else if (q >= 0) {
            const int qq = q, go = qq / TX, cl = qq % TX, g = y0 + go;
            if (g <= n1 && x0 + cl < n0) {
                f_on[p] = true;
                f_d[p] = 1;
                f_b[p] = (go + 1) * HX + cl + 2;
                f_sb[p] = NXS + go * TX + cl;
                f_o[p] = go * TX + cl;
                f_hp[p] = a.m.hp[1][g + 1];
                f_hm[p] = a.m.hm[1][g + 2];
            }
        }
    }
    // update factors of the thread's column
    R axl = R(0), axh = R(0), ayl = R(0), ayh = R(0), tr2 = R(0), ir = R(0), ct = R(0);
    if (live) {
        axl = a.m.alo[0][i];
        axh = a.m.ahi[0][i];
        const R tr1 = a.m.trA[1][i];
        ayl = a.m.alo[1][j] * tr1;
        ayh = a.m.ahi[1][j] * tr1;
        tr2 = a.m.trA[2][i] * a.m.trB[2][j];
        if (GEOM != M1_CARTESIAN) ir = a.m.inv_reff[i];
        if (GEOM == M1_SPHERICAL) ct = a.m.cot_eff[j];
    }

    const int bz0 = a.bc[2][0], bz1 = a.bc[2][1];
    auto zlin = [&](int kk, int c) { return map_index(kk, n2, bz0, bz1) * plane + c; };
    const R *wz = a.m.winv[2], *hpz = a.m.hp[2], *hmz = a.m.hm[2];

    // register window of the thread's column: planes k-1 .. k+2, z slope of
    // plane k.  Plane k+2 is loaded at the top of iteration k and first used
    // after the x/y slopes (LATE): the neighbouring tiles read a plane's
    // edge lines as their halo two planes after it was loaded, and those
    // lines are still in L2.  Loaded a plane earlier (k+3 in iteration k),
    // the halo read came three planes later and often missed: on the
    // 192x96x192 grid the kernel fetched 136 MB per launch instead of
    // 99 MB, and ran 1-2 % slower.  The general FP64 kernels, at the edge
    // of the register file, keep the earlier load (the late one spills).
    constexpr bool LATE = !(GENERAL && sizeof(R) == 8);
    R W[4][4], T1, T2, Fzlo[4], Fzhi[4], Sz0[4];
    Centre<R> C1;                       // f-fix quantities of plane k (W[1])
    {
        R Q0[4], Szm[4];
        load4(a, zlin(z0 - 2, col), Q0);
        load4(a, zlin(z0 - 1, col), W[0]);
        load4(a, zlin(z0, col), W[1]);
        load4(a, zlin(z0 + 1, col), W[2]);
        if constexpr (!LATE) load4(a, zlin(z0 + 2, col), W[3]);
        fix_col(z0 - 2, Q0);
        fix_col(z0 - 1, W[0]);
        fix_col(z0, W[1]);
        fix_col(z0 + 1, W[2]);
        if constexpr (!LATE) fix_col(z0 + 2, W[3]);
        const R Tm = a.tau[zlin(z0 - 1, col)];
        T1 = a.tau[zlin(z0, col)];
        if constexpr (!LATE) T2 = a.tau[zlin(z0 + 1, col)];
        C1 = centre_of(W[1]);
        if constexpr (LIMO3) {
            // the face below plane z0 takes the upper-face slope of plane
            // z0 - 1 and the lower-face slope of plane z0; Sz0 carries the
            // upper-face slope of the current plane
            R lo_m[4], lo_0[4];
            limo3_slopes4(Q0, W[0], W[1], wz[z0 + 1], wz[z0 + 2], lo_m, Szm);
            limo3_slopes4(W[0], W[1], W[2], wz[z0 + 2], wz[z0 + 3], lo_0, Sz0);
            face_flux_s<R>(2, W[0], W[1], Szm, lo_0, centre_of(W[0]), C1, hpz[z0 + 1], hmz[z0 + 2], Tm, T1,
                           a.c_hat, Fzlo, recon, riemann);
        } else {
            slopes4(Q0, W[0], W[1], wz[z0 + 1], wz[z0 + 2], Szm);
            slopes4(W[0], W[1], W[2], wz[z0 + 2], wz[z0 + 3], Sz0);
            face_flux_s<R>(2, W[0], W[1], Szm, Sz0, centre_of(W[0]), C1, hpz[z0 + 1], hmz[z0 + 2], Tm, T1,
                           a.c_hat, Fzlo, recon, riemann);
        }
    }

    // Default kernels: blocks b and b + cus share a compute unit (each XCD
    // hands out its blocks in order, one per compute unit before the
    // second), and the wave arbiter favours the older block: left alone, the
    // first block on a unit finished its chunk in 70 % of the second's time
    // (FP32, measured on the 192x96x192 grid), and the second then ran alone
    // at half occupancy.  The two alternate their wave priority every plane
    // and stay level (FP32: 3-4 % faster transport with one round of blocks,
    // 1 % with several; FP64, two 32 x 8 blocks per unit: 1-1.5 %).  The
    // general kernels run other block counts per unit; for them the
    // alternation did not pay (1-6 % slower).
    constexpr bool ALTERNATE = !GENERAL;
    const int prio_grp = (int(blockIdx.x) / cus) & 1;
    for (int k = z0; k < z1; ++k) {
        if constexpr (ALTERNATE) {
            if (((k - z0) ^ prio_grp) & 1)
                __builtin_amdgcn_s_setprio(1);
            else
                __builtin_amdgcn_s_setprio(0);
        }
        // the plane entering the window (LATE: k+2 now, else k+3 for the
        // next iteration) and this plane's halo
        R Qn[4], Tn = R(0);
        if constexpr (LATE) {
            load4(a, zlin(k + 2, col), W[3]);
            fix_col(k + 2, W[3]);
            T2 = a.tau[zlin(k + 1, col)];
        } else {
            load4(a, zlin(k + 3, col), Qn);
            fix_col(k + 3, Qn);
            Tn = a.tau[zlin(k + 2, col)];
        }
        R Hq[4], Ht = R(0);
        if (tid < NHALO) {
            load4(a, k * plane + hcol, Hq);
            fix_halo(Hq);
            Ht = a.tau[k * plane + hcol];
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) sq[v][ly + 2][lx + 2] = W[1][v];
        st[ly + 2][lx + 2] = T1;
        scf[0][ly + 2][lx + 2] = C1.f2;
        scf[1][ly + 2][lx + 2] = C1.ie;
        if (tid < NHALO) {
#pragma unroll
            for (int v = 0; v < 4; ++v) sq[v][hy][hx] = Hq[v];
            st[hy][hx] = Ht;
            const Centre<R> ch = centre_of(Hq);
            scf[0][hy][hx] = ch.f2;
            scf[1][hy][hx] = ch.ie;
        }
        __syncthreads();

        // slopes of the x and y donor cells
#pragma unroll
        for (int p = 0; p < NSP; ++p) {
            if (!s_on[p]) continue;
            R qm[4], q0[4], qp[4], sl[4];
            const int str = p == 0 ? 1 : (p == 1 ? HX : s_str[p]);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                qm[v] = sqf[v * QS + s_ctr[p] - str];
                q0[v] = sqf[v * QS + s_ctr[p]];
                qp[v] = sqf[v * QS + s_ctr[p] + str];
            }
            if constexpr (LIMO3) {
                R lo[4];
                limo3_slopes4(qm, q0, qp, s_wl[p], s_wr[p], lo, sl);
#pragma unroll
                for (int v = 0; v < 4; ++v) ssl[v][s_slot[p]] = lo[v];
            } else {
                slopes4(qm, q0, qp, s_wl[p], s_wr[p], sl);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) ss[v][s_slot[p]] = sl[v];
        }
        // z slope(s) of plane k+1 (LimO3: Sz1 its upper-face slope, Sz1l
        // its lower-face one)
        R Sz1[4], Sz1l[4];
        if constexpr (LIMO3)
            limo3_slopes4(W[1], W[2], W[3], wz[k + 3], wz[k + 4], Sz1l, Sz1);
        else
            slopes4(W[1], W[2], W[3], wz[k + 3], wz[k + 4], Sz1);
        __syncthreads();

        // x faces (left face of column f) and y faces (lower face of row g)
#pragma unroll
        for (int p = 0; p < NFP; ++p) {
            if (!f_on[p]) continue;
            const int d = p < 2 ? p : f_d[p], b = f_b[p], sb = f_sb[p];
            const int qst = d ? HX : 1, sst = d ? TX : 1;
            R qb[4], qc[4], slb[4], slc[4], fl[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                qb[v] = sqf[v * QS + b];
                qc[v] = sqf[v * QS + b + qst];
                slb[v] = ss[v][sb];
                slc[v] = LIMO3 ? ssl[v][sb + sst] : ss[v][sb + sst];
            }
            face_flux_s<R>(d, qb, qc, slb, slc, Centre<R>{scf2[b], scie[b]}, Centre<R>{scf2[b + qst], scie[b + qst]},
                           f_hp[p], f_hm[p], stf[b], stf[b + qst], a.c_hat, fl, recon, riemann);
            R *dst = d ? &sfy[0][0][0] : &sfx[0][0][0];
            const int fs = d ? (TY + 1) * TX : TY * (TX + 1);
#pragma unroll
            for (int v = 0; v < 4; ++v) dst[v * fs + f_o[p]] = fl[v];
        }
        // z face above the plane from the register window
        const Centre<R> C2 = centre_of(W[2]);
        face_flux_s<R>(2, W[1], W[2], Sz0, LIMO3 ? Sz1l : Sz1, C1, C2, hpz[k + 2], hmz[k + 3], T1, T2, a.c_hat,
                       Fzhi, recon, riemann);
        __syncthreads();

        if (live) {
            R acc[4];
            const R azl = a.m.alo[2][k] * tr2, azh = a.m.ahi[2][k] * tr2;
#pragma unroll
            for (int v = 0; v < 4; ++v)
                acc[v] = face_diff<same_area<GEOM, 0>>(axl, axh, sfx[v][ly][lx], sfx[v][ly][lx + 1]) +
                         face_diff<same_area<GEOM, 1>>(ayl, ayh, sfy[v][ly][lx], sfy[v][ly + 1][lx]) +
                         face_diff<same_area<GEOM, 2>>(azl, azh, Fzlo[v], Fzhi[v]);
            finish_cell<R, GEOM>(a, W[1], C1, acc, ir, ct, (k * n1 + j) * n0 + i);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            Fzlo[v] = Fzhi[v];
            Sz0[v] = Sz1[v];
            W[0][v] = W[1][v];
            W[1][v] = W[2][v];
            W[2][v] = W[3][v];
            if constexpr (!LATE) W[3][v] = Qn[v];
        }
        T1 = T2;
        if constexpr (!LATE) T2 = Tn;
        C1 = C2;
    }
}

// Blocks of a kernel the whole device holds at once (occupancy per compute
// unit times the compute units), cached per kernel and device in a fixed
// table (no heap allocation on any launch path; a full table just stops
// caching).
static int resident_blocks(const void *kern, int block)
{
    struct Entry {
        const void *kern;
        int dev, block, blocks;
    };
    static std::mutex mu;
    static Entry cache[256];
    static int used = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1024;
    std::lock_guard<std::mutex> lock(mu);
    for (int e = 0; e < used; ++e)
        if (cache[e].kern == kern && cache[e].dev == dev && cache[e].block == block) return cache[e].blocks;
    int cus = 0, per = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, block, 0) != hipSuccess || per < 1) per = 1;
    if (used < 256) cache[used++] = Entry{kern, dev, block, per * cus};
    return per * cus;
}

// Tiled 3D launch.  The planes per block (z chunk) minimise rounds x
// (planes + 1): blocks run in rounds of the resident block count, and each
// chunk also pays about one plane of start-up (its first z face and slopes),
// so a chunk that fills the last round evenly beats one that leaves a
// mostly idle tail.  Chunks are kept to at most 16 planes: measured over the
// 128^3, 256^3, 192x96x192 and eight-group workloads (chunks of 4 to 64
// planes), the 28-64-plane chunks this cost picks without the cap were 4-6 %
// slower than 16 (fewer blocks to balance, more halo misses in L2); with the
// cap it lands on the fastest chunk measured or within 3 % of it.
// Launch with tile height TYB; with max_rounds > 0, only if the launch then
// takes at most that many rounds of resident blocks (returns whether it
// launched).
template <typename R, int GEOM, bool GENERAL, int TYB, bool LIMO3 = false>
static bool launch_tile(m1_ctx *c, const TArgs<R> &a, unsigned ngrp, long max_rounds)
{
    using T = Tile<TYB>;
    constexpr int TX = T::TX, TY = T::TY, NT = T::NT;
    const int tiles_x = (c->n[0] + TX - 1) / TX, tiles_y = (c->n[1] + TY - 1) / TY;
    const long slots =
        resident_blocks(reinterpret_cast<const void *>(&k_transport3d<R, GEOM, GENERAL, TYB, LIMO3>), NT);
    int nz = 8;
    double best = 1e300;
    long rounds = 1;
    for (int z = 2; z <= 16; ++z) {
        const long nb = long(tiles_x) * tiles_y * ((c->n[2] + z - 1) / z) * ngrp;
        const long r = (nb + slots - 1) / slots;
        const double cost = double(r) * (z + 1);
        if (cost < best) {
            best = cost;
            nz = z;
            rounds = r;
        }
    }
    if (max_rounds > 0 && rounds > max_rounds) return false;
    const int nblocks = tiles_x * tiles_y * ((c->n[2] + nz - 1) / nz);
    const int launched = ((nblocks + 7) / 8) * 8;
    hipLaunchKernelGGL((k_transport3d<R, GEOM, GENERAL, TYB, LIMO3>), dim3(launched, ngrp), dim3(NT), 0, c->stream, a, nz,
                       tiles_x, tiles_y, nblocks, c->cus);
    return true;
}

// Default FP32 kernel: the 32 x 16 tile where its launch takes at most two
// rounds of resident blocks (the 192x96x192 and 128^3 grids: 1.5 % faster
// transport than 32 x 8), else 32 x 8 (on the 256^3 grid and eight groups
// at 128^3, launches of four to sixteen rounds, the taller blocks were
// 2-4 % slower).  FP64 takes 32 x 8 everywhere: two of its blocks share a
// compute unit and alternate priority (1-1.5 % faster than one 32 x 16
// block per unit, which was 2 % faster than 32 x 8 without alternation).
template <typename R, int GEOM, bool GENERAL, bool LIMO3 = false>
static void launch_tiled(m1_ctx *c, const TArgs<R> &a, unsigned ngrp)
{
    if constexpr (sizeof(R) == 4 && !GENERAL && !LIMO3) {
        if (launch_tile<R, GEOM, GENERAL, 16, LIMO3>(c, a, ngrp, 2)) return;
    }
    launch_tile<R, GEOM, GENERAL, 8, LIMO3>(c, a, ngrp, 0);
}

// One transport launch for every frequency group (grid y = group; one group
// for gray states): the caller's group arrays start at g n0 n1 n2, the
// scratch arrays are laid out per group (transported fields 4 g + v,
// optical depth of group g).
template <typename R>
static hipError_t launch_t(m1_ctx *c, double dt, const Metric<R> &met, const void *const rad[4] = nullptr)
{
    TArgs<R> a;
    const long N = long(c->n[0]) * c->n[1] * c->n[2];
    const unsigned ngrp = unsigned(c->grp.m);
    for (int v = 0; v < 4; ++v) a.out[v] = static_cast<R *>(c->star[v]);
    const void *src[4] = {c->f.E, c->f.Fx, c->f.Fy, c->f.Fz};
    for (int v = 0; v < 4; ++v) a.U[v] = static_cast<const R *>(rad ? rad[v] : src[v]);
    a.tau = static_cast<const R *>(c->tau);
    a.gs_in = N;
    a.gs_out = long(4 * c->plane_bytes / sizeof(R));
    a.gs_tau = long(c->plane_bytes / sizeof(R));
    for (int d = 0; d < 3; ++d) {
        a.n[d] = c->n[d];
        a.bc[d][0] = c->bc[d][0];
        a.bc[d][1] = c->bc[d][1];
        a.ign[d] = c->ign[d];
    }
    a.m = met;
    a.dt = R(dt);
    a.c_hat = R(c->c_hat);
    a.e_floor = R(c->par.e_floor);
    a.recon = c->par.recon;
    a.riemann = c->par.riemann;
    a.limo3 = c->par.limiter == M1_LIMITER_LIMO3;
    a.special = 0;
    for (int d = 0; d < 3; ++d)
        for (int sd = 0; sd < 2; ++sd) {
            if (c->bc[d][sd] == M1_BC_REFLECT || c->bc[d][sd] == M1_BC_FIXED) a.special = 1;
            for (int v = 0; v < 4; ++v) a.bcs[d][sd][v] = R(c->bc_state[d][sd][v]);
        }
    a.cnt = c->cnt;
    if (c->ndim == 3) {
        const bool var = c->par.recon != M1_RECON_FPRESERVE || c->par.riemann != M1_RIEMANN_HLL || a.special;
#define M1_T3D(GM, V, L) launch_tiled<R, GM, V, L>(c, a, ngrp)
#define M1_T3D_ANY(GM)                  \
    if (a.limo3) M1_T3D(GM, true, true);  \
    else if (var) M1_T3D(GM, true, false); \
    else M1_T3D(GM, false, false)
        switch (c->geom) {
        case M1_CARTESIAN: M1_T3D_ANY(M1_CARTESIAN); break;
        case M1_CYLINDRICAL: M1_T3D_ANY(M1_CYLINDRICAL); break;
        default: M1_T3D_ANY(M1_SPHERICAL); break;
        }
#undef M1_T3D_ANY
#undef M1_T3D
        return hipGetLastError();
    }
    dim3 block(256), grid(unsigned((N + 255) / 256), ngrp);
#define M1_LAUNCH(ND, G) \
    hipLaunchKernelGGL((k_transport<R, ND, G>), grid, block, 0, c->stream, a)
#define M1_GEOMS(ND)                                                      \
    switch (c->geom) {                                                    \
    case M1_CARTESIAN: M1_LAUNCH(ND, M1_CARTESIAN); break;                \
    case M1_CYLINDRICAL: M1_LAUNCH(ND, M1_CYLINDRICAL); break;            \
    default: M1_LAUNCH(ND, M1_SPHERICAL); break;                          \
    }
    if (c->ndim == 1) {
        M1_GEOMS(1);
    } else {
        M1_GEOMS(2);
    }
#undef M1_GEOMS
#undef M1_LAUNCH
    return hipGetLastError();
}

hipError_t launch_transport(m1_ctx *c, double dt)
{
    if (c->par.precision == M1_F32) return launch_t<float>(c, dt, c->met32);
    return launch_t<double>(c, dt, c->met64);
}

// transport of a state held elsewhere (the second-order step's U1)
hipError_t launch_transport_from(m1_ctx *c, double dt, const void *const rad[4])
{
    if (c->par.precision == M1_F32) return launch_t<float>(c, dt, c->met32, rad);
    return launch_t<double>(c, dt, c->met64, rad);
}

} // namespace m1
