// Kernels of the step.  Every kernel is a Body with an argument struct and a
// run(args, local block, thread) function; k_one launches it for one box,
// k_many for many boxes at once (the block -> box map is a prefix table of
// per-box block counts), so a box computes bit for bit the same alone or
// batched with others.  Included by mhd.hip only.
#pragma once

#include "mhd_math.hpp"

#include <type_traits>

namespace mhd {

struct StepArgs {
    double dt_val;          // explicit step, or
    const double* dt_dev;   // device-resident CFL step when non-null
    double gamma;
    double h;               // 1 / nx
    double theta;
    double cfl_tol;         // relative slack of the dt <= CFL-bound check
    int ion;                // ionisation network: per-cell gamma_eff (primitive slot 8)
};

__device__ __forceinline__ double step_dt(const StepArgs& a)
{
    return a.dt_dev ? *a.dt_dev : a.dt_val;
}

struct RK { double a, b; };

// ---------------------------------------------------------------- launch wrappers

// Workgroups are dealt to the 8 XCDs round robin (workgroup b runs on XCD
// b % 8) and each XCD has its own L2.  This bijection gives every XCD one
// contiguous range of logical blocks, so stencil neighbours in the next row
// or plane are read through the same L2.
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    constexpr int X = 8;
    int q = nb / X, r = nb % X, x = b % X, i = b / X;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// XCD bands: a launch whose logical blocks are L = (s * nb + y) * ni + i
// (i < ni fastest, then y < nb, then s) deals y in eight contiguous bands, one
// per XCD, over every s: at any moment the eight XCDs work on the same s at
// bands nb / 8 apart, and the neighbours at y +- 1 and s + 1 of a block mostly
// ran on its own XCD shortly before or after it, so their reads hit its L2
// (a single contiguous range per XCD makes the XCDs stream from places far
// apart in memory at once, which was slower).  Identity unless 8 divides nb
// and the grid holds exactly ni * nb * ns blocks (a multi-box launch holds
// more, a resident one fewer); a bijection of [0, ni * nb * ns) either way,
// so the caller's logical blocks must be exactly that range.
__device__ __forceinline__ int xcd_band(int b, int ni, int nb, int ns)
{
    if (nb % 8 != 0 || (int)gridDim.x != ni * nb * ns) return b;
    const int per = ni * (nb / 8);   // blocks of one band and one s
    const int x = b % 8, q = b / 8;
    const int s = q / per, l = q - s * per;
    return (s * nb + x * (nb / 8) + l / ni) * ni + l % ni;
}

// kernels whose stencil spans neighbouring rows of other blocks opt in with
// `static constexpr bool XCD = true`
template <class Body>
__device__ __forceinline__ int logical_block()
{
    return Body::XCD ? xcd_block((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
}

// Cell column (i, j) and z segment of a thread of a z-marching kernel: blocks
// cover tx x ty tiles of the x-y plane, x fastest, then the segments, so the
// y-neighbour rows a thread reads are mostly rows of its own block.  False
// for the idle threads of ragged tiles.
struct ZTile {
    int tx, ty;     // tile shape; tx * ty <= block size
    int ntx, nty;   // tiles per plane along x and y
    int seg;        // z cells per thread
};

__device__ __forceinline__ bool ztile_cell(const Geo& g, const ZTile& z, int blk, int tid, int& i, int& j, int& k0,
                                           int& k1)
{
    int ly = tid / z.tx;
    int lx = tid - ly * z.tx;
    int bx = blk % z.ntx;
    int rest = blk / z.ntx;
    int by = rest % z.nty;
    int sg = rest / z.nty;
    i = bx * z.tx + lx;
    j = by * z.ty + ly;
    k0 = sg * z.seg;
    k1 = min(k0 + z.seg, g.nz);
    return ly < z.ty && i < g.nx && j < g.ny && k0 < g.nz;
}

// occupancy floor: a body may ask for at least MINW waves per SIMD (the
// compiler then caps its registers); default 1
template <class Body, class = void> struct MinWaves { static constexpr int v = 1; };
template <class Body> struct MinWaves<Body, std::void_t<decltype(Body::MINW)>> { static constexpr int v = Body::MINW; };

template <class Body>
__global__ __launch_bounds__(Body::NT) __attribute__((amdgpu_waves_per_eu(MinWaves<Body>::v))) void k_one(typename Body::Args a)
{
    Body::run(a, logical_block<Body>(), (int)threadIdx.x);
}

template <class Body>
__global__ __launch_bounds__(Body::NT) __attribute__((amdgpu_waves_per_eu(MinWaves<Body>::v))) void k_many(const typename Body::Args* __restrict__ tab,
                                                   const int* __restrict__ bstart, int nbox)
{
    int blk = logical_block<Body>();
    int lo = 0, hi = nbox - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (bstart[mid] <= blk) lo = mid;
        else hi = mid - 1;
    }
    const typename Body::Args a = tab[lo];
    Body::run(a, blk - bstart[lo], (int)threadIdx.x);
}

// bodies that opt out of the resident form with `static constexpr bool
// PERSIST = false` keep one workgroup per tile in persistent mode
template <class Body, class = void> struct Persists { static constexpr bool v = true; };
template <class Body> struct Persists<Body, std::void_t<decltype(Body::PERSIST)>> { static constexpr bool v = Body::PERSIST; };

// The same tile list worked through by a grid that stays resident (sized by
// the host to what the chip holds at once): each workgroup claims the next
// `chunk` untaken tiles from the launch's counter (zero at launch) until none
// is left, so the tiles are balanced over the workgroups as they finish, as
// the hardware dispatcher balances one workgroup per tile; claiming several
// tiles at once keeps the traffic on the one counter low when tiles are many
// and small.  The counter only grows, so a workgroup's tiles come in
// increasing order and the search for the tile's box starts at the previous
// one.  The block waits at the end of each tile before the next one reuses
// the LDS (and before the claim slot is rewritten); every body reaches its
// own barriers with all of its waves, so the barrier counts match.
template <class Body>
__global__ __launch_bounds__(Body::NT) __attribute__((amdgpu_waves_per_eu(MinWaves<Body>::v))) void k_persist(const typename Body::Args* __restrict__ tab,
                                                   const int* __restrict__ bstart, int nbox, int total, int chunk,
                                                   int* next)
{
    __shared__ int taken;
    int box = 0;
    for (;;) {
        if (threadIdx.x == 0) taken = atomicAdd(next, chunk);
        __syncthreads();
        const int c0 = taken;
        if (c0 >= total) break;
        const int c1 = min(c0 + chunk, total);
        for (int blk = c0; blk < c1; blk++) {
            int hi = nbox - 1;
            while (box < hi) {
                int mid = (box + hi + 1) >> 1;
                if (bstart[mid] <= blk) box = mid;
                else hi = mid - 1;
            }
            const typename Body::Args a = tab[box];
            Body::run(a, blk - bstart[box], (int)threadIdx.x);
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------- NONADV: primitive recovery

// Primitive variables (Sec. 2: v = m / rho, p = (gamma - 1) e; the cell-centre
// field averages the cell's two faces) are formed where the NONADV face
// kernels read them, from the conserved state, so no primitive array passes
// through memory.  For faces along D a cell contributes the six parabola
// variables (vn, vt1, vt2, Bt1, Bt2, p) with (n, t1, t2) cyclic from D, its
// density and its adiabatic index.

// the conserved values one cell needs: rho, m (normal, t1, t2), e, both faces
// of the two transverse fields (c1, c2: the upper neighbours along t1 and t2)
// and, with the ionisation network, the H2 and H+ densities
template <typename T> struct Raw { T rho, mn, m1, m2, e, b1, b1p, b2, b2p, h2, hp; };

template <typename T, int D, bool ION>
__device__ __forceinline__ void raw_load(const CFields<T>& U, int c, int c1, int c2, Raw<T>& r)
{
    constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
    r.rho = U.f[RHO][c];
    r.mn = U.f[MX + D][c];
    r.m1 = U.f[MX + T1][c];
    r.m2 = U.f[MX + T2][c];
    r.e = U.f[EI][c];
    r.b1 = U.f[BX + T1][c];
    r.b1p = U.f[BX + T1][c1];
    r.b2 = U.f[BX + T2][c];
    r.b2p = U.f[BX + T2][c2];
    if (ION) {
        r.h2 = U.f[H2][c];
        r.hp = U.f[HP][c];
    }
}

// q[0..5] = (vn, vt1, vt2, Bt1, Bt2, p); gam = the cell's gamma (gamma_eff
// of Sec. 4.3 with the network, in FP64 as the tail computes it)
template <typename T, bool ION>
__device__ __forceinline__ void raw_prim(const Raw<T>& r, double gamma, T q[6], T& gam)
{
    const T ir = rcp_nr(r.rho);   // one reciprocal for the three velocities
    q[0] = r.mn * ir;
    q[1] = r.m1 * ir;
    q[2] = r.m2 * ir;
    q[3] = T(0.5) * (r.b1 + r.b1p);
    q[4] = T(0.5) * (r.b2 + r.b2p);
    if (ION) {
        double gc = gamma_cell(1, 0.0, (double)r.rho, (double)r.h2, (double)r.hp);
        gam = T(gc);
        q[5] = T(gc - 1.0) * r.e;
    } else {
        gam = T(gamma);
        q[5] = T(gamma - 1.0) * r.e;
    }
}

// ---------------------------------------------------------------- NONADV faces

template <typename T>
__device__ __forceinline__ void store_face(T* __restrict__ F, size_t N, int c, const T out[7])
{
#pragma unroll
    for (int q = 0; q < 7; q++) F[q * N + c] = out[q];
}

template <typename T>
struct FaceArgs {
    Geo g;
    CFields<T> U;            // substage input state
    T* F;
    StepArgs a;
    int rpb;                 // x rows per block (row kernel)
    int seg;                 // faces per thread (marching kernel)
    uint32_t* flags;
    const double* dt_cfl;    // non-null: check the explicit dt against this CFL bound
    // the x-row kernel also updates m, E, e (the NONADV update of Sec. 2.2,
    // 2.5 without the face fields): Runge-Kutta inputs and output, the y and
    // z face outputs, and the gravitational potential (null without gravity)
    CFields<T> S;
    Fields<T> O;
    const T* Fy;
    const T* Fz;
    RK rk;
    int dbg;                 // 1: write tau R(U) instead of the combination
    const T* phi;
};

// an explicit dt above the device CFL bound (with its relative slack) latches
// flag bit 2 for the next synchronising call; one thread of the box checks
template <typename T>
__device__ __forceinline__ void check_dt(const FaceArgs<T>& A, int blk, int tid)
{
    if (blk == 0 && tid == 0 && A.dt_cfl && !A.a.dt_dev && A.a.dt_val > *A.dt_cfl * (1.0 + A.a.cfl_tol))
        atomicOr(A.flags, 2u);
}

// NONADV faces along D, one face per thread, both adjacent parabolas computed
// by the thread from the primitives of the six cells of its line (general
// fallback for any box)
template <typename T, int D, bool ION>
struct BFacePair {
    static constexpr int NT = NTH;
    static constexpr bool XCD = false;
    using Args = FaceArgs<T>;
    static __device__ __forceinline__ void run(const Args& A, int blk, int tid)
    {
        const Geo& g = A.g;
        check_dt(A, blk, tid);
        int c = blk * NT + tid;
        if (c >= g.n) return;
        constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
        int i, j, k;
        decompose(g, c, i, j, k);
        const size_t N = (size_t)g.n;
        // the cells of the line share their transverse coordinates, so their
        // upper transverse neighbours sit at the same offsets
        const int o1 = nbr<T1>(g, c, i, j, k, 1) - c, o2 = nbr<T2>(g, c, i, j, k, 1) - c;
        T q[6][6], rho[6], gam[6];
#pragma unroll
        for (int m = 0; m < 6; m++) {
            int cm = nbr<D>(g, c, i, j, k, m - 3);
            Raw<T> rw;
            raw_load<T, D, ION>(A.U, cm, cm + o1, cm + o2, rw);
            T qm[6];
            raw_prim<T, ION>(rw, A.a.gamma, qm, gam[m]);
#pragma unroll
            for (int v = 0; v < 6; v++) q[v][m] = qm[v];
            rho[m] = rw.rho;
        }
        Side<T> L, R;
#pragma unroll
        for (int v = 0; v < 6; v++) {
            Par<T> PL, PR;
            parabola_pair(q[v][0], q[v][1], q[v][2], q[v][3], q[v][4], q[v][5], PL, PR);
            side_left(PL, L, v);
            side_right(PR, R, v);
        }
        T out[7];
        const T gm = T(A.a.gamma);
        face_solve(rho[2], q[5][2], q[3][2], q[4][2], rho[3], q[5][3], q[3][3], q[4][3], A.U.f[BX + D][c], L, R,
                   gm, gam[2], gam[3], ION, T(A.a.theta * (step_dt(A.a) / A.a.h)), root_nr(rho[2]), root_nr(rho[3]),
                   out);
        store_face(A.F, N, c, out);
    }
};

// The y and z face kernels store, for FP32 state, the per-cell difference of
// the five fluxes between a cell's upper and lower face (what the update
// reads) instead of the face values, so the update reads one value per flux;
// the two edge-field components are stored per face either way.  (For FP64
// the carried fluxes would not fit the marching kernel's registers.)
template <typename T> struct FluxDiff { static constexpr bool v = sizeof(T) == 4; };

// NONADV faces along x with whole x rows per block, fused with the update of
// m, E and e.  Each thread owns one cell, forms its primitives and computes,
// once each, its limited slopes, the interface values at its lower face and
// its parabolas (Sec. 2.1); neighbours' primitives, slopes, interface values
// and parabola sides come through LDS (periodic wrap inside the row).  After
// the face solve the row's x-face fluxes are exchanged the same way, so the
// thread forms the flux differences of its cell (y and z faces from the face
// kernels that ran before), the p dV work, the gravity sources and the
// Runge-Kutta combination of m, E, e (Sec. 2.2).  Only the edge-field
// components of the x faces are stored, for the face-field update.  Dynamic
// LDS: XROW_SLOTS x NT values, value k of thread t at k * NT + t: primitives
// in slots 0-7 with sqrt(rho) in 14, slopes 8-13, the two edge values of each
// parabola in 0-7 and 14-17 (the right neighbour forms the left cell's jump
// and curvature from them and the mean it holds, with the expressions of
// parabola_finish, so the same bits) and x-face fluxes 8-12, so each exchange
// needs one barrier.
constexpr int XROW_SLOTS = 18;

template <typename T, int MAXT, bool ION>
struct BFaceXRows {
    static constexpr int NT = MAXT;
    static constexpr bool XCD = false;
    // FP64 rows of 512 cells: two blocks per CU (72 KB of LDS each) need four
    // waves per SIMD, i.e. at most 128 registers; the few values that spill
    // cost less than the waiting of a single block at its barriers
    static constexpr int MINW = (MAXT == 512 && sizeof(T) == 8) ? 4 : 1;
    // FP32 256-thread rows keep one workgroup per tile in the persistent
    // multi-box form: the tile loop costs three registers (83 instead of 80),
    // five waves per SIMD instead of six, and these small tiles run 8%
    // slower (held to six waves, the spills cost more)
    static constexpr bool PERSIST = !(MAXT == 256 && sizeof(T) == 4);
    using Args = FaceArgs<T>;
    // LDS slot of edge value k (qL, qR) of variable v's published parabola:
    // slots 0-7 and 14-17, around the slopes in 8-13
    static __device__ __forceinline__ constexpr int sslot(int v, int k)
    {
        return 2 * v + k < 8 ? 2 * v + k : 2 * v + k + 6;
    }
    static __device__ __forceinline__ void run(const Args& A, int blk, int tid)
    {
        extern __shared__ unsigned char smem_raw[];
        T* sm = reinterpret_cast<T*>(smem_raw);
        const Geo& g = A.g;
        const size_t N = (size_t)g.n;
        const int nx = g.nx;
        check_dt(A, blk, tid);
        // one row per block: rows in XCD bands, so the next row's and the next
        // plane's y and z fluxes are mostly read through this XCD's L2 (a fifth
        // of the reads fewer, about 1% slower).  Only then are the row indices
        // the block indices: with several rows per block the band's domain
        // (ny nz) would exceed the blocks
        if (A.rpb == 1) blk = xcd_band(blk, 1, g.ny, g.nz);
        // row r of the block, cell i of the row (one row per block: no
        // per-thread division)
        int r, i;
        if (nx == NT) {
            r = 0;
            i = tid;
        } else {
            r = tid / nx;
            i = tid - r * nx;
        }
        const int row = blk * A.rpb + r;
        // the row's y and z indices: with rows of a multiple of 64 cells each
        // wave lies in one row and divides once, on the scalar unit (unsigned
        // there, so that the compiler does not merge the two divisions into
        // one per-thread division after the branch)
        int j, k;
        if ((nx & 63) == 0) {
            const unsigned wrow = (unsigned)__builtin_amdgcn_readfirstlane(row);
            j = (int)(wrow % (unsigned)g.ny);
            k = (int)(wrow / (unsigned)g.ny);
        } else {
            j = row % g.ny;
            k = row / g.ny;
        }
        bool act = r < A.rpb && row < g.ny * g.nz;
        const int rowbase = row * nx;
        const int c = rowbase + i;
        const int rb = r * nx;
        const int tl = rb + (i == 0 ? nx - 1 : i - 1);   // thread of the left cell
        const int tr = rb + (i + 1 == nx ? 0 : i + 1);   // thread of the right cell
        const int tm2 = rb + wrapc(i - 2, nx), tp2 = rb + wrapc(i + 2, nx);
        const T gm = T(A.a.gamma);
        // periodic offsets of the upper neighbours along y and z
        const int dyp = ((j + 1 == g.ny ? 0 : j + 1) - j) * nx;
        const int dzp = ((k + 1 == g.nz ? 0 : k + 1) - k) * g.nxy;
        // the step's dt (device-resident under the CFL step), read before any
        // store of this kernel: read later, each wave would wait for the load
        // after a barrier, with every other wave of the block (FP64 rows of
        // 512 cells, held to 128 registers, read it where it is used: the
        // two registers would spill)
        constexpr bool DT_EARLY = !(sizeof(T) == 8 && MAXT == 512);
        const double dt_early = DT_EARLY ? step_dt(A.a) : 0.0;
        auto dt_now = [&]() { return DT_EARLY ? dt_early : step_dt(A.a); };

        // own cell: conserved values, primitives
        // uc, sc: the cell's m, E, e at the substage input and at the stage
        // start, for the update at the end.  With EARLY they are taken here
        // (FP64 rows of 256 cells: the registers still fit three waves per
        // SIMD, and the stores of the face outputs in between would make the
        // compiler load them again); otherwise loaded at the update (FP32
        // would drop from six to five waves, the 512-cell rows would spill)
        constexpr bool EARLY = sizeof(T) == 8 && MAXT == 256;
        T q2[6], rho = T(0), gam = gm, bn = T(0), srho = T(0), uc[5], sc[5];
        const int upd[5] = { MX, MY, MZ, EN, EI };
        if (act) {
            Raw<T> rw;
            raw_load<T, 0, ION>(A.U, c, c + dyp, c + dzp, rw);
            bn = A.U.f[BX][c];
            if constexpr (EARLY) {
                uc[0] = rw.mn;
                uc[1] = rw.m1;
                uc[2] = rw.m2;
                uc[3] = A.U.f[EN][c];
                uc[4] = rw.e;
#pragma unroll
                for (int q = 0; q < 5; q++) sc[q] = A.S.f[upd[q]][c];
            }
            raw_prim<T, ION>(rw, A.a.gamma, q2, gam);
            rho = rw.rho;
#pragma unroll
            for (int v = 0; v < 6; v++) sm[v * NT + tid] = q2[v];
            sm[6 * NT + tid] = rho;
            if (ION) sm[7 * NT + tid] = gam;
            srho = root_nr(rho);
            sm[14 * NT + tid] = srho;
        }
        __syncthreads();
        // the 5-cell line of each variable; the left cell's density (and
        // gamma); slopes of the own cell
        T q0[6], q1[6], q3[6], q4[6], dm[6], fl[6];
        T rl = T(0), gl = gm, srl = T(0);
        if (act) {
#pragma unroll
            for (int v = 0; v < 6; v++) {
                q0[v] = sm[v * NT + tm2];
                q1[v] = sm[v * NT + tl];
                q3[v] = sm[v * NT + tr];
                q4[v] = sm[v * NT + tp2];
            }
            rl = sm[6 * NT + tl];
            srl = sm[14 * NT + tl];
            if (ION) gl = sm[7 * NT + tl];
#pragma unroll
            for (int v = 0; v < 6; v++) {
                dm[v] = limited_slope(q1[v], q2[v], q3[v]);
                sm[(8 + v) * NT + tid] = dm[v];
            }
        }
        __syncthreads();
        // interface values at both faces from the neighbours' slopes (the
        // upper one is the right cell's lower one, formed from the same
        // operands), then the own cell's parabolas; their edge values are
        // published in the slots sslot(v, 0..1) (0-7 and 14-17: the
        // primitives, densities and gamma there are no longer read; the
        // slopes in 8-13 are read until the barrier below)
        Side<T> R;
        if (act) {
#pragma unroll
            for (int v = 0; v < 6; v++) {
                fl[v] = interface_value(q1[v], q2[v], sm[(8 + v) * NT + tl], dm[v]);
                T fr = interface_value(q2[v], q3[v], dm[v], sm[(8 + v) * NT + tr]);
                Par<T> P = parabola_finish(q0[v], q1[v], q2[v], q3[v], q4[v], fl[v], fr, dm[v]);
                side_right(P, R, v);
                sm[sslot(v, 0) * NT + tid] = P.qL;
                sm[sslot(v, 1) * NT + tid] = P.qR;
            }
        }
        __syncthreads();
        // the face solve; its fluxes go to slots 8-12 (the slopes there were
        // read before the barrier)
        T out[7];
        // the update's y and z flux values (per-cell differences when the
        // marches stored them) and, without EARLY, its m, E, e inputs: loaded
        // after the face solve, before this thread's stores (outputs may alias
        // inputs as far as the compiler knows) and, with LOADS_AHEAD, before
        // the barrier, so their latency overlaps the wait (FP64 rows of 512
        // cells, held to 128 registers, would spill more: they load after it)
        constexpr bool DIFF = FluxDiff<T>::v;
        constexpr bool LOADS_AHEAD = !(sizeof(T) == 8 && MAXT == 512);
        T fy[5], fz[5], fyp[DIFF ? 1 : 5], fzp[DIFF ? 1 : 5];
        auto load_update_inputs = [&]() {
#pragma unroll
            for (int v = 0; v < 5; v++) {
                fy[v] = A.Fy[v * N + c];
                fz[v] = A.Fz[v * N + c];
                if constexpr (!DIFF) {
                    fyp[v] = A.Fy[v * N + c + dyp];
                    fzp[v] = A.Fz[v * N + c + dzp];
                }
            }
            if constexpr (!EARLY) {
#pragma unroll
                for (int q = 0; q < 5; q++) {
                    uc[q] = A.U.f[upd[q]][c];
                    sc[q] = A.S.f[upd[q]][c];
                }
            }
        };
        if (act) {
            // the left cell's right side (Step 5 of parabola_finish on its
            // edge values and its mean q1)
            Side<T> L;
#pragma unroll
            for (int v = 0; v < 6; v++) {
                const T fL = sm[sslot(v, 0) * NT + tl], fR = sm[sslot(v, 1) * NT + tl];
                L.e[v] = fR;
                L.dq[v] = fR - fL;
                L.q6[v] = T(6) * (q1[v] - T(0.5) * (fL + fR));
            }
            // parabola variables 3, 4, 5 are Bt1, Bt2, p
            face_solve(rl, q1[5], q1[3], q1[4], rho, q2[5], q2[3], q2[4], bn, L, R, gm, gl, gam, ION,
                       T(A.a.theta * (dt_now() / A.a.h)), srl, srho, out);
            if constexpr (LOADS_AHEAD) load_update_inputs();
            A.F[5 * N + c] = out[5];
            A.F[6 * N + c] = out[6];
#pragma unroll
            for (int v = 0; v < 5; v++) sm[(8 + v) * NT + tid] = out[v];
        }
        __syncthreads();
        if (!act) return;
        if constexpr (!LOADS_AHEAD) load_update_inputs();

        // update of m, E, e: flux differences of the x faces (the right
        // cell's lower face from LDS), y and z faces (loaded above)
        const T dtdx = T(dt_now() / A.a.h);
        T dF[3][5];
#pragma unroll
        for (int v = 0; v < 5; v++) {
            dF[0][v] = sm[(8 + v) * NT + tr] - out[v];
            if constexpr (DIFF) {
                dF[1][v] = fy[v];
                dF[2][v] = fz[v];
            } else {
                dF[1][v] = fyp[v] - fy[v];
                dF[2][v] = fzp[v] - fz[v];
            }
        }
        T inc[5];
        // momentum component a takes slot (a - d) mod 3 from direction d
        inc[0] = -dtdx * ((dF[0][0] + dF[1][2]) + dF[2][1]);
        inc[1] = -dtdx * ((dF[0][1] + dF[1][0]) + dF[2][2]);
        inc[2] = -dtdx * ((dF[0][2] + dF[1][1]) + dF[2][0]);
        inc[3] = -dtdx * ((dF[0][3] + dF[1][3]) + dF[2][3]);
        T divv = (dF[0][4] + dF[1][4]) + dF[2][4];
        // (gamma - 1) e, with the cell's gamma_eff under the network
        const T gm1 = ION ? gam - T(1) : T(A.a.gamma - 1.0);
        inc[4] = -gm1 * uc[4] * dtdx * divv;
        if (A.phi) {
            // self-gravity (Sec. 2 equations, Sec. 2.4): -rho grad(Phi) on
            // m and -m . grad(Phi) on E, central differences
            const T* ph = A.phi;
            const T i2h = T(0.5 / A.a.h);
            const T dt = T(dt_now());
            const int dxp = tr - tid, dxm = tl - tid;
            const int dym = ((j == 0 ? g.ny - 1 : j - 1) - j) * nx;
            const int dzm = ((k == 0 ? g.nz - 1 : k - 1) - k) * g.nxy;
            T gv[3] = { (ph[c + dxp] - ph[c + dxm]) * i2h, (ph[c + dyp] - ph[c + dym]) * i2h,
                        (ph[c + dzp] - ph[c + dzm]) * i2h };
            T work = T(0);
#pragma unroll
            for (int a = 0; a < 3; a++) {
                inc[a] -= dt * rho * gv[a];
                work += uc[a] * gv[a];
            }
            inc[3] -= dt * work;
        }
        if (A.dbg) {
#pragma unroll
            for (int q = 0; q < 5; q++) A.O.f[upd[q]][c] = inc[q];
            A.O.f[RHO][c] = T(0);
            A.O.f[H2][c] = T(0);
            if (ION) A.O.f[HP][c] = T(0);   // H+ is a field of its own only with the network
        } else {
            const T ra = T(A.rk.a), rb = T(A.rk.b);
#pragma unroll
            for (int q = 0; q < 5; q++) A.O.f[upd[q]][c] = (uc[q] + ra * (sc[q] - uc[q])) + rb * inc[q];
        }
    }
};

// NONADV faces along D = y or z: each thread marches along one grid line over
// a segment of `seg` faces with a sliding 5-cell window of primitives in
// registers, so each cell's primitives and parabolas are formed once per
// segment (seg + 1 per seg faces); threads are consecutive in x, so every load
// is coalesced.  With per-cell differences the thread also solves the upper
// face of its segment's last cell; the previous face's fluxes wait in LDS.
template <typename T, int D, bool ION>
struct BFaceMarch {
    static constexpr int NT = NTH;
    static constexpr bool XCD = false;
    using Args = FaceArgs<T>;
    static __device__ __forceinline__ void run(const Args& A, int blk, int tid)
    {
        const Geo& g = A.g;
        const size_t N = (size_t)g.n;
        const int seg = A.seg;
        const int nd = D == 1 ? g.ny : g.nz;
        const int no = D == 1 ? g.nz : g.ny;
        const int nseg = (nd + seg - 1) / seg;
        int t = blk * NT + tid;
        int i = t % g.nx;
        int rest = t / g.nx;
        int o = rest % no;
        int sgi = rest / no;
        if (sgi >= nseg) return;
        const int base = D == 1 ? i + g.nxy * o : i + g.nx * o;
        const int stride = D == 1 ? g.nx : g.nxy;
        const int x0 = sgi * seg;
        const int x1 = min(x0 + seg, nd);
        const T gm = T(A.a.gamma);
        const T ydx = T(A.a.theta * (step_dt(A.a) / A.a.h));
        // offsets of the upper neighbours along t1, t2 (the same for every
        // cell of the line): y march t1 = z, t2 = x; z march t1 = x, t2 = y
        const int dxp = (i + 1 == g.nx ? 0 : i + 1) - i;
        const int dop = ((o + 1 == no ? 0 : o + 1) - o) * (D == 1 ? g.nxy : g.nx);
        const int o1 = D == 1 ? dop : dxp, o2 = D == 1 ? dxp : dop;

        // window: w[v][m] = variable v of cell x-2+m; v = 0..5 parabola
        // variables, 6 = rho; gw[m] its gamma (network only)
        T w[7][5];
        T gw[5];
#pragma unroll
        for (int m = 0; m < 5; m++) {
            int cc = base + wrapc(x0 - 3 + m, nd) * stride;
            Raw<T> rw;
            raw_load<T, D, ION>(A.U, cc, cc + o1, cc + o2, rw);
            T qm[6];
            raw_prim<T, ION>(rw, A.a.gamma, qm, gw[m]);
#pragma unroll
            for (int v = 0; v < 6; v++) w[v][m] = qm[v];
            w[6][m] = rw.rho;
        }
        // parabolas of cell x0 - 1 (the left side of the first face).  Along
        // the march each cell's limited slope and each face's interface value
        // is computed once and carried: dmc = slope of the current cell,
        // fl = interface value at its lower face (Step 1, the same calls as
        // in parabola())
        Side<T> L;
        T dmc[6], fl[6];
#pragma unroll
        for (int v = 0; v < 6; v++) {
            T d0 = limited_slope(w[v][0], w[v][1], w[v][2]);
            T d1 = limited_slope(w[v][1], w[v][2], w[v][3]);
            T d2 = limited_slope(w[v][2], w[v][3], w[v][4]);
            T f0 = interface_value(w[v][1], w[v][2], d0, d1);
            T f1 = interface_value(w[v][2], w[v][3], d1, d2);
            side_left(parabola_finish(w[v][0], w[v][1], w[v][2], w[v][3], w[v][4], f0, f1, d1), L, v);
            dmc[v] = d2;
            fl[v] = f1;
        }

        // the conserved values of the cell entering the window (x + 2 for
        // face x) are loaded one face ahead, so the loads are in flight while
        // the previous face is solved
        Raw<T> nr;
        auto fetch = [&](int x) {
            int cn = base + wrapc(x + 2, nd) * stride;
            raw_load<T, D, ION>(A.U, cn, cn + o1, cn + o2, nr);
        };
        constexpr bool DIFF = FluxDiff<T>::v;
        const int xe = DIFF ? x1 + 1 : x1;   // faces solved: x0 .. xe - 1
        __shared__ T prev[DIFF ? 5 : 1][NT];
        // sqrt(rho) of the face's left cell, carried (window slot 2 before
        // the first slide is slot 1 of the first face)
        T srl = root_nr(w[6][2]);
        fetch(x0);
        // the face's normal field, loaded one face ahead with the entering
        // cell (loaded at the face, its latency stood before the face solve);
        // FP64 with the ionisation network has no registers left for it
        constexpr bool BN_AHEAD = !ION || sizeof(T) == 4;
        auto bn_of = [&](int x) { return A.U.f[BX + D][base + (DIFF ? wrapc(x, nd) : x) * stride]; };
        T bnn = BN_AHEAD ? bn_of(x0) : T(0);
        auto face = [&](int x) {
            const T bnx = BN_AHEAD ? bnn : bn_of(x);
            T qn[6], gn;
            raw_prim<T, ION>(nr, A.a.gamma, qn, gn);
#pragma unroll
            for (int v = 0; v < 7; v++) {
#pragma unroll
                for (int m = 0; m < 4; m++) w[v][m] = w[v][m + 1];
                w[v][4] = v < 6 ? qn[v] : nr.rho;
            }
            if (ION) {
#pragma unroll
                for (int m = 0; m < 4; m++) gw[m] = gw[m + 1];
                gw[4] = gn;
            }
            if (x + 1 < xe) {
                fetch(x + 1);
                if constexpr (BN_AHEAD) bnn = bn_of(x + 1);
            }
            Side<T> R, Ln;
#pragma unroll
            for (int v = 0; v < 6; v++) {
                // window slots 0..4 = cells x-2 .. x+2
                T dn = limited_slope(w[v][2], w[v][3], w[v][4]);
                T fr = interface_value(w[v][2], w[v][3], dmc[v], dn);
                Par<T> P = parabola_finish(w[v][0], w[v][1], w[v][2], w[v][3], w[v][4], fl[v], fr, dmc[v]);
                side_right(P, R, v);
                side_left(P, Ln, v);
                dmc[v] = dn;
                fl[v] = fr;
            }
            // face x is the lower face of cell x (with differences, x = x1 is
            // the upper face of the last cell, periodic)
            int c = base + (DIFF ? wrapc(x, nd) : x) * stride;
            T out[7];
            // left cell x-1 is window slot 1, right cell x is slot 2
            const T srr = root_nr(w[6][2]);
            face_solve(w[6][1], w[5][1], w[3][1], w[4][1], w[6][2], w[5][2], w[3][2], w[4][2], bnx, L,
                       R, gm, ION ? gw[1] : gm, ION ? gw[2] : gm, ION, ydx, srl, srr, out);
            srl = srr;
            if (!DIFF) {
                store_face(A.F, N, c, out);
            } else {
                if (x < x1) {
                    A.F[5 * N + c] = out[5];
                    A.F[6 * N + c] = out[6];
                }
                if (x > x0) {
                    const int cm = base + (x - 1) * stride;
#pragma unroll
                    for (int v = 0; v < 5; v++) A.F[v * N + cm] = out[v] - prev[v][tid];
                }
#pragma unroll
                for (int v = 0; v < 5; v++) prev[v][tid] = out[v];
            }
            L = Ln;
        };
        // FP32 (without the network) takes two faces per loop trip: the
        // window, slopes and sides are renamed instead of moved between them
        // (about 8% fewer VALU instructions per face, still three waves per
        // SIMD; the scheduling barrier keeps the two faces' work apart, which
        // holds the registers to one face's).  FP64 has no registers for it.
        int x = x0;
        if constexpr (sizeof(T) == 4 && !ION) {
            for (; x + 1 < xe; x += 2) {
                face(x);
                __builtin_amdgcn_sched_barrier(0);
                face(x + 1);
            }
        }
        for (; x < xe; x++) face(x);
    }
};

// NONADV update: flux differences, p dV work, face-field update from edge
// fields (Sec. 2.5), Runge-Kutta combination (Sec. 2.2).  dbg != 0 writes
// tau R(U) instead of the combination.  Each thread marches along z over a
// segment of cells (ZTile); the Ex, Ey on the upper z edges of cell k, the
// edge-field components they read, and (full update, FP64) the z-face fluxes
// at its upper face are the lower ones of cell k+1, so they are carried
// instead of read or formed again (same arithmetic).
template <typename T>
struct NonadvUpdateArgs {
    Geo g;
    CFields<T> U, S;
    Fields<T> O;
    const T* Fx;
    const T* Fy;
    const T* Fz;
    StepArgs a;
    RK rk;
    int dbg;
    ZTile zt;
    const T* phi;   // gravitational potential, or null without self-gravity
};

// threads per block of the NONADV update and the x width of its x-y tile
// (UPD_TX x UPD_NT / UPD_TX cells)
constexpr int UPD_NT = 256;
constexpr int UPD_TX = 64;

// FULL: all eight fields (the update of boxes whose x faces come from the
// one-face-per-thread kernel); otherwise only the face fields b_x, b_y, b_z,
// after the x-row face kernel has updated m, E and e
template <typename T, bool ION, bool FULL>
struct BNonadvUpdate {
    static constexpr int NT = UPD_NT;
    static constexpr bool XCD = false;
    static constexpr int MINW = ION ? 1 : 4;
    using Args = NonadvUpdateArgs<T>;
    static __device__ __forceinline__ void run(const Args& A, int blk, int tid)
    {
        const Geo& g = A.g;
        const int nx = g.nx, ny = g.ny, nz = g.nz, nxy = g.nxy;
        int i, j, k0, k1;
        // the y-neighbour rows at the tile edges and the z-neighbour
        // segment are read through the same L2 (a quarter of the reads
        // fewer, 2% faster)
        blk = xcd_band(blk, A.zt.ntx, A.zt.nty, (g.nz + A.zt.seg - 1) / A.zt.seg);
        if (!ztile_cell(g, A.zt, blk, tid, i, j, k0, k1)) return;
        const size_t N = (size_t)g.n;
        const T dtdx = T(step_dt(A.a) / A.a.h);
        const T* Fx = A.Fx;
        const T* Fy = A.Fy;
        const T* Fz = A.Fz;
        // periodic neighbour offsets in the x-y plane
        const int dxp = (i + 1 == nx ? 0 : i + 1) - i, dxm = (i == 0 ? nx - 1 : i - 1) - i;
        const int dyp = ((j + 1 == ny ? 0 : j + 1) - j) * nx, dym = ((j == 0 ? ny - 1 : j - 1) - j) * nx;

        // edge fields (electric-field appendix): Ex at (i, j-1/2, k-1/2) from
        // z faces at j-1, j and y faces at k, k-1; Ey at (i-1/2, j, k-1/2) from
        // z faces at i-1, i and x faces at k-1, k; Ez at (i-1/2, j-1/2, k) from
        // x faces at j-1, j and y faces at i-1, i.
        const T* ezx = Fz + 5 * N;   // z faces, E along x
        const T* ezy = Fz + 6 * N;   // z faces, E along y
        const T* eyz = Fy + 5 * N;   // y faces, E along z
        const T* eyx = Fy + 6 * N;   // y faces, E along x
        const T* exy = Fx + 5 * N;   // x faces, E along y
        const T* exz = Fx + 6 * N;   // x faces, E along z
        auto Ez = [&](int cc, int cym, int cxm) { return T(0.25) * (((exz[cym] + exz[cc]) + eyz[cxm]) + eyz[cc]); };

        // carried from the cell below: the z-face values at the lower face of
        // the current cell, the Ex, Ey on its lower z edges, and the face
        // edge-field values of the current plane (and of the plane below at
        // x+1, y+1) that the cell below read as its upper-plane values
        T fzc[5];
        T Ex_c, Ey_c;
        T ezx_c, eyx_c, ezy_c, exy_c, eyx_ypm, exy_xpm;
        {
            int c = i + nx * j + nxy * k0;
            int zm = c + ((k0 == 0 ? nz - 1 : k0 - 1) - k0) * nxy;
            if (FULL && !FluxDiff<T>::v) {
#pragma unroll
                for (int v = 0; v < 5; v++) fzc[v] = Fz[v * N + c];
            }
            ezx_c = ezx[c];
            eyx_c = eyx[c];
            ezy_c = ezy[c];
            exy_c = exy[c];
            eyx_ypm = eyx[zm + dyp];
            exy_xpm = exy[zm + dxp];
            Ex_c = T(0.25) * (((ezx[c + dym] + ezx_c) + eyx_c) + eyx[zm]);
            Ey_c = T(0.25) * (((ezy[c + dxm] + ezy_c) + exy[zm]) + exy_c);
        }
        const T ra = T(A.rk.a), rb = T(A.rk.b);
        // two (FP64) or four (FP32) planes per loop trip: the loads of the
        // later planes are in flight with the earlier planes' arithmetic
        // (the kernel waits on memory latency, not bandwidth)
#pragma unroll(sizeof(T) == 8 ? 2 : 4)
        for (int k = k0; k < k1; k++) {
            const int c = i + nx * j + nxy * k;
            const int dzp = ((k + 1 == nz ? 0 : k + 1) - k) * nxy;
            const int dzm = ((k == 0 ? nz - 1 : k - 1) - k) * nxy;
            const int xp = c + dxp, xm = c + dxm, yp = c + dyp, ym = c + dym, zp = c + dzp;
            constexpr int Q0 = FULL ? 0 : 5;
            const int upd[8] = { MX, MY, MZ, EN, EI, BX, BY, BZ };
            // the face fields' Runge-Kutta inputs, all loaded before the
            // plane's stores (a load issued after a store waits for the store
            // as well: one memory counter, in order); the full update, with
            // eight fields, keeps them at the combination (here it would
            // spill)
            T uo[8], so[8];
            if (!FULL && !A.dbg) {
#pragma unroll
                for (int q = Q0; q < 8; q++) {
                    uo[q] = A.U.f[upd[q]][c];
                    so[q] = A.S.f[upd[q]][c];
                }
            }
            T inc[NF];
            if (FULL) {
                T dF[3][5], fzp[5];
#pragma unroll
                for (int v = 0; v < 5; v++) {
                    dF[0][v] = Fx[v * N + xp] - Fx[v * N + c];
                    if (FluxDiff<T>::v) {   // the marches stored per-cell differences
                        dF[1][v] = Fy[v * N + c];
                        dF[2][v] = Fz[v * N + c];
                    } else {
                        dF[1][v] = Fy[v * N + yp] - Fy[v * N + c];
                        fzp[v] = Fz[v * N + zp];
                        dF[2][v] = fzp[v] - fzc[v];
                    }
                }
                // momentum component a takes slot (a - d) mod 3 from direction d
                inc[MX] = -dtdx * ((dF[0][0] + dF[1][2]) + dF[2][1]);
                inc[MY] = -dtdx * ((dF[0][1] + dF[1][0]) + dF[2][2]);
                inc[MZ] = -dtdx * ((dF[0][2] + dF[1][1]) + dF[2][0]);
                inc[EN] = -dtdx * ((dF[0][3] + dF[1][3]) + dF[2][3]);
                T divv = (dF[0][4] + dF[1][4]) + dF[2][4];
                // with the network, gamma_eff of the cell (FP64, as the tail forms it)
                T gm1 = T(A.a.gamma - 1.0);
                if (ION)
                    gm1 = T(gamma_cell(1, 0.0, (double)A.U.f[RHO][c], (double)A.U.f[H2][c], (double)A.U.f[HP][c])) -
                          T(1);
                inc[EI] = -gm1 * A.U.f[EI][c] * dtdx * divv;
                if (A.phi) {
                    // self-gravity (Sec. 2 equations, Sec. 2.4): -rho grad(Phi) on
                    // m and -m . grad(Phi) on E, central differences
                    const T* ph = A.phi;
                    const T i2h = T(0.5 / A.a.h);
                    const T dt = T(step_dt(A.a));
                    T gv[3] = { (ph[xp] - ph[xm]) * i2h, (ph[yp] - ph[ym]) * i2h, (ph[zp] - ph[c + dzm]) * i2h };
                    T rho = A.U.f[RHO][c];
                    T work = T(0);
#pragma unroll
                    for (int a = 0; a < 3; a++) {
                        inc[MX + a] -= dt * rho * gv[a];
                        work += A.U.f[MX + a][c] * gv[a];
                    }
                    inc[EN] -= dt * work;
                }
                if (!FluxDiff<T>::v) {
#pragma unroll
                    for (int v = 0; v < 5; v++) fzc[v] = fzp[v];
                }
            }

            // edge fields on the upper edges (Ex, Ey at z+1/2; Ex at y+1/2, Ey
            // at x+1/2): the same sums as for the carried lower edges
            const T ezx_zp = ezx[zp], eyx_zp = eyx[zp], ezy_zp = ezy[zp], exy_zp = exy[zp];
            const T eyx_yp = eyx[yp], exy_xp = exy[xp];
            T Ex_yp = T(0.25) * (((ezx_c + ezx[yp]) + eyx_yp) + eyx_ypm);
            T Ex_zp = T(0.25) * (((ezx[zp + dym] + ezx_zp) + eyx_zp) + eyx_c);
            T Ey_xp = T(0.25) * (((ezy_c + ezy[xp]) + exy_xpm) + exy_xp);
            T Ey_zp = T(0.25) * (((ezy[zp + dxm] + ezy_zp) + exy_c) + exy_zp);
            T Ez_c = Ez(c, ym, xm);
            T Ez_xp = Ez(xp, xp + dym, c);
            T Ez_yp = Ez(yp, c, yp + dxm);
            inc[BX] = -dtdx * (Ez_yp - Ez_c) + dtdx * (Ey_zp - Ey_c);
            inc[BY] = -dtdx * (Ex_zp - Ex_c) + dtdx * (Ez_xp - Ez_c);
            inc[BZ] = -dtdx * (Ey_xp - Ey_c) + dtdx * (Ex_yp - Ex_c);

            if (A.dbg) {
#pragma unroll
                for (int q = Q0; q < 8; q++) A.O.f[upd[q]][c] = inc[upd[q]];
                if (FULL) {
                    A.O.f[RHO][c] = T(0);
                    A.O.f[H2][c] = T(0);
                    if (ION) A.O.f[HP][c] = T(0);   // H+ is a field of its own only with the network
                }
            } else {
#pragma unroll
                for (int q = Q0; q < 8; q++) {
                    if constexpr (FULL) {
                        uo[q] = A.U.f[upd[q]][c];
                        so[q] = A.S.f[upd[q]][c];
                    }
                    A.O.f[upd[q]][c] = (uo[q] + ra * (so[q] - uo[q])) + rb * inc[upd[q]];
                }
            }
            Ex_c = Ex_zp;
            Ey_c = Ey_zp;
            ezx_c = ezx_zp;
            eyx_c = eyx_zp;
            ezy_c = ezy_zp;
            exy_c = exy_zp;
            eyx_ypm = eyx_yp;
            exy_xpm = exy_xp;
        }
    }
};

// ---------------------------------------------------------------- Poisson (Sec. 2.9)

template <typename T> struct Cx { T re, im; };

template <typename T>
__device__ __forceinline__ Cx<T> cmul(const Cx<T>& a, const Cx<T>& b)
{
    return { a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re };
}

// Values (lines x length) one block transforms: 1024 in the x passes, 2048 in
// the y/z passes, i.e. at most VALUES / 1024 radix-4 butterflies per thread of
// a 256-thread block in a stage (twice that in the radix-2 stage)
constexpr int FFT_X_VALUES = 1024;
constexpr int FFT_YZ_VALUES = 2048;

// Stockham transform of nl lines of length n = 2^logn held in the LDS buffer
// a (line l at l * ls), in place: every thread first reads the inputs of all
// its butterflies of a stage into registers, the block waits, then every
// thread writes its outputs, and the block waits again.  Radix-4 stages, with
// one radix-2 stage first when logn is odd; the result is in natural order.
// tw[m] = exp(-2 pi i m / n), m < n; inv conjugates the twiddles (no 1/n
// scaling).  Needs nl * n <= VALUES and nt = NTH.
template <typename T, int VALUES>
__device__ void stockham(Cx<T>* a, int logn, int nl, int ls, const Cx<T>* __restrict__ tw, bool inv, int tid,
                         int nt)
{
    const int n = 1 << logn;
    int Ns = 1;
    if (logn & 1) {
        // radix-2 stage with Ns = 1 (no twiddles)
        constexpr int MB = VALUES / 2 / NTH;
        const int half = n >> 1;
        Cx<T> v[MB][2];
#pragma unroll
        for (int c = 0; c < MB; c++) {
            const int t = tid + c * nt;
            if (t < nl * half) {
                const int l = t >> (logn - 1), j = t & (half - 1);
                v[c][0] = a[l * ls + j];
                v[c][1] = a[l * ls + j + half];
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < MB; c++) {
            const int t = tid + c * nt;
            if (t < nl * half) {
                const int l = t >> (logn - 1), j = t & (half - 1);
                a[l * ls + 2 * j] = { v[c][0].re + v[c][1].re, v[c][0].im + v[c][1].im };
                a[l * ls + 2 * j + 1] = { v[c][0].re - v[c][1].re, v[c][0].im - v[c][1].im };
            }
        }
        __syncthreads();
        Ns = 2;
    }
    constexpr int MB = VALUES / 4 / NTH;
    const int q = n >> 2;   // butterflies per line in a radix-4 stage
    const int lq = logn - 2;
    const T sgn = inv ? T(1) : T(-1);   // exp(sgn i pi / 2) = sgn i
    for (; Ns < n; Ns <<= 2) {
        const int tstep = n / (4 * Ns);   // twiddle index step of k
        Cx<T> v[MB][4];
#pragma unroll
        for (int c = 0; c < MB; c++) {
            const int t = tid + c * nt;
            if (t < nl * q) {
                const int l = t >> lq, j = t & (q - 1), k = j & (Ns - 1);
#pragma unroll
                for (int r = 0; r < 4; r++) v[c][r] = a[l * ls + j + r * q];
#pragma unroll
                for (int r = 1; r < 4; r++) {
                    Cx<T> w = tw[r * k * tstep];
                    if (inv) w.im = -w.im;
                    v[c][r] = cmul(v[c][r], w);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < MB; c++) {
            const int t = tid + c * nt;
            if (t < nl * q) {
                const int l = t >> lq, j = t & (q - 1), k = j & (Ns - 1);
                // radix-4 DFT: X_r = sum_s v_s (sgn i)^(r s)
                const Cx<T> s02 = { v[c][0].re + v[c][2].re, v[c][0].im + v[c][2].im };
                const Cx<T> d02 = { v[c][0].re - v[c][2].re, v[c][0].im - v[c][2].im };
                const Cx<T> s13 = { v[c][1].re + v[c][3].re, v[c][1].im + v[c][3].im };
                const Cx<T> d13 = { v[c][1].re - v[c][3].re, v[c][1].im - v[c][3].im };
                const Cx<T> rd = { -sgn * d13.im, sgn * d13.re };   // (sgn i) d13
                const int o = l * ls + ((j - k) << 2) + k;
                a[o] = { s02.re + s13.re, s02.im + s13.im };
                a[o + Ns] = { d02.re + rd.re, d02.im + rd.im };
                a[o + 2 * Ns] = { s02.re - s13.re, s02.im - s13.im };
                a[o + 3 * Ns] = { d02.re - rd.re, d02.im - rd.im };
            }
        }
        __syncthreads();
    }
}

template <typename T>
struct FftArgs {
    Geo g;
    const T* rho;             // density (forward x pass)
    Cx<T>* Z;                 // complex scratch, N values, cell order
    T* phi;                   // potential (inverse x pass)
    const Cx<T>* tw[3];       // per-axis twiddles exp(-2 pi i m / n), m < n
    const double* sf[3];      // per-axis 27-point stencil factors (3 - 2 sin^2(pi m / n)) / 3
    double gscale;            // -(2/3) pi G h^2 / N (Green's numerator with the 1/N of the inverse)
    int logn[3];
    int lpb;                  // x lines per block
    int tx;                   // x columns per block of the y/z passes
};

// Transforms along x: INV = 0 reads the density and writes its transform to
// Z; INV = 1 inverts Z and writes the real part, the potential.  Dynamic LDS:
// lpb x nx complex values.
template <typename T, int INV>
struct BFftX {
    static constexpr int NT = NTH;
    static constexpr bool XCD = false;
    using Args = FftArgs<T>;
    static __device__ __forceinline__ void run(const Args& A, int blk, int tid)
    {
        extern __shared__ unsigned char smem_raw[];
        const int n = A.g.nx, logn = A.logn[0];
        Cx<T>* a = reinterpret_cast<Cx<T>*>(smem_raw);
        const int lines = A.g.ny * A.g.nz;
        const int l0 = blk * A.lpb;
        for (int t = tid; t < A.lpb * n; t += NT) {
            const int line = l0 + (t >> logn);
            T re = T(0), im = T(0);
            if (line < lines) {
                const size_t c = (size_t)line * n + (t & (n - 1));
                if (INV) {
                    re = A.Z[c].re;
                    im = A.Z[c].im;
                } else {
                    re = A.rho[c];
                }
            }
            a[t].re = re;
            a[t].im = im;
        }
        __syncthreads();
        stockham<T, FFT_X_VALUES>(a, logn, A.lpb, n, A.tw[0], INV != 0, tid, NT);
        const Cx<T>* r = a;
        for (int t = tid; t < A.lpb * n; t += NT) {
            const int line = l0 + (t >> logn);
            if (line >= lines) continue;
            const size_t c = (size_t)line * n + (t & (n - 1));
            if (INV) A.phi[c] = r[t].re;
            else A.Z[c] = r[t];
        }
    }
};

// Transforms along D = y or z of tx adjacent x columns per block (row
// segments of tx values are read and written together).  MODE 0: forward;
// 1: inverse; 2 (D = z): forward, multiply by the Green's function of the
// 27-point stencil, inverse.  Dynamic LDS: tx x (n + 1) complex values (a
// padded line stride).
template <typename T, int D, int MODE>
struct BFftYZ {
    static constexpr int NT = NTH;
    static constexpr bool XCD = false;
    using Args = FftArgs<T>;
    static __device__ __forceinline__ void run(const Args& A, int blk, int tid)
    {
        extern __shared__ unsigned char smem_raw[];
        const Geo& g = A.g;
        const int n = D == 1 ? g.ny : g.nz, logn = A.logn[D];
        const int tx = A.tx, ls = n + 1;
        Cx<T>* a = reinterpret_cast<Cx<T>*>(smem_raw);
        const int ntx = (g.nx + tx - 1) / tx;
        const int x0 = (blk % ntx) * tx;
        const int o = blk / ntx;   // z index (D = y) or y index (D = z)
        const size_t stride = D == 1 ? (size_t)g.nx : (size_t)g.nxy;
        const size_t base = (size_t)x0 + (D == 1 ? (size_t)o * g.nxy : (size_t)o * g.nx);
        for (int t = tid; t < tx * n; t += NT) {
            const int p = t / tx, c = t - p * tx;
            T re = T(0), im = T(0);
            if (x0 + c < g.nx) {
                re = A.Z[base + p * stride + c].re;
                im = A.Z[base + p * stride + c].im;
            }
            a[c * ls + p].re = re;
            a[c * ls + p].im = im;
        }
        __syncthreads();
        stockham<T, FFT_YZ_VALUES>(a, logn, tx, ls, A.tw[D], MODE == 1, tid, NT);
        Cx<T>* r = a;
        if (MODE == 2) {
            // mode (kx, ky, kz) = (x0 + c, o, p); the zero mode (the mean
            // density of the periodic box) has no potential
            for (int t = tid; t < tx * n; t += NT) {
                const int c = t / n, p = t - c * n;
                const int kx = x0 + c;
                if (kx >= g.nx) continue;
                double f = 0.0;
                if (kx != 0 || o != 0 || p != 0)
                    f = A.gscale / (1.0 - A.sf[0][kx] * A.sf[1][o] * A.sf[2][p]);
                Cx<T>& v = r[c * ls + p];
                v.re *= T(f);
                v.im *= T(f);
            }
            __syncthreads();
            stockham<T, FFT_YZ_VALUES>(a, logn, tx, ls, A.tw[D], true, tid, NT);
        }
        for (int t = tid; t < tx * n; t += NT) {
            const int p = t / tx, c = t - p * tx;
            if (x0 + c < g.nx) A.Z[base + p * stride + c] = r[c * ls + p];
        }
    }
};

// ---------------------------------------------------------------- tail of the step, per cell

// The tail of the step for one cell (after ADV): H2 (and H+) clamped to the
// cell's hydrogen, FP64 chemistry, heating/cooling, the pressure-gated
// dual-energy sync (Sec. 2.8); E, e, h2, hp in and out, each output rounded
// to the storage type T as it is stored.  The caller stores E only with
// heating/cooling (nothing else changes it).
template <typename T>
__device__ __forceinline__ void tail_cell(const StepArgs& a, const ChemArgs& ch, double rho, double mx, double my,
                                          double mz, double bx, double by, double bz, double& E, double& e, double& h2,
                                          double& hp)
{
    const int ion = a.ion;
    const double dt = step_dt(a);
    h2 = h2 > rho ? rho : h2;
    h2 = h2 < 0.0 ? 0.0 : h2;
    if (ion) {
        hp = hp > rho - h2 ? rho - h2 : hp;
        hp = hp < 0.0 ? 0.0 : hp;
    }
    if (ch.on) {
        if (ion) chem_ion(ch, rho, e, h2, hp, dt, h2, hp);
        else h2 = chem_h2(ch, a.gamma, rho, e, h2, dt);
    }
    if (ch.cool) {
        double en = ion ? cooled_e_ion(ch, rho, e, h2, hp, dt) : cooled_e(ch, a.gamma, rho, e, h2, dt);
        E += en - e;
        e = en;
        E = (double)(T)E;
    }
    double K = 0.5 * (mx * mx + my * my + mz * mz) / rho;
    double M = 0.5 * (bx * bx + by * by + bz * bz);
    double ei = E - K - M;
    if (ei >= 1e-3 * E && (gamma_cell(ion, a.gamma, rho, h2, hp) - 1.0) * ei > M) e = ei;
    e = (double)(T)e;
    h2 = (double)(T)h2;
    if (ion) hp = (double)(T)hp;
}

// validity of a cell (flag bit 0 when not) and its CFL signal speed (zero
// for an invalid cell)
__device__ __forceinline__ double tail_speed(const StepArgs& a, double rho, double mx, double my, double mz, double E,
                                             double e, double bx, double by, double bz, double h2, double hp,
                                             uint32_t* flags)
{
    bool ok = rho > 0.0 && e > 0.0 && isfinite(rho) && isfinite(e) && isfinite(E) && isfinite(mx) && isfinite(my) &&
              isfinite(mz) && isfinite(bx) && isfinite(by) && isfinite(bz);
    if (!ok) atomicOr(flags, 1u);
    return ok ? cell_speed(gamma_cell(a.ion, a.gamma, rho, h2, hp), rho, mx, my, mz, e, bx, by, bz) : 0.0;
}

// ---------------------------------------------------------------- ADV

// ADV fluxes at the lower x face of every cell (Sec. 2.6): the sqrt(rho)-
// weighted face velocity and the upwind parabola average of NQ fields (NQ =
// 7, or 8 with the ionisation network), in the order rho, mx, my, mz, E, e,
// h2, hp; outputs NQ x N.  A block holds rpb segments of tx cells of x rows
// (whole rows when nx <= 256, else 256-cell pieces), each with three cells of
// its periodic row on either side, loaded coalesced into LDS behind one
// barrier; each thread then forms its face from the staged row, its 5-cell
// window read at fixed offsets (no per-neighbour wrap or address
// arithmetic).  Dynamic LDS: NQ x rpb x (tx + 6) values.
template <typename T, int NQ>
struct BAdvFaceXRow {
    static constexpr int NT = NTH;
    static constexpr bool XCD = false;
    struct Args {
        Geo g;
        CFields<T> U;
        T* F;
        StepArgs a;
        int tx, rpb, spr;   // segment width, segments per block, segments per row
    };
    static __device__ __forceinline__ void run(const Args& A, int blk, int tid)
    {
        extern __shared__ unsigned char smem_raw[];
        T* L = reinterpret_cast<T*>(smem_raw);
        const Geo& g = A.g;
        const int nx = g.nx, tx = A.tx, cw = tx + 6;
        const int LS = A.rpb * cw;   // staged cells per field
        const int nseg = g.ny * g.nz * A.spr;   // below 2^31: at most one segment per cell
        const int fld[8] = { RHO, MX, MY, MZ, EN, EI, H2, HP };
        // own cell
        const int sl = tid / tx, pos = tid - sl * tx;
        const int sg = blk * A.rpb + sl;
        bool act = false;
        size_t c = 0;
        int p = 0;
        if (sl < A.rpb && sg < nseg) {
            const int row = sg / A.spr, s0 = (sg - row * A.spr) * tx;
            const int w = min(tx, nx - s0);
            if (pos < w) {
                act = true;
                c = (size_t)row * nx + s0 + pos;
                p = sl * cw + pos + 3;
#pragma unroll
                for (int q = 0; q < NQ; q++) L[q * LS + p] = A.U.f[fld[q]][c];
            }
        }
        // halo: three cells of the periodic row on each side of each segment
        if (tid < 6 * A.rpb) {
            const int hs = tid / 6, k = tid - 6 * hs;
            const int hg = blk * A.rpb + hs;
            if (hg < nseg) {
                const int row = hg / A.spr, s0 = (hg - row * A.spr) * tx;
                const int w = min(tx, nx - s0);
                const int x = k < 3 ? s0 - 3 + k : s0 + w + k - 3;
                const int hp = hs * cw + (k < 3 ? k : w + k);
                const size_t hc = (size_t)row * nx + wrapc(x, nx);
#pragma unroll
                for (int q = 0; q < NQ; q++) L[q * LS + hp] = A.U.f[fld[q]][hc];
            }
        }
        __syncthreads();
        if (!act) return;
        const T ydx = T(A.a.theta * (step_dt(A.a) / A.a.h));
        // sqrt(rho)-weighted face velocity; sqrt(rho) v = m / sqrt(rho)
        const T* rho = L;
        const T* mx = L + LS;
        const T rl = rho[p - 1], rr = rho[p];
        const T rsl = rsqrt_nr(rl), rsr = rsqrt_nr(rr);
        const T vf = (mx[p - 1] * rsl + mx[p] * rsr) * rcp_nr(rl * rsl + rr * rsr);
        const bool upw = vf >= T(0);
        const T y = upw ? ydx * vf : ydx * (-vf);
        const int b = upw ? p - 3 : p - 2;
        const size_t N = (size_t)g.n;
        T out[NQ];
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            const T* u = L + q * LS;
            Par<T> P = parabola(u[b], u[b + 1], u[b + 2], u[b + 3], u[b + 4]);
            T qup = upw ? avg_right(P, y) : avg_left(P, y);
            out[q] = vf * qup;
        }
#pragma unroll
        for (int q = 0; q < NQ; q++) A.F[q * N + c] = out[q];
    }
};

// ADV faces along y, marched: each thread walks one y line over a segment of
// `seg` cells with a sliding 5-cell window of the NQ fields, so each cell's
// limited slope, lower interface value and parabola are formed once (the
// per-face kernel forms three slopes, two interface values and a parabola per
// face); the previous cell's right side and sqrt(rho) are carried.  The face
// takes the upwind average: the left cell's right part for vf >= 0, the right
// cell's left part otherwise (the same arithmetic as the x faces).  What is
// stored is each cell's flux difference F(upper face) - F(lower face), the
// value the update takes, so the segment forms one face more than it has
// cells (the upper face of its last cell, also formed by the next segment
// from the same window) and the update reads one value per field instead of
// two.
template <typename T, int NQ>
struct BAdvFaceMarchY {
    static constexpr int NT = NTH;
    static constexpr bool XCD = false;
    // two waves per SIMD (FP64 needs 220-230 registers; unbounded, the
    // scheduler may take a few more and halve that)
    static constexpr int MINW = sizeof(T) == 8 ? 2 : 1;
    struct Args {
        Geo g;
        CFields<T> U;
        T* F;
        StepArgs a;
        int seg;
    };
    static __device__ __forceinline__ void run(const Args& A, int blk, int tid)
    {
        const Geo& g = A.g;
        const size_t N = (size_t)g.n;
        const int seg = A.seg;
        const int nd = g.ny, no = g.nz;
        const int nseg = (nd + seg - 1) / seg;
        int t = blk * NT + tid;
        int i = t % g.nx;
        int rest = t / g.nx;
        int o = rest % no;
        int sgi = rest / no;
        if (sgi >= nseg) return;
        const int base = i + g.nxy * o;
        const int stride = g.nx;
        const int x0 = sgi * seg;
        const int x1 = min(x0 + seg, nd);
        const T ydx = T(A.a.theta * (step_dt(A.a) / A.a.h));
        const int fld[8] = { RHO, MX, MY, MZ, EN, EI, H2, HP };

        // window: w[q][m] = field q of cell x-2+m (after the slide of face x)
        T w[NQ][5];
#pragma unroll
        for (int m = 0; m < 5; m++) {
            int cc = base + wrapc(x0 - 3 + m, nd) * stride;
#pragma unroll
            for (int q = 0; q < NQ; q++) w[q][m] = A.U.f[fld[q]][cc];
        }
        // parabola of cell x0 - 1 (its right side is read by the first face),
        // the slope of cell x0 and the interface value at its lower face
        T pR[NQ], pdq[NQ], p6[NQ], dmc[NQ], fl[NQ];
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            T d0 = limited_slope(w[q][0], w[q][1], w[q][2]);
            T d1 = limited_slope(w[q][1], w[q][2], w[q][3]);
            T d2 = limited_slope(w[q][2], w[q][3], w[q][4]);
            T f0 = interface_value(w[q][1], w[q][2], d0, d1);
            T f1 = interface_value(w[q][2], w[q][3], d1, d2);
            Par<T> P = parabola_finish(w[q][0], w[q][1], w[q][2], w[q][3], w[q][4], f0, f1, d1);
            pR[q] = P.qR;
            pdq[q] = P.dq;
            p6[q] = P.q6;
            dmc[q] = d2;
            fl[q] = f1;
        }
        // 1 / sqrt(rho) of the face's left cell (window slot 2 before the
        // first slide is slot 1 of the first face)
        T rsl = rsqrt_nr(w[0][2]);
        // the cell entering the window, loaded one face ahead
        T nw[NQ];
        auto fetch = [&](int x) {
            int cn = base + wrapc(x + 2, nd) * stride;
#pragma unroll
            for (int q = 0; q < NQ; q++) nw[q] = A.U.f[fld[q]][cn];
        };
        fetch(x0);
        // the flux of the lower face of the cell before x: in registers, or
        // in the thread's own LDS slots where registers would not leave two
        // waves per SIMD (FP64 with the H+ field)
        constexpr bool PREV_LDS = sizeof(T) == 8 && NQ == 8;
        __shared__ T prev_lds[PREV_LDS ? NQ * NT : 1];
        T prev[PREV_LDS ? 1 : NQ];
        auto prev_of = [&](int q) -> T { return PREV_LDS ? prev_lds[q * NT + tid] : prev[q]; };
        for (int x = x0; x <= x1; x++) {
#pragma unroll
            for (int q = 0; q < NQ; q++) {
#pragma unroll
                for (int m = 0; m < 4; m++) w[q][m] = w[q][m + 1];
                w[q][4] = nw[q];
            }
            if (x < x1) fetch(x + 1);
            // sqrt(rho)-weighted face velocity from cells x-1 (slot 1) and x
            // (slot 2); sqrt(rho) v = m / sqrt(rho), m_y is field 2
            const T rsr = rsqrt_nr(w[0][2]);
            const T vf = (w[2][1] * rsl + w[2][2] * rsr) * rcp_nr(w[0][1] * rsl + w[0][2] * rsr);
            const bool upw = vf >= T(0);
            const T y = upw ? ydx * vf : ydx * (-vf);
            T flux[NQ];
#pragma unroll
            for (int q = 0; q < NQ; q++) {
                // the parabola of cell x (window slots 0..4 = cells x-2..x+2)
                T dn = limited_slope(w[q][2], w[q][3], w[q][4]);
                T fr = interface_value(w[q][2], w[q][3], dmc[q], dn);
                Par<T> P = parabola_finish(w[q][0], w[q][1], w[q][2], w[q][3], w[q][4], fl[q], fr, dmc[q]);
                Par<T> Pl;
                Pl.qR = pR[q];
                Pl.dq = pdq[q];
                Pl.q6 = p6[q];
                Pl.qL = T(0);
                T qup = upw ? avg_right(Pl, y) : avg_left(P, y);
                flux[q] = vf * qup;
                pR[q] = P.qR;
                pdq[q] = P.dq;
                p6[q] = P.q6;
                dmc[q] = dn;
                fl[q] = fr;
            }
            if (x > x0) {
                // cell x - 1: its upper face is face x
                const int c = base + (x - 1) * stride;
#pragma unroll
                for (int q = 0; q < NQ; q++) {
                    const T d = flux[q] - prev_of(q);
                    A.F[q * N + c] = d;
                }
            }
#pragma unroll
            for (int q = 0; q < NQ; q++) {
                if constexpr (PREV_LDS) prev_lds[q * NT + tid] = flux[q];
                else prev[q] = flux[q];
            }
            rsl = rsr;
        }
    }
};

// ADV z faces fused with the ADV update, for the advected fields Q0 ..
// Q0+NQ-1 of the order rho, mx, my, mz, E, e, h2, hp: each thread marches along z
// over a segment of cells with a sliding 6-cell window of those fields, so
// the flux at the upper z face of cell k is the lower one of cell k+1, and the
// update reads the x and y fluxes written by the x/y face kernels.  Same
// arithmetic as the x/y face kernels followed by a plain update.  The fields
// are split over several launches so that a thread holds a small window and
// more waves fit on a SIMD; every launch reads rho and mz of the two cells at
// each face for the face velocity.
template <typename T>
struct AdvZArgs {
    Geo g;
    CFields<T> U, S;
    Fields<T> O;
    const T* Fx;
    const T* Fy;
    StepArgs a;
    RK rk;
    int dbg;
    ZTile zt;
    // the tail of the step (TAIL launches only)
    ChemArgs ch;
    double* part;
    uint32_t* flags;
};

// TAIL (the field group E, e, h2 [, hp] of the step's last substage): the
// tail of the step runs on each cell as its new values are formed (rho and m
// are the substage's outputs of the first group, launched before; B is not
// changed by ADV), and the block's CFL speed maximum goes to part[blk]; the
// same arithmetic as BTail after the update.
template <typename T, int Q0, int NQ, bool TAIL = false>
struct BAdvZUpdate {
    static constexpr int NT = NTH;
    static constexpr bool XCD = false;
    static_assert(!TAIL || Q0 == 4, "the tail runs with the energy group");
    static constexpr int MINW = TAIL ? 2 : 1;
    static constexpr int UNROLL = TAIL ? 1 : 2;   // cells per trip of the march
    using Args = AdvZArgs<T>;
    // Along the march each cell's limited slope, lower interface value and
    // parabola are formed once: for the face between window slots 2 and 3
    // (cells k, k+1 of a window that starts at k-2) the parabola of cell k
    // was formed at the face below (pc: its right side), and the thread forms
    // that of cell k+1 from the carried slope d1 of cell k+1 and interface
    // value f1 at k+1/2; the face takes the upwind average.
    static __device__ __forceinline__ void zflux(const T w[NQ][6], T vf, T ydx, T pR[NQ], T pdq[NQ], T p6[NQ],
                                                 T d1[NQ], T f1[NQ], T out[NQ])
    {
        bool upw = vf >= T(0);
        T y = upw ? ydx * vf : ydx * (-vf);
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            T d2 = limited_slope(w[q][3], w[q][4], w[q][5]);
            T f2 = interface_value(w[q][3], w[q][4], d1[q], d2);
            Par<T> Pn = parabola_finish(w[q][1], w[q][2], w[q][3], w[q][4], w[q][5], f1[q], f2, d1[q]);
            Par<T> Pc;
            Pc.qR = pR[q];
            Pc.dq = pdq[q];
            Pc.q6 = p6[q];
            Pc.qL = T(0);
            T qup = upw ? avg_right(Pc, y) : avg_left(Pn, y);
            out[q] = vf * qup;
            pR[q] = Pn.qR;
            pdq[q] = Pn.dq;
            p6[q] = Pn.q6;
            d1[q] = d2;
            f1[q] = f2;
        }
    }
    static __device__ __forceinline__ void run(const Args& A, int blk, int tid)
    {
        int i, j, x0, x1;
        double smax = 0.0;
        if (ztile_cell(A.g, A.zt, blk, tid, i, j, x0, x1)) march(A, i, j, x0, x1, smax);
        if constexpr (TAIL) block_max_store(smax, A.part, blk);
    }
    static __device__ __forceinline__ void march(const Args& A, int i, int j, int x0, int x1, double& smax)
    {
        const Geo& g = A.g;
        const int nd = g.nz;
        const size_t N = (size_t)g.n;
        const int base = i + g.nx * j;
        const int stride = g.nxy;
        const T ydx = T(A.a.theta * (step_dt(A.a) / A.a.h));
        const T dtdx = T(step_dt(A.a) / A.a.h);
        const int fld[8] = { RHO, MX, MY, MZ, EN, EI, H2, HP };
        const T ra = T(A.rk.a), rb = T(A.rk.b);
        int ip = i + 1 == g.nx ? 0 : i + 1;
        int jp = j + 1 == g.ny ? 0 : j + 1;

        // window cells z = x0-3 .. x0+2 (slots 0..5): the first face is
        // x0-1/2.  vr, vm: rho and mz of slots 2 and 3, for the face velocity.
        T w[NQ][6];
        T vr[2], vm[2];
#pragma unroll
        for (int m = 0; m < 6; m++) {
            int cc = base + wrapc(x0 - 3 + m, nd) * stride;
#pragma unroll
            for (int q = 0; q < NQ; q++) w[q][m] = A.U.f[fld[Q0 + q]][cc];
            if (m == 2 || m == 3) {   // constant after unrolling
                vr[m - 2] = A.U.f[RHO][cc];
                vm[m - 2] = A.U.f[MZ][cc];
            }
        }
        auto velocity = [&]() {
            // sqrt(rho)-weighted face velocity; sqrt(rho) v = m / sqrt(rho)
            T rsl = rsqrt_nr(vr[0]), rsr = rsqrt_nr(vr[1]);
            return (vm[0] * rsl + vm[1] * rsr) * rcp_nr(vr[0] * rsl + vr[1] * rsr);
        };
        // the first face (slots 2, 3): both adjacent parabolas; then carry the
        // upper cell's right side, the slope of the cell above it and the
        // interface value between them
        T Flo[NQ], pR[NQ], pdq[NQ], p6[NQ], d1[NQ], f1[NQ];
        {
            const T vf = velocity();
            const bool upw = vf >= T(0);
            const T y = upw ? ydx * vf : ydx * (-vf);
#pragma unroll
            for (int q = 0; q < NQ; q++) {
                T s0 = limited_slope(w[q][0], w[q][1], w[q][2]);
                T s1 = limited_slope(w[q][1], w[q][2], w[q][3]);
                T s2 = limited_slope(w[q][2], w[q][3], w[q][4]);
                T s3 = limited_slope(w[q][3], w[q][4], w[q][5]);
                T i0 = interface_value(w[q][1], w[q][2], s0, s1);
                T i1 = interface_value(w[q][2], w[q][3], s1, s2);
                T i2 = interface_value(w[q][3], w[q][4], s2, s3);
                Par<T> Pl = parabola_finish(w[q][0], w[q][1], w[q][2], w[q][3], w[q][4], i0, i1, s1);
                Par<T> Pr = parabola_finish(w[q][1], w[q][2], w[q][3], w[q][4], w[q][5], i1, i2, s2);
                T qup = upw ? avg_right(Pl, y) : avg_left(Pr, y);
                Flo[q] = vf * qup;
                pR[q] = Pr.qR;
                pdq[q] = Pr.dq;
                p6[q] = Pr.q6;
                d1[q] = s3;
                f1[q] = i2;
            }
        }
        // the values cell x needs from beyond the window (cell x+3 entering
        // it; rho and mz of cell x+1 when the group holds neither) are loaded
        // one cell ahead, so the loads are in flight during the previous cell
        constexpr bool own_v = Q0 == 0 && NQ >= 4;   // rho and mz are window fields 0 and 3
        T nw[NQ], nvr = T(0), nvm = T(0);
        auto fetch = [&](int x) {
            int cn = base + wrapc(x + 3, nd) * stride;
#pragma unroll
            for (int q = 0; q < NQ; q++) nw[q] = A.U.f[fld[Q0 + q]][cn];
            if (!own_v) {
                int c1 = base + wrapc(x + 1, nd) * stride;
                nvr = A.U.f[RHO][c1];
                nvm = A.U.f[MZ][c1];
            }
        };
        fetch(x0);
        // two cells per trip halve the register moves of the window slide
        // (measured faster here; the face marches lose by it); one with the
        // tail, whose chemistry would double the registers
#pragma unroll UNROLL
        for (int x = x0; x < x1; x++) {
            // slide: window slots 0..5 = cells x-2 .. x+3
#pragma unroll
            for (int q = 0; q < NQ; q++) {
#pragma unroll
                for (int m = 0; m < 5; m++) w[q][m] = w[q][m + 1];
                w[q][5] = nw[q];
            }
            vr[0] = vr[1];
            vm[0] = vm[1];
            if constexpr (own_v) {
                vr[1] = w[0][3];
                vm[1] = w[3][3];
            } else {
                vr[1] = nvr;
                vm[1] = nvm;
            }
            if (x + 1 < x1) fetch(x + 1);
            // the cell's x/y flux differences and Runge-Kutta input, loaded
            // before the z flux is formed so the loads overlap it, and before
            // any store (the output fields may alias the inputs as far as the
            // compiler knows)
            int c = base + x * stride;
            int cxp = c - i + ip;
            int cyp = c + (jp - j) * g.nx;
            T dx[NQ], dy[NQ], sv[NQ];
#pragma unroll
            for (int q = 0; q < NQ; q++) {
                const size_t o = (size_t)(Q0 + q) * N;
                dx[q] = A.Fx[o + cxp] - A.Fx[o + c];
                dy[q] = A.Fy[o + c];   // the y march stored the difference
                sv[q] = A.S.f[fld[Q0 + q]][c];
            }
            // the tail's inputs: the first group's new rho and m, the face
            // field at the cell's lower and upper faces
            T tr[4], tb[6];
            if constexpr (TAIL) {
                tr[0] = A.O.f[RHO][c];
                tr[1] = A.O.f[MX][c];
                tr[2] = A.O.f[MY][c];
                tr[3] = A.O.f[MZ][c];
                tb[0] = A.O.f[BX][c];
                tb[1] = A.O.f[BX][cxp];
                tb[2] = A.O.f[BY][c];
                tb[3] = A.O.f[BY][cyp];
                tb[4] = A.O.f[BZ][c];
                tb[5] = A.O.f[BZ][c + (wrapc(x + 1, nd) - x) * stride];
            }
            // upper face of cell x: between slots 2 (cell x) and 3 (cell x+1)
            T Fup[NQ], nv[NQ];
            zflux(w, velocity(), ydx, pR, pdq, p6, d1, f1, Fup);
#pragma unroll
            for (int q = 0; q < NQ; q++) {
                T dz = Fup[q] - Flo[q];
                T inc = -dtdx * ((dx[q] + dy[q]) + dz);
                if (A.dbg) {
                    nv[q] = inc;
                } else {
                    T u = w[q][2];
                    nv[q] = (u + ra * (sv[q] - u)) + rb * inc;
                }
                Flo[q] = Fup[q];
            }
            if constexpr (TAIL) {
                // group fields E, e, h2 (, hp)
                const double rho = (double)tr[0], mx = (double)tr[1], my = (double)tr[2], mz = (double)tr[3];
                const double bx = 0.5 * ((double)tb[0] + (double)tb[1]);
                const double by = 0.5 * ((double)tb[2] + (double)tb[3]);
                const double bz = 0.5 * ((double)tb[4] + (double)tb[5]);
                double E = (double)nv[0], e = (double)nv[1], h2 = (double)nv[2];
                double hp = 0.0;
                if constexpr (NQ > 3) hp = (double)nv[3];
                tail_cell<T>(A.a, A.ch, rho, mx, my, mz, bx, by, bz, E, e, h2, hp);
                nv[0] = (T)E;
                nv[1] = (T)e;
                nv[2] = (T)h2;
                if constexpr (NQ > 3) nv[3] = (T)hp;
                const double spd = tail_speed(A.a, rho, mx, my, mz, E, e, bx, by, bz, h2, hp, A.flags);
                smax = spd > smax ? spd : smax;
            }
#pragma unroll
            for (int q = 0; q < NQ; q++) A.O.f[fld[Q0 + q]][c] = nv[q];
            if (Q0 == 0 && A.dbg) {
                A.O.f[BX][c] = T(0);
                A.O.f[BY][c] = T(0);
                A.O.f[BZ][c] = T(0);
            }
        }
    }
};

// ADV update with the x faces formed in the same kernel (boxes whose x rows
// fit a block).  A block holds rpb whole x rows (nx <= NT), one thread per
// column, and marches its rows along z over a segment of cells, like
// BAdvZUpdate (z faces from the sliding window, y fluxes from memory, the
// Runge-Kutta update; the tail of the step follows as a pass of its own).  At each plane the threads publish
// their cell's values in LDS and form the flux of their lower x face exactly
// as BAdvFaceXRow does (sqrt(rho)-weighted velocity, the upwind cell's
// parabola from its 5-cell window at fixed row offsets, periodic inside the
// row); the fluxes are exchanged through LDS for the x difference, so the x
// fluxes never pass through memory.  Each cell's limited slope is formed once
// by its own thread and shared through LDS (the per-face form computes the
// three slopes of the upwind window from the same operands, so the results
// are the same bits).  Three block barriers per plane (values, slopes,
// fluxes); the LDS is double-buffered by plane parity, so a buffer is
// rewritten only after every thread has passed the barriers that follow its
// last reads.  Dynamic LDS: 2 x (NV + 2 NQ) x NT values.  Threads beyond the block's rows (and the rows
// of a last, partial row group) reach every barrier: they read row 0 of the
// block, which is always a real row, and write nothing, to LDS or memory.
template <typename T>
struct AdvXZArgs {
    Geo g;
    CFields<T> U, S;
    Fields<T> O;
    const T* Fy;
    StepArgs a;
    RK rk;
    int dbg;
    int rpb;    // x rows per block (nx * rpb <= NT)
    int nrg;    // row groups: ceil(ny / rpb)
    int seg;    // z cells per block
};

template <typename T, int Q0, int NQ, int MAXT>
struct BAdvXZUpdate {
    static constexpr int NT = MAXT;
    static constexpr bool XCD = false;
    // rho and m of the cell are window fields 0-3 of the first group;
    // the energy group stages rho and mx of the cell as two more values
    static constexpr bool own_v = Q0 == 0 && NQ >= 4;
    static constexpr int NV = own_v ? NQ : NQ + 2;
    static constexpr int RI = own_v ? 0 : NQ;       // staged slot of rho
    static constexpr int MXI = own_v ? 1 : NQ + 1;  // staged slot of mx
    static constexpr int MINW = (sizeof(T) == 8 && Q0 == 0 && MAXT == 256) ? 3 : 1;
    using Args = AdvXZArgs<T>;
    static __device__ __forceinline__ void run(const Args& A, int blk, int tid)
    {
        extern __shared__ unsigned char smem_raw[];
        T* sm = reinterpret_cast<T*>(smem_raw);
        const Geo& g = A.g;
        const int nx = g.nx;
        const int r = tid / nx;
        const int i = tid - r * nx;
        const int rg = blk % A.nrg, sgi = blk / A.nrg;
        const int j0 = rg * A.rpb + r;
        const bool act = r < A.rpb && j0 < g.ny;
        // threads beyond the rows follow a column of row 0 of the block
        const int rr = act ? r : 0;
        const int j = act ? j0 : rg * A.rpb;
        const int k0 = sgi * A.seg, k1 = min(k0 + A.seg, g.nz);
        // threads of cells i-3 .. i+2 of the row
        int tx[6];
#pragma unroll
        for (int m = 0; m < 6; m++) tx[m] = rr * nx + wrapc(i + m - 3, nx);
        const int tme = rr * nx + i;
        march(A, sm, act, i, j, k0, k1, tx, tme);
    }
    static __device__ __forceinline__ void march(const Args& A, T* sm, bool act, int i, int j, int x0, int x1,
                                                 const int tx[6], int tme)
    {
        const Geo& g = A.g;
        const int nd = g.nz;
        const size_t N = (size_t)g.n;
        const int base = i + g.nx * j;
        const int stride = g.nxy;
        const T ydx = T(A.a.theta * (step_dt(A.a) / A.a.h));
        const T dtdx = T(step_dt(A.a) / A.a.h);
        const int fld[8] = { RHO, MX, MY, MZ, EN, EI, H2, HP };
        const T ra = T(A.rk.a), rb = T(A.rk.b);

        // window cells z = x0-3 .. x0+2 (slots 0..5); vr, vm: rho and mz of
        // slots 2 and 3 (z-face velocity); vx: mx of slots 2 and 3 (the
        // energy group's x-face velocity; the first group holds it in w)
        T w[NQ][6];
        T vr[2], vm[2], vx[2] = { T(0), T(0) };
#pragma unroll
        for (int m = 0; m < 6; m++) {
            int cc = base + wrapc(x0 - 3 + m, nd) * stride;
#pragma unroll
            for (int q = 0; q < NQ; q++) w[q][m] = A.U.f[fld[Q0 + q]][cc];
            if (m == 2 || m == 3) {
                vr[m - 2] = A.U.f[RHO][cc];
                vm[m - 2] = A.U.f[MZ][cc];
                if (!own_v) vx[m - 2] = A.U.f[MX][cc];
            }
        }
        auto velocity = [&]() {
            T rsl = rsqrt_nr(vr[0]), rsr = rsqrt_nr(vr[1]);
            return (vm[0] * rsl + vm[1] * rsr) * rcp_nr(vr[0] * rsl + vr[1] * rsr);
        };
        // the first z face (slots 2, 3), as BAdvZUpdate
        T Flo[NQ], pR[NQ], pdq[NQ], p6[NQ], d1[NQ], f1[NQ];
        {
            const T vf = velocity();
            const bool upw = vf >= T(0);
            const T y = upw ? ydx * vf : ydx * (-vf);
#pragma unroll
            for (int q = 0; q < NQ; q++) {
                T s0 = limited_slope(w[q][0], w[q][1], w[q][2]);
                T s1 = limited_slope(w[q][1], w[q][2], w[q][3]);
                T s2 = limited_slope(w[q][2], w[q][3], w[q][4]);
                T s3 = limited_slope(w[q][3], w[q][4], w[q][5]);
                T i0 = interface_value(w[q][1], w[q][2], s0, s1);
                T i1 = interface_value(w[q][2], w[q][3], s1, s2);
                T i2 = interface_value(w[q][3], w[q][4], s2, s3);
                Par<T> Pl = parabola_finish(w[q][0], w[q][1], w[q][2], w[q][3], w[q][4], i0, i1, s1);
                Par<T> Pr = parabola_finish(w[q][1], w[q][2], w[q][3], w[q][4], w[q][5], i1, i2, s2);
                T qup = upw ? avg_right(Pl, y) : avg_left(Pr, y);
                Flo[q] = vf * qup;
                pR[q] = Pr.qR;
                pdq[q] = Pr.dq;
                p6[q] = Pr.q6;
                d1[q] = s3;
                f1[q] = i2;
            }
        }
        T nw[NQ], nvr = T(0), nvm = T(0), nvx = T(0);
        auto fetch = [&](int x) {
            int cn = base + wrapc(x + 3, nd) * stride;
#pragma unroll
            for (int q = 0; q < NQ; q++) nw[q] = A.U.f[fld[Q0 + q]][cn];
            if (!own_v) {
                int c1 = base + wrapc(x + 1, nd) * stride;
                nvr = A.U.f[RHO][c1];
                nvm = A.U.f[MZ][c1];
                nvx = A.U.f[MX][c1];
            }
        };
        fetch(x0);
        auto plane = [&](int x) {
            // slide: window slots 0..5 = cells x-2 .. x+3
#pragma unroll
            for (int q = 0; q < NQ; q++) {
#pragma unroll
                for (int m = 0; m < 5; m++) w[q][m] = w[q][m + 1];
                w[q][5] = nw[q];
            }
            vr[0] = vr[1];
            vm[0] = vm[1];
            vx[0] = vx[1];
            if constexpr (own_v) {
                vr[1] = w[0][3];
                vm[1] = w[3][3];
            } else {
                vr[1] = nvr;
                vm[1] = nvm;
                vx[1] = nvx;
            }
            if (x + 1 < x1) fetch(x + 1);
            const int c = base + x * stride;
            // x faces of plane x: publish the cell, then its limited slope,
            // form the flux of its lower x face, exchange the fluxes
            T* vb = sm + (x & 1) * ((NV + 2 * NQ) * NT);
            T* db = vb + NV * NT;
            T* fb = db + NQ * NT;
            if (act) {
#pragma unroll
                for (int q = 0; q < NQ; q++) vb[q * NT + tme] = w[q][2];
                if constexpr (!own_v) {
                    vb[RI * NT + tme] = vr[0];
                    vb[MXI * NT + tme] = vx[0];
                }
            }
            __syncthreads();
            if (act) {
#pragma unroll
                for (int q = 0; q < NQ; q++) {
                    const T* u = vb + q * NT;
                    db[q * NT + tme] = limited_slope(u[tx[2]], w[q][2], u[tx[4]]);
                }
            }
            __syncthreads();
            T fx[NQ];
            {
                // sqrt(rho)-weighted face velocity; sqrt(rho) v = m / sqrt(rho)
                const T rl = vb[RI * NT + tx[2]], rr = vb[RI * NT + tme];
                const T rsl = rsqrt_nr(rl), rsr = rsqrt_nr(rr);
                const T vf = (vb[MXI * NT + tx[2]] * rsl + vb[MXI * NT + tme] * rsr) * rcp_nr(rl * rsl + rr * rsr);
                const bool upw = vf >= T(0);
                const T y = upw ? ydx * vf : ydx * (-vf);
                // the upwind cell's window: cells i-3 .. i+1 or i-2 .. i+2;
                // its slopes and those of its neighbours from LDS
                int ix[5];
#pragma unroll
                for (int m = 0; m < 5; m++) ix[m] = upw ? tx[m] : tx[m + 1];
#pragma unroll
                for (int q = 0; q < NQ; q++) {
                    const T* u = vb + q * NT;
                    const T* d = db + q * NT;
                    const T u0 = u[ix[0]], u1 = u[ix[1]], u2 = u[ix[2]], u3 = u[ix[3]], u4 = u[ix[4]];
                    const T dm_m = d[ix[1]], dm_0 = d[ix[2]], dm_p = d[ix[3]];
                    Par<T> P = parabola_finish(u0, u1, u2, u3, u4, interface_value(u1, u2, dm_m, dm_0),
                                               interface_value(u2, u3, dm_0, dm_p), dm_0);
                    T qup = upw ? avg_right(P, y) : avg_left(P, y);
                    fx[q] = vf * qup;
                    if (act) fb[q * NT + tme] = fx[q];
                }
            }
            __syncthreads();
            // the cell's y flux difference and Runge-Kutta input: loaded here,
            // before this plane's stores, so the z flux below hides their
            // latency; loaded at the top of the plane they lived through the
            // x faces and cost the registers of a third wave per SIMD (the
            // first FP64 group then spilled, and the reload of a spilled
            // address waited for the previous plane's stores)
            T dy[NQ], sv[NQ];
#pragma unroll
            for (int q = 0; q < NQ; q++) {
                const size_t o = (size_t)(Q0 + q) * N;
                dy[q] = A.Fy[o + c];   // the y march stored the difference
                sv[q] = A.S.f[fld[Q0 + q]][c];
            }
            // upper face of cell x along z: between slots 2 and 3
            T Fup[NQ], nv[NQ];
            BAdvZUpdate<T, Q0, NQ>::zflux(w, velocity(), ydx, pR, pdq, p6, d1, f1, Fup);
#pragma unroll
            for (int q = 0; q < NQ; q++) {
                T dx = fb[q * NT + tx[4]] - fx[q];
                T dz = Fup[q] - Flo[q];
                T inc = -dtdx * ((dx + dy[q]) + dz);
                if (A.dbg) {
                    nv[q] = inc;
                } else {
                    T u = w[q][2];
                    nv[q] = (u + ra * (sv[q] - u)) + rb * inc;
                }
                Flo[q] = Fup[q];
            }
            if (act) {
#pragma unroll
                for (int q = 0; q < NQ; q++) A.O.f[fld[Q0 + q]][c] = nv[q];
                if (Q0 == 0 && A.dbg) {
                    A.O.f[BX][c] = T(0);
                    A.O.f[BY][c] = T(0);
                    A.O.f[BZ][c] = T(0);
                }
            }
        };
        // FP32 groups without the H+ field take two planes per loop trip: the
        // window and the carried z-face values are renamed instead of moved
        // (four waves per SIMD instead of five; 7% faster at 512 and 1024
        // cells per row, level at 256).  FP64 and the H+ group keep one.
        int x = x0;
        if constexpr (sizeof(T) == 4 && Q0 + NQ <= 7) {
            for (; x + 1 < x1; x += 2) {
                plane(x);
                __builtin_amdgcn_sched_barrier(0);
                plane(x + 1);
            }
        }
        for (; x < x1; x++) plane(x);
    }
};

// ---------------------------------------------------------------- tail and reductions

// Tail of the step (after ADV) as a pass of its own: tail_cell on every cell,
// validity flag, per-block CFL speed maximum.  mode: 1 = full tail, 0 = speed
// only (state unchanged).  The step itself runs the tail inside its last ADV
// launch (BAdvZUpdate with TAIL).
template <typename T>
struct BTail {
    static constexpr int NT = NTH;
    static constexpr bool XCD = false;
    // in a resident loop the compiler keeps the chemistry's FP64 constants in
    // registers across tiles (174 instead of 98: half the waves per SIMD)
    static constexpr bool PERSIST = false;
    struct Args {
        Geo g;
        Fields<T> U;
        StepArgs a;
        ChemArgs ch;
        int mode;
        double* part;
        uint32_t* flags;
    };
    static __device__ __forceinline__ void run(const Args& A, int blk, int tid)
    {
        const Geo& g = A.g;
        int c = blk * NT + tid;
        double spd = 0.0;
        if (c < g.n) {
            int i, j, k;
            if ((g.nx & 63) == 0) {
                // every wave lies in one x row: its row is divided once, on
                // the scalar unit (signed there, so that the compiler does
                // not merge it with the per-thread division below)
                const int c0 = __builtin_amdgcn_readfirstlane(c);
                const int row = c0 / g.nx;
                j = row % g.ny;
                k = row / g.ny;
                i = (c0 - row * g.nx) + (c - c0);
            } else {
                decompose(g, c, i, j, k);
            }
            const Fields<T>& U = A.U;
            double rho = (double)U.f[RHO][c];
            double mx = (double)U.f[MX][c], my = (double)U.f[MY][c], mz = (double)U.f[MZ][c];
            double E = (double)U.f[EN][c];
            double e = (double)U.f[EI][c];
            double bx = 0.5 * ((double)U.f[BX][c] + (double)U.f[BX][nbr<0>(g, c, i, j, k, 1)]);
            double by = 0.5 * ((double)U.f[BY][c] + (double)U.f[BY][nbr<1>(g, c, i, j, k, 1)]);
            double bz = 0.5 * ((double)U.f[BZ][c] + (double)U.f[BZ][nbr<2>(g, c, i, j, k, 1)]);
            const int ion = A.a.ion;
            double h2 = (double)U.f[H2][c];
            double hp = ion ? (double)U.f[HP][c] : 0.0;
            if (A.mode == 1) {
                tail_cell<T>(A.a, A.ch, rho, mx, my, mz, bx, by, bz, E, e, h2, hp);
                if (A.ch.cool) U.f[EN][c] = (T)E;
                U.f[H2][c] = (T)h2;
                U.f[EI][c] = (T)e;
                if (ion) U.f[HP][c] = (T)hp;
            }
            spd = tail_speed(A.a, rho, mx, my, mz, E, e, bx, by, bz, h2, hp, A.flags);
        }
        block_max_store(spd, A.part, blk);
    }
};

// dt = cfl h / max speed over the per-block maxima (max is exact, so the
// result equals the minimum over cells of cfl h / speed)
struct BReduceDt {
    static constexpr int NT = 1024;
    static constexpr bool XCD = false;
    struct Args {
        const double* part;
        int nparts;
        double cflh;
        double* dt;
    };
    static __device__ __forceinline__ void run(const Args& A, int blk, int tid)
    {
        __shared__ double red[16];
        double m = 0.0;
        // unrolled so that several independent loads are in flight
#pragma unroll 8
        for (int t = tid; t < A.nparts; t += NT) m = A.part[t] > m ? A.part[t] : m;
        m = wave_max(m);
        if ((tid & 63) == 0) red[tid >> 6] = m;
        __syncthreads();
        if (tid == 0) {
            double r = red[0];
            for (int w = 1; w < 16; w++) r = red[w] > r ? red[w] : r;
            *A.dt = r > 0.0 ? A.cflh / r : 0.0;
        }
    }
};

// FP64 totals: per-block fixed-order sums of the NF fields
template <typename T>
struct BTotalsPartial {
    static constexpr int NT = NTH;
    static constexpr bool XCD = false;
    struct Args {
        Geo g;
        CFields<T> U;
        double* part;
    };
    static __device__ __forceinline__ void run(const Args& A, int blk, int tid)
    {
        __shared__ double red[NF][NTH / 64];
        int c = blk * NT + tid;
        int lane = tid & 63, wv = tid >> 6;
#pragma unroll
        for (int f = 0; f < NF; f++) {
            double v = c < A.g.n ? (double)A.U.f[f][c] : 0.0;
            v = wave_sum(v);
            if (lane == 0) red[f][wv] = v;
        }
        __syncthreads();
        if (tid < NF) {
            double s = 0.0;
            for (int w = 0; w < NTH / 64; w++) s += red[tid][w];
            A.part[(size_t)blk * NF + tid] = s;
        }
    }
};

struct BTotalsFinal {
    static constexpr int NT = 1024;
    static constexpr bool XCD = false;
    struct Args {
        const double* part;
        int nparts;
        double* out;
    };
    static __device__ __forceinline__ void run(const Args& A, int blk, int tid)
    {
        __shared__ double red[NF][16];
        int lane = tid & 63, wv = tid >> 6;
        for (int f = 0; f < NF; f++) {
            double s = 0.0;
            for (int t = tid; t < A.nparts; t += NT) s += A.part[(size_t)t * NF + f];
            s = wave_sum(s);
            if (lane == 0) red[f][wv] = s;
        }
        __syncthreads();
        if (tid < NF) {
            double s = 0.0;
            for (int w = 0; w < 16; w++) s += red[tid][w];
            A.out[tid] = s;
        }
    }
};

// ---------------------------------------------------------------- state conversion

// primitive (host order rho, vx, vy, vz, p, bx_f, by_f, bz_f, x_h2, x_hp) -> conserved
template <typename T>
struct BInit {
    static constexpr int NT = NTH;
    static constexpr bool XCD = false;
    struct Args {
        Geo g;
        const double* Wp;
        Fields<T> U;
        double gamma;
        int ion;
    };
    static __device__ __forceinline__ void run(const Args& A, int blk, int tid)
    {
        const Geo& g = A.g;
        int c = blk * NT + tid;
        if (c >= g.n) return;
        int i, j, k;
        decompose(g, c, i, j, k);
        const size_t N = (size_t)g.n;
        const double* Wp = A.Wp;
        double rho = Wp[c];
        double vx = Wp[N + c], vy = Wp[2 * N + c], vz = Wp[3 * N + c];
        double p = Wp[4 * N + c];
        double bxf = Wp[5 * N + c], byf = Wp[6 * N + c], bzf = Wp[7 * N + c];
        double bx = 0.5 * (bxf + Wp[5 * N + nbr<0>(g, c, i, j, k, 1)]);
        double by = 0.5 * (byf + Wp[6 * N + nbr<1>(g, c, i, j, k, 1)]);
        double bz = 0.5 * (bzf + Wp[7 * N + nbr<2>(g, c, i, j, k, 1)]);
        double h2 = Wp[8 * N + c] * rho, hp = Wp[9 * N + c] * rho;
        double e = p / (gamma_cell(A.ion, A.gamma, rho, h2, hp) - 1.0);
        A.U.f[RHO][c] = (T)rho;
        A.U.f[MX][c] = (T)(rho * vx);
        A.U.f[MY][c] = (T)(rho * vy);
        A.U.f[MZ][c] = (T)(rho * vz);
        A.U.f[EI][c] = (T)e;
        A.U.f[EN][c] = (T)(e + 0.5 * rho * (vx * vx + vy * vy + vz * vz) + 0.5 * (bx * bx + by * by + bz * bz));
        A.U.f[BX][c] = (T)bxf;
        A.U.f[BY][c] = (T)byf;
        A.U.f[BZ][c] = (T)bzf;
        A.U.f[H2][c] = (T)h2;
        A.U.f[HP][c] = (T)hp;
    }
};

template <typename T>
struct BFromF64 {
    static constexpr int NT = NTH;
    static constexpr bool XCD = false;
    struct Args {
        Geo g;
        const double* src;
        Fields<T> U;
    };
    static __device__ __forceinline__ void run(const Args& A, int blk, int tid)
    {
        int c = blk * NT + tid;
        if (c >= A.g.n) return;
        const size_t N = (size_t)A.g.n;
#pragma unroll
        for (int f = 0; f < NF; f++) A.U.f[f][c] = (T)A.src[f * N + c];
    }
};

template <typename T>
struct BToF64 {
    static constexpr int NT = NTH;
    static constexpr bool XCD = false;
    struct Args {
        Geo g;
        CFields<T> U;
        double* dst;
    };
    static __device__ __forceinline__ void run(const Args& A, int blk, int tid)
    {
        int c = blk * NT + tid;
        if (c >= A.g.n) return;
        const size_t N = (size_t)A.g.n;
#pragma unroll
        for (int f = 0; f < NF; f++) A.dst[f * N + c] = (double)A.U.f[f][c];
    }
};

struct BClearFlags {
    static constexpr int NT = 64;
    static constexpr bool XCD = false;
    struct Args {
        uint32_t* flags;
    };
    static __device__ __forceinline__ void run(const Args& A, int blk, int tid)
    {
        if (blk == 0 && tid == 0) *A.flags = 0u;
    }
};

}  // namespace mhd
