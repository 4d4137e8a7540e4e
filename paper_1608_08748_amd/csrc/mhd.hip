// Host runtime and C ABI (include/mhdchem.h) of the HIP implementation of one
// operator-split step of ideal MHD with H/H2 chemistry on a uniform periodic
// grid (Kulikov, Chernykh & Protasov, arXiv:1608.08748), for AMD MI355X.
//
// Stage names: NONADV is the paper's "eulerian" stage (Sec. 2.4, 2.5: pressure,
// Lorentz force, p dV work, face-field update); ADV is its "lagrangian" stage
// (Sec. 2.6: advection).
//
// Data layout in HBM: structure of arrays, one array of n cells per field,
// x fastest.  The state is split into three groups that are updated by
// different stages, each with three Runge-Kutta slots:
//   H = (rho, h2)            updated by ADV and the tail
//   M = (mx, my, mz, E, e)   updated by NONADV, ADV and the tail
//   B = (bx, by, bz)         updated by NONADV (face-centred, lower faces)
// so no stage copies a field it does not change.
//
// A step is a fixed program of kernel launches (mhd_kernels.hpp).  One box
// sends the program to its stream; the server runs the same program for every
// box in flight and merges the launches (one launch per program position over
// all boxes), so a box gets the same bits alone or in a batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "mhd_kernels.hpp"
#include "mhdchem.h"

static_assert(mhd::NF == MHD_NFIELDS, "conserved field count of the kernels and the C ABI");

using namespace mhd;

// ---------------------------------------------------------------- box

// launches whose event pairs the timing ring holds (a step makes at most a
// few dozen)
constexpr int EVCAP = 1024;

struct mhd_box {
    mhd_params p;
    Geo g;
    hipStream_t s;
    int prec;          // MHD_FP64 / MHD_FP32_MIXED
    size_t esz;        // bytes per stored value
    int nblocks;       // cell-parallel blocks of NTH threads
    char* slot[3];     // three Runge-Kutta copies of the NF fields
    char* F[3];        // per-direction face outputs, 7 x N each (8 x N with the ionisation network)
    double* part;      // per-block partials: NF x nblocks
    uint32_t* flags;
    double* dt_dev;
    double* tot_dev;
    int grav;          // self-gravity on
    char* phi;         // gravitational potential, N values
    char* tw[3];       // per-axis FFT twiddles (n complex values)
    double* sf[3];     // per-axis 27-point stencil factors (n values)
    int cur[3];        // current slot of the groups H, M, B
    // per-launch event timing (mhd_set_timing)
    int timing;
    int nev;
    hipEvent_t ev[2 * EVCAP];
    int evcls[EVCAP];
    int ev_ready;
    double tms[MHD_NKCLASS];
    int64_t tcnt[MHD_NKCLASS];
};

namespace {

enum { GH = 0, GM = 1, GB = 2 };
int group_of(int f)
{
    if (f == RHO || f == H2 || f == HP) return GH;
    if (f >= BX && f <= BZ) return GB;
    return GM;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t slot, F, part, misc, grav, total;
};

bool pow2_upto(int n, int cap) { return n >= 1 && n <= cap && (n & (n - 1)) == 0; }

// the FFT Poisson solve handles power-of-two axes up to 1024 cells
constexpr int FFT_MAX = 1024;

bool valid_physics(int32_t precision, double gamma, double cfl, double theta, int32_t chem, int32_t cool,
                   double nu, double Tu, double tu)
{
    if (!(gamma > 1.0) || !std::isfinite(gamma)) return false;
    if (!(cfl > 0.0) || !std::isfinite(cfl)) return false;
    if (!(theta >= 0.0) || !std::isfinite(theta)) return false;
    if (precision != MHD_FP64 && precision != MHD_FP32_MIXED) return false;
    if (chem != 0 && chem != 1) return false;
    if (cool != 0 && cool != 1) return false;
    if ((chem || cool) && !(nu > 0.0 && Tu > 0.0 && tu > 0.0)) return false;
    return true;
}

bool valid_dims(const int32_t n[3])
{
    for (int d = 0; d < 3; d++)
        if (n[d] < 1) return false;
    double c = (double)n[0] * n[1] * n[2];
    return c < 2147483647.0;
}

bool valid_params(const mhd_params* p)
{
    if (!p || !valid_dims(p->n)) return false;
    if (p->ionisation != 0 && p->ionisation != 1) return false;
    if (p->ionisation && !(p->n_unit_cm3 > 0.0 && p->T_unit_K > 0.0 && p->t_unit_s > 0.0)) return false;
    if (!(p->grav_G >= 0.0) || !std::isfinite(p->grav_G)) return false;
    if (p->grav_G > 0.0)
        for (int d = 0; d < 3; d++)
            if (!pow2_upto(p->n[d], FFT_MAX)) return false;
    return valid_physics(p->precision, p->gamma, p->cfl, p->theta, p->chemistry, p->cooling, p->n_unit_cm3,
                         p->T_unit_K, p->t_unit_s);
}

// face outputs per direction: 7 NONADV values, or 8 ADV fluxes with the
// ionisation network
size_t face_values(bool ion) { return ion ? NFACE + 1 : NFACE; }

ZTile ztile_of(const Geo& g, int nt, int txmax = 64);
int ztile_blocks(const Geo& g, const ZTile& z);

Layout layout_of(const int32_t n[3], int precision, bool grav, bool ion)
{
    Layout L;
    size_t N = (size_t)n[0] * n[1] * n[2];
    size_t esz = precision == MHD_FP64 ? 8 : 4;
    size_t nb = (N + NTH - 1) / NTH;
    L.slot = align256(NF * N * esz);
    size_t fbytes = align256(face_values(ion) * N * esz);
    // the face scratch doubles as host staging (MHD_NPRIM or NF FP64 fields)
    size_t stage = align256((size_t)NF * N * 8);
    L.F = 3 * fbytes > stage ? 3 * fbytes : stage;
    // per-block partials: the totals (NF per cell-parallel block) and the
    // CFL speed maxima of the z-marching update that runs the tail
    Geo g;
    g.nx = n[0];
    g.ny = n[1];
    g.nz = n[2];
    g.nxy = n[0] * n[1];
    g.n = (int)N;
    size_t zb = (size_t)ztile_blocks(g, ztile_of(g, NTH));
    L.part = align256((nb * NF > zb ? nb * NF : zb) * sizeof(double));
    L.misc = 3 * 256;
    // self-gravity: the potential and the FFT tables (the complex scratch of
    // the Poisson solve is the x face scratch, free at that point)
    L.grav = 0;
    if (grav) {
        L.grav = align256(N * esz);
        for (int d = 0; d < 3; d++) L.grav += align256((size_t)n[d] * 2 * esz) + align256(n[d] * 8);
    }
    L.total = 3 * L.slot + L.F + L.part + L.misc + L.grav;
    return L;
}

void box_bind(mhd_box* b, const mhd_params* p, const Layout& L)
{
    b->p = *p;
    b->g.nx = p->n[0];
    b->g.ny = p->n[1];
    b->g.nz = p->n[2];
    b->g.nxy = p->n[0] * p->n[1];
    b->g.n = p->n[0] * p->n[1] * p->n[2];
    b->s = reinterpret_cast<hipStream_t>(p->stream);
    b->prec = p->precision;
    b->esz = p->precision == MHD_FP64 ? 8 : 4;
    b->nblocks = (b->g.n + NTH - 1) / NTH;
    char* w = reinterpret_cast<char*>(p->workspace);
    for (int s = 0; s < 3; s++) {
        b->slot[s] = w;
        w += L.slot;
    }
    size_t fbytes = align256(face_values(p->ionisation != 0) * (size_t)b->g.n * b->esz);
    for (int d = 0; d < 3; d++) b->F[d] = w + d * fbytes;
    w += L.F;
    b->part = reinterpret_cast<double*>(w);
    w += L.part;
    b->flags = reinterpret_cast<uint32_t*>(w);
    b->dt_dev = reinterpret_cast<double*>(w + 256);
    b->tot_dev = reinterpret_cast<double*>(w + 512);
    w += L.misc;
    b->grav = p->grav_G > 0.0;
    b->phi = nullptr;
    for (int d = 0; d < 3; d++) {
        b->tw[d] = nullptr;
        b->sf[d] = nullptr;
    }
    if (b->grav) {
        b->phi = w;
        w += align256((size_t)b->g.n * b->esz);
        for (int d = 0; d < 3; d++) {
            b->tw[d] = w;
            w += align256((size_t)p->n[d] * 2 * b->esz);
            b->sf[d] = reinterpret_cast<double*>(w);
            w += align256((size_t)p->n[d] * 8);
        }
    }
    b->cur[0] = b->cur[1] = b->cur[2] = 0;
    b->timing = 0;
    b->nev = 0;
    b->ev_ready = 0;
    for (int c = 0; c < MHD_NKCLASS; c++) {
        b->tms[c] = 0.0;
        b->tcnt[c] = 0;
    }
}

template <typename T>
Fields<T> view(mhd_box* b, int sH, int sM, int sB)
{
    Fields<T> v;
    size_t N = (size_t)b->g.n;
    for (int f = 0; f < NF; f++) {
        int grp = group_of(f);
        int s = grp == GH ? sH : (grp == GM ? sM : sB);
        // without the ionisation network no kernel writes H+: it stays in
        // slot 0, where the state was loaded, whatever slot is current
        if (f == HP && !b->p.ionisation) s = 0;
        v.f[f] = reinterpret_cast<T*>(b->slot[s]) + f * N;
    }
    return v;
}

template <typename T>
CFields<T> cview(const Fields<T>& v)
{
    CFields<T> c;
    for (int f = 0; f < NF; f++) c.f[f] = v.f[f];
    return c;
}

int launch_status() { return hipGetLastError() == hipSuccess ? MHD_OK : MHD_EDEVICE; }

StepArgs step_args(mhd_box* b, double dt, bool dev)
{
    StepArgs a;
    a.dt_val = dt;
    a.dt_dev = dev ? b->dt_dev : nullptr;
    a.gamma = b->p.gamma;
    a.h = 1.0 / (double)b->p.n[0];
    a.theta = b->p.theta;
    // the bound is computed from the stored state: FP32 storage moves it by ~1e-7
    a.cfl_tol = b->prec == MHD_FP64 ? 1e-12 : 1e-4;
    a.ion = b->p.ionisation;
    return a;
}

ChemArgs chem_args(mhd_box* b)
{
    ChemArgs c;
    c.on = b->p.chemistry;
    c.cool = b->p.cooling;
    c.ion = b->p.ionisation;
    c.n_unit = b->p.n_unit_cm3;
    c.T_unit = b->p.T_unit_K;
    c.t_unit = b->p.t_unit_s;
    return c;
}

const RK rk_coef[3] = { { 0.0, 1.0 }, { 0.75, 0.25 }, { 1.0 / 3.0, 2.0 / 3.0 } };

struct Slots { int h, m, b; };

// ---------------------------------------------------------------- emitters

// event pair around one launch of class cls (no-op unless timing is on)
struct KTimer {
    mhd_box* b;
    int slot;
    KTimer(mhd_box* box, int cls) : b(box), slot(-1)
    {
        if (b && b->timing && b->nev < EVCAP) {
            slot = b->nev++;
            b->evcls[slot] = cls;
            (void)hipEventRecord(b->ev[2 * slot], b->s);
        }
    }
    ~KTimer()
    {
        if (slot >= 0) (void)hipEventRecord(b->ev[2 * slot + 1], b->s);
    }
};

int timing_collect(mhd_box* b)
{
    if (!b->timing || b->nev == 0) return MHD_OK;
    if (hipEventSynchronize(b->ev[2 * (b->nev - 1) + 1]) != hipSuccess) return MHD_EDEVICE;
    for (int i = 0; i < b->nev; i++) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, b->ev[2 * i], b->ev[2 * i + 1]) != hipSuccess) return MHD_EDEVICE;
        b->tms[b->evcls[i]] += ms;
        b->tcnt[b->evcls[i]] += 1;
    }
    b->nev = 0;
    return MHD_OK;
}

// sends each launch of the program straight to the box's stream
struct OneEmit {
    mhd_box* b;
    template <class Body>
    void launch(int cls, int blocks, size_t shm, const typename Body::Args& a)
    {
        if (blocks <= 0) return;
        KTimer t(b, cls);
        if (shm > 65536)
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_one<Body>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        k_one<Body><<<blocks, Body::NT, shm, b->s>>>(a);
    }
};

// one program position merged over many boxes
struct MultiRec {
    void (*go)(const void* tab, const int* bstart, int nbox, int blocks, size_t shm, hipStream_t s);
    int (*go_persist)(const void* tab, const int* bstart, int nbox, int blocks, size_t shm, hipStream_t s, int ncu,
                      int cap, int* next);
    std::vector<char> args;
    std::vector<int> bstart;
    int total;
    size_t shm;
    size_t off_args, off_bstart;   // offsets in the uploaded table
    size_t off_next;               // the launch's tile counter (uploaded as 0; persistent launches)
};

template <class Body>
void go_many(const void* tab, const int* bstart, int nbox, int blocks, size_t shm, hipStream_t s)
{
    if (shm > 65536)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_many<Body>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    k_many<Body><<<blocks, Body::NT, shm, s>>>(reinterpret_cast<const typename Body::Args*>(tab), bstart, nbox);
}

// resident workgroups per CU of k_persist<Body> with shm bytes of dynamic
// LDS (the occupancy query runs once per body and LDS size)
template <class Body>
int persist_per_cu(size_t shm)
{
    static std::mutex mu;
    static std::vector<std::pair<size_t, int>> known;
    std::lock_guard<std::mutex> lk(mu);
    for (const auto& kv : known)
        if (kv.first == shm) return kv.second;
    const void* f = reinterpret_cast<const void*>(&k_persist<Body>);
    if (shm > 65536) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, Body::NT, shm) != hipSuccess || nb < 1) return 0;
    known.push_back(std::make_pair(shm, nb));
    return nb;
}

// claims of tiles per workgroup of a persistent launch: the last claims
// balance the workgroups to within 1 / PERSIST_CLAIMS of their share
constexpr int PERSIST_CLAIMS = 8;

template <class Body>
int go_persist(const void* tab, const int* bstart, int nbox, int blocks, size_t shm, hipStream_t s, int ncu,
               int max_wg, int* next)
{
    if constexpr (!Persists<Body>::v) {
        go_many<Body>(tab, bstart, nbox, blocks, shm, s);
        return MHD_OK;
    } else {
        const int per_cu = persist_per_cu<Body>(shm);
        if (per_cu < 1) return MHD_EDEVICE;
        long cap = (long)per_cu * ncu;
        if (max_wg > 0 && max_wg < cap) cap = max_wg;
        const int grid = blocks < cap ? blocks : (int)cap;
        // about PERSIST_CLAIMS claims per workgroup
        const int chunk = std::max(1, blocks / (grid * PERSIST_CLAIMS));
        k_persist<Body><<<grid, Body::NT, shm, s>>>(reinterpret_cast<const typename Body::Args*>(tab), bstart, nbox,
                                                   blocks, chunk, next);
        return MHD_OK;
    }
}

struct MultiEmit {
    std::vector<MultiRec>* recs;
    size_t k;        // program position within the current box
    bool first;      // the first box defines the program
    bool mismatch;
    template <class Body>
    void launch(int, int blocks, size_t shm, const typename Body::Args& a)
    {
        if (first) {
            MultiRec r;
            r.go = &go_many<Body>;
            r.go_persist = &go_persist<Body>;
            r.total = 0;
            r.shm = 0;
            r.off_args = r.off_bstart = r.off_next = 0;
            recs->push_back(r);
        }
        if (k >= recs->size() || (*recs)[k].go != &go_many<Body>) {
            mismatch = true;
            return;
        }
        MultiRec& r = (*recs)[k++];
        const char* p = reinterpret_cast<const char*>(&a);
        r.args.insert(r.args.end(), p, p + sizeof(a));
        r.bstart.push_back(r.total);
        r.total += blocks > 0 ? blocks : 0;
        r.shm = shm > r.shm ? shm : r.shm;
    }
};

// ---------------------------------------------------------------- the step program

// z cells per thread in the z-marching update kernels
constexpr int ZMARCH_SEG = 32;

// tiles of the z-marching update kernels: 64 x cells (a wave) by nt / 64
// rows for blocks of nt threads, narrower for thin boxes
ZTile ztile_of(const Geo& g, int nt, int txmax)
{
    ZTile z;
    z.tx = g.nx < txmax ? g.nx : txmax;
    z.ty = nt / z.tx;
    z.ntx = (g.nx + z.tx - 1) / z.tx;
    z.nty = (g.ny + z.ty - 1) / z.ty;
    z.seg = g.nz < ZMARCH_SEG ? g.nz : ZMARCH_SEG;
    return z;
}

int ztile_blocks(const Geo& g, const ZTile& z)
{
    return z.ntx * z.nty * ((g.nz + z.seg - 1) / z.seg);
}

// The ADV update forms the x faces itself when whole x rows fit its block:
// blocks of 256 threads, or 512 for longer rows, or 1024 for FP32 state (the
// FP64 kernels need more than the 128 registers a 1024-thread block allows).
int xz_block_threads(const Geo& g, size_t esz)
{
    if (g.nx <= 256) return 256;
    if (g.nx <= 512) return 512;
    if (g.nx <= 1024 && esz == 4) return 1024;
    return 0;
}

bool adv_xz(const Geo& g, size_t esz) { return xz_block_threads(g, esz) > 0; }

// rows per block, row groups and z segment of the fused ADV update
void xz_tiling(const Geo& g, size_t esz, int& rpb, int& nrg, int& seg)
{
    rpb = xz_block_threads(g, esz) / g.nx;
    nrg = (g.ny + rpb - 1) / rpb;
    seg = g.nz < ZMARCH_SEG ? g.nz : ZMARCH_SEG;
}

int xz_blocks(const Geo& g, size_t esz)
{
    int rpb, nrg, seg;
    xz_tiling(g, esz, rpb, nrg, seg);
    return nrg * ((g.nz + seg - 1) / seg);
}

// One NONADV substage.  y and z faces first (marching kernels); then, for
// boxes whose x rows fit a block, the x-row face kernel, which also updates
// m, E and e, and the face-field update; otherwise the one-face-per-thread x
// kernel and the full update.  The primitives are formed inside the face
// kernels from the substage input state.
template <typename T, bool ION, class Emit>
void emit_nonadv_substage_t(mhd_box* b, Emit& e, Slots sin, Slots sS, Slots sout, const StepArgs& a, RK rk,
                            int dbg, bool first)
{
    Fields<T> in = view<T>(b, sin.h, sin.m, sin.b);
    Fields<T> S = view<T>(b, sS.h, sS.m, sS.b);
    Fields<T> out = view<T>(b, sout.h, sout.m, sout.b);
    const Geo& g = b->g;
    T* F0 = reinterpret_cast<T*>(b->F[0]);
    T* F1 = reinterpret_cast<T*>(b->F[1]);
    T* F2 = reinterpret_cast<T*>(b->F[2]);
    const T* phi = b->grav ? reinterpret_cast<const T*>(b->phi) : nullptr;
    FaceArgs<T> fa{};
    fa.g = g;
    fa.U = cview(in);
    fa.a = a;
    fa.flags = b->flags;
    fa.dt_cfl = nullptr;
    fa.S = cview(S);
    fa.O = out;
    fa.Fy = F1;
    fa.Fz = F2;
    fa.rk = rk;
    fa.dbg = dbg;
    fa.phi = phi;
    // y and z faces: marching segments
    constexpr int MARCH_SEG = 32;
    for (int D = 1; D <= 2; D++) {
        const int nd = D == 1 ? g.ny : g.nz;
        const int no = D == 1 ? g.nz : g.ny;
        fa.seg = nd < MARCH_SEG ? nd : MARCH_SEG;
        fa.rpb = 0;
        fa.F = D == 1 ? F1 : F2;
        long long threads = (long long)g.nx * no * ((nd + fa.seg - 1) / fa.seg);
        int blocks = (int)((threads + NTH - 1) / NTH);
        if (D == 1)
            e.template launch<BFaceMarch<T, 1, ION>>(MHD_K_NONADV_FACE, blocks, 0, fa);
        else
            e.template launch<BFaceMarch<T, 2, ION>>(MHD_K_NONADV_FACE, blocks, 0, fa);
    }
    // x faces; the launch of the first substage checks an explicit dt
    // against the last device CFL bound
    fa.F = F0;
    fa.seg = 0;
    fa.dt_cfl = first ? b->dt_dev : nullptr;
    const int maxt = sizeof(T) == 8 ? 512 : 1024;
    const bool rows = g.nx <= maxt;
    if (rows) {
        int rpb = g.nx >= 256 ? 1 : 256 / g.nx;
        fa.rpb = rpb;
        int blocks = (g.ny * g.nz + rpb - 1) / rpb;
        if (g.nx <= 256)
            e.template launch<BFaceXRows<T, 256, ION>>(MHD_K_NONADV_FACE, blocks, 256 * XROW_SLOTS * sizeof(T), fa);
        else if (g.nx <= 512)
            e.template launch<BFaceXRows<T, 512, ION>>(MHD_K_NONADV_FACE, blocks, 512 * XROW_SLOTS * sizeof(T), fa);
        else if constexpr (sizeof(T) == 4)   // 1024-thread rows only in FP32 (register budget)
            e.template launch<BFaceXRows<T, 1024, ION>>(MHD_K_NONADV_FACE, blocks, 1024 * XROW_SLOTS * sizeof(T), fa);
    } else {
        fa.rpb = 0;
        e.template launch<BFacePair<T, 0, ION>>(MHD_K_NONADV_FACE, b->nblocks, 0, fa);
    }
    NonadvUpdateArgs<T> ua;
    ua.g = g;
    ua.U = cview(in);
    ua.S = cview(S);
    ua.O = out;
    ua.Fx = F0;
    ua.Fy = F1;
    ua.Fz = F2;
    ua.a = a;
    ua.rk = rk;
    ua.dbg = dbg;
    ua.zt = ztile_of(g, UPD_NT, UPD_TX);
    ua.phi = phi;
    const int ublocks = ztile_blocks(g, ua.zt);
    if (rows)
        e.template launch<BNonadvUpdate<T, ION, false>>(MHD_K_NONADV_UPDATE, ublocks, 0, ua);
    else
        e.template launch<BNonadvUpdate<T, ION, true>>(MHD_K_NONADV_UPDATE, ublocks, 0, ua);
}

template <typename T, class Emit>
void emit_nonadv_substage(mhd_box* b, Emit& e, Slots sin, Slots sS, Slots sout, const StepArgs& a, RK rk, int dbg,
                          bool first)
{
    if (b->p.ionisation)
        emit_nonadv_substage_t<T, true>(b, e, sin, sS, sout, a, rk, dbg, first);
    else
        emit_nonadv_substage_t<T, false>(b, e, sin, sS, sout, a, rk, dbg, first);
}

template <typename T, int D, int NQ, class Emit>
void emit_adv_face(mhd_box* b, Emit& e, const Fields<T>& in, const StepArgs& a)
{
    if constexpr (D == 1) {
        // y faces: marched along y
        typename BAdvFaceMarchY<T, NQ>::Args ma;
        ma.g = b->g;
        ma.U = cview(in);
        ma.a = a;
        ma.F = reinterpret_cast<T*>(b->F[1]);
        constexpr int SEG = 32;
        ma.seg = b->g.ny < SEG ? b->g.ny : SEG;
        long long threads = (long long)b->g.nx * b->g.nz * ((b->g.ny + ma.seg - 1) / ma.seg);
        e.template launch<BAdvFaceMarchY<T, NQ>>(MHD_K_ADV_FACE, (int)((threads + NTH - 1) / NTH), 0, ma);
    } else {
        // x faces from row segments staged in LDS
        static_assert(D == 0, "y faces are marched");
        typename BAdvFaceXRow<T, NQ>::Args fa;
        const Geo& g = b->g;
        fa.g = g;
        fa.U = cview(in);
        fa.a = a;
        fa.F = reinterpret_cast<T*>(b->F[0]);
        fa.tx = g.nx < NTH ? g.nx : NTH;
        fa.spr = (g.nx + fa.tx - 1) / fa.tx;
        fa.rpb = NTH / fa.tx < NTH / 6 ? NTH / fa.tx : NTH / 6;   // 6 halo cells per segment, one per thread
        const long long nseg = (long long)g.ny * g.nz * fa.spr;
        const size_t shm = (size_t)NQ * fa.rpb * (fa.tx + 6) * sizeof(T);
        e.template launch<BAdvFaceXRow<T, NQ>>(MHD_K_ADV_FACE, (int)((nseg + fa.rpb - 1) / fa.rpb), shm, fa);
    }
}


// the two field-group launches of the fused ADV update with blocks of NT
// threads (dynamic LDS: 2 x (NV + 2 NQ) x NT values)
template <typename T, int NT, class Emit>
void emit_adv_xz(Emit& e, const AdvXZArgs<T>& xa, int blocks, bool ion)
{
    auto shm = [](int nv, int nq) { return (size_t)2 * (nv + 2 * nq) * NT * sizeof(T); };
    e.template launch<BAdvXZUpdate<T, 0, 4, NT>>(MHD_K_ADV_UPDATE, blocks, shm(4, 4), xa);   // rho, m
    if (ion) e.template launch<BAdvXZUpdate<T, 4, 4, NT>>(MHD_K_ADV_UPDATE, blocks, shm(6, 4), xa);
    else e.template launch<BAdvXZUpdate<T, 4, 3, NT>>(MHD_K_ADV_UPDATE, blocks, shm(5, 3), xa);
}

// tail: the step's last substage, whose energy-group launch runs the tail of
// the step and leaves the CFL speed maxima in b->part
template <typename T, class Emit>
void emit_adv_substage(mhd_box* b, Emit& e, Slots sin, Slots sS, Slots sout, const StepArgs& a, RK rk, int dbg,
                       bool tail = false)
{
    Fields<T> in = view<T>(b, sin.h, sin.m, sin.b);
    Fields<T> S = view<T>(b, sS.h, sS.m, sS.b);
    Fields<T> out = view<T>(b, sout.h, sout.m, sout.b);
    const bool ion = b->p.ionisation != 0;
    if (adv_xz(b->g, sizeof(T))) {
        // y faces marched along y; the x faces inside the z-marching update
        if (ion) emit_adv_face<T, 1, 8>(b, e, in, a);
        else emit_adv_face<T, 1, 7>(b, e, in, a);
        AdvXZArgs<T> xa;
        xa.g = b->g;
        xa.U = cview(in);
        xa.S = cview(S);
        xa.O = out;
        xa.Fy = reinterpret_cast<T*>(b->F[1]);
        xa.a = a;
        xa.rk = rk;
        xa.dbg = dbg;
        xz_tiling(b->g, sizeof(T), xa.rpb, xa.nrg, xa.seg);
        const int nt = xz_block_threads(b->g, sizeof(T));
        if (nt == 256) emit_adv_xz<T, 256>(e, xa, xz_blocks(b->g, sizeof(T)), ion);
        else if (nt == 512) emit_adv_xz<T, 512>(e, xa, xz_blocks(b->g, sizeof(T)), ion);
        else if constexpr (sizeof(T) == 4) emit_adv_xz<T, 1024>(e, xa, xz_blocks(b->g, sizeof(T)), ion);
        return;
    }
    // x faces from staged row segments, one face per thread; y faces marched
    // along y, each cell's parabola formed once
    if (ion) {
        emit_adv_face<T, 0, 8>(b, e, in, a);
        emit_adv_face<T, 1, 8>(b, e, in, a);
    } else {
        emit_adv_face<T, 0, 7>(b, e, in, a);
        emit_adv_face<T, 1, 7>(b, e, in, a);
    }
    // z faces marched together with the update of every cell
    AdvZArgs<T> ua;
    ua.g = b->g;
    ua.U = cview(in);
    ua.S = cview(S);
    ua.O = out;
    ua.Fx = reinterpret_cast<T*>(b->F[0]);
    ua.Fy = reinterpret_cast<T*>(b->F[1]);
    ua.a = a;
    ua.rk = rk;
    ua.dbg = dbg;
    ua.zt = ztile_of(b->g, NTH);
    ua.ch = chem_args(b);
    ua.part = b->part;
    ua.flags = b->flags;
    const int blocks = ztile_blocks(b->g, ua.zt);
    e.template launch<BAdvZUpdate<T, 0, 4>>(MHD_K_ADV_UPDATE, blocks, 0, ua);   // rho, m
    if (b->p.ionisation) {
        if (tail) e.template launch<BAdvZUpdate<T, 4, 4, true>>(MHD_K_ADV_UPDATE, blocks, 0, ua);
        else e.template launch<BAdvZUpdate<T, 4, 4>>(MHD_K_ADV_UPDATE, blocks, 0, ua);   // E, e, h2, hp
    } else {
        if (tail) e.template launch<BAdvZUpdate<T, 4, 3, true>>(MHD_K_ADV_UPDATE, blocks, 0, ua);
        else e.template launch<BAdvZUpdate<T, 4, 3>>(MHD_K_ADV_UPDATE, blocks, 0, ua);   // E, e, h2
    }
}

// NONADV stage: the M and B groups each rotate through their three slots
// (stage start S, then A, B, A); H is read from its current slot.
template <typename T, class Emit>
void emit_nonadv_stage(mhd_box* b, Emit& e, const StepArgs& a, bool first)
{
    int h = b->cur[GH], Sm = b->cur[GM], Sb = b->cur[GB];
    Slots S0 = { h, Sm, Sb };
    Slots A = { h, (Sm + 1) % 3, (Sb + 1) % 3 };
    Slots B2 = { h, (Sm + 2) % 3, (Sb + 2) % 3 };
    emit_nonadv_substage<T>(b, e, S0, S0, A, a, rk_coef[0], 0, first);
    emit_nonadv_substage<T>(b, e, A, S0, B2, a, rk_coef[1], 0, false);
    emit_nonadv_substage<T>(b, e, B2, S0, A, a, rk_coef[2], 0, false);
    b->cur[GM] = A.m;
    b->cur[GB] = A.b;
}

// ADV stage: the H and M groups rotate; B is read from its current slot
// tail: run the tail of the step inside the last substage (the step itself)
template <typename T, class Emit>
void emit_adv_stage(mhd_box* b, Emit& e, const StepArgs& a, bool tail = false)
{
    int Sh = b->cur[GH], Sm = b->cur[GM], bb = b->cur[GB];
    Slots S0 = { Sh, Sm, bb };
    Slots A = { (Sh + 1) % 3, (Sm + 1) % 3, bb };
    Slots B2 = { (Sh + 2) % 3, (Sm + 2) % 3, bb };
    emit_adv_substage<T>(b, e, S0, S0, A, a, rk_coef[0], 0);
    emit_adv_substage<T>(b, e, A, S0, B2, a, rk_coef[1], 0);
    emit_adv_substage<T>(b, e, B2, S0, A, a, rk_coef[2], 0, tail);
    b->cur[GH] = A.h;
    b->cur[GM] = A.m;
}

// dt from the per-block CFL speed maxima in b->part
template <class Emit>
void emit_reduce_dt(mhd_box* b, Emit& e, int nparts)
{
    BReduceDt::Args ra;
    ra.part = b->part;
    ra.nparts = nparts;
    ra.cflh = b->p.cfl * (1.0 / (double)b->p.n[0]);
    ra.dt = b->dt_dev;
    e.template launch<BReduceDt>(MHD_K_REDUCE, 1, 0, ra);
}

template <typename T, class Emit>
void emit_tail(mhd_box* b, Emit& e, const StepArgs& a, int mode)
{
    typename BTail<T>::Args ta;
    ta.g = b->g;
    ta.U = view<T>(b, b->cur[GH], b->cur[GM], b->cur[GB]);
    ta.a = a;
    ta.ch = chem_args(b);
    ta.mode = mode;
    ta.part = b->part;
    ta.flags = b->flags;
    e.template launch<BTail<T>>(MHD_K_TAIL, b->nblocks, 0, ta);
    emit_reduce_dt(b, e, b->nblocks);
}

int ilog2(int n)
{
    int l = 0;
    while ((1 << l) < n) l++;
    return l;
}

// Poisson stage (Sec. 2.9) on the current density: x forward, y forward,
// z forward + Green's function + z inverse, y inverse, x inverse
template <typename T, class Emit>
void emit_poisson(mhd_box* b, Emit& e)
{
    const Geo& g = b->g;
    FftArgs<T> fa;
    fa.g = g;
    fa.rho = reinterpret_cast<const T*>(b->slot[b->cur[GH]]) + (size_t)RHO * g.n;
    fa.Z = reinterpret_cast<Cx<T>*>(b->F[0]);
    fa.phi = reinterpret_cast<T*>(b->phi);
    for (int d = 0; d < 3; d++) {
        fa.tw[d] = reinterpret_cast<const Cx<T>*>(b->tw[d]);
        fa.sf[d] = b->sf[d];
        fa.logn[d] = ilog2(b->p.n[d]);
    }
    const double h = 1.0 / (double)b->p.n[0];
    fa.gscale = -(2.0 / 3.0) * M_PI * b->p.grav_G * h * h / (double)g.n;
    fa.lpb = g.nx >= FFT_X_VALUES ? 1 : FFT_X_VALUES / g.nx;
    const int lines = g.ny * g.nz;
    const int xb = (lines + fa.lpb - 1) / fa.lpb;
    const size_t xshm = (size_t)fa.lpb * g.nx * sizeof(Cx<T>);
    e.template launch<BFftX<T, 0>>(MHD_K_POISSON, xb, xshm, fa);
    // y and z passes: tx columns of a line set, tx x (n + 1) complex in LDS
    auto tx_of = [&](int n) {
        int t = FFT_YZ_VALUES / n;
        t = t < 1 ? 1 : t;
        return t > g.nx ? g.nx : t;
    };
    fa.tx = tx_of(g.ny);
    e.template launch<BFftYZ<T, 1, 0>>(MHD_K_POISSON, ((g.nx + fa.tx - 1) / fa.tx) * g.nz,
                                       (size_t)fa.tx * (g.ny + 1) * sizeof(Cx<T>), fa);
    fa.tx = tx_of(g.nz);
    e.template launch<BFftYZ<T, 2, 2>>(MHD_K_POISSON, ((g.nx + fa.tx - 1) / fa.tx) * g.ny,
                                       (size_t)fa.tx * (g.nz + 1) * sizeof(Cx<T>), fa);
    fa.tx = tx_of(g.ny);
    e.template launch<BFftYZ<T, 1, 1>>(MHD_K_POISSON, ((g.nx + fa.tx - 1) / fa.tx) * g.nz,
                                       (size_t)fa.tx * (g.ny + 1) * sizeof(Cx<T>), fa);
    e.template launch<BFftX<T, 1>>(MHD_K_POISSON, xb, xshm, fa);
}

// host-built FFT tables of a self-gravity box, uploaded on the box's stream;
// the caller synchronises before `host` goes out of scope
template <typename T>
int upload_grav_tables(mhd_box* b, std::vector<double>& host)
{
    if (!b->grav) return MHD_OK;
    for (int d = 0; d < 3; d++) {
        const int n = b->p.n[d];
        std::vector<T> tw((size_t)n * 2, T(0));
        for (int m = 0; m < n; m++) {
            const double t = 2.0 * M_PI * (double)m / (double)n;
            tw[2 * m] = (T)std::cos(t);
            tw[2 * m + 1] = (T)(-std::sin(t));
        }
        const size_t off = host.size();
        host.resize(off + (tw.size() * sizeof(T) + 7) / 8 + n);
        std::memcpy(host.data() + off, tw.data(), tw.size() * sizeof(T));
        double* sfh = host.data() + off + (tw.size() * sizeof(T) + 7) / 8;
        for (int m = 0; m < n; m++) {
            const double s = std::sin(M_PI * (double)m / (double)n);
            sfh[m] = (3.0 - 2.0 * s * s) / 3.0;
        }
    }
    size_t off = 0;
    for (int d = 0; d < 3; d++) {
        const int n = b->p.n[d];
        const size_t twb = (size_t)n * 2 * sizeof(T);
        if (hipMemcpyAsync(b->tw[d], host.data() + off, twb, hipMemcpyHostToDevice, b->s) != hipSuccess)
            return MHD_EDEVICE;
        off += (twb + 7) / 8;
        if (hipMemcpyAsync(b->sf[d], host.data() + off, (size_t)n * 8, hipMemcpyHostToDevice, b->s) !=
            hipSuccess)
            return MHD_EDEVICE;
        off += n;
    }
    return MHD_OK;
}

template <typename T, class Emit>
void emit_step(mhd_box* b, Emit& e, const StepArgs& a)
{
    if (b->grav) emit_poisson<T>(b, e);
    emit_nonadv_stage<T>(b, e, a, true);
    if (adv_xz(b->g, sizeof(T))) {
        // the fused ADV update forms x faces at every plane; with the tail's
        // FP64 chemistry on top it would spill, so the tail is a pass of its
        // own (the same arithmetic)
        emit_adv_stage<T>(b, e, a, false);
        emit_tail<T>(b, e, a, 1);
    } else {
        // the tail of the step runs inside the last ADV launch
        emit_adv_stage<T>(b, e, a, true);
        emit_reduce_dt(b, e, ztile_blocks(b->g, ztile_of(b->g, NTH)));
    }
}

// ---------------------------------------------------------------- single-box operations

template <typename T>
int full_step(mhd_box* b, double dt, bool dev)
{
    StepArgs a = step_args(b, dt, dev);
    OneEmit e{ b };
    emit_step<T>(b, e, a);
    int st = launch_status();
    if (st) return st;
    // the event ring is read (a wait on its last event) only once half of it
    // is used, so timed steps stay asynchronous
    return b->nev >= EVCAP / 2 ? timing_collect(b) : MHD_OK;
}

int sync_and_flags(mhd_box* b)
{
    uint32_t fl = 0;
    if (hipMemcpyAsync(&fl, b->flags, sizeof(fl), hipMemcpyDeviceToHost, b->s) != hipSuccess) return MHD_EDEVICE;
    if (hipStreamSynchronize(b->s) != hipSuccess) return MHD_EDEVICE;
    if (fl & 1u) return MHD_ENONPHYS;
    if (fl & 2u) return MHD_ECFL;
    return MHD_OK;
}

template <typename T>
int load_f64(mhd_box* b, const double* host, bool prim, bool wait = true)
{
    size_t N = (size_t)b->g.n;
    double* stage = reinterpret_cast<double*>(b->F[0]);
    size_t nf = prim ? MHD_NPRIM : NF;
    if (hipMemcpyAsync(stage, host, nf * N * sizeof(double), hipMemcpyHostToDevice, b->s) != hipSuccess)
        return MHD_EDEVICE;
    std::vector<double> tables;
    int tst = upload_grav_tables<T>(b, tables);
    if (tst) return tst;
    b->cur[GH] = b->cur[GM] = b->cur[GB] = 0;
    Fields<T> u = view<T>(b, 0, 0, 0);
    int saved = b->timing;
    b->timing = 0;
    OneEmit e{ b };
    if (prim) {
        typename BInit<T>::Args ia;
        ia.g = b->g;
        ia.Wp = stage;
        ia.U = u;
        ia.gamma = b->p.gamma;
        ia.ion = b->p.ionisation;
        e.template launch<BInit<T>>(MHD_K_SETUP, b->nblocks, 0, ia);
    } else {
        typename BFromF64<T>::Args ia;
        ia.g = b->g;
        ia.src = stage;
        ia.U = u;
        e.template launch<BFromF64<T>>(MHD_K_SETUP, b->nblocks, 0, ia);
    }
    BClearFlags::Args ca;
    ca.flags = b->flags;
    e.template launch<BClearFlags>(0, 1, 0, ca);
    StepArgs a = step_args(b, 0.0, false);
    emit_tail<T>(b, e, a, 0);
    b->timing = saved;
    int st = launch_status();
    if (st) return st;
    if (wait && hipStreamSynchronize(b->s) != hipSuccess) return MHD_EDEVICE;
    return MHD_OK;
}

template <typename T>
int get_f64(mhd_box* b, double* host)
{
    size_t N = (size_t)b->g.n;
    double* stage = reinterpret_cast<double*>(b->F[0]);
    typename BToF64<T>::Args ta;
    ta.g = b->g;
    ta.U = cview(view<T>(b, b->cur[GH], b->cur[GM], b->cur[GB]));
    ta.dst = stage;
    k_one<BToF64<T>><<<b->nblocks, NTH, 0, b->s>>>(ta);
    if (launch_status()) return MHD_EDEVICE;
    if (hipMemcpyAsync(host, stage, NF * N * sizeof(double), hipMemcpyDeviceToHost, b->s) != hipSuccess)
        return MHD_EDEVICE;
    return sync_and_flags(b);
}

template <typename T>
int totals_launch(mhd_box* b)
{
    typename BTotalsPartial<T>::Args pa;
    pa.g = b->g;
    pa.U = cview(view<T>(b, b->cur[GH], b->cur[GM], b->cur[GB]));
    pa.part = b->part;
    k_one<BTotalsPartial<T>><<<b->nblocks, NTH, 0, b->s>>>(pa);
    BTotalsFinal::Args fa;
    fa.part = b->part;
    fa.nparts = b->nblocks;
    fa.out = b->tot_dev;
    k_one<BTotalsFinal><<<1, BTotalsFinal::NT, 0, b->s>>>(fa);
    return launch_status();
}

template <typename T>
int totals(mhd_box* b, double* out)
{
    if (totals_launch<T>(b)) return MHD_EDEVICE;
    if (hipMemcpyAsync(out, b->tot_dev, NF * sizeof(double), hipMemcpyDeviceToHost, b->s) != hipSuccess)
        return MHD_EDEVICE;
    return sync_and_flags(b);
}

template <typename T>
int debug_stage(mhd_box* b, int stage, double dt)
{
    StepArgs a = step_args(b, dt, false);
    OneEmit e{ b };
    if (b->grav && (stage == MHD_STAGE_NONADV || stage == MHD_STAGE_NONADV_RHS)) emit_poisson<T>(b, e);
    switch (stage) {
    case MHD_STAGE_NONADV: emit_nonadv_stage<T>(b, e, a, false); break;
    case MHD_STAGE_ADV: emit_adv_stage<T>(b, e, a); break;
    case MHD_STAGE_TAIL: emit_tail<T>(b, e, a, 1); break;
    case MHD_STAGE_NONADV_RHS:
    case MHD_STAGE_ADV_RHS: {
        // tau R(U) of one substage into all ten fields of a free slot; needs
        // the three groups in one slot (true right after mhd_set_state)
        int S = b->cur[GM];
        if (b->cur[GH] != S || b->cur[GB] != S) return MHD_EINVAL;
        int O = (S + 1) % 3;
        Slots s0 = { S, S, S }, so = { O, O, O };
        if (stage == MHD_STAGE_NONADV_RHS)
            emit_nonadv_substage<T>(b, e, s0, s0, so, a, rk_coef[0], 1, false);
        else
            emit_adv_substage<T>(b, e, s0, s0, so, a, rk_coef[0], 1);
        b->cur[GH] = b->cur[GM] = b->cur[GB] = O;
        break;
    }
    default: return MHD_EINVAL;
    }
    return launch_status();
}

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// ---------------------------------------------------------------- server

struct mhd_server {
    mhd_server_params p;
    hipStream_t s;
    char* dtab;                // device launch tables (start of the workspace)
    char* htab;                // pinned host copy of the tables
    char* pool;                // the rest of the workspace: box allocations
    size_t pool_bytes;
    std::vector<std::pair<size_t, size_t>> freel;   // (offset, size), sorted by offset
    size_t used, peak;
    struct Pending {
        uint64_t id;
        mhd_request r;
        std::vector<double> prim;       // copied state, or
        const double* src = nullptr;    // the caller's state, borrowed
        double t_submit;
    };
    struct Active {
        uint64_t id;
        mhd_box* box;
        size_t off, bytes;
        int steps, done, keep;
        double t_submit, t_admit;
    };
    std::deque<Pending> pending;
    std::vector<Active> active;
    std::deque<mhd_completion> done;
    std::unordered_map<uint64_t, std::vector<double>> results;
    uint64_t next_id;
    double t0;
    std::vector<MultiRec> recs;
    // pipelined rounds: a call launches its round and then waits for the one
    // before; the boxes that finished in the last launched round have their
    // totals and flags on the way to pinned slots (slot k of the round's half)
    struct Retiring {
        Active a;
        int slot;
    };
    std::vector<Retiring> retiring;
    hipEvent_t ev[2];
    int ev_ready;
    int64_t rounds;        // rounds launched
    int ncu;               // compute units of the server's device (persistent launches)
    bool prev_launched;    // the previous call launched a round (event ev[(rounds - 1) & 1])
};

namespace {

constexpr size_t SERVER_TAB_BYTES = (size_t)32 << 20;   // launch tables of one round
constexpr int SERVER_MAX_SLOTS = 1024;
// pinned return slot of a finished box: NF totals and the fault flags
constexpr size_t SERVER_RET_BYTES = (NF + 1) * sizeof(double);
// pinned host area: two table halves (consecutive rounds alternate) and two
// sets of return slots
constexpr size_t SERVER_HOST_BYTES = 2 * SERVER_TAB_BYTES + 2 * SERVER_MAX_SLOTS * SERVER_RET_BYTES;
constexpr int SERVER_MAX_NX = 256;

bool pool_alloc(mhd_server* sv, size_t bytes, size_t* off)
{
    bytes = align256(bytes);
    for (size_t i = 0; i < sv->freel.size(); i++) {
        if (sv->freel[i].second >= bytes) {
            *off = sv->freel[i].first;
            sv->freel[i].first += bytes;
            sv->freel[i].second -= bytes;
            if (sv->freel[i].second == 0) sv->freel.erase(sv->freel.begin() + i);
            sv->used += bytes;
            if (sv->used > sv->peak) sv->peak = sv->used;
            return true;
        }
    }
    return false;
}

void pool_free(mhd_server* sv, size_t off, size_t bytes)
{
    bytes = align256(bytes);
    sv->used -= bytes;
    size_t i = 0;
    while (i < sv->freel.size() && sv->freel[i].first < off) i++;
    sv->freel.insert(sv->freel.begin() + i, std::make_pair(off, bytes));
    if (i + 1 < sv->freel.size() && sv->freel[i].first + sv->freel[i].second == sv->freel[i + 1].first) {
        sv->freel[i].second += sv->freel[i + 1].second;
        sv->freel.erase(sv->freel.begin() + i + 1);
    }
    if (i > 0 && sv->freel[i - 1].first + sv->freel[i - 1].second == sv->freel[i].first) {
        sv->freel[i - 1].second += sv->freel[i].second;
        sv->freel.erase(sv->freel.begin() + i);
    }
}

mhd_params box_params(const mhd_server* sv, const int32_t n[3], void* ws, size_t bytes)
{
    mhd_params bp;
    bp.n[0] = n[0];
    bp.n[1] = n[1];
    bp.n[2] = n[2];
    bp.gamma = sv->p.gamma;
    bp.cfl = sv->p.cfl;
    bp.precision = sv->p.precision;
    bp.theta = sv->p.theta;
    bp.chemistry = sv->p.chemistry;
    bp.cooling = sv->p.cooling;
    bp.grav_G = 0.0;   // served boxes run without self-gravity
    bp.ionisation = 0; // and without the ionisation network
    bp.n_unit_cm3 = sv->p.n_unit_cm3;
    bp.T_unit_K = sv->p.T_unit_K;
    bp.t_unit_s = sv->p.t_unit_s;
    bp.stream = sv->p.stream;
    bp.workspace = ws;
    bp.workspace_bytes = bytes;
    return bp;
}

int server_admit(mhd_server* sv)
{
    while (!sv->pending.empty() && (int)sv->active.size() < sv->p.max_slots) {
        mhd_server::Pending& q = sv->pending.front();
        Layout L = layout_of(q.r.n, sv->p.precision, false, false);
        size_t off;
        if (!pool_alloc(sv, L.total, &off)) break;   // first come, first served: wait for memory
        mhd_box* b = new (std::nothrow) mhd_box;
        if (!b) {
            pool_free(sv, off, L.total);
            return MHD_ENOMEM;
        }
        mhd_params bp = box_params(sv, q.r.n, sv->pool + off, L.total);
        box_bind(b, &bp, L);
        // a copied state is freed below, so its upload completes first; a
        // borrowed one stays valid until the completion is polled
        const double* src = q.src ? q.src : q.prim.data();
        const bool wait = q.src == nullptr;
        int st = sv->p.precision == MHD_FP64 ? load_f64<double>(b, src, true, wait)
                                             : load_f64<float>(b, src, true, wait);
        if (st) {
            delete b;
            pool_free(sv, off, L.total);
            return st;
        }
        mhd_server::Active a;
        a.id = q.id;
        a.box = b;
        a.off = off;
        a.bytes = L.total;
        a.steps = q.r.steps;
        a.done = 0;
        a.keep = q.r.keep_state;
        a.t_submit = q.t_submit;
        a.t_admit = now_s() - sv->t0;
        sv->active.push_back(a);
        sv->pending.pop_front();
    }
    return MHD_OK;
}

// one step of every active box, merged into one launch per program position
template <typename T>
int server_step(mhd_server* sv, int half)
{
    sv->recs.clear();
    MultiEmit e{ &sv->recs, 0, true, false };
    for (size_t i = 0; i < sv->active.size(); i++) {
        mhd_box* b = sv->active[i].box;
        e.k = 0;
        e.first = i == 0;
        StepArgs a = step_args(b, 0.0, true);
        emit_step<T>(b, e, a);
        if (e.mismatch || e.k != sv->recs.size()) return MHD_EINVAL;
    }
    // pack the tables into this round's half and upload them once
    size_t off = 0;
    for (MultiRec& r : sv->recs) {
        off = align256(off);
        r.off_args = off;
        off += r.args.size();
        off = align256(off);
        r.off_bstart = off;
        off += r.bstart.size() * sizeof(int);
        off = align256(off);
        r.off_next = off;
        off += sizeof(int);
    }
    if (off > SERVER_TAB_BYTES) return MHD_ENOMEM;
    char* h = sv->htab + (size_t)half * SERVER_TAB_BYTES;
    char* d = sv->dtab + (size_t)half * SERVER_TAB_BYTES;
    for (MultiRec& r : sv->recs) {
        memcpy(h + r.off_args, r.args.data(), r.args.size());
        memcpy(h + r.off_bstart, r.bstart.data(), r.bstart.size() * sizeof(int));
        memset(h + r.off_next, 0, sizeof(int));
    }
    if (hipMemcpyAsync(d, h, off, hipMemcpyHostToDevice, sv->s) != hipSuccess) return MHD_EDEVICE;
    int nbox = (int)sv->active.size();
    for (MultiRec& r : sv->recs) {
        if (r.total == 0) continue;
        const int* bs = reinterpret_cast<const int*>(d + r.off_bstart);
        if (sv->p.persistent) {
            int st = r.go_persist(d + r.off_args, bs, nbox, r.total, r.shm, sv->s, sv->ncu, sv->p.max_workgroups,
                                  reinterpret_cast<int*>(d + r.off_next));
            if (st) return st;
        } else {
            r.go(d + r.off_args, bs, nbox, r.total, r.shm, sv->s);
        }
    }
    return launch_status();
}

double* ret_slot(mhd_server* sv, int half, int k)
{
    return reinterpret_cast<double*>(sv->htab + 2 * SERVER_TAB_BYTES +
                                     ((size_t)half * SERVER_MAX_SLOTS + k) * SERVER_RET_BYTES);
}

// completion record of a box whose last round has finished (its totals and
// flags are in its return slot)
int server_retire(mhd_server* sv, mhd_server::Retiring& r, int half)
{
    mhd_server::Active& a = r.a;
    const double* slot = ret_slot(sv, half, r.slot);
    uint32_t fl;
    memcpy(&fl, slot + NF, sizeof(fl));
    mhd_completion c;
    memset(&c, 0, sizeof(c));
    c.id = a.id;
    c.steps = a.done;
    c.t_submit = a.t_submit;
    c.t_admit = a.t_admit;
    c.cells = (int64_t)a.box->g.n;
    c.bytes = a.bytes;
    memcpy(c.totals, slot, NF * sizeof(double));
    int s2 = (fl & 1u) ? MHD_ENONPHYS : (fl & 2u) ? MHD_ECFL : MHD_OK;
    c.status = s2;
    if (a.keep) {
        // the kept state is copied out before the box's memory is released
        std::vector<double> buf((size_t)NF * a.box->g.n);
        int s3 = sv->p.precision == MHD_FP64 ? get_f64<double>(a.box, buf.data())
                                             : get_f64<float>(a.box, buf.data());
        if (s3 == MHD_OK || s3 == s2) sv->results[a.id].swap(buf);
        else if (s3 == MHD_EDEVICE) return s3;
        pool_free(sv, a.off, a.bytes);
    }
    c.t_done = now_s() - sv->t0;
    sv->done.push_back(c);
    delete a.box;
    return MHD_OK;
}

int server_progress(mhd_server* sv, int* nact, int* npend)
{
    int st = server_admit(sv);
    if (st) return st;
    std::vector<mhd_server::Retiring> now_ret;
    const int half = (int)(sv->rounds & 1);
    bool launched = false;
    if (!sv->active.empty()) {
        st = sv->p.precision == MHD_FP64 ? server_step<double>(sv, half) : server_step<float>(sv, half);
        if (st) return st;
        // boxes that have run their steps leave the round: their totals and
        // flags go to pinned slots behind the round on the stream, and (unless
        // their state is kept) their memory returns to the pool at once, since
        // anything that reuses it is queued behind
        std::vector<mhd_server::Active> keep;
        for (mhd_server::Active& a : sv->active) {
            a.done++;
            if (a.done < a.steps) {
                keep.push_back(a);
                continue;
            }
            const int k = (int)now_ret.size();
            double* slot = ret_slot(sv, half, k);
            int s2 = sv->p.precision == MHD_FP64 ? totals_launch<double>(a.box) : totals_launch<float>(a.box);
            if (s2 ||
                hipMemcpyAsync(slot, a.box->tot_dev, NF * sizeof(double), hipMemcpyDeviceToHost, sv->s) != hipSuccess ||
                hipMemcpyAsync(slot + NF, a.box->flags, sizeof(uint32_t), hipMemcpyDeviceToHost, sv->s) != hipSuccess)
                return MHD_EDEVICE;
            now_ret.push_back({ a, k });
            if (!a.keep) pool_free(sv, a.off, a.bytes);
        }
        sv->active.swap(keep);
        if (hipEventRecord(sv->ev[half], sv->s) != hipSuccess) return MHD_EDEVICE;
        sv->rounds++;
        launched = true;
    }
    // the previous round: wait for it and report the boxes that finished in it
    if (sv->prev_launched) {
        const int ph = half ^ 1;   // round rounds - 1 (launched by the previous call)
        if (hipEventSynchronize(sv->ev[ph]) != hipSuccess) return MHD_EDEVICE;
        for (mhd_server::Retiring& r : sv->retiring) {
            st = server_retire(sv, r, ph);
            if (st) return st;
        }
        sv->retiring.clear();
    }
    sv->retiring.swap(now_ret);
    sv->prev_launched = launched;
    if (nact) *nact = (int)sv->active.size();
    if (npend) *npend = (int)sv->pending.size();
    return MHD_OK;
}

}  // namespace

// ---------------------------------------------------------------- C ABI

// ---------------------------------------------------------------- allocation-free totals

// Per-block partial sums of mhd_conserved_totals_noalloc: NF doubles for each
// 256-cell block of a box of at most MHD_NOALLOC_MAX_CELLS cells (5.5 MiB).
// Each device that loads the library holds its own copy until the process
// ends.  Host code never passes the array's name to a kernel (on the host it
// is a stand-in, not a device address): it uses the address that
// hipGetSymbolAddress returned for the current device.
constexpr size_t NOALLOC_BLOCKS = ((size_t)MHD_NOALLOC_MAX_CELLS + NTH - 1) / NTH;
static __device__ __align__(256) double scratch[NOALLOC_BLOCKS * NF];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[NOALLOC_MAX_DEVICES];

// device address of this device's scratch array, looked up once per device
// with that device current
int scratch_of_current_device(double** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) return MHD_EDEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MHD_EDEVICE;
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return MHD_OK;
}

template <typename T>
int totals_noalloc(const void* state, const Geo& g, hipStream_t s, double* part, double* out)
{
    typename BTotalsPartial<T>::Args pa;
    pa.g = g;
    const T* base = static_cast<const T*>(state);
    for (int f = 0; f < NF; f++) pa.U.f[f] = base + (size_t)f * (size_t)g.n;
    pa.part = part;
    const int nblocks = (g.n + NTH - 1) / NTH;
    k_one<BTotalsPartial<T>><<<nblocks, NTH, 0, s>>>(pa);
    BTotalsFinal::Args fa;
    fa.part = part;
    fa.nparts = nblocks;
    fa.out = out;
    k_one<BTotalsFinal><<<1, BTotalsFinal::NT, 0, s>>>(fa);
    return launch_status();
}

}  // namespace

extern "C" {

size_t mhd_workspace_bytes(const mhd_params* p)
{
    if (!valid_params(p)) return 0;
    return layout_of(p->n, p->precision, p->grav_G > 0.0, p->ionisation != 0).total;
}

int mhd_create(const mhd_params* p, mhd_box** out)
{
    if (!out) return MHD_EINVAL;
    *out = nullptr;
    if (!valid_params(p)) return MHD_EINVAL;
    Layout L = layout_of(p->n, p->precision, p->grav_G > 0.0, p->ionisation != 0);
    if (!p->workspace || p->workspace_bytes < L.total) return MHD_ENOMEM;
    if (((uintptr_t)p->workspace) & 255) return MHD_EINVAL;
    mhd_box* b = new (std::nothrow) mhd_box;
    if (!b) return MHD_ENOMEM;
    box_bind(b, p, L);
    *out = b;
    return MHD_OK;
}

int mhd_set_timing(mhd_box* b, int enable)
{
    if (!b) return MHD_EINVAL;
    if (enable && !b->ev_ready) {
        for (int i = 0; i < 2 * EVCAP; i++)
            if (hipEventCreate(&b->ev[i]) != hipSuccess) return MHD_EDEVICE;
        b->ev_ready = 1;
    }
    b->timing = enable ? 1 : 0;
    b->nev = 0;
    for (int c = 0; c < MHD_NKCLASS; c++) {
        b->tms[c] = 0.0;
        b->tcnt[c] = 0;
    }
    return MHD_OK;
}

int mhd_get_timing(mhd_box* b, double* ms, int64_t* counts)
{
    if (!b || !ms || !counts) return MHD_EINVAL;
    int st = timing_collect(b);
    if (st) return st;
    for (int c = 0; c < MHD_NKCLASS; c++) {
        ms[c] = b->tms[c];
        counts[c] = b->tcnt[c];
    }
    return MHD_OK;
}

int mhd_init_state(mhd_box* b, const double* prim)
{
    if (!b || !prim) return MHD_EINVAL;
    return b->prec == MHD_FP64 ? load_f64<double>(b, prim, true) : load_f64<float>(b, prim, true);
}

int mhd_set_state(mhd_box* b, const double* cons)
{
    if (!b || !cons) return MHD_EINVAL;
    return b->prec == MHD_FP64 ? load_f64<double>(b, cons, false) : load_f64<float>(b, cons, false);
}

int mhd_get_state(mhd_box* b, double* cons_out)
{
    if (!b || !cons_out) return MHD_EINVAL;
    return b->prec == MHD_FP64 ? get_f64<double>(b, cons_out) : get_f64<float>(b, cons_out);
}

int mhd_get_potential(mhd_box* b, double* phi_out)
{
    if (!b || !phi_out || !b->grav) return MHD_EINVAL;
    OneEmit e{ b };
    const size_t N = (size_t)b->g.n;
    if (b->prec == MHD_FP64) {
        emit_poisson<double>(b, e);
        if (launch_status()) return MHD_EDEVICE;
        if (hipMemcpyAsync(phi_out, b->phi, N * 8, hipMemcpyDeviceToHost, b->s) != hipSuccess) return MHD_EDEVICE;
        return sync_and_flags(b);
    }
    emit_poisson<float>(b, e);
    if (launch_status()) return MHD_EDEVICE;
    std::vector<float> tmp(N);
    if (hipMemcpyAsync(tmp.data(), b->phi, N * 4, hipMemcpyDeviceToHost, b->s) != hipSuccess) return MHD_EDEVICE;
    int st = sync_and_flags(b);
    for (size_t c = 0; c < N; c++) phi_out[c] = (double)tmp[c];
    return st;
}

int mhd_cfl_dt(mhd_box* b, double* dt_out)
{
    if (!b || !dt_out) return MHD_EINVAL;
    if (hipMemcpyAsync(dt_out, b->dt_dev, sizeof(double), hipMemcpyDeviceToHost, b->s) != hipSuccess)
        return MHD_EDEVICE;
    return sync_and_flags(b);
}

int mhd_step(mhd_box* b, double dt)
{
    if (!b || !std::isfinite(dt) || !(dt > 0.0)) return MHD_EINVAL;
    return b->prec == MHD_FP64 ? full_step<double>(b, dt, false) : full_step<float>(b, dt, false);
}

int mhd_step_cfl(mhd_box* b)
{
    if (!b) return MHD_EINVAL;
    return b->prec == MHD_FP64 ? full_step<double>(b, 0.0, true) : full_step<float>(b, 0.0, true);
}

int mhd_conserved_totals(mhd_box* b, double out[MHD_NFIELDS])
{
    if (!b || !out) return MHD_EINVAL;
    return b->prec == MHD_FP64 ? totals<double>(b, out) : totals<float>(b, out);
}

int mhd_conserved_totals_noalloc(const void* state, int32_t precision, const int32_t n[3], void* stream,
                                 double* out)
{
    if (!state || !n || !out || (precision != MHD_FP64 && precision != MHD_FP32_MIXED)) return MHD_EINVAL;
    if (!valid_dims(n)) return MHD_EINVAL;
    const int64_t cells = (int64_t)n[0] * n[1] * n[2];
    if (cells > MHD_NOALLOC_MAX_CELLS) return MHD_ETOOLARGE;
    double* part = nullptr;
    int st = scratch_of_current_device(&part);
    if (st) return st;
    Geo g;
    g.nx = n[0];
    g.ny = n[1];
    g.nz = n[2];
    g.nxy = n[0] * n[1];
    g.n = (int)cells;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    return precision == MHD_FP64 ? totals_noalloc<double>(state, g, s, part, out)
                                 : totals_noalloc<float>(state, g, s, part, out);
}

int mhd_debug_stage(mhd_box* b, int stage, double dt)
{
    if (!b) return MHD_EINVAL;
    if (stage != MHD_STAGE_TAIL && (!std::isfinite(dt) || !(dt > 0.0))) return MHD_EINVAL;
    if (stage == MHD_STAGE_TAIL && (!std::isfinite(dt) || dt < 0.0)) return MHD_EINVAL;
    return b->prec == MHD_FP64 ? debug_stage<double>(b, stage, dt) : debug_stage<float>(b, stage, dt);
}

int mhd_destroy(mhd_box* b)
{
    if (b && b->ev_ready)
        for (int i = 0; i < 2 * EVCAP; i++) (void)hipEventDestroy(b->ev[i]);
    delete b;
    return MHD_OK;
}

const char* mhd_strerror(int status)
{
    switch (status) {
    case MHD_OK: return "ok";
    case MHD_EINVAL: return "invalid argument";
    case MHD_ENOMEM: return "workspace missing or too small";
    case MHD_EDEVICE: return "HIP runtime error";
    case MHD_ECFL: return "time step above the CFL bound";
    case MHD_ENONPHYS: return "non-finite or non-positive density or internal energy";
    case MHD_ETOOLARGE: return "box larger than the static scratch of the allocation-free entry point";
    default: return "unknown status";
    }
}

size_t mhd_server_reserved_bytes(void) { return 2 * SERVER_TAB_BYTES; }

size_t mhd_server_box_bytes(const mhd_server_params* p, const int32_t n[3])
{
    if (!p || !n || !valid_dims(n)) return 0;
    if (p->precision != MHD_FP64 && p->precision != MHD_FP32_MIXED) return 0;
    return align256(layout_of(n, p->precision, false, false).total);
}

int mhd_server_create(const mhd_server_params* p, mhd_server** out)
{
    if (!out) return MHD_EINVAL;
    *out = nullptr;
    if (!p) return MHD_EINVAL;
    if (!valid_physics(p->precision, p->gamma, p->cfl, p->theta, p->chemistry, p->cooling, p->n_unit_cm3,
                       p->T_unit_K, p->t_unit_s))
        return MHD_EINVAL;
    if (p->max_slots < 1 || p->max_slots > SERVER_MAX_SLOTS) return MHD_EINVAL;
    if (p->persistent != 0 && p->persistent != 1) return MHD_EINVAL;
    if (p->max_workgroups < 0) return MHD_EINVAL;
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
        return MHD_EDEVICE;
    if (!p->workspace || p->workspace_bytes < 2 * SERVER_TAB_BYTES + 4096) return MHD_ENOMEM;
    if (((uintptr_t)p->workspace) & 255) return MHD_EINVAL;
    mhd_server* sv = new (std::nothrow) mhd_server;
    if (!sv) return MHD_ENOMEM;
    sv->p = *p;
    sv->s = reinterpret_cast<hipStream_t>(p->stream);
    sv->dtab = reinterpret_cast<char*>(p->workspace);
    sv->pool = sv->dtab + 2 * SERVER_TAB_BYTES;
    sv->pool_bytes = (p->workspace_bytes - 2 * SERVER_TAB_BYTES) & ~(size_t)255;
    sv->freel.push_back(std::make_pair((size_t)0, sv->pool_bytes));
    sv->used = sv->peak = 0;
    sv->next_id = 1;
    sv->t0 = now_s();
    sv->htab = nullptr;
    sv->rounds = 0;
    sv->ncu = ncu;
    sv->prev_launched = false;
    sv->ev_ready = 0;
    if (hipHostMalloc(reinterpret_cast<void**>(&sv->htab), SERVER_HOST_BYTES, hipHostMallocDefault) != hipSuccess) {
        delete sv;
        return MHD_EDEVICE;
    }
    if (hipEventCreateWithFlags(&sv->ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&sv->ev[1], hipEventDisableTiming) != hipSuccess) {
        (void)hipHostFree(sv->htab);
        delete sv;
        return MHD_EDEVICE;
    }
    sv->ev_ready = 1;
    *out = sv;
    return MHD_OK;
}

int mhd_server_submit(mhd_server* sv, const mhd_request* r, const double* prim, uint64_t* id)
{
    if (!sv || !r || !prim || !id) return MHD_EINVAL;
    if (!valid_dims(r->n) || r->steps < 1) return MHD_EINVAL;
    if (r->n[0] > SERVER_MAX_NX) return MHD_EINVAL;
    if (align256(layout_of(r->n, sv->p.precision, false, false).total) > sv->pool_bytes) return MHD_ENOMEM;
    mhd_server::Pending q;
    if (r->borrow != 0 && r->borrow != 1) return MHD_EINVAL;
    q.id = sv->next_id++;
    q.r = *r;
    size_t n = (size_t)r->n[0] * r->n[1] * r->n[2];
    if (r->borrow)
        q.src = prim;
    else
        q.prim.assign(prim, prim + (size_t)MHD_NPRIM * n);
    q.t_submit = now_s() - sv->t0;
    sv->pending.push_back(std::move(q));
    *id = sv->pending.back().id;
    return MHD_OK;
}

int mhd_server_progress(mhd_server* sv, int* n_active, int* n_pending)
{
    if (!sv) return MHD_EINVAL;
    return server_progress(sv, n_active, n_pending);
}

int mhd_server_poll(mhd_server* sv, mhd_completion* out, int cap, int* n)
{
    if (!sv || !n || (cap > 0 && !out)) return MHD_EINVAL;
    int k = 0;
    while (k < cap && !sv->done.empty()) {
        out[k++] = sv->done.front();
        sv->done.pop_front();
    }
    *n = k;
    return MHD_OK;
}

int mhd_server_result(mhd_server* sv, uint64_t id, double* cons_out, size_t count)
{
    if (!sv || !cons_out) return MHD_EINVAL;
    auto it = sv->results.find(id);
    if (it == sv->results.end()) return MHD_EINVAL;
    if (count != it->second.size()) return MHD_EINVAL;
    memcpy(cons_out, it->second.data(), count * sizeof(double));
    sv->results.erase(it);
    return MHD_OK;
}

int mhd_server_memory(mhd_server* sv, size_t* used, size_t* peak, size_t* capacity)
{
    if (!sv) return MHD_EINVAL;
    if (used) *used = sv->used;
    if (peak) *peak = sv->peak;
    if (capacity) *capacity = sv->pool_bytes;
    return MHD_OK;
}

int mhd_server_destroy(mhd_server* sv)
{
    if (!sv) return MHD_OK;
    (void)hipStreamSynchronize(sv->s);
    for (mhd_server::Active& a : sv->active) delete a.box;
    for (mhd_server::Retiring& r : sv->retiring) delete r.a.box;
    if (sv->ev_ready) {
        (void)hipEventDestroy(sv->ev[0]);
        (void)hipEventDestroy(sv->ev[1]);
    }
    if (sv->htab) (void)hipHostFree(sv->htab);
    delete sv;
    return MHD_OK;
}

}  // extern "C"
