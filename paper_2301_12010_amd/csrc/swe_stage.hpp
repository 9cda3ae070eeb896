// swe_stage.hpp - device code of one TVD-RK3 stage on one tile (gfx950).
//
// One stage computes out = a_n u^n + a_w (w + dt L(w)) (Methods, Eq. (8)) for
// every cell of a TX x TY tile, where L is the explicit operator of Eq. (7):
// the divergence of WENO5-reconstructed Lax-Friedrichs split fluxes
// (Methods, WENO and Lax-Friedrichs paragraphs) plus the cell-centred bed and
// Manning sources of Eqs. (2)-(3), with the bed taken relative to the datum.
//
// Work layout, per block:
//   1. the tile's input state (s, hu, hv, b) with a 3-cell halo is staged in
//      LDS in coalesced row passes (s is the stored level, see Geo); ghosts
//      are mirrored or read from frozen planes on the fly, so no separate
//      ghost pass exists.  The per-cell global reads that step 3 combines
//      (g n^2, u^n, residuals, the maximum-depth map) are issued next, so
//      their latency hides behind both sweeps;
//   2. x sweep: each thread walks R consecutive cells of one row, keeping a
//      3-cell window of split fluxes in registers.  Every cell centre's
//      second and first differences, the three smoothness indicators and the
//      four stencil polynomials are computed once and shared by the three
//      faces that use them; a face's WENO sums complete two centres later.
//      The x part of L goes to LDS;
//   3. y sweep: the same along columns; as soon as a cell's y part of L is
//      complete, its friction, RK combination, wet/dry fix-up and store
//      follow (no per-cell results wait in registers), then the epilogue
//      reductions (wave shuffles -> LDS -> at most one atomic per block and
//      quantity) of the next stage's wave speeds, the clamped mass and the
//      runup.  The FP64 mass is not on the step path: a separate
//      deterministic reduction computes it when the state is read.
// The arithmetic of a cell does not depend on the tile shape or on which
// launch runs the tile, so every tile variant and launch mode gives bitwise
// identical states.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swe {

constexpr int HALO = 3;
constexpr int BC_REFLECT = 0;
constexpr int BC_FIXED = 1;
constexpr int MASS_BLOCKS = 256;

// Per-scenario device scalars.  alpha[s] holds the float bits of the wave
// speeds of the input of stage s+1 (slot 0: u^n, 1: u^(1), 2: u^(2)).
struct alignas(64) DevScen {
    unsigned int alpha[3][2];
    float dt;              // step size of the step in flight (written by stage 1)
    unsigned int runup;    // float bits of the running max runup elevation
    unsigned int flags;    // bit 0: non-finite state seen
    unsigned int pad0;
    double t;              // simulated time (FP64)
    long long step;        // completed steps
    double mass_sum;       // sum of h over the grid (x dx dy), refreshed by the mass kernel
    double clamp_sum;      // weighted sum of clamped depth deficits (x dx dy on read)
    double pad1[2];
};

// Geometry, parameters and buffers of one scenario.
struct Geo {
    int nx, ny, pitch;       // pitch: row stride of every plane (elements)
    int bc[4];               // west, east, south, north
    float dx, dy, inv_dx, inv_dy;
    float g, half_g, h_dry, eps16;  // eps16 = 16 * weno_eps (the kernels' indicator scale)
    float kappa_cap, cfl, dt_fixed;
    int fric_implicit;       // 1: point-implicit friction (the host launches the IMP kernels)
    int local_split;         // 1: local Lax-Friedrichs splitting (the host launches the LLF kernels)
    const float *b, *gn2;    // bed and g n^2 planes
    // u^n, u^(1), u^(2): planes of (s, hu, hv) where s = h + min(b, 0) is the
    // stored level: the surface elevation h + b where the bed lies below the
    // datum, the depth h on land.  In deep water s stays small, so FP32 keeps
    // the surface to ~1e-7 m instead of an ulp of the depth (8e-6 m at 80 m),
    // and thin films on land keep their own precision.
    float *U[3], *A[3], *B[3];
    // optional residual planes of the stored level of U, A and B (null when
    // off): with them the level is kept as s + r, r the FP32 rounding error
    // of s, and the RK combination adds with error-free sums, so increments
    // below half an ulp of s are not lost (mass balance in shallow water)
    float *Rl[3];
    const float *ghost;      // frozen FIXED ghosts (s, hu, hv, b), see ghost_index()
    DevScen *sd;
    double *mass_part;       // MASS_BLOCKS partial sums of the mass kernel
    float *hmax;             // maximum-depth plane (same pitch), or null
};

// Frozen ghosts of a FIXED side: [field s,hu,hv,b][layer 0..2][position along the side].
// West/east sides have length ny and start at 0 and 12*ny; south/north have
// length nx and start at 24*ny and 24*ny + 12*nx.
__device__ __forceinline__ int ghost_index(const Geo &G, int side, int field, int layer, int pos)
{
    const int len = side < 2 ? G.ny : G.nx;
    const int base = side == 0 ? 0 : side == 1 ? 12 * G.ny : side == 2 ? 24 * G.ny : 24 * G.ny + 12 * G.nx;
    return base + (field * 3 + layer) * len + pos;
}

__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
// Hardware square root (v_sqrt_f32, within 1 ulp; no correctly-rounded
// expansion, which costs about ten more instructions).  It only enters wave
// speeds and the friction's |q|, whose results the FP64 checker bounds.
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
// min(x, 0) as one v_min_f32.  fminf on a value loaded from memory costs two
// instructions in IEEE mode (the compiler first quiets a possible signalling
// NaN); the bed values this takes are finite (checked at creation).
__device__ __forceinline__ float min0(float x)
{
    float r;
    asm("v_min_f32 %0, 0, %1" : "=v"(r) : "v"(x));
    return r;
}

// Error-free sum (Knuth): s + e == a + b exactly, s = fl(a + b).
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e)
{
    s = a + b;
    const float bv = s - a;
    e = (a - (s - bv)) + (b - bv);
}

// Plane element access by a 32-bit element index.  A plane holds fewer than
// 2^30 elements (checked at creation), so the byte offset fits 32 bits and the
// access takes the scalar-base + 32-bit vector-offset form: one offset
// register serves every plane, with no 64-bit address arithmetic per plane.
// The access is declared global: for a Geo read from a table (the batched
// kernels) the compiler cannot infer where its plane pointers point and
// would emit flat accesses, which count on the same wait counter as LDS
// reads, so every LDS wait of the sweeps would also wait for HBM loads.
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) char gchar;
__device__ __forceinline__ float pld(const float *p, unsigned i)
{
    return *(const gfloat *)((const gchar *)p + (size_t)(i << 2));
}
__device__ __forceinline__ void pst(float *p, unsigned i, float v)
{
    *(gfloat *)((gchar *)p + (size_t)(i << 2)) = v;
}

template <int TX_, int TY_, int R_>
struct TileCfg {
    static constexpr int TX = TX_, TY = TY_, R = R_;
    static constexpr int NT = TX * TY / R;         // threads per block
    static constexpr int WX = TX + 2 * HALO;       // staged columns
    static constexpr int WY = TY + 2 * HALO;       // staged rows
    static constexpr int SX = WX + 1;              // odd LDS row stride
    static constexpr int PLANE = SX * WY;
    static constexpr int XR = TX + 1;              // row stride of the x-sweep results
    static constexpr int XPLANE = XR * TY;
    static constexpr int LDS_FLOATS = 4 * PLANE + 3 * XPLANE;
    static_assert(TX % R == 0 && TY % R == 0, "R must divide the tile");
    static_assert(NT % 64 == 0, "whole wavefronts");
};

// Sweep constants shared by the x and y sweeps.
struct SweepK {
    float a;        // alpha of the sweep direction
    float hinv_ds;  // 1/(2 dx) or 1/(2 dy)
    float ghinv_ds; // -g/(2 dx) or -g/(2 dy)
    float g, half_g, h_dry;
    float e0, e1, e2;  // 16 eps / sqrt(d_k)
};

// Scales.  The sweeps reconstruct the doubled split fluxes F +- alpha u~
// (twice the split fluxes); the halving is folded into the final difference.
// A centre's smoothness indicators are carried as (13/3) D^2 + s^2 of the
// doubled values, i.e. 16 beta, so epsilon enters as 16 eps.  Scaling all
// three indicators and epsilon by one factor scales the unnormalised weights
// by one factor, which the normalisation removes.
//
// WENO5 linear weights d = (1/10, 6/10, 3/10) enter as 1/sqrt(d_k): the
// unnormalised weight d_k / (eps + beta_k)^2 is computed as 1/t^2 with
// t = (eps + beta_k) / sqrt(d_k).
constexpr float KD0 = 3.16227766016838f;  // 1/sqrt(0.1)
constexpr float KD1 = 1.29099444873581f;  // 1/sqrt(0.6)
constexpr float KD2 = 1.82574185835055f;  // 1/sqrt(0.3)

__device__ __forceinline__ float wt(float beta12, float kd, float ek)
{
    const float r = frcp(fmaf(beta12, kd, ek));
    return r * r;
}

// One sweep along x (DIR 0) or y (DIR 1) over R cells.  li0 is the LDS index
// of the window cell 3 before the first cell, st the LDS step between cells.
// emit(k, L0, L1, L2) receives, as soon as cell k's second face completes,
// the sweep's part of L for that cell: -(Fhat_{k+1/2} - Fhat_{k-1/2})/ds, plus
// the bed term -g (h + min(b, 0))(bhat_{k+1/2} - bhat_{k-1/2})/ds on the momentum
// component normal to the faces.
template <int R, int DIR, class Emit>
__device__ __forceinline__ void sweep(const float *__restrict__ Ls, const float *__restrict__ Lhu,
                                      const float *__restrict__ Lhv, const float *__restrict__ Lb,
                                      int li0, int st, const SweepK &K, Emit &&emit)
{
    constexpr int NF = R + 1;                 // faces k-1/2 for k = 0..R
    constexpr int MB = DIR == 0 ? 1 : 2;      // component whose weights reconstruct b
    // accumulators start at -0, the additive identity the compiler may fold
    // away (x + -0 == x for every x), so a first contribution costs no add
    float np_[NF][3], dp_[NF][3], nm_[NF][3], dm_[NF][3], nbp[NF], nbm[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
#pragma unroll
        for (int m = 0; m < 3; ++m) np_[f][m] = dp_[f][m] = nm_[f][m] = dm_[f][m] = -0.f;
        nbp[f] = nbm[f] = -0.f;
    }
    float win[3][7];   // rolling window: F+ (3), F- (3), b
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int q = 0; q < 7; ++q) win[s][q] = 0.f;
    float eta[R];
    float fprev[3] = {0.f, 0.f, 0.f}, bprev = 0.f;

#pragma unroll
    for (int w = -HALO; w < R + HALO; ++w) {
        const int li = li0 + (w + HALO) * st;
        const float sv = Ls[li], hu = Lhu[li], hv = Lhv[li], b = Lb[li];
        // the bed enters relative to the datum: lo = min(b, 0), the level of
        // zero depth below it.  The stored level is sv = h + lo (see Geo), the
        // pressure 1/2 g (h^2 - lo^2) = 1/2 g (h - lo) sv, the LF split vector
        // u~ = (sv, hu, hv) and the bed term's coefficient sv: the printed
        // (h + b) form below the datum, the depth form on land, where dry
        // cells then carry no flux at all
        const float lo = min0(b);
        const float h = sv - lo;
        const float inv = h > K.h_dry ? frcp(h) : 0.f;
        const float pres = K.half_g * (h - lo) * sv;
        float F0, F1, F2;
        if (DIR == 0) {
            F0 = hu;
            F1 = fmaf(hu, hu * inv, pres);
            F2 = hu * (hv * inv);
        } else {
            F0 = hv;
            F1 = hv * (hu * inv);
            F2 = fmaf(hv, hv * inv, pres);
        }
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            win[0][q] = win[1][q];
            win[1][q] = win[2][q];
        }
        win[2][0] = fmaf(K.a, sv, F0);
        win[2][1] = fmaf(K.a, hu, F1);
        win[2][2] = fmaf(K.a, hv, F2);
        win[2][3] = fmaf(-K.a, sv, F0);
        win[2][4] = fmaf(-K.a, hu, F1);
        win[2][5] = fmaf(-K.a, hv, F2);
        win[2][6] = b;
        if (w >= 0 && w < R) eta[w >= 0 && w < R ? w : 0] = sv;
        if (w < -1) continue;

        const int c = w - 1;  // cell centre whose three cells are now in the window
        // stencil polynomials of b at this centre (shared by both directions)
        float bRR, bR, bL, bLL;
        {
            const float D = fmaf(-2.f, win[1][6], win[0][6] + win[2][6]);
            const float E = win[2][6] - win[0][6];
            const float t0 = fmaf(D, 1.f / 12.f, win[1][6]);
            const float t1 = t0 + D;
            bR = fmaf(E, 0.25f, t0);
            bL = fmaf(E, -0.25f, t0);
            bRR = fmaf(E, 0.75f, t1);
            bLL = fmaf(E, -0.75f, t1);
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const float vm = win[0][q], v0 = win[1][q], vp = win[2][q];
            const float D = fmaf(-2.f, v0, vm + vp);
            const float E = vp - vm;
            const float base = ((13.f / 3.f) * D) * D;
            const float sR = fmaf(2.f, D, E);
            const float sL = fmaf(2.f, D, -E);
            const float bM_ = fmaf(E, E, base);     // 16 x indicator, centred stencil
            const float bR_ = fmaf(sR, sR, base);   // stencil whose right end is the face side
            const float bL_ = fmaf(sL, sL, base);
            const float t0 = fmaf(D, 1.f / 12.f, v0);
            const float pR = fmaf(E, 0.25f, t0);          // value at c + 1/2
            const float pL = fmaf(E, -0.25f, t0);         // value at c - 1/2
            if (q < 3) {
                const int m = q;
                // R+ at face f (index f <-> face f-1/2): roles 0, 1, 2 from centres f-2, f-1, f
                const float pRR = fmaf(E, 0.75f, t0 + D); // value at c + 3/2
                if (c + 2 >= 0 && c + 2 <= R) {
                    const int f = (c + 2 >= 0 && c + 2 <= R) ? c + 2 : 0;
                    const float a = wt(bR_, KD0, K.e0);
                    np_[f][m] = fmaf(a, pRR, np_[f][m]);
                    dp_[f][m] += a;
                    if (m == MB) nbp[f] = fmaf(a, bRR, nbp[f]);
                }
                if (c + 1 >= 0 && c + 1 <= R) {
                    const int f = (c + 1 >= 0 && c + 1 <= R) ? c + 1 : 0;
                    const float a = wt(bM_, KD1, K.e1);
                    np_[f][m] = fmaf(a, pR, np_[f][m]);
                    dp_[f][m] += a;
                    if (m == MB) nbp[f] = fmaf(a, bR, nbp[f]);
                }
                if (c >= 0 && c <= R) {
                    const int f = (c >= 0 && c <= R) ? c : 0;
                    const float a = wt(bL_, KD2, K.e2);
                    np_[f][m] = fmaf(a, pL, np_[f][m]);
                    dp_[f][m] += a;
                    if (m == MB) nbp[f] = fmaf(a, bL, nbp[f]);
                }
            } else {
                const int m = q - 3;
                // R- at face f: roles 0, 1, 2 from centres f+1, f, f-1 (mirrored stencil)
                const float pLL = fmaf(E, -0.75f, t0 + D); // value at c - 3/2
                if (c - 1 >= 0 && c - 1 <= R) {
                    const int f = (c - 1 >= 0 && c - 1 <= R) ? c - 1 : 0;
                    const float a = wt(bL_, KD0, K.e0);
                    nm_[f][m] = fmaf(a, pLL, nm_[f][m]);
                    dm_[f][m] += a;
                    if (m == MB) nbm[f] = fmaf(a, bLL, nbm[f]);
                }
                if (c >= 0 && c <= R) {
                    const int f = (c >= 0 && c <= R) ? c : 0;
                    const float a = wt(bM_, KD1, K.e1);
                    nm_[f][m] = fmaf(a, pL, nm_[f][m]);
                    dm_[f][m] += a;
                    if (m == MB) nbm[f] = fmaf(a, bL, nbm[f]);
                }
                if (c + 1 >= 0 && c + 1 <= R) {
                    const int f = (c + 1 >= 0 && c + 1 <= R) ? c + 1 : 0;
                    const float a = wt(bR_, KD2, K.e2);
                    nm_[f][m] = fmaf(a, pR, nm_[f][m]);
                    dm_[f][m] += a;
                    if (m == MB) nbm[f] = fmaf(a, bR, nbm[f]);
                }
            }
        }
        // face c-1 has received all six contributions
        if (c - 1 >= 0 && c - 1 <= R) {
            const int f = (c - 1 >= 0 && c - 1 <= R) ? c - 1 : 0;
            float Fh[3], rp_b = 0.f, rm_b = 0.f;
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const float rp = frcp(dp_[f][m]);
                const float rm = frcp(dm_[f][m]);
                Fh[m] = fmaf(np_[f][m], rp, nm_[f][m] * rm);
                if (m == MB) {
                    rp_b = rp;
                    rm_b = rm;
                }
            }
            // twice the face value of b (mean of the two reconstructions)
            const float bh = fmaf(nbp[f], rp_b, nbm[f] * rm_b);
            if (f >= 1) {
                const int k = f - 1;
                float r3[3];
#pragma unroll
                for (int m = 0; m < 3; ++m) r3[m] = (fprev[m] - Fh[m]) * K.hinv_ds;
                r3[MB] = fmaf(eta[k], (bh - bprev) * K.ghinv_ds, r3[MB]);
                emit(k, r3[0], r3[1], r3[2]);
            }
#pragma unroll
            for (int m = 0; m < 3; ++m) fprev[m] = Fh[m];
            bprev = bh;
        }
    }
}

// The three candidate stencils of a five-value stencil v (read in the upwind
// direction; the face lies between v[2] and v[3]), in the centre form of
// sweep(): the stencils are centred on v[1], v[2], v[3]; D and E are each
// centre's second and central differences, and q the candidates' values at
// the face, t + D + 3E/4, t + E/4 and t - E/4 with t = v_c + D/12.
__device__ __forceinline__ void weno5_cands(const float v[5], float D[3], float E[3], float q[3])
{
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        D[k] = fmaf(-2.f, v[k + 1], v[k] + v[k + 2]);
        E[k] = v[k + 2] - v[k];
    }
    q[0] = fmaf(E[0], 0.75f, fmaf(D[0], 1.f / 12.f, v[1]) + D[0]);
    q[1] = fmaf(E[1], 0.25f, fmaf(D[1], 1.f / 12.f, v[2]));
    q[2] = fmaf(E[2], -0.25f, fmaf(D[2], 1.f / 12.f, v[3]));
}

// WENO5-JS of one five-value stencil v (doubled split values): the
// unnormalised weights a0..a2 (indicators carried 16-fold as in sweep(),
// from the same centre differences) and the numerator sum a_k q_k; the
// reconstruction is num / (a0 + a1 + a2).
__device__ __forceinline__ void weno5_face(const float v[5], const SweepK &K, float &num, float a[3])
{
    float D[3], E[3], q[3];
    weno5_cands(v, D, E, q);
    const float sR = fmaf(2.f, D[0], E[0]), sL = fmaf(2.f, D[2], -E[2]);
    a[0] = wt(fmaf(sR, sR, ((13.f / 3.f) * D[0]) * D[0]), KD0, K.e0);
    a[1] = wt(fmaf(E[1], E[1], ((13.f / 3.f) * D[1]) * D[1]), KD1, K.e1);
    a[2] = wt(fmaf(sL, sL, ((13.f / 3.f) * D[2]) * D[2]), KD2, K.e2);
    num = fmaf(a[2], q[2], fmaf(a[1], q[1], a[0] * q[0]));
}

// The same candidates of a stencil of b, combined with given weights.
__device__ __forceinline__ float weno5_with(const float v[5], const float a[3])
{
    float D[3], E[3], q[3];
    weno5_cands(v, D, E, q);
    return fmaf(a[2], q[2], fmaf(a[1], q[1], a[0] * q[0]));
}

// One sweep with local Lax-Friedrichs splitting (an option; the paper splits
// with the global speed of the stage, Methods, Lax-Friedrichs paragraph).
// Face-based: face f of the segment (between cells f-1 and f, f = 0..R)
// takes the largest normal speed |u_n| + sqrt(g h+) over the six cells its
// two reconstructions read (f-3..f+2), splits those cells with it and runs
// both reconstructions of every component itself: with a speed per face the
// split values differ from face to face, so the per-centre sharing of
// sweep() does not apply.  Same interface and emitted quantities as sweep().
template <int R, int DIR, class Emit>
__device__ __forceinline__ void sweep_llf(const float *__restrict__ Ls, const float *__restrict__ Lhu,
                                          const float *__restrict__ Lhv, const float *__restrict__ Lb,
                                          int li0, int st, const SweepK &K, Emit &&emit)
{
    constexpr int MB = DIR == 0 ? 1 : 2;
    float wf[6][3], wu[6][3], wb[6], ws[6];  // cells f-3..f+2: flux, split vector, bed, speed
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        wf[q][0] = wf[q][1] = wf[q][2] = wu[q][0] = wu[q][1] = wu[q][2] = 0.f;
        wb[q] = ws[q] = 0.f;
    }
    float eta[R];
    float fprev[3] = {0.f, 0.f, 0.f}, bprev = 0.f;
#pragma unroll
    for (int w = -HALO; w < R + HALO; ++w) {
        const int li = li0 + (w + HALO) * st;
        const float sv = Ls[li], hu = Lhu[li], hv = Lhv[li], b = Lb[li];
        const float lo = min0(b);
        const float h = sv - lo;
        const float inv = h > K.h_dry ? frcp(h) : 0.f;
        const float pres = K.half_g * (h - lo) * sv;
        float F0, F1, F2, un;
        if (DIR == 0) {
            un = hu * inv;
            F0 = hu;
            F1 = fmaf(hu, un, pres);
            F2 = hu * (hv * inv);
        } else {
            un = hv * inv;
            F0 = hv;
            F1 = hv * (hu * inv);
            F2 = fmaf(hv, un, pres);
        }
#pragma unroll
        for (int q = 0; q < 5; ++q) {
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                wf[q][m] = wf[q + 1][m];
                wu[q][m] = wu[q + 1][m];
            }
            wb[q] = wb[q + 1];
            ws[q] = ws[q + 1];
        }
        wf[5][0] = F0;
        wf[5][1] = F1;
        wf[5][2] = F2;
        wu[5][0] = sv;
        wu[5][1] = hu;
        wu[5][2] = hv;
        wb[5] = b;
        ws[5] = fabsf(un) + fsqrt(K.g * fmaxf(h, 0.f));
        if (w >= 0 && w < R) eta[w >= 0 && w < R ? w : 0] = sv;
        if (w < 2) continue;
        const int f = w - 2;  // face between cells f-1 and f: its window is complete
        const float a = fmaxf(fmaxf(fmaxf(ws[0], ws[1]), fmaxf(ws[2], ws[3])), fmaxf(ws[4], ws[5]));
        float Fh[3], ap_b[3], am_b[3], rp_b = 0.f, rm_b = 0.f;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            float vp[5], vm[5], ap[3], am[3], np_, nm_;
#pragma unroll
            for (int s = 0; s < 5; ++s) {
                vp[s] = fmaf(a, wu[s][m], wf[s][m]);            // cells f-3 .. f+1
                vm[s] = fmaf(-a, wu[5 - s][m], wf[5 - s][m]);   // cells f+2 .. f-2
            }
            weno5_face(vp, K, np_, ap);
            weno5_face(vm, K, nm_, am);
            const float rp = frcp(ap[0] + ap[1] + ap[2]);
            const float rm = frcp(am[0] + am[1] + am[2]);
            Fh[m] = fmaf(np_, rp, nm_ * rm);
            if (m == MB) {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    ap_b[k] = ap[k];
                    am_b[k] = am[k];
                }
                rp_b = rp;
                rm_b = rm;
            }
        }
        float bp[5], bm[5];
#pragma unroll
        for (int s = 0; s < 5; ++s) {
            bp[s] = wb[s];
            bm[s] = wb[5 - s];
        }
        // twice the face value of b (mean of the two reconstructions)
        const float bh = fmaf(weno5_with(bp, ap_b), rp_b, weno5_with(bm, am_b) * rm_b);
        if (f >= 1) {
            const int k = f - 1;
            float r3[3];
#pragma unroll
            for (int m = 0; m < 3; ++m) r3[m] = (fprev[m] - Fh[m]) * K.hinv_ds;
            r3[MB] = fmaf(eta[k], (bh - bprev) * K.ghinv_ds, r3[MB]);
            emit(k, r3[0], r3[1], r3[2]);
        }
#pragma unroll
        for (int m = 0; m < 3; ++m) fprev[m] = Fh[m];
        bprev = bh;
    }
}

// ---------------------------------------------------------------------------
// wave64 reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned int wave_max_u32(unsigned int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const unsigned int u = __shfl_xor(v, o, 64);
        v = u > v ? u : v;
    }
    return v;
}

__device__ __forceinline__ double wave_sum_f64(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Float bits of a non-negative speed; any non-finite value maps to +inf so
// that the unsigned max keeps it.
__device__ __forceinline__ unsigned int speed_bits(float s)
{
    return (s <= 3.4e38f) ? __float_as_uint(s) : 0x7f800000u;
}

// ---------------------------------------------------------------------------
// The stage on one tile
// ---------------------------------------------------------------------------
// STAGE 1: w = u^n -> A;  2: w = A -> B;  3: w = B -> u^n (in place: each
// cell of u^n is read and then written by the same thread, and no halo of
// stage 3 reads u^n).  A tile is processed in four parts: tile_load (every
// global load of the tile in flight at once, into registers), tile_store
// (registers -> LDS), tile_compute (sweeps, sources, RK combination, store;
// per-thread partials) and stage_publish (block reduction, at most one
// atomic per quantity).

// Per-stage scalars, identical in every block.
struct StageScalars {
    int stage;
    float ax, ay, dt, kcap;
};

__device__ __forceinline__ StageScalars stage_scalars(const Geo &G, int STAGE)
{
    StageScalars sc;
    DevScen *sd = G.sd;
    sc.stage = STAGE;
    sc.ax = __uint_as_float(__hip_atomic_load(&sd->alpha[STAGE - 1][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    sc.ay = __uint_as_float(__hip_atomic_load(&sd->alpha[STAGE - 1][1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (STAGE == 1) {
        if (G.cfl > 0.f) {
            const double den = (double)sc.ax * (double)G.inv_dx + (double)sc.ay * (double)G.inv_dy;
            sc.dt = (den > 0.0 && den < 1e300) ? (float)((double)G.cfl / den) : 0.f;
        } else {
            sc.dt = G.dt_fixed;
        }
    } else {
        sc.dt = __hip_atomic_load(&sd->dt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    sc.kcap = (G.kappa_cap > 0.f && sc.dt > 0.f) ? G.kappa_cap / sc.dt : 3.0e38f;
    return sc;
}

// Per-thread partial reductions of a stage.
struct StagePartials {
    unsigned int sxb = 0, syb = 0, rub = 0;
    float deficit = 0.f;
};

template <class C>
struct TileRegs {
    // passes over the first TX staged columns, RPI rows per pass (thread =
    // (row q, column c)), then the 2 HALO last columns
    static constexpr int RPI = C::NT / C::TX;
    static constexpr int MI = (C::WY + RPI - 1) / RPI;
    static constexpr int NR = 2 * HALO * C::WY;
    static constexpr int RI = (NR + C::NT - 1) / C::NT;
    static constexpr int IT = MI + RI;
    static_assert(C::NT % C::TX == 0, "whole rows of threads per pass");
    float h[IT], hu[IT], hv[IT], b[IT];
};

// A tile whose halo lies inside the grid: staged without mirroring, frozen
// ghosts or index clamping.
template <class C>
__device__ __forceinline__ bool tile_inner(const Geo &G, int tx, int ty)
{
    const int x0 = tx * C::TX, y0 = ty * C::TY;
    return x0 >= HALO && y0 >= HALO && x0 + C::TX + HALO <= G.nx && y0 + C::TY + HALO <= G.ny;
}

// Grid index of staged coordinate g along a side of n cells: ghosts of a
// mirrored side read the mirror cell; clamped into the grid.
__device__ __forceinline__ int mirror_index(int g, int n)
{
    int m = g < 0 ? -1 - g : (g >= n ? 2 * n - 1 - g : g);
    return m < 0 ? 0 : (m >= n ? n - 1 : m);
}

// Global loads of a tile and its halo.  Ghost cells of mirrored sides read
// the mirror cell; indices are clamped into the grid, so the cells beyond
// three ghost layers that only ragged tail tiles touch read finite values
// whose results are discarded.  All loads are issued back to back.
template <class C, bool INNER>
__device__ __forceinline__ void tile_load(const Geo &G, int STAGE, int tx, int ty, TileRegs<C> &v)
{
    const float *const *W = STAGE == 1 ? G.U : STAGE == 2 ? G.A : G.B;
    const float *w0 = W[0], *w1 = W[1], *w2 = W[2];
    const int nx = G.nx, ny = G.ny, pitch = G.pitch;
    const int x0 = tx * C::TX, y0 = ty * C::TY;
    using T = TileRegs<C>;
    const int c = threadIdx.x % C::TX, q = threadIdx.x / C::TX;
    if (INNER) {
        // every pass whose rows lie in the window reads the four planes at
        // one per-thread 32-bit offset (the pass's rows added once), so a
        // load is the plane's scalar base plus that offset; rows of a last,
        // partial pass are clamped to the window's last row
        const unsigned off = (unsigned)((y0 - HALO + q) * pitch + x0 - HALO + c);
#pragma unroll
        for (int k = 0; k < T::MI; ++k) {
            if ((k + 1) * T::RPI <= C::WY) {
                const unsigned ok = off + (unsigned)(k * T::RPI * pitch);
                v.h[k] = pld(w0, ok);
                v.hu[k] = pld(w1, ok);
                v.hv[k] = pld(w2, ok);
                v.b[k] = pld(G.b, ok);
            } else {
                const int r = q + k * T::RPI < C::WY ? q + k * T::RPI : C::WY - 1;
                const unsigned i = (unsigned)((y0 - HALO + r) * pitch + x0 - HALO + c);
                v.h[k] = pld(w0, i);
                v.hu[k] = pld(w1, i);
                v.hv[k] = pld(w2, i);
                v.b[k] = pld(G.b, i);
            }
        }
#pragma unroll
        for (int j = 0; j < T::RI; ++j) {
            int e = threadIdx.x + j * C::NT;
            e = (T::RI * C::NT == T::NR || e < T::NR) ? e : T::NR - 1;
            const int r = e / (2 * HALO), cc = C::TX + e % (2 * HALO);
            const unsigned i = (unsigned)((y0 - HALO + r) * pitch + x0 - HALO + cc);
            v.h[T::MI + j] = pld(w0, i);
            v.hu[T::MI + j] = pld(w1, i);
            v.hv[T::MI + j] = pld(w2, i);
            v.b[T::MI + j] = pld(G.b, i);
        }
        return;
    }
    // edge tiles: the same passes.  Ghost cells of mirrored sides read the
    // mirror cell and indices are clamped into the grid, so the cells beyond
    // three ghost layers that only ragged tail tiles touch read finite values
    // whose results are discarded.  A thread's column, and so its mirrored
    // column, is the same in every pass.
    const int mx = mirror_index(x0 - HALO + c, nx);
#pragma unroll
    for (int k = 0; k < T::MI; ++k) {
        const int r = q + k * T::RPI < C::WY ? q + k * T::RPI : C::WY - 1;
        const unsigned i = (unsigned)(mirror_index(y0 - HALO + r, ny) * pitch + mx);
        v.h[k] = pld(w0, i);
        v.hu[k] = pld(w1, i);
        v.hv[k] = pld(w2, i);
        v.b[k] = pld(G.b, i);
    }
#pragma unroll
    for (int j = 0; j < T::RI; ++j) {
        int e = threadIdx.x + j * C::NT;
        e = (T::RI * C::NT == T::NR || e < T::NR) ? e : T::NR - 1;
        const int r = e / (2 * HALO), cc = C::TX + e % (2 * HALO);
        const unsigned i = (unsigned)(mirror_index(y0 - HALO + r, ny) * pitch + mirror_index(x0 - HALO + cc, nx));
        v.h[T::MI + j] = pld(w0, i);
        v.hu[T::MI + j] = pld(w1, i);
        v.hv[T::MI + j] = pld(w2, i);
        v.b[T::MI + j] = pld(G.b, i);
    }
}

// LDS stores of a loaded tile: normal momentum negated on mirrored ghosts,
// frozen values on FIXED sides.
template <class C, bool INNER>
__device__ __forceinline__ void tile_store(const Geo &G, int tx, int ty, const TileRegs<C> &v, float *lds)
{
    float *Lh = lds, *Lhu = lds + C::PLANE, *Lhv = lds + 2 * C::PLANE, *Lb = lds + 3 * C::PLANE;
    const int nx = G.nx, ny = G.ny;
    const int x0 = tx * C::TX, y0 = ty * C::TY;
    using T = TileRegs<C>;
    const int c = threadIdx.x % C::TX, q = threadIdx.x / C::TX;
    if (INNER) {
        // the pass layout of tile_load: one LDS index plus a constant per pass
#pragma unroll
        for (int k = 0; k < T::MI; ++k) {
            const int r = (k + 1) * T::RPI <= C::WY || q + k * T::RPI < C::WY ? q + k * T::RPI : C::WY - 1;
            const int li = r * C::SX + c;
            Lh[li] = v.h[k];
            Lhu[li] = v.hu[k];
            Lhv[li] = v.hv[k];
            Lb[li] = v.b[k];
        }
#pragma unroll
        for (int j = 0; j < T::RI; ++j) {
            int e = threadIdx.x + j * C::NT;
            e = (T::RI * C::NT == T::NR || e < T::NR) ? e : T::NR - 1;
            const int li = (e / (2 * HALO)) * C::SX + C::TX + e % (2 * HALO);
            Lh[li] = v.h[T::MI + j];
            Lhu[li] = v.hu[T::MI + j];
            Lhv[li] = v.hv[T::MI + j];
            Lb[li] = v.b[T::MI + j];
        }
        return;
    }
    // edge tiles: the same passes; a FIXED side's frozen values are looked
    // up only when the tile reaches into that side's ghosts (decided once
    // for the tile)
    const bool fixed_near = (x0 < HALO && G.bc[0] == BC_FIXED) || (x0 + C::TX + HALO > nx && G.bc[1] == BC_FIXED) ||
                            (y0 < HALO && G.bc[2] == BC_FIXED) || (y0 + C::TY + HALO > ny && G.bc[3] == BC_FIXED);
    auto put = [&](int r, int cc, float h, float hu, float hv, float b) {
        const int gx = x0 - HALO + cc, gy = y0 - HALO + r;
        const bool inx = (unsigned)gx < (unsigned)nx, iny = (unsigned)gy < (unsigned)ny;
        if (!inx) hu = -hu;
        if (!iny) hv = -hv;
        if (fixed_near && inx != iny) {
            // a ghost of exactly one side: frozen values if that side is FIXED
            const int side = !inx ? (gx < 0 ? 0 : 1) : (gy < 0 ? 2 : 3);
            const int layer = !inx ? (gx < 0 ? -1 - gx : gx - nx) : (gy < 0 ? -1 - gy : gy - ny);
            if (G.bc[side] == BC_FIXED && layer < HALO) {
                const int pos = side < 2 ? gy : gx;
                h = pld(G.ghost, (unsigned)ghost_index(G, side, 0, layer, pos));
                hu = pld(G.ghost, (unsigned)ghost_index(G, side, 1, layer, pos));
                hv = pld(G.ghost, (unsigned)ghost_index(G, side, 2, layer, pos));
                b = pld(G.ghost, (unsigned)ghost_index(G, side, 3, layer, pos));
            }
        }
        const int li = r * C::SX + cc;
        Lh[li] = h;
        Lhu[li] = hu;
        Lhv[li] = hv;
        Lb[li] = b;
    };
#pragma unroll
    for (int k = 0; k < T::MI; ++k) {
        const int r = q + k * T::RPI < C::WY ? q + k * T::RPI : C::WY - 1;
        put(r, c, v.h[k], v.hu[k], v.hv[k], v.b[k]);
    }
#pragma unroll
    for (int j = 0; j < T::RI; ++j) {
        int e = threadIdx.x + j * C::NT;
        e = (T::RI * C::NT == T::NR || e < T::NR) ? e : T::NR - 1;
        put(e / (2 * HALO), C::TX + e % (2 * HALO), v.h[T::MI + j], v.hu[T::MI + j], v.hv[T::MI + j],
            v.b[T::MI + j]);
    }
}

// Sweeps, sources, RK combination and store of a tile staged in LDS.  Ends
// with the LDS tile still in use: the caller synchronises before overwriting
// it.  PF: issue the combination's global reads before the x sweep (costs
// 4R registers across both sweeps; off for variants whose register budget is
// tight, those launched for three waves per SIMD).
// IMP: point-implicit friction.  Each stage takes its own friction term
// backward in time with the rate kappa of its input, uncapped:
// q_out = [a_n q^n + a_w (q + dt L')] / (1 + a_w dt kappa), L' without
// friction, a_w = 1, 1/4, 2/3 (an option; the paper's friction is explicit).
template <class C, bool PF, bool CMP, bool IMP, bool LLF = false>
__device__ __forceinline__ void tile_compute(const Geo &G, const StageScalars &sc, int tx, int ty, float *lds,
                                             StagePartials &acc)
{
    constexpr int TX = C::TX, TY = C::TY, R = C::R;
    const int STAGE = sc.stage;
    const float *Ls = lds, *Lhu = lds + C::PLANE, *Lhv = lds + 2 * C::PLANE, *Lb = lds + 3 * C::PLANE;
    float *Xr = lds + 4 * C::PLANE;
    const int tid = threadIdx.x;
    const int x0 = tx * TX, y0 = ty * TY;
    const int nx = G.nx, ny = G.ny, pitch = G.pitch;
    float *const *O = STAGE == 1 ? G.A : STAGE == 2 ? G.B : G.U;

    SweepK K;
    K.g = G.g;
    K.half_g = G.half_g;
    K.h_dry = G.h_dry;
    K.e0 = G.eps16 * KD0;
    K.e1 = G.eps16 * KD1;
    K.e2 = G.eps16 * KD2;

    // y-sweep thread -> (column, segment of R cells)
    const int col = tid % TX, seg = tid / TX;
    const int gx = x0 + col;
    // the per-cell global reads of the combination in the y sweep (g n^2,
    // u^n in stages 2 and 3, with the compensated level the residuals of the
    // input's level and of u^n's, and in stage 3 the maximum-depth map when
    // one is kept) are issued before the x sweep, so their HBM latency hides
    // behind both sweeps; indices are clamped into the grid (cells outside
    // it are skipped)
    const bool track_max = STAGE == 3 && G.hmax != nullptr;
    float pgn2[R], pun[R][3], prin[R], prun[R], phm[R];
    const float *rin = CMP ? (STAGE == 1 ? G.Rl[0] : STAGE == 2 ? G.Rl[1] : G.Rl[2]) : nullptr;
    if (PF) {
        const int cx = gx < nx ? gx : nx - 1;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int gy = y0 + seg * R + k;
            const unsigned gi = (unsigned)((gy < ny ? gy : ny - 1) * pitch + cx);
            pgn2[k] = pld(G.gn2, gi);
            if (STAGE != 1) {
                pun[k][0] = pld(G.U[0], gi);
                pun[k][1] = pld(G.U[1], gi);
                pun[k][2] = pld(G.U[2], gi);
            }
            if (CMP) {
                prin[k] = pld(rin, gi);
                if (STAGE != 1) prun[k] = pld(G.Rl[0], gi);
            }
            if (track_max) phm[k] = pld(G.hmax, gi);
        }
    }

    // ---- x sweep: thread -> (row, segment of R cells) ------------------------
    {
        const int row = tid % TY, xseg = tid / TY;
        K.a = sc.ax;
        K.hinv_ds = 0.5f * G.inv_dx;
        K.ghinv_ds = -G.g * K.hinv_ds;
        float *xo = Xr + row * C::XR + xseg * R;
        auto xput = [&](int k, float l0, float l1, float l2) {
            xo[k] = l0;
            xo[C::XPLANE + k] = l1;
            xo[2 * C::XPLANE + k] = l2;
        };
        if constexpr (LLF)
            sweep_llf<R, 0>(Ls, Lhu, Lhv, Lb, (row + HALO) * C::SX + xseg * R, 1, K, xput);
        else
            sweep<R, 0>(Ls, Lhu, Lhv, Lb, (row + HALO) * C::SX + xseg * R, 1, K, xput);
    }
    __syncthreads();

    // ---- y sweep, sources, RK combination, store ------------------------------
    K.a = sc.ay;
    K.hinv_ds = 0.5f * G.inv_dy;
    K.ghinv_ds = -G.g * K.hinv_ds;
    const float h_dry = G.h_dry, dt = sc.dt;
    // cell k of the thread's column segment, as soon as the y sweep has its
    // part of L (ry0..2): friction, RK combination, fix-up, store, partials.
    // Done inside the sweep, so no per-cell results wait in registers.
    auto cell = [&](int k, float ry0, float ry1, float ry2) {
        const int ly = seg * R + k;
        const int gy = y0 + ly;
        if (gx >= nx || gy >= ny) return;
        const unsigned gi = (unsigned)(gy * pitch + gx);
        const int li = (ly + HALO) * C::SX + col + HALO;
        const int xi = ly * C::XR + col;
        const float sv = Ls[li], hu = Lhu[li], hv = Lhv[li], bb = Lb[li];
        const float lo = min0(bb);  // level of zero depth
        const float h = sv - lo;
        float Lh_ = Xr[xi] + ry0;
        float Lhu_ = Xr[C::XPLANE + xi] + ry1;
        float Lhv_ = Xr[2 * C::XPLANE + xi] + ry2;
        // explicit Manning friction, wet cells only, rate capped at kappa_cap/dt
        // (IMP: the uncapped rate, taken after the combination)
        const float gn2 = PF ? pgn2[k] : pld(G.gn2, gi);
        float kimp = 0.f;
        if (h > h_dry && gn2 > 0.f) {
            // |q| as a sum of two rounded squares: the same for (hu, hv) and
            // (hv, hu), so the step commutes with exchanging x and y
            const float qn = fsqrt(hu * hu + hv * hv);
            const float hm73 = __builtin_amdgcn_exp2f(-2.33333333333333f * __builtin_amdgcn_logf(h));
            if (IMP) {
                kimp = gn2 * qn * hm73;
            } else {
                const float kap = fminf(gn2 * qn * hm73, sc.kcap);
                Lhu_ = fmaf(-kap, hu, Lhu_);
                Lhv_ = fmaf(-kap, hv, Lhv_);
            }
        }
        // the combination acts on the stored level: it differs from the depth
        // by a per-cell constant and the stage weights sum to one
        float os = fmaf(dt, Lh_, sv), ohu = fmaf(dt, Lhu_, hu), ohv = fmaf(dt, Lhv_, hv);
        float osl = 0.f;  // residual of the level (compensated kernels)
        if (!CMP) {
            if (STAGE == 2) {
                os = fmaf(0.75f, PF ? pun[k][0] : pld(G.U[0], gi), 0.25f * os);
                ohu = fmaf(0.75f, PF ? pun[k][1] : pld(G.U[1], gi), 0.25f * ohu);
                ohv = fmaf(0.75f, PF ? pun[k][2] : pld(G.U[2], gi), 0.25f * ohv);
            }
            if (STAGE == 3) {
                // u^n + (2/3)(w + dt L - u^n): the FP32 weights 1/3 and 2/3 sum
                // to 1 + 3e-8, which would create mass every step; this form
                // keeps the two weights summing to exactly one
                const float un0 = PF ? pun[k][0] : pld(G.U[0], gi);
                const float un1 = PF ? pun[k][1] : pld(G.U[1], gi);
                const float un2 = PF ? pun[k][2] : pld(G.U[2], gi);
                os = fmaf(2.f / 3.f, os - un0, un0);
                ohu = fmaf(2.f / 3.f, ohu - un1, un1);
                ohv = fmaf(2.f / 3.f, ohv - un2, un2);
            }
        } else {
            // the same combination on (s, r) pairs with error-free sums and
            // products; the value s + r is carried to ~2^-46 relative
            const float slo = PF ? prin[k] : pld(rin, gi);
            float yh, yl;
            two_sum(sv, fmaf(dt, Lh_, slo), yh, yl);
            os = yh;
            osl = yl;
            if (STAGE == 2) {
                const float uh = PF ? pun[k][0] : pld(G.U[0], gi), ul = PF ? prun[k] : pld(G.Rl[0], gi);
                const float p1 = 0.75f * uh, e1 = fmaf(0.75f, uh, -p1);
                float s2, e2;
                two_sum(p1, 0.25f * yh, s2, e2);
                const float l2 = ((e2 + e1) + 0.75f * ul) + 0.25f * yl;
                os = s2 + l2;
                osl = l2 - (os - s2);
                ohu = fmaf(0.75f, PF ? pun[k][1] : pld(G.U[1], gi), 0.25f * ohu);
                ohv = fmaf(0.75f, PF ? pun[k][2] : pld(G.U[2], gi), 0.25f * ohv);
            }
            if (STAGE == 3) {
                const float uh = PF ? pun[k][0] : pld(G.U[0], gi), ul = PF ? prun[k] : pld(G.Rl[0], gi);
                const float un1 = PF ? pun[k][1] : pld(G.U[1], gi);
                const float un2 = PF ? pun[k][2] : pld(G.U[2], gi);
                float dh, dl;
                two_sum(yh, -uh, dh, dl);
                dl += yl - ul;
                const float p3 = (2.f / 3.f) * dh, e3 = fmaf(2.f / 3.f, dh, -p3);
                float s3, e4;
                two_sum(uh, p3, s3, e4);
                const float l3 = ((e4 + e3) + (2.f / 3.f) * dl) + ul;
                os = s3 + l3;
                osl = l3 - (os - s3);
                ohu = fmaf(2.f / 3.f, ohu - un1, un1);
                ohv = fmaf(2.f / 3.f, ohv - un2, un2);
            }
        }
        if (IMP && kimp > 0.f) {
            const float aw = STAGE == 1 ? 1.f : STAGE == 2 ? 0.25f : 2.f / 3.f;
            const float rden = frcp(fmaf(aw * dt, kimp, 1.f));
            ohu *= rden;
            ohv *= rden;
        }
        float oh = CMP ? (os - lo) + osl : os - lo;
        if (oh < 0.f) {
            acc.deficit -= oh;
            oh = 0.f;
            os = lo;
            osl = 0.f;
        }
        if (CMP) pst(STAGE == 1 ? G.Rl[1] : STAGE == 2 ? G.Rl[2] : G.Rl[0], gi, osl);
        const bool wet = oh > h_dry;
        if (!wet) {
            ohu = 0.f;
            ohv = 0.f;
        }
        pst(O[0], gi, os);
        pst(O[1], gi, ohu);
        pst(O[2], gi, ohv);
        if (track_max) {
            // maximum-depth map over the states after completed steps
            if (oh > (PF ? phm[k] : pld(G.hmax, gi))) pst(G.hmax, gi, oh);
        }
        // wave speeds of the output (the next stage's input), as float bits:
        // a speed is +0 or more, so its bits order as unsigned integers, and a
        // non-finite output gives an infinite or NaN speed (a NaN depth fails
        // the wet test and leaves cel NaN; an infinite momentum meets inv = 0
        // or a finite inv), whose bits are 0x7f800000 or above; the block
        // reduction clamps those to the bits of +inf
        const float cel = fsqrt(G.g * oh);
        const float inv = wet ? frcp(oh) : 0.f;
        const unsigned int bx = __float_as_uint(fabsf(ohu * inv) + cel);
        const unsigned int by = __float_as_uint(fabsf(ohv * inv) + cel);
        acc.sxb = bx > acc.sxb ? bx : acc.sxb;
        acc.syb = by > acc.syb ? by : acc.syb;
        if (STAGE == 3) {
            if (wet && bb > 0.f) {
                const unsigned int u = __float_as_uint(bb);
                acc.rub = u > acc.rub ? u : acc.rub;
            }
        }
    };
    if constexpr (LLF)
        sweep_llf<R, 1>(Ls, Lhu, Lhv, Lb, (seg * R) * C::SX + col + HALO, C::SX, K, cell);
    else
        sweep<R, 1>(Ls, Lhu, Lhv, Lb, (seg * R) * C::SX + col + HALO, C::SX, K, cell);
}

// Block reduction of the partials and the stage's atomics.  `first` marks
// the block that processed tile (0, 0): it does the once-per-stage
// bookkeeping.  Uses the first bytes of LDS; synchronises before and after.
template <class C>
__device__ __forceinline__ void stage_publish(const Geo &G, const StageScalars &sc, StagePartials acc, bool first,
                                              float *lds)
{
    constexpr int NT = C::NT;
    const int STAGE = sc.stage;
    DevScen *sd = G.sd;
    const int tid = threadIdx.x;
    // NaN bits (above those of +inf) become +inf, the value a non-finite
    // speed publishes
    unsigned int sxb = min(wave_max_u32(acc.sxb), 0x7f800000u);
    unsigned int syb = min(wave_max_u32(acc.syb), 0x7f800000u);
    const bool any_def = __any(acc.deficit > 0.f);
    double dsum = any_def ? wave_sum_f64((double)acc.deficit) : 0.0;
    unsigned int rub = STAGE == 3 ? wave_max_u32(acc.rub) : 0u;
    __syncthreads();  // LDS tile no longer needed
    constexpr int NW = NT / 64;
    unsigned int *ru = reinterpret_cast<unsigned int *>(lds);
    double *rd = reinterpret_cast<double *>(lds + 4 * NW);
    const int lane = tid & 63, wv = tid >> 6;
    if (lane == 0) {
        ru[wv] = sxb;
        ru[NW + wv] = syb;
        ru[2 * NW + wv] = rub;
        rd[wv] = dsum;
    }
    __syncthreads();
    if (tid == 0) {
        unsigned int mx = 0, my = 0, mr = 0;
        double ds = 0.0;
        for (int i = 0; i < NW; ++i) {
            mx = ru[i] > mx ? ru[i] : mx;
            my = ru[NW + i] > my ? ru[NW + i] : my;
            mr = ru[2 * NW + i] > mr ? ru[2 * NW + i] : mr;
            ds += rd[i];
        }
        // Same-address atomics from every block serialise; the running maxima
        // only grow, so a block whose partial does not exceed the value
        // already there skips its atomic (the load may lag, never lead).
        const int out_slot = STAGE % 3;  // stage 1 -> slot 1, 2 -> 2, 3 -> 0
        unsigned int *ax_slot = &sd->alpha[out_slot][0], *ay_slot = &sd->alpha[out_slot][1];
        if (mx > __hip_atomic_load(ax_slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(ax_slot, mx);
        if (my > __hip_atomic_load(ay_slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(ay_slot, my);
        const double wgt = STAGE == 1 ? 1.0 / 6.0 : STAGE == 2 ? 2.0 / 3.0 : 1.0;
        if (ds != 0.0) atomicAdd(&sd->clamp_sum, wgt * ds);
        if (STAGE == 3 && mr > __hip_atomic_load(&sd->runup, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(&sd->runup, mr);
        if ((mx >= 0x7f800000u || my >= 0x7f800000u)) atomicOr(&sd->flags, 1u);
        // bookkeeping done once per stage
        if (first) {
            if (STAGE == 1) {
                sd->dt = sc.dt;
                sd->alpha[2][0] = 0u;
                sd->alpha[2][1] = 0u;
            } else if (STAGE == 2) {
                sd->alpha[0][0] = 0u;
                sd->alpha[0][1] = 0u;
            } else {
                sd->alpha[1][0] = 0u;
                sd->alpha[1][1] = 0u;
                sd->t += (double)sc.dt;
                sd->step += 1;
            }
        }
    }
}

// The whole stage on one tile (one block, one tile).
// PF and IMP as for tile_compute; CMP: the compensated level (Geo::Rl set).
template <class C, bool PF, bool CMP = false, bool IMP = false, bool LLF = false>
__device__ __forceinline__ void stage_tile(const Geo &G, int tx, int ty, float *lds, const int STAGE)
{
    const StageScalars sc = stage_scalars(G, STAGE);
    if (tile_inner<C>(G, tx, ty)) {
        TileRegs<C> v;
        tile_load<C, true>(G, STAGE, tx, ty, v);
        tile_store<C, true>(G, tx, ty, v, lds);
    } else {
        TileRegs<C> v;
        tile_load<C, false>(G, STAGE, tx, ty, v);
        tile_store<C, false>(G, tx, ty, v, lds);
    }
    __syncthreads();
    StagePartials acc;
    tile_compute<C, PF, CMP, IMP, LLF>(G, sc, tx, ty, lds, acc);
    stage_publish<C>(G, sc, acc, tx == 0 && ty == 0, lds);
}

// Blocks are dispatched round-robin over the 8 XCDs; renumber them so that
// each XCD receives a contiguous band of tiles and shares halo rows in its L2.
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7, l = b >> 3;
    return x * q + (x < r ? x : r) + l;
}

// The stage kernel: one tile per block.  CMP selects the compensated level,
// IMP the point-implicit friction, LLF the local Lax-Friedrichs splitting.
template <class C, int S, int W, bool CMP = false, bool IMP = false, bool LLF = false>
__global__ __launch_bounds__(C::NT, W) void k_stage(Geo G, int ntx, int nblocks)
{
    __shared__ float lds[C::LDS_FLOATS];
    const int id = xcd_remap(blockIdx.x, nblocks);
    stage_tile<C, (W <= 2), CMP, IMP, LLF>(G, id % ntx, id / ntx, lds, S);
}

}  // namespace swe
