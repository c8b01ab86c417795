// Device-side building blocks of the Shan-Chen D3Q19 update for gfx950.
//
// Method: Section 2 of Chiappini, Xue, Falcucci & Sbragaglia (ligament
// break-up with the pseudo-potential lattice Boltzmann method): BGK collision
// (Eq. 3) towards the second-order equilibrium (Eq. 2, with its leading 1)
// evaluated at the shifted velocity u' = u + tau F / rho (Eq. 6), F the
// single-belt Shan-Chen force (Eq. 5) with psi = rho0 (1 - exp(-rho/rho0)).
// Lattice units, c_s^2 = 1/3.
//
// Population order: 0 rest; 1..6 = +x,-x,+y,-y,+z,-z; 7..18 = +x+y,-x-y,
// +x-y,-x+y, +x+z,-x-z, +x-z,-x+z, +y+z,-y-z, +y-z,-y+z.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int Q = 19;
constexpr int kCX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int kCY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int kCZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

__host__ __device__ constexpr double weight(int a) {
    return a == 0 ? 1.0 / 3.0 : (a <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}

enum StorageKind { kF64 = 0, kF32 = 1, kF16S = 2, kBF16S = 3 };

// Storage traits: T is what lives in HBM, C what the arithmetic uses.
// Shifted kinds hold f_a - w_a rho_ref, rounded to nearest even.
template <int ST> struct Storage;
template <> struct Storage<kF64> {
    using T = double;
    using C = double;
    static constexpr bool kShifted = false;
    __device__ static C decode(T v, C) { return v; }
    __device__ static T encode(C f, C) { return f; }
};
template <> struct Storage<kF32> {
    using T = float;
    using C = float;
    static constexpr bool kShifted = false;
    __device__ static C decode(T v, C) { return v; }
    __device__ static T encode(C f, C) { return f; }
};
template <> struct Storage<kF16S> {
    using T = _Float16;
    using C = float;
    static constexpr bool kShifted = true;
    __device__ static C decode(T v, C shift) { return shift + static_cast<float>(v); }
    __device__ static T encode(C f, C shift) { return static_cast<_Float16>(f - shift); }
};
template <> struct Storage<kBF16S> {
    using T = __bf16;
    using C = float;
    static constexpr bool kShifted = true;
    __device__ static C decode(T v, C shift) { return shift + static_cast<float>(v); }
    __device__ static T encode(C f, C shift) { return static_cast<__bf16>(f - shift); }
};

__device__ inline float expm1_c(float v) { return expm1f(v); }
__device__ inline double expm1_c(double v) { return expm1(v); }

// psi = rho0 (1 - exp(-rho/rho0)), written with expm1 to keep digits at small rho.
template <typename C>
__device__ inline C pseudo_potential(C rho, C rho0, C inv_rho0) {
    return -rho0 * expm1_c(-rho * inv_rho0);
}

// Density as the zeroth moment (Eq. 4), summed in a fixed order so every
// place that needs rho of a node gets the same bits.
template <typename C>
__device__ inline C density(const C (&f)[Q]) {
    C r = f[0];
#pragma unroll
    for (int a = 1; a < Q; ++a) r += f[a];
    return r;
}

// Shan-Chen force of Eq. (5) from the 18 neighbour values of psi.
// P(dx,dy,dz) returns psi at x + (dx,dy,dz).
template <typename C, typename PsiAt>
__device__ inline void sc_force(C psi_c, C G, const PsiAt &P, C &Fx, C &Fy, C &Fz) {
    const C w1 = C(1.0 / 18.0), w2 = C(1.0 / 36.0);
    const C pxp = P(1, 0, 0), pxm = P(-1, 0, 0), pyp = P(0, 1, 0), pym = P(0, -1, 0);
    const C pzp = P(0, 0, 1), pzm = P(0, 0, -1);
    const C ppx = P(1, 1, 0), pmm = P(-1, -1, 0), ppm = P(1, -1, 0), pmp = P(-1, 1, 0);
    const C xpz = P(1, 0, 1), xmz = P(-1, 0, -1), xpzm = P(1, 0, -1), xmzp = P(-1, 0, 1);
    const C ypz = P(0, 1, 1), ymz = P(0, -1, -1), ypzm = P(0, 1, -1), ymzp = P(0, -1, 1);
    const C sx = w1 * (pxp - pxm) + w2 * ((ppx - pmm) + (ppm - pmp) + (xpz - xmz) + (xpzm - xmzp));
    const C sy = w1 * (pyp - pym) + w2 * ((ppx - pmm) - (ppm - pmp) + (ypz - ymz) + (ypzm - ymzp));
    const C sz = w1 * (pzp - pzm) + w2 * ((xpz - xmz) - (xpzm - xmzp) + (ypz - ymz) - (ypzm - ymzp));
    const C g = -G * psi_c;
    Fx = g * sx;
    Fy = g * sy;
    Fz = g * sz;
}

// BGK relaxation (Eq. 3, forcing term zero) towards f^eq(rho, u') (Eq. 2)
// with u' = (j + tau F) / rho (Eqs. 4 and 6).  In place on f.
template <typename C>
__device__ inline void collide(C (&f)[Q], C Fx, C Fy, C Fz, C tau, C omega) {
    const C rho = density(f);
    const C jx = (f[1] - f[2]) + (f[7] - f[8]) + (f[9] - f[10]) + (f[11] - f[12]) + (f[13] - f[14]);
    const C jy = (f[3] - f[4]) + (f[7] - f[8]) - (f[9] - f[10]) + (f[15] - f[16]) + (f[17] - f[18]);
    const C jz = (f[5] - f[6]) + (f[11] - f[12]) - (f[13] - f[14]) + (f[15] - f[16]) - (f[17] - f[18]);
    const C inv = C(1) / rho;
    const C ux = (jx + tau * Fx) * inv;
    const C uy = (jy + tau * Fy) * inv;
    const C uz = (jz + tau * Fz) * inv;
    const C base = C(1) - C(1.5) * (ux * ux + uy * uy + uz * uz);
    // opposite pairs (a, a+1) share |c.u'|: f^eq = w rho (base + 4.5 cu^2 +- 3 cu)
#define LBM_PAIR(A, CU, W)                                           \
    {                                                                \
        const C cu = (CU);                                           \
        const C wr = C(W) * rho;                                     \
        const C sym = wr * (base + C(4.5) * cu * cu);                \
        const C asym = wr * C(3) * cu;                               \
        f[A] += omega * ((sym + asym) - f[A]);                       \
        f[A + 1] += omega * ((sym - asym) - f[A + 1]);               \
    }
    LBM_PAIR(1, ux, 1.0 / 18.0)
    LBM_PAIR(3, uy, 1.0 / 18.0)
    LBM_PAIR(5, uz, 1.0 / 18.0)
    LBM_PAIR(7, ux + uy, 1.0 / 36.0)
    LBM_PAIR(9, ux - uy, 1.0 / 36.0)
    LBM_PAIR(11, ux + uz, 1.0 / 36.0)
    LBM_PAIR(13, ux - uz, 1.0 / 36.0)
    LBM_PAIR(15, uy + uz, 1.0 / 36.0)
    LBM_PAIR(17, uy - uz, 1.0 / 36.0)
#undef LBM_PAIR
    // Rest population: in exact arithmetic f*_0 = f_0 + omega (w_0 rho base - f_0),
    // and sum_a f*_a = rho because sum_a f^eq_a = rho.  Taking f*_0 as rho minus
    // the 18 moving populations keeps that identity through rounding, so the
    // collision adds no systematic mass error (in FP32 this is the dominant
    // error source over hundreds of steps, near the interface).
    C moving = f[1];
#pragma unroll
    for (int a = 2; a < Q; ++a) moving += f[a];
    f[0] = rho - moving;
}

__device__ inline int wrapi(int v, int n) {
    int r = v % n;
    return r < 0 ? r + n : r;
}

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b mod 8).  Renumber so each XCD receives a contiguous range of logical
// work items: spatial neighbours then share that XCD's L2.
__device__ inline int xcd_contiguous(int b, int nblk) {
    const int q = nblk >> 3, r = nblk & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

}  // namespace lbm
