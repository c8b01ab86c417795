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

// 1.0f in a register whose value the compiler does not see: a fused
// multiply-add with it is an addition rounded once, and one that takes a
// half-precision operand directly (v_fma_mix_f32), where a plain addition
// converts the half first (two instructions).
__device__ inline float opaque_one() {
    float o = 1.0f;
    asm("" : "+v"(o));
    return o;
}
// acc + v in FP32 for a 16-bit storage value v (the conversion is exact).
__device__ inline float add16(_Float16 v, float acc) { return __builtin_fmaf(static_cast<float>(v), opaque_one(), acc); }
__device__ inline float add16(__bf16 v, float acc) { return static_cast<float>(v) + acc; }

enum StorageKind { kF64 = 0, kF32 = 1, kF16S = 2, kBF16S = 3, kF16M = 4, kBF16M = 5 };
constexpr int kNumStorage = 6;

// Storage traits: T is what lives in HBM, C what the arithmetic uses.
// Shifted kinds hold f_a - w_a rho_ref, rounded to nearest even.
//
// kMassRest (F16M, BF16M): the 18 moving populations are stored shifted in
// 16 bits (stochastically rounded) and the rest population, shifted, in FP32;
// the arithmetic works on the shifted values h_a = f_a - w_a rho_ref
// themselves (decode returns h_a), and the collision sets the rest
// population from the node's mass minus the moving populations as they are
// stored (collide_shifted).  A node's stored
// mass then equals the mass the collision conserves to FP32 rounding, where
// with every population in 16 bits it moved by up to 19 half-precision
// roundings per step, one-signed wherever the values repeat from step to step.
template <int ST> struct Storage;
template <> struct Storage<kF64> {
    using T = double;
    using C = double;
    static constexpr bool kShifted = false, kMassRest = false;
    __device__ static C decode(T v, C) { return v; }
    __device__ static T encode(C f, C) { return f; }
};
template <> struct Storage<kF32> {
    using T = float;
    using C = float;
    static constexpr bool kShifted = false, kMassRest = false;
    __device__ static C decode(T v, C) { return v; }
    __device__ static T encode(C f, C) { return f; }
};
template <> struct Storage<kF16S> {
    using T = _Float16;
    using C = float;
    static constexpr bool kShifted = true, kMassRest = false;
    __device__ static C decode(T v, C shift) { return add16(v, shift); }
    __device__ static T encode(C f, C shift) { return static_cast<_Float16>(f - shift); }
};
template <> struct Storage<kBF16S> {
    using T = __bf16;
    using C = float;
    static constexpr bool kShifted = true, kMassRest = false;
    __device__ static C decode(T v, C shift) { return shift + static_cast<float>(v); }
    __device__ static T encode(C f, C shift) { return static_cast<__bf16>(f - shift); }
};
template <> struct Storage<kF16M> {
    using T = _Float16;
    using C = float;
    static constexpr bool kShifted = true, kMassRest = true;
    static constexpr int kDropBits = 13;  // FP32 mantissa bits below the half's last bit
    __device__ static C decode(T v, C) { return static_cast<float>(v); }
    __device__ static T encode(C h, C) { return static_cast<_Float16>(h); }
};
template <> struct Storage<kBF16M> {
    using T = __bf16;
    using C = float;
    static constexpr bool kShifted = true, kMassRest = true;
    static constexpr int kDropBits = 16;  // FP32 mantissa bits below the bfloat16's last bit
    __device__ static C decode(T v, C) { return static_cast<float>(v); }
    __device__ static T encode(C h, C) { return static_cast<__bf16>(h); }
};

// Counter-based random bits for the stochastic rounding of the FP32-rest
// kinds: the "lowbias32" integer hash (C. Wellons, "Prospecting for hash
// functions", 2018), applied to the node index xor a per-step key.
__host__ __device__ inline uint32_t hash32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// FP32 sum of the 18 moving populations as stored (slots 1..18 of v), in the
// order 1, 2, ..., 18.  The values are multiples of 2^-24 (half) or carry 8
// significant bits (bfloat16), so the sum is exact unless their magnitudes
// span more than the 24 bits of FP32.
template <typename T>
__device__ inline float moving_sum16(const T (&v)[Q]) {
    float s = static_cast<float>(v[1]);
#pragma unroll
    for (int a = 2; a < Q; ++a) s = add16(v[a], s);
    return s;
}

// Stochastic rounding of the 18 moving populations h[1..18] (FP32) to the
// 16-bit storage type, into out[1..18], returning their FP32 sum (moving_sum16).  A value
// is rounded up in magnitude with probability (distance to the lower
// neighbour) / (spacing), so the rounding error has zero mean: increments
// smaller than the 16-bit spacing survive on average instead of being
// rounded away step after step (round-to-nearest holds a slowly changing
// population at the same stored value, and a slowly growing flow with it).
// Population a takes a window of D random bits (D = the number of FP32
// mantissa bits the 16-bit type drops: 13 for half, 16 for bfloat16) from
// word (a - 1) / 6 at offset ((a - 1) mod 6) (32 - D) / 5 (overlapping
// windows, each uniform), adds it to the FP32 bit pattern and truncates.
// Below the half-precision normal range (|h| < 2^-14, a spacing of 2^-24)
// F16M truncates toward zero.
template <typename Tr>
__device__ inline float round_moving_sr(const float (&h)[Q], typename Tr::T (&out)[Q], const uint32_t (&rnd)[3]) {
    using T = typename Tr::T;
    constexpr int D = Tr::kDropBits;
    auto perturbed = [&](int a) -> uint32_t {
        return __float_as_uint(h[a]) + __builtin_amdgcn_ubfe(rnd[(a - 1) / 6], ((a - 1) % 6) * (32 - D) / 5, D);
    };
#pragma unroll
    for (int a = 1; a < Q; a += 2) {
        if constexpr (D == 16) {  // bfloat16: the upper half of the FP32 pattern
            out[a] = __builtin_bit_cast(T, static_cast<uint16_t>(perturbed(a) >> 16));
            out[a + 1] = __builtin_bit_cast(T, static_cast<uint16_t>(perturbed(a + 1) >> 16));
        } else {  // half: truncating conversion of the perturbed values, two at a time
            const auto p = __builtin_amdgcn_cvt_pkrtz(__uint_as_float(perturbed(a)), __uint_as_float(perturbed(a + 1)));
            out[a] = static_cast<T>(p[0]);
            out[a + 1] = static_cast<T>(p[1]);
        }
    }
    return moving_sum16(out);
}

// Slots of 16-bit elements per node and population index -> slot: with an
// FP32 rest population the rest takes two slots (0 and 1) and population
// a >= 1 sits in slot a + 1.
__host__ __device__ constexpr int storage_slots(bool mass_rest) { return mass_rest ? Q + 1 : Q; }
__host__ __device__ constexpr int pop_slot(int a, bool mass_rest) { return (mass_rest && a > 0) ? a + 1 : a; }

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
// rho is density(f), passed in by callers that already have it.
template <typename C>
__device__ inline void collide(C (&f)[Q], C rho, C Fx, C Fy, C Fz, C tau, C omega) {
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

template <typename C>
__device__ inline void collide(C (&f)[Q], C Fx, C Fy, C Fz, C tau, C omega) {
    collide<C>(f, density(f), Fx, Fy, Fz, tau, omega);
}

// The same BGK relaxation for the shifted variables h_a = f_a - w_a rho_ref
// of the kMassRest storage kinds.  m = rho - rho_ref is the sum of the h_a,
// passed in (moving_sum16 of the stored values plus the FP32 rest);
// j = sum c_a h_a (sum_a c_a w_a = 0); the equilibrium minus the shift is
// w_a (m + rho (4.5 (c.u')^2 - 1.5 u'^2)) +- 3 w_a rho c.u'.  The moving
// populations leave stochastically rounded to the storage type (`out`,
// slots 1..18, round_moving_sr with the node's random words `rnd`); the rest
// population becomes m minus their FP32 sum (exact as a rule), so the node's
// stored mass is m to within one FP32 rounding.
template <typename Tr>
__device__ inline void collide_shifted(float (&h)[Q], float m, typename Tr::T (&out)[Q], float Fx, float Fy,
                                       float Fz, float tau, float omega, float rho_ref, const uint32_t (&rnd)[3]) {
    using C = float;
    const C rho = rho_ref + m;
    const C jx = (h[1] - h[2]) + (h[7] - h[8]) + (h[9] - h[10]) + (h[11] - h[12]) + (h[13] - h[14]);
    const C jy = (h[3] - h[4]) + (h[7] - h[8]) - (h[9] - h[10]) + (h[15] - h[16]) + (h[17] - h[18]);
    const C jz = (h[5] - h[6]) + (h[11] - h[12]) - (h[13] - h[14]) + (h[15] - h[16]) - (h[17] - h[18]);
    const C inv = C(1) / rho;
    const C ux = (jx + tau * Fx) * inv;
    const C uy = (jy + tau * Fy) * inv;
    const C uz = (jz + tau * Fz) * inv;
    const C q = C(-1.5) * (ux * ux + uy * uy + uz * uz);
#define LBM_SPAIR(A, CU, W)                                          \
    {                                                                \
        const C cu = (CU);                                           \
        const C wr = C(W) * rho;                                     \
        const C sym = C(W) * m + wr * (q + C(4.5) * cu * cu);        \
        const C asym = wr * C(3) * cu;                               \
        h[A] += omega * ((sym + asym) - h[A]);                       \
        h[A + 1] += omega * ((sym - asym) - h[A + 1]);               \
    }
    LBM_SPAIR(1, ux, 1.0 / 18.0)
    LBM_SPAIR(3, uy, 1.0 / 18.0)
    LBM_SPAIR(5, uz, 1.0 / 18.0)
    LBM_SPAIR(7, ux + uy, 1.0 / 36.0)
    LBM_SPAIR(9, ux - uy, 1.0 / 36.0)
    LBM_SPAIR(11, ux + uz, 1.0 / 36.0)
    LBM_SPAIR(13, ux - uz, 1.0 / 36.0)
    LBM_SPAIR(15, uy + uz, 1.0 / 36.0)
    LBM_SPAIR(17, uy - uz, 1.0 / 36.0)
#undef LBM_SPAIR
    h[0] = m - round_moving_sr<Tr>(h, out, rnd);
}

// ---------------------------------------------------------------------------
// Multiple-relaxation-time collision, the operator the paper's conclusion
// names as the next step (it lets the viscosity change at a fixed density
// ratio).  Moment basis of d'Humieres, Ginzburg, Krafczyk, Lallemand and Luo
// (2002) for D3Q19; row k of M is the polynomial of c defining moment k:
//   rho, e, eps, jx, qx, jy, qy, jz, qz, 3pxx, 3pixx, pww, piww, pxy, pyz,
//   pxz, mx, my, mz.
// The rows are orthogonal, so M^-1 = M^T diag(1 / |row k|^2).  The equilibrium
// moments are those of the second-order equilibrium of Eq. (2), so equal
// rates reproduce BGK.  The force enters as the velocity shift of Eq. (6)
// carried to moment space: the equilibrium is taken at j' = j + F / s_j, so
// a collision adds exactly F to the momentum (s_j = 1/tau is BGK's shift).
__host__ __device__ constexpr int mrt_row(int k, int a) {
    const int x = kCX[a], y = kCY[a], z = kCZ[a];
    const int c2 = x * x + y * y + z * z;
    switch (k) {
        case 0: return 1;
        case 1: return 19 * c2 - 30;
        case 2: return (21 * c2 * c2 - 53 * c2 + 24) / 2;
        case 3: return x;
        case 4: return (5 * c2 - 9) * x;
        case 5: return y;
        case 6: return (5 * c2 - 9) * y;
        case 7: return z;
        case 8: return (5 * c2 - 9) * z;
        case 9: return 3 * x * x - c2;
        case 10: return (3 * c2 - 5) * (3 * x * x - c2);
        case 11: return y * y - z * z;
        case 12: return (3 * c2 - 5) * (y * y - z * z);
        case 13: return x * y;
        case 14: return y * z;
        case 15: return x * z;
        case 16: return (y * y - z * z) * x;
        case 17: return (z * z - x * x) * y;
        default: return (x * x - y * y) * z;
    }
}

__host__ __device__ constexpr int mrt_norm2(int k) {
    int s = 0;
    for (int a = 0; a < Q; ++a) s += mrt_row(k, a) * mrt_row(k, a);
    return s;
}

// Sum over a of mrt_row(k, a) * v[a] with the integer coefficients folded
// at compile time (k, a are constants after unrolling).
template <typename C>
__device__ inline C mrt_moment(int k, const C (&v)[Q]) {
    C acc = C(0);
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        const int c = mrt_row(k, a);
        if (c == 1) acc += v[a];
        else if (c == -1) acc -= v[a];
        else if (c != 0) acc += C(c) * v[a];
    }
    return acc;
}

// Rates of the moments: s[k] for moment k (s[0] unused), inv_sj = 1 / s_j.
template <typename C>
struct MrtRates {
    C s[Q];
    C inv_sj;
};

// Rates of every moment from the viscous rate omega = 1/tau and the other
// rates (s_j <= 0 selects s_j = omega, the BGK velocity shift).
template <typename C>
__device__ inline MrtRates<C> mrt_rates(double omega, double s_e, double s_eps, double s_q, double s_pi,
                                        double s_m, double s_j) {
    const double sj = s_j > 0.0 ? s_j : omega;
    const double v[Q] = {0.0, s_e, s_eps, sj, s_q, sj, s_q, sj, s_q, omega, s_pi, omega, s_pi,
                         omega, omega, omega, s_m, s_m, s_m};
    MrtRates<C> r;
#pragma unroll
    for (int k = 0; k < Q; ++k) r.s[k] = C(v[k]);
    r.inv_sj = C(1.0 / sj);
    return r;
}

// MRT relaxation of f in place: m = M f, m* = m - S (m - m^eq(rho, j + F/s_j)),
// f* = M^-1 m*, then the rest population from the exact mass (as in collide).
template <typename C>
__device__ inline void collide_mrt(C (&f)[Q], C Fx, C Fy, C Fz, const MrtRates<C> &r) {
    C m[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) m[k] = mrt_moment(k, f);
    const C rho = m[0], ir = C(1) / rho;
    const C jx = m[3] + Fx * r.inv_sj, jy = m[5] + Fy * r.inv_sj, jz = m[7] + Fz * r.inv_sj;
    const C jj = jx * jx + jy * jy + jz * jz;
    C meq[Q];
    meq[0] = rho;
    meq[1] = C(-11) * rho + C(19) * jj * ir;
    meq[2] = C(3) * rho - C(5.5) * jj * ir;
    meq[3] = jx;
    meq[4] = C(-2.0 / 3.0) * jx;
    meq[5] = jy;
    meq[6] = C(-2.0 / 3.0) * jy;
    meq[7] = jz;
    meq[8] = C(-2.0 / 3.0) * jz;
    meq[9] = (C(3) * jx * jx - jj) * ir;
    meq[10] = C(-0.5) * meq[9];
    meq[11] = (jy * jy - jz * jz) * ir;
    meq[12] = C(-0.5) * meq[11];
    meq[13] = jx * jy * ir;
    meq[14] = jy * jz * ir;
    meq[15] = jx * jz * ir;
    meq[16] = meq[17] = meq[18] = C(0);
    // relaxed moments divided by the squared row norms (rho is conserved)
    C w[Q];
    w[0] = rho * C(1.0 / mrt_norm2(0));
#pragma unroll
    for (int k = 1; k < Q; ++k) w[k] = (m[k] - r.s[k] * (m[k] - meq[k])) * C(1.0 / mrt_norm2(k));
    // f*_a = sum_k M_ka w_k: column a of M, i.e. row a of M^T
#pragma unroll
    for (int a = 1; a < Q; ++a) {
        C acc = C(0);
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            const int c = mrt_row(k, a);
            if (c == 1) acc += w[k];
            else if (c == -1) acc -= w[k];
            else if (c != 0) acc += C(c) * w[k];
        }
        f[a] = acc;
    }
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
