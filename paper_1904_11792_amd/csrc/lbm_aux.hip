// Auxiliary kernels of liblbm: ligament set-up, FP64 import/export of the
// state, diagnostics reductions, the flat-interface coexistence run and a
// plain copy kernel used as the bandwidth ceiling.
//
// All of them read or write the pull layout of the step kernel: lattice
// population a at node y holds f_a(y + c_a, t), so f_a(x, t) = lat_a(x - c_a).
#include <float.h>

#include "lbm_internal.h"

namespace lbm {

namespace {

constexpr int kBlock = 256;

__device__ inline int64_t node_index(int x, int y, int z, int nx, int ny) {
    return (int64_t(z) * ny + y) * nx + x;
}

// Node loop of the auxiliary kernels: blocks stride over (y, z) rows, threads
// over x; defines x, y, z and the node index i (32-bit coordinate arithmetic).
#define LBM_FOR_EACH_NODE(L)                                                        \
    for (int row = blockIdx.x; row < (L).ny * (L).nz; row += gridDim.x)            \
        for (int x = threadIdx.x, y = row % (L).ny, z = row / (L).ny; x < (L).nx;   \
             x += kBlock)                                                            \
            if (const int64_t i = int64_t(row) * (L).nx + x; true)

// Offset, in storage elements, of population a at the lattice site that
// holds f_a(x, t) under pull streaming: site x - c_a.  With an FP32 rest
// population (kMassRest) population a >= 1 sits in slot a + 1.
template <int ST>
__device__ inline int64_t pull_source(int a, int x, int y, int z, const LatticeRef &L) {
    return pop_slot(a, Storage<ST>::kMassRest) * L.pop_stride + int64_t(wrapi(z - kCZ[a], L.nz)) * L.plane_stride +
           row_offset(wrapi(y - kCY[a], L.ny), L.row_stride, L.rec_shift, L.nx) + wrapi(x - kCX[a], L.nx);
}

// Index, in floats, of the FP32 rest population of node (x, y, z)
// (kMassRest; the rest population does not move).
__device__ inline int64_t rest_index(int x, int y, int z, const LatticeRef &L) {
    return int64_t(z) * (L.plane_stride / 2) + row_offset(y, L.row_stride / 2, L.rec_shift, L.nx) + x;
}

template <int ST>
__device__ inline double shift_of(const LatticeRef &L, int a) {
    using C = typename Storage<ST>::C;
    return Storage<ST>::kShifted ? double(C(weight(a) * L.rho_ref)) : 0.0;
}

// f_a(x, t) as FP64.  kMassRest kinds: w_a rho_ref (as the kernels round it
// to FP32) plus the stored shifted value, added exactly in FP64.
template <int ST>
__device__ inline double read_pop(const LatticeRef &L, int a, int x, int y, int z) {
    using Tr = Storage<ST>;
    using C = typename Tr::C;
    if constexpr (Tr::kMassRest) {
        if (a == 0) return shift_of<ST>(L, 0) + double(static_cast<const float *>(L.lat)[rest_index(x, y, z, L)]);
        const auto *p = static_cast<const typename Tr::T *>(L.lat);
        return shift_of<ST>(L, a) + double(static_cast<float>(p[pull_source<ST>(a, x, y, z, L)]));
    } else {
        const auto *p = static_cast<const typename Tr::T *>(L.lat);
        const C shift = Tr::kShifted ? C(weight(a) * L.rho_ref) : C(0);
        return double(Tr::decode(p[pull_source<ST>(a, x, y, z, L)], shift));
    }
}

// Store the populations v[a] = f_a(x, t) of one node.  kMassRest kinds round
// the moving populations to 16 bits and give the rest population what that
// rounding took from them, so the node keeps its mass to FP32 rounding (and
// values read by read_pop come back unchanged).
template <int ST>
__device__ inline void write_node(const LatticeRef &L, int x, int y, int z, const double (&v)[Q]) {
    using Tr = Storage<ST>;
    using C = typename Tr::C;
    auto *p = static_cast<typename Tr::T *>(L.lat);
    if constexpr (Tr::kMassRest) {
        double rest = v[0] - shift_of<ST>(L, 0);
#pragma unroll
        for (int a = 1; a < Q; ++a) {
            const double h = v[a] - shift_of<ST>(L, a);
            const typename Tr::T stored = Tr::encode(float(h), 0.0f);
            p[pull_source<ST>(a, x, y, z, L)] = stored;
            rest += h - double(static_cast<float>(stored));
        }
        static_cast<float *>(L.lat)[rest_index(x, y, z, L)] = float(rest);
    } else {
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            const C shift = Tr::kShifted ? C(weight(a) * L.rho_ref) : C(0);
            p[pull_source<ST>(a, x, y, z, L)] = Tr::encode(C(v[a]), shift);
        }
    }
}

// SplitMix64 (Steele, Lea & Flood 2014) used counter-based: first output of
// a generator whose state is s.
__device__ inline uint64_t splitmix64(uint64_t s) {
    uint64_t z = s + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Ligament of Section 3 (radius modulated by a whole number of cosine waves),
// tanh interface, optional seeded noise, populations at rest equilibrium.
template <int ST>
__global__ __launch_bounds__(kBlock) void k_init_ligament(LatticeRef L, LigamentArgs g) {
    LBM_FOR_EACH_NODE(L) {
        // s: coordinate along the axis; p1, p2: the in-plane coordinates in axis order
        const int xyz[3] = {x, y, z};
        const double s = xyz[g.axis];
        const double p1 = xyz[g.axis == 0 ? 1 : 0];
        const double p2 = xyz[g.axis == 2 ? 1 : 2];
        const double d1 = p1 - g.c1, d2 = p2 - g.c2;
        const double r = sqrt(d1 * d1 + d2 * d2);
        const double R = g.R0 * (1.0 + g.amp_rel * cos(6.283185307179586476925286766559 * s / g.wavelength));
        double rho = 0.5 * (g.rho_l + g.rho_v) - 0.5 * (g.rho_l - g.rho_v) * tanh(2.0 * (r - R) / g.width);
        if (g.noise_amp != 0.0) {
            const double U = double(splitmix64(g.seed + uint64_t(i)) >> 11) * (1.0 / 9007199254740992.0);
            rho += g.noise_amp * (2.0 * U - 1.0);
        }
        double v[Q];
#pragma unroll
        for (int a = 0; a < Q; ++a) v[a] = weight(a) * rho;
        write_node<ST>(L, x, y, z, v);
    }
}

template <int ST>
__global__ __launch_bounds__(kBlock) void k_import(LatticeRef L, const double *__restrict__ pop) {
    const int64_t n = int64_t(L.nx) * L.ny * L.nz;
    LBM_FOR_EACH_NODE(L) {
        double v[Q];
#pragma unroll
        for (int a = 0; a < Q; ++a) v[a] = pop[a * n + i];
        write_node<ST>(L, x, y, z, v);
    }
}

template <int ST>
__global__ __launch_bounds__(kBlock) void k_export_pop(LatticeRef L, double *__restrict__ pop) {
    const int64_t n = int64_t(L.nx) * L.ny * L.nz;
    LBM_FOR_EACH_NODE(L) {
#pragma unroll
        for (int a = 0; a < Q; ++a) pop[a * n + i] = read_pop<ST>(L, a, x, y, z);
    }
}

template <int ST>
__global__ __launch_bounds__(kBlock) void k_export_rho(LatticeRef L, double *__restrict__ rho) {
    LBM_FOR_EACH_NODE(L) {
        double f[Q];
#pragma unroll
        for (int a = 0; a < Q; ++a) f[a] = read_pop<ST>(L, a, x, y, z);
        rho[i] = density(f);
    }
}

// Force (Eq. 5) from the exported density field, and the physical velocity
// (j + F/2) / rho.
template <int ST>
__global__ __launch_bounds__(kBlock) void k_export_force_u(LatticeRef L, const double *__restrict__ rho,
                                                          double G, double rho0,
                                                          double *__restrict__ force,
                                                          double *__restrict__ u) {
    const int64_t n = int64_t(L.nx) * L.ny * L.nz;
    const double inv_rho0 = 1.0 / rho0;
    LBM_FOR_EACH_NODE(L) {
        auto P = [&](int dx, int dy, int dz) -> double {
            const int64_t j = node_index(wrapi(x + dx, L.nx), wrapi(y + dy, L.ny), wrapi(z + dz, L.nz),
                                         L.nx, L.ny);
            return pseudo_potential(rho[j], rho0, inv_rho0);
        };
        double Fx, Fy, Fz;
        sc_force<double>(pseudo_potential(rho[i], rho0, inv_rho0), G, P, Fx, Fy, Fz);
        if (force) {
            force[i] = Fx;
            force[n + i] = Fy;
            force[2 * n + i] = Fz;
        }
        if (u) {
            double jx = 0, jy = 0, jz = 0;
#pragma unroll
            for (int a = 0; a < Q; ++a) {
                const double v = read_pop<ST>(L, a, x, y, z);
                jx += kCX[a] * v;
                jy += kCY[a] * v;
                jz += kCZ[a] * v;
            }
            const double r = rho[i];
            u[i] = (jx + 0.5 * Fx) / r;
            u[n + i] = (jy + 0.5 * Fy) / r;
            u[2 * n + i] = (jz + 0.5 * Fz) / r;
        }
    }
}

// ---------------------------------------------------------------------------
// Diagnostics: each block reduces a range of (y, z) rows in FP64; the
// per-slice maximum density (for the neck) is combined with 64-bit atomic
// max on the bit patterns of non-negative doubles (order-independent, hence
// reproducible); the final pass sums the block partials in a fixed order.

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ inline unsigned long long max_bits(double v) {
    // negative or NaN densities count as 0 here (they are flagged separately)
    return (v > 0.0) ? (unsigned long long)__double_as_longlong(v) : 0ull;
}

__device__ inline void flush_slice(double smax, unsigned long long *slice_max, int slice) {
    const double m = wave_max(smax);
    if ((threadIdx.x & 63) == 0 && slice >= 0) atomicMax(&slice_max[slice], max_bits(m));
}

template <int ST>
__global__ __launch_bounds__(kBlock) void k_diag(LatticeRef L, int axis, int rows_per_block,
                                                 DiagPartial *__restrict__ partials,
                                                 unsigned long long *__restrict__ slice_max) {
    if (L.frozen) {
        const int32_t fz = *L.frozen;
        if (fz) L.lat = L.pair[fz - 1];
    }
    const int nrows = L.ny * L.nz;
    const int r0 = blockIdx.x * rows_per_block;
    const int r1 = min(r0 + rows_per_block, nrows);
    double m = 0, px = 0, py = 0, pz = 0, bad = 0;
    double mn = DBL_MAX, mx = -DBL_MAX;
    double smax = 0;          // running max for the current slice (axis 1 or 2)
    int slice = -1;
    double xmax = 0;          // axis 0 with nx <= block: max over rows of my column
    for (int r = r0; r < r1; ++r) {
        const int y = r % L.ny, z = r / L.ny;
        if (axis != 0) {
            const int sl = axis == 2 ? z : y;
            if (sl != slice) {
                flush_slice(smax, slice_max, slice);
                smax = 0;
                slice = sl;
            }
        }
        for (int x = threadIdx.x; x < L.nx; x += kBlock) {
            double f[Q];
            bool finite = true;
#pragma unroll
            for (int a = 0; a < Q; ++a) {
                f[a] = read_pop<ST>(L, a, x, y, z);
                finite = finite && isfinite(f[a]);
            }
            const double rho = density(f);
            const double jx = (f[1] - f[2]) + (f[7] - f[8]) + (f[9] - f[10]) + (f[11] - f[12]) + (f[13] - f[14]);
            const double jy = (f[3] - f[4]) + (f[7] - f[8]) - (f[9] - f[10]) + (f[15] - f[16]) + (f[17] - f[18]);
            const double jz = (f[5] - f[6]) + (f[11] - f[12]) - (f[13] - f[14]) + (f[15] - f[16]) - (f[17] - f[18]);
            if (!finite || !(rho > 0.0)) bad += 1.0;
            m += rho;
            px += jx;
            py += jy;
            pz += jz;
            mn = fmin(mn, rho);
            mx = fmax(mx, rho);
            if (axis == 0) {
                if (L.nx <= kBlock)
                    xmax = fmax(xmax, rho);
                else
                    atomicMax(&slice_max[x], max_bits(rho));
            } else {
                smax = fmax(smax, rho);
            }
        }
    }
    if (axis != 0) flush_slice(smax, slice_max, slice);
    else if (L.nx <= kBlock && int(threadIdx.x) < L.nx && r1 > r0)
        atomicMax(&slice_max[threadIdx.x], max_bits(xmax));

    // block reduction in a fixed order: waves, then wave 0 over the waves
    __shared__ double red[7][kBlock / 64];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    double v[7] = {wave_sum(m), wave_sum(px), wave_sum(py), wave_sum(pz), wave_min(mn),
                   wave_max(mx), wave_sum(bad)};
    if (l == 0)
        for (int k = 0; k < 7; ++k) red[k][w] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        DiagPartial p;
        p.mass = red[0][0]; p.mom[0] = red[1][0]; p.mom[1] = red[2][0]; p.mom[2] = red[3][0];
        p.rho_min = red[4][0]; p.rho_max = red[5][0]; p.nonfinite = red[6][0];
        for (int k = 1; k < kBlock / 64; ++k) {
            p.mass += red[0][k]; p.mom[0] += red[1][k]; p.mom[1] += red[2][k]; p.mom[2] += red[3][k];
            p.rho_min = fmin(p.rho_min, red[4][k]); p.rho_max = fmax(p.rho_max, red[5][k]);
            p.nonfinite += red[6][k];
        }
        p.pad_ = 0;
        partials[blockIdx.x] = p;
    }
}

// Final pass: one block sums the partials (thread t takes t, t+256, ...
// in order, then a fixed tree), takes the neck, and clears the slice maxima
// for the next evaluation.
__global__ __launch_bounds__(kBlock) void k_diag_final(const DiagPartial *__restrict__ partials,
                                                       int nparts,
                                                       unsigned long long *__restrict__ slice_max,
                                                       int nslices, DiagRecord *__restrict__ out,
                                                       int64_t step, int32_t *frozen_flag,
                                                       int32_t freeze_value) {
    __shared__ double s[8][kBlock];
    double m = 0, px = 0, py = 0, pz = 0, bad = 0, mn = DBL_MAX, mx = -DBL_MAX, neck = DBL_MAX;
    for (int i = threadIdx.x; i < nparts; i += kBlock) {
        const DiagPartial p = partials[i];
        m += p.mass; px += p.mom[0]; py += p.mom[1]; pz += p.mom[2];
        mn = fmin(mn, p.rho_min); mx = fmax(mx, p.rho_max); bad += p.nonfinite;
    }
    for (int i = threadIdx.x; i < nslices; i += kBlock) {
        neck = fmin(neck, __longlong_as_double((long long)slice_max[i]));
        slice_max[i] = 0ull;
    }
    s[0][threadIdx.x] = m; s[1][threadIdx.x] = px; s[2][threadIdx.x] = py; s[3][threadIdx.x] = pz;
    s[4][threadIdx.x] = mn; s[5][threadIdx.x] = mx; s[6][threadIdx.x] = bad; s[7][threadIdx.x] = neck;
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if (int(threadIdx.x) < h) {
            const int t = threadIdx.x;
            for (int k = 0; k < 4; ++k) s[k][t] += s[k][t + h];
            s[4][t] = fmin(s[4][t], s[4][t + h]);
            s[5][t] = fmax(s[5][t], s[5][t + h]);
            s[6][t] += s[6][t + h];
            s[7][t] = fmin(s[7][t], s[7][t + h]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        DiagRecord r;
        r.step = step;
        r.mass = s[0][0]; r.mom[0] = s[1][0]; r.mom[1] = s[2][0]; r.mom[2] = s[3][0];
        r.rho_min = s[4][0]; r.rho_max = s[5][0]; r.neck_rho = s[7][0];
        r.nonfinite = (int64_t)s[6][0];
        *out = r;
        if (frozen_flag && r.nonfinite > 0 && *frozen_flag == 0) *frozen_flag = freeze_value;
    }
}

__global__ __launch_bounds__(kBlock) void k_fill_u64(unsigned long long *p, size_t count,
                                                     unsigned long long v) {
    for (size_t i = blockIdx.x * size_t(kBlock) + threadIdx.x; i < count; i += size_t(gridDim.x) * kBlock)
        p[i] = v;
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Streaming copy: one 16-byte vector per thread, 64-thread workgroups in
// address order (non-temporal stores).  Of the copy shapes measured on
// MI355X (1 to 8 vectors per thread, 64 to 1024 threads, other workgroup
// orders) this one moved the most bytes per second: small workgroups
// dispatched in address order keep the memory traffic of each XCD within one
// advancing window.
constexpr int kCopyBlock = 64;
__global__ __launch_bounds__(kCopyBlock) void k_copy16(u32x4 *__restrict__ dst, const u32x4 *__restrict__ src,
                                                       size_t count) {
    const size_t i = blockIdx.x * size_t(kCopyBlock) + threadIdx.x;
    if (i < count) __builtin_nontemporal_store(src[i], &dst[i]);
}

// ---------------------------------------------------------------------------
// Flat interface on a 1 x 1 x n periodic slab, whole state in LDS, one
// thread per node.  The x and y neighbours of a node are the node itself,
// so the same force stencil and collision as the 3-D step apply unchanged.
// State convention here: f_a(z, t) at z (push streaming inside LDS).
// One workgroup per flat-interface run: case blockIdx.x of the table.
__global__ __launch_bounds__(1024) void k_coexistence(const CoexCase *__restrict__ cases, int n, int chunk) {
    const CoexCase &cc = cases[blockIdx.x];
    double *__restrict__ state = cc.state;
    double *__restrict__ out = cc.out;
    const double G = cc.G, tau = cc.tau, rho0 = cc.rho0, hi = cc.hi, lo = cc.lo;
    const MrtParams mrt = cc.mrt;
    const int init = cc.init;
    extern __shared__ double sm[];
    double *fa = sm;              // [19][n]
    double *fb = sm + Q * n;      // [19][n]
    double *psi = sm + 2 * Q * n; // [n]
    double *red = psi + n;        // [n]
    const int z = threadIdx.x;
    const double inv_rho0 = 1.0 / rho0, omega = 1.0 / tau;
    const MrtRates<double> rates = mrt_rates<double>(omega, mrt.s_e, mrt.s_eps, mrt.s_q, mrt.s_pi, mrt.s_m, mrt.s_j);
    if (z < n) {
        if (init) {
            const double W = 4.0;
            const double z1 = n / 4 - 0.5, z2 = 3 * (n / 4) - 0.5;
            const double rho = lo + (hi - lo) * 0.5 * (tanh(2.0 * (z - z1) / W) - tanh(2.0 * (z - z2) / W));
            for (int a = 0; a < Q; ++a) fa[a * n + z] = weight(a) * rho;
        } else {
            for (int a = 0; a < Q; ++a) fa[a * n + z] = state[a * n + z];
        }
    }
    __syncthreads();
    double before = 0;
    if (z < n) {
        double f[Q];
        for (int a = 0; a < Q; ++a) f[a] = fa[a * n + z];
        before = density(f);
    }
    double *cur = fa, *nxt = fb;
    for (int s = 0; s < chunk; ++s) {
        double f[Q];
        if (z < n) {
#pragma unroll
            for (int a = 0; a < Q; ++a) f[a] = cur[a * n + z];
            psi[z] = pseudo_potential(density(f), rho0, inv_rho0);
        }
        __syncthreads();
        if (z < n) {
            auto P = [&](int, int, int dz) -> double { return psi[wrapi(z + dz, n)]; };
            double Fx, Fy, Fz;
            sc_force<double>(psi[z], G, P, Fx, Fy, Fz);
            if (mrt.on)
                collide_mrt<double>(f, Fx, Fy, Fz, rates);
            else
                collide<double>(f, Fx, Fy, Fz, tau, omega);
#pragma unroll
            for (int a = 0; a < Q; ++a) nxt[a * n + wrapi(z + kCZ[a], n)] = f[a];
        }
        __syncthreads();
        double *t = cur;
        cur = nxt;
        nxt = t;
    }
    double after = 0;
    if (z < n) {
        double f[Q];
        for (int a = 0; a < Q; ++a) {
            f[a] = cur[a * n + z];
            state[a * n + z] = f[a];
        }
        after = density(f);
        red[z] = isfinite(after) ? fabs(after - before) : INFINITY;
        psi[z] = after;
    }
    __syncthreads();
    if (z == 0) {
        double mx = 0;
        int bad = 0;
        for (int i = 0; i < n; ++i) {
            if (!isfinite(red[i])) bad = 1;
            else mx = fmax(mx, red[i]);
        }
        out[0] = psi[n / 2];
        out[1] = psi[0];
        out[2] = mx;
        out[3] = bad;
    }
}

// Blocks for a row loop over a grid: one block per (y, z) row, capped.
// ---------------------------------------------------------------------------
// Droplets: 6-connected components of {rho > rho_mid} on the periodic grid
// (the droplet count of the break-up analysis), labelled on the device by a
// lock-free union-find over node indices.
//
// parent[i] is -1 for a background node and a node index <= i for a
// foreground one; a root has parent[i] == i.  Every value ever stored keeps
// parent[i] <= i (stores only lower it, to the smaller of two roots or to an
// ancestor), so a find walks strictly decreasing indices and ends.  A union links the larger
// root under the smaller with an atomic minimum; if the larger one had been
// linked meanwhile, it retries with the value found there, which is smaller:
// max(a, b) falls at every retry, so it ends as well.  When the union pass
// has finished, each component is one tree whose root is its smallest node
// index.  Loads of parent go to the device-coherent level (agent scope), so
// a find never follows a value older than what this CU's cache held.

__device__ inline int cc_load(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline int cc_find(const int32_t *parent, int i) {
    int p = cc_load(&parent[i]);
    while (p != i) {
        i = p;
        p = cc_load(&parent[i]);
    }
    return i;
}

// Find with path halving: each visited node is re-pointed (atomic minimum, so
// a lower value stored meanwhile is kept) at its grandparent, an ancestor in
// the same tree.  Without it, row roots linked one after another form chains
// as long as the number of rows in a large drop.
__device__ inline int cc_find_halving(int32_t *parent, int x) {
    while (true) {
        const int p = cc_load(&parent[x]);
        if (p == x) return x;
        const int gp = cc_load(&parent[p]);
        if (gp == p) return p;
        atomicMin(&parent[x], gp);
        x = gp;
    }
}

__device__ inline void cc_union(int32_t *parent, int a, int b) {
    while (true) {
        a = cc_find_halving(parent, a);
        b = cc_find_halving(parent, b);
        if (a == b) return;
        if (a > b) {
            const int t = a;
            a = b;
            b = t;
        }
        const int old = atomicMin(&parent[b], a);
        if (old == b) return;
        b = old;
    }
}

// Density of every node (FP64), the initial forest, zeroed per-root sums and
// the two counters of the compaction.
template <int ST>
__global__ __launch_bounds__(kBlock) void k_cc_init(LatticeRef L, double rho_mid, double *__restrict__ rho,
                                                    int32_t *__restrict__ parent, int32_t *__restrict__ vol,
                                                    double *__restrict__ mass, int32_t *__restrict__ counters) {
    if (blockIdx.x == 0 && threadIdx.x < 2) counters[threadIdx.x] = 0;
    LBM_FOR_EACH_NODE(L) {
        double f[Q];
#pragma unroll
        for (int a = 0; a < Q; ++a) f[a] = read_pop<ST>(L, a, x, y, z);
        const double r = density(f);
        rho[i] = r;
        parent[i] = r > rho_mid ? int32_t(i) : -1;  // NaN is background
        vol[i] = 0;
        mass[i] = 0.0;
    }
}

// Union of every foreground node with its +x, +y and +z neighbours (periodic);
// the -x, -y, -z links are the same pairs seen from the other node.
__global__ __launch_bounds__(kBlock) void k_cc_union(int32_t *parent, int nx, int ny, int nz) {
    for (int row = blockIdx.x; row < ny * nz; row += gridDim.x) {
        const int y = row % ny, z = row / ny;
        const int yn = y + 1 == ny ? 0 : y + 1, zn = z + 1 == nz ? 0 : z + 1;
        for (int x = threadIdx.x; x < nx; x += kBlock) {
            const int i = row * nx + x;
            if (cc_load(&parent[i]) < 0) continue;
            const int xn = x + 1 == nx ? 0 : x + 1;
            const int nb[3] = {row * nx + xn, (z * ny + yn) * nx + x, (zn * ny + y) * nx + x};
#pragma unroll
            for (int k = 0; k < 3; ++k)
                if (cc_load(&parent[nb[k]]) >= 0) cc_union(parent, i, nb[k]);
        }
    }
}

// Every foreground node points at its root.
__global__ __launch_bounds__(kBlock) void k_cc_compress(int32_t *parent, int n) {
    for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
        if (cc_load(&parent[i]) >= 0)
            __hip_atomic_store(&parent[i], cc_find(parent, int(i)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Volume (nodes) and mass (sum of rho) per root.  The FP64 atomic sums make
// the last bits of a mass depend on the order of the additions.
__global__ __launch_bounds__(kBlock) void k_cc_accumulate(const int32_t *__restrict__ parent,
                                                          const double *__restrict__ rho, int n,
                                                          int32_t *vol, double *mass) {
    for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
        const int r = parent[i];
        if (r >= 0) {
            atomicAdd(&vol[r], 1);
            atomicAdd(&mass[r], rho[i]);
        }
    }
}

// Number of roots (nodes with a non-zero volume): one atomic per wave.
__global__ __launch_bounds__(kBlock) void k_cc_count(const int32_t *__restrict__ vol, int n,
                                                     int32_t *counter) {
    const int lane = threadIdx.x & 63;
    for (int64_t base = (blockIdx.x * int64_t(kBlock) + threadIdx.x) & ~int64_t(63); base < n;
         base += int64_t(gridDim.x) * kBlock) {
        const int64_t i = base + lane;
        const unsigned long long m = __ballot(i < n && vol[i] > 0);
        if (lane == 0 && m) atomicAdd(counter, int32_t(__popcll(m)));
    }
}

// One table entry per root, in no particular order (the host sorts).
__global__ __launch_bounds__(kBlock) void k_cc_write(const int32_t *__restrict__ vol,
                                                     const double *__restrict__ mass, int n,
                                                     int32_t *counter, DropletEntry *out, int cap) {
    for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
        const int v = vol[i];
        if (v > 0) {
            const int k = atomicAdd(counter, 1);
            if (k < cap) {
                out[k].first_node = i;
                out[k].volume = v;
                out[k].mass = mass[i];
            }
        }
    }
}

int flat_grid(int64_t n) {
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    return int(b);
}

int rows_grid(const LatticeRef &L) {
    int64_t b = int64_t(L.ny) * L.nz;
    if (b > 65536) b = 65536;
    return int(b);
}

}  // namespace

#define LBM_DISPATCH(ST_VAR, KERNEL, ...)                         \
    switch (ST_VAR) {                                             \
        case kF64: hipLaunchKernelGGL(KERNEL<kF64>, __VA_ARGS__); break;   \
        case kF32: hipLaunchKernelGGL(KERNEL<kF32>, __VA_ARGS__); break;   \
        case kF16S: hipLaunchKernelGGL(KERNEL<kF16S>, __VA_ARGS__); break; \
        case kBF16S: hipLaunchKernelGGL(KERNEL<kBF16S>, __VA_ARGS__); break; \
        case kF16M: hipLaunchKernelGGL(KERNEL<kF16M>, __VA_ARGS__); break; \
        default: hipLaunchKernelGGL(KERNEL<kBF16M>, __VA_ARGS__); break;   \
    }

hipError_t launch_init_ligament(const LatticeRef &L, const LigamentArgs &g, hipStream_t s) {
    const int nb = rows_grid(L);
    LBM_DISPATCH(L.storage, k_init_ligament, dim3(nb), dim3(kBlock), 0, s, L, g);
    return hipGetLastError();
}

hipError_t launch_import(const LatticeRef &L, const double *pop, hipStream_t s) {
    const int nb = rows_grid(L);
    LBM_DISPATCH(L.storage, k_import, dim3(nb), dim3(kBlock), 0, s, L, pop);
    return hipGetLastError();
}

hipError_t launch_export_pop(const LatticeRef &L, double *pop, hipStream_t s) {
    const int nb = rows_grid(L);
    LBM_DISPATCH(L.storage, k_export_pop, dim3(nb), dim3(kBlock), 0, s, L, pop);
    return hipGetLastError();
}

hipError_t launch_export_rho(const LatticeRef &L, double *rho, hipStream_t s) {
    const int nb = rows_grid(L);
    LBM_DISPATCH(L.storage, k_export_rho, dim3(nb), dim3(kBlock), 0, s, L, rho);
    return hipGetLastError();
}

hipError_t launch_export_force_u(const LatticeRef &L, const double *rho, double G, double rho0,
                                 double *force, double *u, hipStream_t s) {
    const int nb = rows_grid(L);
    LBM_DISPATCH(L.storage, k_export_force_u, dim3(nb), dim3(kBlock), 0, s, L, rho, G, rho0, force, u);
    return hipGetLastError();
}

static int rows_per_block(int ny, int nz) {
    const int nrows = ny * nz;
    int rpb = nrows / 2048;
    return rpb < 1 ? 1 : rpb;
}

int diag_blocks(int nx, int ny, int nz) {
    (void)nx;
    const int rpb = rows_per_block(ny, nz);
    return (ny * nz + rpb - 1) / rpb;
}

hipError_t launch_diag(const LatticeRef &L, int axis, DiagPartial *partials,
                       unsigned long long *slice_max, DiagRecord *out, int64_t step,
                       int32_t *frozen_flag, int32_t freeze_value, hipStream_t s) {
    const int rpb = rows_per_block(L.ny, L.nz);
    const int nb = diag_blocks(L.nx, L.ny, L.nz);
    LBM_DISPATCH(L.storage, k_diag, dim3(nb), dim3(kBlock), 0, s, L, axis, rpb, partials, slice_max);
    const int nslices = axis == 0 ? L.nx : (axis == 1 ? L.ny : L.nz);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kBlock), 0, s, (const DiagPartial *)partials, nb,
                       slice_max, nslices, out, step, frozen_flag, freeze_value);
    return hipGetLastError();
}

__global__ void k_counter(uint32_t *p, uint32_t v, int add) {
    if (threadIdx.x == 0) *p = add ? *p + v : v;
}

hipError_t launch_counter(uint32_t *p, uint32_t v, bool add, hipStream_t s) {
    hipLaunchKernelGGL(k_counter, dim3(1), dim3(64), 0, s, p, v, add ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, size_t count, unsigned long long v, hipStream_t s) {
    int64_t nbl = int64_t((count + kBlock - 1) / kBlock);
    const int nb = int(nbl < 1 ? 1 : (nbl > 65536 ? 65536 : nbl));
    hipLaunchKernelGGL(k_fill_u64, dim3(nb), dim3(kBlock), 0, s, p, count, v);
    return hipGetLastError();
}

hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s) {
    const size_t count = bytes / 16;
    const size_t nb = (count + kCopyBlock - 1) / kCopyBlock;
    if (nb == 0) return hipSuccess;
    if (nb > 0x7fffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy16, dim3(unsigned(nb)), dim3(kCopyBlock), 0, s, (u32x4 *)dst, (const u32x4 *)src, count);
    return hipGetLastError();
}

hipError_t launch_droplets_label(const LatticeRef &L, double rho_mid, const DropletScratch &w, hipStream_t s) {
    const int n = L.nx * L.ny * L.nz;
    const int nb = rows_grid(L);
    LBM_DISPATCH(L.storage, k_cc_init, dim3(nb), dim3(kBlock), 0, s, L, rho_mid, w.rho, w.parent, w.vol, w.mass,
                 w.counters);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cc_union, dim3(nb), dim3(kBlock), 0, s, w.parent, L.nx, L.ny, L.nz);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int fb = flat_grid(n);
    hipLaunchKernelGGL(k_cc_compress, dim3(fb), dim3(kBlock), 0, s, w.parent, n);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_cc_accumulate, dim3(fb), dim3(kBlock), 0, s, w.parent, w.rho, n, w.vol, w.mass);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_cc_count, dim3(fb), dim3(kBlock), 0, s, w.vol, n, w.counters);
    return hipGetLastError();
}

hipError_t launch_droplets_table(const DropletScratch &w, int n, DropletEntry *out, int cap, hipStream_t s) {
    hipLaunchKernelGGL(k_cc_write, dim3(flat_grid(n)), dim3(kBlock), 0, s, w.vol, w.mass, n, w.counters + 1, out,
                       cap);
    return hipGetLastError();
}

hipError_t launch_coexistence_chunk(const CoexCase *cases, int ncases, int n, int chunk, hipStream_t s) {
    const size_t lds = sizeof(double) * (2 * Q * n + 2 * n);
    hipLaunchKernelGGL(k_coexistence, dim3(ncases), dim3(n), lds, s, cases, n, chunk);
    return hipGetLastError();
}

}  // namespace lbm
