// Fused Shan-Chen D3Q19 step for gfx950: psi, force, collision and streaming
// of one time step in a single kernel (Section 2, Eqs. 2-6).
//
// Layout: population a of node (x, y, z) at a * S + z * P + row_offset(y) + x.
// The host lays the lattice out in records of k rows, [z][y / k][a][y % k][x]
// (S = k nx, record stride 19 k nx): the 19 population segments of k grid rows
// are contiguous, so a workgroup's gathers for a plane stay within a few
// contiguous blocks of DRAM instead of 19 arrays far apart (k = 1 measured 11%
// faster than one array per population on MI355X), and k > 1 lengthens the
// segments of narrow rows.
// Streaming is PULL between two lattices: the launch reads src and writes dst,
// and a node gathers f_a(x, t) = src_a(x - c_a), i.e. src holds the
// post-collision values of the previous step at their source nodes.
//
// The psi stencil of Eq. (5) needs psi, hence rho, of all 18 neighbours at
// the same time level.  Each workgroup owns a tile_x * tile_y column of the
// grid (one thread per node) and marches it over `zchunk` planes along z.
// Per plane it gathers the populations of its tile (kept in registers for the
// collision one plane later; in the prefetching march the loads go out two
// planes ahead) and of a one-node ring around the tile (only their mass sum
// is kept), and writes psi into a four-plane window in LDS; the force then
// reads psi(z-1), psi(z), psi(z+1) from LDS.  HBM traffic stays near 19
// loads + 19 stores per node: the ring and the two extra planes of a z chunk
// are re-reads of lines that neighbouring tiles, scheduled on the same XCD
// at the same time, have mostly just brought into L2 (rocprofv3 FETCH_SIZE,
// FP32 on 256 x 256 x 1024: 82 B per node read from HBM against the 76 B of
// algorithmic reads).
#include <algorithm>
#include <atomic>

#include "lbm_internal.h"

namespace lbm {

// Access to one z plane of a lattice: element at byte offset soff + voff
// from the plane's base, soff wave-uniform (population segment), voff per
// lane (row and column, below 4 GiB).
//
// BUF = false: a 64-bit pointer and global instructions (one 64-bit vector
// add per access forms the address).  BUF = true: a raw buffer resource
// holding the plane's base, with soff and voff as the instruction's scalar
// and vector offsets, so an access needs no vector address arithmetic.  No
// range limit is set (every offset the step forms lies inside the plane);
// the last resource word is the raw-buffer format of the gfx9 family (32-bit
// data format, no swizzle, no per-lane index).
//
// Stores go through global instructions except for FP64; loads go through
// buffer resources except in the plain march of the single-grid launches
// of the other kinds (MRT, and FP32 on planes with more tiles than the
// device keeps resident).  Measured on MI355X on 256 x 256 x 1024 (one
// GPU call per comparison): buffer stores made FP32, FP16S and F16M 3-5%
// slower and FP64 faster; buffer loads were 2-5% slower for those kinds in
// the plain march but are the faster choice in the prefetching one (with
// 64-bit addresses its registers spill) and in the batched launch.
template <bool BUF>
struct PlaneRef;

template <>
struct PlaneRef<false> {
    char *p;
    __device__ explicit PlaneRef(const void *base) : p(static_cast<char *>(const_cast<void *>(base))) {}
    template <typename V>
    __device__ V load(uint32_t voff, uint32_t soff) const {
        return *reinterpret_cast<const V *>(p + soff + voff);
    }
    template <typename V>
    __device__ void store_nt(V v, uint32_t voff, uint32_t soff) const {
        __builtin_nontemporal_store(v, reinterpret_cast<V *>(p + soff + voff));
    }
};

template <>
struct PlaneRef<true> {
    __amdgpu_buffer_rsrc_t r;
    __device__ explicit PlaneRef(const void *base)
        : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, -1, 0x00020000)) {}
    template <typename V>
    __device__ V load(uint32_t voff, uint32_t soff) const {
        if constexpr (sizeof(V) == 2)
            return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
        else if constexpr (sizeof(V) == 4)
            return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
        else
            return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    }
    // non-temporal: cache-policy bit NT of gfx94x / gfx950
    template <typename V>
    __device__ void store_nt(V v, uint32_t voff, uint32_t soff) const {
        constexpr int kNT = 2;
        if constexpr (sizeof(V) == 2)
            __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, voff, soff, kNT);
        else if constexpr (sizeof(V) == 4)
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, kNT);
        else {
            typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, kNT);
        }
    }
};

// Tile shape: compile-time (TXS x TYS), or with TXS = 0 chosen per grid at
// run time (A.tile_w x A.tile_h) for a workgroup of TYS threads: tile_w at
// most 128 (512 threads) or 256 (1024 threads), tile_h at most 64 and
// tile_w * tile_h at most TYS.  Then (tile_w + 2)(tile_h + 2) is at most
// 900 (512 threads) or 1548 (1024 threads) and the ring fits the threads.
__host__ __device__ constexpr int dyn_window(int threads) { return threads == 512 ? 900 : 1600; }
__host__ __device__ constexpr int dyn_width_cap(int threads) { return threads == 512 ? 128 : 256; }

// PRIO: gathers issued at raised wave priority (single-lattice launches).
// PF: the prefetching march allowed (where the kind and tile have it).
// tstep: the step number (keys the stochastic rounding of the FP32-rest kinds).
template <int ST, int TXS, int TYS, bool MRT, bool PRIO, bool PF>
__device__ __forceinline__ void step_tile(const StepArgs &A, int tile_x, int tile_y, int chunk, uint32_t tstep) {
    using Tr = Storage<ST>;
    using T = typename Tr::T;
    using C = typename Tr::C;
    static_assert(TXS == 0 || 2 * (TXS + 2) + 2 * TYS <= TXS * TYS, "ring must fit the thread count");
    static_assert(TXS != 0 || TYS == 512 || TYS == 1024, "run-time tiles use 512 or 1024 threads");
    const int TX = TXS ? TXS : A.tile_w;
    const int TY = TXS ? TYS : A.tile_h;
    const int PX = TX + 2;
    const int RING = 2 * PX + 2 * TY;
    constexpr int WIN = TXS ? (TXS + 2) * (TYS + 2) : dyn_window(TYS);
    __shared__ C win[4 * WIN];  // psi window: 4 planes of (TY + 2) x (TX + 2)
    auto W = [&](int s, int yy, int xx) -> C & { return win[s * WIN + yy * PX + xx]; };

    const int nx = A.nx, ny = A.ny, nz = A.nz;
    const int64_t plane = A.plane_stride;
    const int rowst = A.row_stride;
    const int S = int(A.pop_stride);
    const C rho0 = C(A.rho0), inv_rho0 = C(1.0 / A.rho0);
    const C G = C(A.G), tau = C(A.tau), omega = C(1.0 / A.tau);
    MrtRates<C> rates;
    if constexpr (MRT)
        rates = mrt_rates<C>(1.0 / A.tau, A.mrt.s_e, A.mrt.s_eps, A.mrt.s_q, A.mrt.s_pi, A.mrt.s_m, A.mrt.s_j);
    constexpr bool MR = Tr::kMassRest;
    static_assert(!(MRT && MR), "the MRT collision is not provided for the FP32-rest storage kinds");
    C shift[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) shift[a] = Tr::kShifted ? C(weight(a) * A.rho_ref) : C(0);
    const C rho_ref = C(A.rho_ref);
    // per-step keys of the node hashes (wave-uniform)
    uint32_t skey[3] = {0u, 0u, 0u};
    if constexpr (MR) {
#pragma unroll
        for (int k = 0; k < 3; ++k) skey[k] = hash32(3u * tstep + uint32_t(k) + 0x9E3779B9u);
    }
    // A gather returns the node's mass sum d: the density, or with kMassRest
    // the excess m = sum h_a (the moving populations as stored, in order,
    // then the FP32 rest), from which density_of gives the density.
    // The tile's sums are kept from the gather to the collision one plane
    // later.
    auto density_of = [&](C d) -> C { return MR ? rho_ref + d : d; };
    // z +- 1 wrapped, for z in [-1, nz] (no division)
    auto wrapz = [&](int z) { return z < 0 ? z + nz : (z >= nz ? z - nz : z); };

    const int x0 = tile_x * TX, y0 = tile_y * TY;
    const int z0 = chunk * A.zchunk;
    const int kend = min(A.zchunk, nz - z0);

    const int t = threadIdx.x;
    // Threads beyond a run-time tile only take part in the barriers.  The test
    // uses the run-time tile size for fixed tiles too: as a compile-time
    // constant it lets the compiler merge the tile and ring gathers, which
    // made the 16-bit storage kernels up to 1.7x slower on MI355X.
    const bool inside = t < A.tile_w * A.tile_h;
    const int lx = inside ? t % TX : 0, ly = inside ? t / TX : 0;
    const bool active = inside && (x0 + lx < nx) && (y0 + ly < ny);
    // Source columns/rows of the pull: index (1 - c) selects x - c.
    const int gx = wrapi(x0 + lx, nx), gy = wrapi(y0 + ly, ny);
    const int X[3] = {wrapi(gx - 1, nx), gx, wrapi(gx + 1, nx)};
    const int rsh = A.rec_shift;
    const int Y[3] = {row_offset(wrapi(gy - 1, ny), rowst, rsh, nx), row_offset(gy, rowst, rsh, nx),
                      row_offset(wrapi(gy + 1, ny), rowst, rsh, nx)};
    // kMassRest: FP32 rest population, indexed in floats from the plane base
    // (records of rowst 16-bit slots are rowst / 2 floats apart)
    const int YR = MR ? row_offset(gy, rowst / 2, rsh, nx) : 0;

    // A tile that spans whole rows (TX == nx) finds the psi of its left and
    // right ring columns among its own nodes (periodic in x), and one that
    // spans the whole cross-section its top and bottom rows as well: those
    // ring nodes are not gathered; the owning threads copy their psi into
    // the ghost cells of the window instead (same values, fewer gathers).
    const bool full_w = TX == nx, full_h = full_w && TY == ny;
    // Ring node handled by this thread (t < RING), in tile coordinates [-1, TX] x [-1, TY]:
    // the whole ring; the top and bottom rows without corners when full_w;
    // none when full_h.
    const int RING_N = full_h ? 0 : (full_w ? 2 * TX : RING);
    const bool ring = t < RING_N;
    int rx = 0, ry = 0;
    if (full_w) {
        rx = t < TX ? t : t - TX;
        ry = t < TX ? -1 : TY;
    } else if (t < PX) {
        rx = t - 1;
        ry = -1;
    } else if (t < 2 * PX) {
        rx = t - PX - 1;
        ry = TY;
    } else {
        const int r = t - 2 * PX;
        rx = (r < TY) ? -1 : TX;
        ry = (r < TY) ? r : r - TY;
    }
    const int rgx = wrapi(x0 + rx, nx), rgy = wrapi(y0 + ry, ny);
    const int RX[3] = {wrapi(rgx - 1, nx), rgx, wrapi(rgx + 1, nx)};
    const int RY[3] = {row_offset(wrapi(rgy - 1, ny), rowst, rsh, nx), row_offset(rgy, rowst, rsh, nx),
                       row_offset(wrapi(rgy + 1, ny), rowst, rsh, nx)};
    const int RYR = MR ? row_offset(rgy, rowst / 2, rsh, nx) : 0;

    // Addresses: a z plane (PlaneRef: a buffer resource or a 64-bit pointer,
    // chosen below per access kind), the population segment as the
    // wave-uniform offset and a 32-bit byte offset within the segment (the
    // host keeps a plane below 4 GiB).  The byte offsets of the nine (row,
    // column) combinations a pull reads from -- index (1 - c_y) 3 + (1 - c_x)
    // -- and of the FP32 rest population are fixed for the whole march.
    using u32 = uint32_t;
    // The prefetching march (below) for the single-grid BGK launches, FP64
    // only with at most 512 threads per workgroup: FP64 values at 1024
    // threads and the MRT collision leave too few registers for it, and the
    // batched launch measured 2% slower with it.
    constexpr bool kPrefetch = PF && PRIO && !MRT && (ST != kF64 || (TXS ? TXS * TYS : TYS) <= 512);
    // The bfloat16 kernels of the plain single-grid march (global loads)
    // would spill with eighteen offsets held over the march; they keep the
    // three row and three column offsets instead and form the nine byte
    // offsets at each gather (one add and shift each).  With buffer loads
    // they hold them (no spill; BF16S 1.8% and BF16M 1.2% faster on
    // 256 x 256 x 1024, MI355X).
    constexpr bool kHoldOffsets = !(ST == kBF16S || ST == kBF16M) || kPrefetch || !PRIO;
    using SrcPlane = PlaneRef<ST == kF64 || !PRIO || kPrefetch>;
    using DstPlane = PlaneRef<ST == kF64>;
    auto offsets9 = [&](const int(&XX)[3], const int(&YY)[3], u32(&o)[9]) {
        int yy[3] = {YY[0], YY[1], YY[2]}, xx[3] = {XX[0], XX[1], XX[2]};
        if constexpr (!kHoldOffsets)  // opaque copies: formed here, not hoisted
            asm volatile("" : "+v"(yy[0]), "+v"(yy[1]), "+v"(yy[2]), "+v"(xx[0]), "+v"(xx[1]), "+v"(xx[2]));
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) o[r * 3 + c] = u32(yy[r] + xx[c]) * u32(sizeof(T));
    };
    u32 OT[9], OR[9];
    if constexpr (kHoldOffsets) {
        offsets9(X, Y, OT);
        offsets9(RX, RY, OR);
    }
    const u32 OTR = MR ? u32(YR + X[1]) * 4u : 0u, ORR = MR ? u32(RYR + RX[1]) * 4u : 0u;
    const int64_t plane_b = plane * int64_t(sizeof(T));
    const u32 S_b = u32(S) * u32(sizeof(T));
    const char *const srcb = static_cast<const char *>(A.src);
    char *const dstb = static_cast<char *>(A.dst);

    // The 19 loads of a node's pull (raw storage values; with kMassRest the
    // FP32 rest population in `rest`), all issued before any use: the
    // scheduler would otherwise interleave load, wait and convert for 16-bit
    // storage.  With PRIO the wave issues them at raised priority, ahead of
    // other waves' collision arithmetic.  Measured on MI355X: single grids
    // FP16S 1-2% and narrow FP32 grids up to 7% faster, wide FP32 and FP64
    // unchanged; the batched launch, whose workgroups belong to many small
    // grids, 3-5% slower, so it keeps the default priority.
    auto issue = [&](int zc, const u32(&o_held)[9], const int(&XX)[3], const int(&YY)[3], u32 orest, T(&raw)[Q],
                     float &rest) {
        const SrcPlane pz[3] = {SrcPlane(srcb + wrapz(zc - 1) * plane_b), SrcPlane(srcb + zc * plane_b),
                                SrcPlane(srcb + wrapz(zc + 1) * plane_b)};  // index 1 + dz
        u32 o[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) o[q] = o_held[q];
        if constexpr (!kHoldOffsets) offsets9(XX, YY, o);
        if constexpr (PRIO) __builtin_amdgcn_s_setprio(2);
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            if (MR && a == 0)
                rest = pz[1].template load<float>(orest, 0);
            else
                raw[a] = pz[1 - kCZ[a]].template load<T>(o[(1 - kCY[a]) * 3 + (1 - kCX[a])], u32(pop_slot(a, MR)) * S_b);
        }
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
    };
    auto decode = [&](const T(&raw)[Q], float rest, C(&f)[Q]) {
#pragma unroll
        for (int a = 0; a < Q; ++a) f[a] = (MR && a == 0) ? C(rest) : Tr::decode(raw[a], shift[a]);
    };
    // mass sum of decoded populations, or with kMassRest of the stored values
    auto mass_of = [&](const T(&raw)[Q], float rest, const C(&f)[Q]) -> C {
        if constexpr (MR)
            return moving_sum16(raw) + rest;
        else
            return density(f);
    };
    auto gather = [&](int zc, const u32(&o_held)[9], const int(&XX)[3], const int(&YY)[3], u32 orest, C(&f)[Q]) -> C {
        T raw[Q];
        float rest = 0.0f;
        issue(zc, o_held, XX, YY, orest, raw, rest);
        decode(raw, rest, f);
        return mass_of(raw, rest, f);
    };
    // psi of the node at window cell (yy, xx) into slot s, and into the ghost
    // cells that hold the same node when the tile spans whole rows or the
    // whole cross-section.
    auto put_row = [&](int s, int yy, int xx, C v) {
        W(s, yy, xx) = v;
        if (full_w && xx == TX) W(s, yy, 0) = v;
        if (full_w && xx == 1) W(s, yy, TX + 1) = v;
    };
    auto put = [&](int s, int yy, int xx, C v) {
        put_row(s, yy, xx, v);
        if (full_h && yy == TY) put_row(s, 0, xx, v);
        if (full_h && yy == 1) put_row(s, TY + 1, xx, v);
    };
    // psi of plane zc for the tile (pops kept in f, mass sum in d) and the
    // ring, into window slot s.
    auto load_plane = [&](int zc, int s, C(&f)[Q], C &d) {
        if (inside) {
            d = gather(zc, OT, X, Y, OTR, f);
            put(s, ly + 1, lx + 1, pseudo_potential(density_of(d), rho0, inv_rho0));
        }
        if (ring) {
            C g[Q];  // only the mass sum is used
            const C dr = gather(zc, OR, RX, RY, ORR, g);
            put(s, ry + 1, rx + 1, pseudo_potential(density_of(dr), rho0, inv_rho0));
        }
    };

    // Odd chunks march towards -z.  Two neighbouring chunks then read the
    // planes around their common boundary at the same time (both at their
    // start or both at their end), so the second read tends to hit L2; with
    // short chunks those boundary planes are a large part of the gathers
    // (measured: +3% on narrow grids at z chunks of 8-32 on MI355X).
    const int dir = (chunk & 1) ? -1 : 1;
    const int zfirst = dir > 0 ? z0 : z0 + kend - 1;

    // Window slots: (k + 3) & 3 the plane behind, k & 3 the current one,
    // (k + 1) & 3 the plane ahead (in the marching direction).
    auto collide_store = [&](int k, C(&f)[Q], C d) {
        const int zc = zfirst + dir * k;
        const int behind = (k + 3) & 3, s0 = k & 3, ahead = (k + 1) & 3;
        const int s_lo = dir > 0 ? behind : ahead, s_hi = dir > 0 ? ahead : behind;  // planes z-1, z+1
        auto P = [&](int dx, int dy, int dz) -> C {
            const int s = dz < 0 ? s_lo : (dz > 0 ? s_hi : s0);
            return W(s, ly + 1 + dy, lx + 1 + dx);
        };
        C Fx, Fy, Fz;
        sc_force<C>(W(s0, ly + 1, lx + 1), G, P, Fx, Fy, Fz);
        const DstPlane pd(dstb + zc * plane_b);
        if constexpr (MR) {
            T out[Q];
            // random words of this node and step (node index as in the canonical layout)
            const uint32_t node = (uint32_t(zc) * uint32_t(ny) + uint32_t(gy)) * uint32_t(nx) + uint32_t(gx);
            const uint32_t rnd[3] = {hash32(node ^ skey[0]), hash32(node ^ skey[1]), hash32(node ^ skey[2])};
            collide_shifted<Tr>(f, d, out, Fx, Fy, Fz, tau, omega, rho_ref, rnd);
            pd.store_nt(f[0], OTR, 0);
            const u32 oc = kHoldOffsets ? OT[4] : u32(Y[1] + X[1]) * u32(sizeof(T));
#pragma unroll
            for (int a = 1; a < Q; ++a) pd.store_nt(out[a], oc, u32(pop_slot(a, MR)) * S_b);
        } else {
            if constexpr (MRT)
                collide_mrt<C>(f, Fx, Fy, Fz, rates);
            else
                collide<C>(f, d, Fx, Fy, Fz, tau, omega);
            const u32 oc = kHoldOffsets ? OT[4] : u32(Y[1] + X[1]) * u32(sizeof(T));
#pragma unroll
            for (int a = 0; a < Q; ++a) pd.store_nt(Tr::encode(f[a], shift[a]), oc, u32(a) * S_b);
        }
    };

    if constexpr (!kPrefetch) {
        // Two register sets take turns as the plane being collided and the
        // plane ahead: the march is unrolled by two, so nothing is copied
        // between them.
        C fa[Q], fb[Q], da = C(0), db = C(0);
        load_plane(wrapz(zfirst - dir), 3, fb, db);
        load_plane(zfirst, 0, fa, da);
        auto advance = [&](int k, C(&cur)[Q], C dcur, C(&nxt)[Q], C &dnxt) {
            load_plane(wrapz(zfirst + dir * (k + 1)), (k + 1) & 3, nxt, dnxt);
            __syncthreads();
            if (active) collide_store(k, cur, dcur);
        };
        for (int k = 0; k < kend; k += 2) {
            advance(k, fa, da, fb, db);
            if (k + 1 < kend) advance(k + 1, fb, db, fa, da);
        }
    } else {
        // Prefetching march: the tile's loads for plane k + 2 are issued
        // right after the barrier of plane k, once plane k's values are
        // decoded, and fly during plane k's collision and stores; plane
        // k + 1's values (issued one plane earlier) only need their mass sum
        // for psi before the barrier.  The tile keeps its planes as stored
        // values (two sets, taking turns) and decodes at the collision.
        T ra[Q], rb[Q];
        float sa = 0.0f, sb = 0.0f;
        C da = C(0), db = C(0);
        {
            C f[Q], d = C(0);
            load_plane(wrapz(zfirst - dir), 3, f, d);  // psi only
        }
        auto tile_psi = [&](int s, const T(&raw)[Q], float rest, C &d) {
            C f[Q];
            if constexpr (!MR) decode(raw, rest, f);
            d = mass_of(raw, rest, f);
            put(s, ly + 1, lx + 1, pseudo_potential(density_of(d), rho0, inv_rho0));
        };
        auto ring_psi = [&](int zc, int s) {
            C g[Q];  // only the mass sum is used
            const C dr = gather(zc, OR, RX, RY, ORR, g);
            put(s, ry + 1, rx + 1, pseudo_potential(density_of(dr), rho0, inv_rho0));
        };
        if (inside) {
            issue(zfirst, OT, X, Y, OTR, ra, sa);
            tile_psi(0, ra, sa, da);
        }
        if (ring) ring_psi(zfirst, 0);
        if (inside) issue(wrapz(zfirst + dir), OT, X, Y, OTR, rb, sb);
        // plane k collided from (rc, scur, dcur); plane k + 1 in (rn, sn)
        auto advance = [&](int k, T(&rc)[Q], float &scur, C dcur, T(&rn)[Q], float sn, C &dn) {
            if (ring) ring_psi(wrapz(zfirst + dir * (k + 1)), (k + 1) & 3);
            if (inside) tile_psi((k + 1) & 3, rn, sn, dn);
            __syncthreads();
            C f[Q];
            decode(rc, scur, f);
            if (inside && k + 1 < kend) issue(wrapz(zfirst + dir * (k + 2)), OT, X, Y, OTR, rc, scur);
            if (active) collide_store(k, f, dcur);
        };
        for (int k = 0; k < kend; k += 2) {
            advance(k, ra, sa, da, rb, sb, db);
            if (k + 1 < kend) advance(k + 1, rb, sb, db, ra, sa, da);
        }
    }
}

template <int ST, int TX, int TY, bool MRT, bool PF = true>
__device__ __forceinline__ void step_grid(const StepArgs &A) {
    const int lb = xcd_contiguous(blockIdx.x, gridDim.x);
    const int ntile = A.tiles_x * A.tiles_y;
    const int tile = lb % ntile, chunk = lb / ntile;
    uint32_t tstep = 0;
    if constexpr (Storage<ST>::kMassRest) tstep = *A.step_base + A.step_add;
    step_tile<ST, TX, TY, MRT, true, PF>(A, tile % A.tiles_x, tile / A.tiles_x, chunk, tstep);
}

template <int ST, int TX, int TY>
__global__ __launch_bounds__(TX ? TX * TY : TY) void k_step_bgk(StepArgs A) {
    step_grid<ST, TX, TY, false>(A);
}

// The plain march (no prefetch), for grids whose planes hold more tiles than
// the device keeps resident (launch_step).
template <int ST, int TX, int TY>
__global__ __launch_bounds__(TX ? TX * TY : TY) void k_step_bgk_plain(StepArgs A) {
    step_grid<ST, TX, TY, false, false>(A);
}

template <int ST, int TX, int TY>
__global__ __launch_bounds__(TX ? TX * TY : TY) void k_step_mrt(StepArgs A) {
    step_grid<ST, TX, TY, true>(A);
}

// Batched form: one launch covers every case's work items.  Items are
// (case, tile, chunk) triples; case parameters and lattice pointers come from
// a device table; frozen cases and padding items (case -1) are skipped.  The
// host orders the list by XCD (workgroup b runs on XCD b mod 8), so the
// workgroup index is used as is.
template <int ST, int TX, int TY>
__global__ __launch_bounds__(TX ? TX * TY : TY) void k_step_batch(const BatchCase *__restrict__ cases,
                                                       const int4 *__restrict__ items,
                                                       const int32_t *__restrict__ frozen,
                                                       int parity, const uint32_t *step_base,
                                                       uint32_t step_add) {
    const int4 it = items[blockIdx.x];
    if (it.x < 0 || frozen[it.x]) return;
    const BatchCase &bc = cases[it.x];
    StepArgs A = bc.args;
    A.src = bc.lat[parity];
    A.dst = bc.lat[parity ^ 1];
    uint32_t tstep = 0;
    if constexpr (Storage<ST>::kMassRest) tstep = *step_base + step_add;
    step_tile<ST, TX, TY, false, false, false>(A, it.y % A.tiles_x, it.y / A.tiles_x, it.z, tstep);
}

// ---------------------------------------------------------------------------
// Launch tables.

struct TileEntry {
    int tx, ty;
    const void *fn[kNumStorage];
    const void *batch_fn[kNumStorage];
    const void *mrt_fn[kNumStorage];    // MRT collision: run-time tiles, storages 0-3 only
    const void *plain_fn[kNumStorage];  // the plain march: run-time tiles, FP64 and FP32
};

// Every tile has the four storage kinds of the first round of kernels; the
// FP32-rest kinds (F16M, BF16M) are compiled for the run-time tiles only.
#define LBM_TILE_FNS4(K, TXV, TYV) \
    (const void *)K<kF64, TXV, TYV>, (const void *)K<kF32, TXV, TYV>, (const void *)K<kF16S, TXV, TYV>, \
        (const void *)K<kBF16S, TXV, TYV>
#define LBM_TILE(TXV, TYV)                                                                          \
    {TXV, TYV, {LBM_TILE_FNS4(k_step_bgk, TXV, TYV), nullptr, nullptr},                             \
     {LBM_TILE_FNS4(k_step_batch, TXV, TYV), nullptr, nullptr},                                     \
     {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr},                                        \
     {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr}}
#define LBM_TILE_RT(TXV, TYV)                                                                       \
    {TXV, TYV,                                                                                      \
     {LBM_TILE_FNS4(k_step_bgk, TXV, TYV), (const void *)k_step_bgk<kF16M, TXV, TYV>,              \
      (const void *)k_step_bgk<kBF16M, TXV, TYV>},                                                  \
     {LBM_TILE_FNS4(k_step_batch, TXV, TYV), (const void *)k_step_batch<kF16M, TXV, TYV>,          \
      (const void *)k_step_batch<kBF16M, TXV, TYV>},                                                \
     {LBM_TILE_FNS4(k_step_mrt, TXV, TYV), nullptr, nullptr},                                       \
     {(const void *)k_step_bgk_plain<kF64, TXV, TYV>, (const void *)k_step_bgk_plain<kF32, TXV, TYV>, \
      nullptr, nullptr, nullptr, nullptr}}

// Entries (0, 512) and (0, 1024) are the run-time shaped tiles.
static const TileEntry kTiles[] = {
    LBM_TILE_RT(0, 512), LBM_TILE_RT(0, 1024), LBM_TILE(256, 4), LBM_TILE(128, 8), LBM_TILE(128, 4), LBM_TILE(64, 16), LBM_TILE(64, 8),
    LBM_TILE(64, 4), LBM_TILE(32, 16), LBM_TILE(32, 8), LBM_TILE(16, 16),
};
#undef LBM_TILE
#undef LBM_TILE_RT
#undef LBM_TILE_FNS4

// Width: nx split into the fewest tiles of at most the cap, as evenly as
// possible, so that the tiles carry equal work (a 24-wide remainder tile beside
// 256-wide ones marches as long for a tenth of the nodes); when nx is a
// multiple of 32 the width is rounded up to a multiple of 32, so that the
// tiles' row segments start on the same 32-element boundaries as the rows.
// With the round-aware z chunk of the default launch this made non-256 grids
// 3-45% faster on MI355X (e.g. 280 x 280 x 628 FP32 3.30 -> 2.00 ms,
// 288 x 288 x 512 2.39 -> 1.40 ms; 256 x 256 x 1024 unchanged).
void dynamic_tile(int threads, int nx, int ny, int *tw, int *th) {
    const int cap = dyn_width_cap(threads);
    const int ntx = (nx + cap - 1) / cap;
    int w = (nx + ntx - 1) / ntx;
    if (nx % 32 == 0) w = std::min(cap, (w + 31) / 32 * 32);
    int hmax = threads / w;
    if (hmax > 64) hmax = 64;
    const int ntile_y = (ny + hmax - 1) / hmax;
    *tw = w;
    *th = (ny + ntile_y - 1) / ntile_y;
}

int num_tiles() { return int(sizeof(kTiles) / sizeof(kTiles[0])); }
void tile_shape(int i, int *tx, int *ty) {
    *tx = kTiles[i].tx;
    *ty = kTiles[i].ty;
}
int find_tile(int tx, int ty) {
    for (int i = 0; i < num_tiles(); ++i)
        if (kTiles[i].tx == tx && kTiles[i].ty == ty) return i;
    return -1;
}

bool tile_has_mrt(int tile_index) { return kTiles[tile_index].mrt_fn[0] != nullptr; }
bool tile_has_storage(int tile_index, int storage) { return kTiles[tile_index].fn[storage] != nullptr; }

int launch_slots(int tile_index, int storage) {
    const TileEntry &e = kTiles[tile_index];
    const int threads = e.tx ? e.tx * e.ty : e.ty;
    int dev = 0, cus = 0, per_cu = 0;
    if (!e.fn[storage]) return 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, e.fn[storage], threads, 0) != hipSuccess)
        return 0;
    return cus * per_cu;
}

// Workgroups of the (prefetching) step kernel resident at once on the current
// device, cached per device, tile and storage kind.
static int resident_slots(int tile_index, int storage) {
    constexpr int kMaxDev = 64, kMaxTiles = 16;
    static std::atomic<int> cache[kMaxDev][kMaxTiles][kNumStorage];  // 0: not yet known
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev || tile_index >= kMaxTiles)
        return launch_slots(tile_index, storage);
    int v = cache[dev][tile_index][storage].load(std::memory_order_relaxed);
    if (v == 0) {
        v = launch_slots(tile_index, storage);
        if (v > 0) cache[dev][tile_index][storage].store(v, std::memory_order_relaxed);
    }
    return v;
}

hipError_t launch_step(int tile_index, int storage, const StepArgs &A, hipStream_t s) {
    const TileEntry &e = kTiles[tile_index];
    const void *fn = A.mrt.on ? e.mrt_fn[storage] : e.fn[storage];
    if (!fn) return hipErrorInvalidDeviceFunction;
    // The prefetching march holds a third plane per workgroup in flight.
    // When a plane has more tiles than the device keeps resident, the
    // workgroups that share ring rows are not all resident together and the
    // larger footprint evicts those rows from L2 before the neighbour reads
    // them: FP32 on 1024 x 1024 x 1024 read 96 instead of 81 B per node from
    // HBM and ran 5.6% slower (rocprofv3 FETCH_SIZE, MI355X).  Such grids take
    // the plain march (measured on MI355X, FP32: prefetch faster up to 256
    // tiles of 1024 threads per plane -- 256x256, 512x512, 1024x256 -- and
    // slower from 512 tiles -- 1024x512, 768x768, 1024x1024).  The 16-bit
    // kinds, with half the bytes per plane, keep the prefetch: 1-2% faster
    // on 1024x512x1024, 768x768x1024 and 1024x1024x2047.
    if (!A.mrt.on && e.plain_fn[storage] && int64_t(A.tiles_x) * A.tiles_y > resident_slots(tile_index, storage))
        fn = e.plain_fn[storage];
    const int nblk = A.tiles_x * A.tiles_y * A.nchunks;
    StepArgs args = A;
    void *kargs[] = {&args};
    const int threads = e.tx ? e.tx * e.ty : e.ty;
    return hipLaunchKernel(fn, dim3(nblk), dim3(threads), kargs, 0, s);
}

hipError_t launch_step_batch(int tile_index, int storage, const BatchCase *cases,
                             const int4 *items, int nitems, const int32_t *frozen, int parity,
                             const uint32_t *step_base, uint32_t step_add, hipStream_t s) {
    const TileEntry &e = kTiles[tile_index];
    if (!e.batch_fn[storage]) return hipErrorInvalidDeviceFunction;
    void *kargs[] = {(void *)&cases, (void *)&items, (void *)&frozen, &parity, (void *)&step_base, &step_add};
    const int threads = e.tx ? e.tx * e.ty : e.ty;
    return hipLaunchKernel(e.batch_fn[storage], dim3(nitems), dim3(threads), kargs, 0, s);
}

}  // namespace lbm
