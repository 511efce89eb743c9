// Mesh-based surface measures per object: the baseline the paper compares its
// local-thickness sphericity against (Related work; Experiments, Benchmark
// methods: the object mask is meshed -- marching cubes in 3D, marching squares in
// 2D -- and the mesh area or contour length replaces the surface / perimeter in
// Wadell's sphericity, Background Eq. 1, or the perimeter sphericity P_c / P_o).
//
// Surface used here: the iso-surface at level 1/2 of each object's own 0/1 mask
// (every other label and everything outside the image is 0), linearly
// interpolated inside the simplices of the lattice.
//   3D: every unit cube is split into the six tetrahedra of the Freudenthal (Kuhn)
//       subdivision along its (0,0,0)-(1,1,1) diagonal: for each ordering (a, b, c)
//       of the axes, the tetrahedron 0 -> e_a -> e_a + e_b -> e_a + e_b + e_c.  In
//       a tetrahedron the surface passes through the midpoints of the edges that
//       join an inside and an outside corner: a triangle when one corner differs
//       from the other three, a parallelogram for two against two.  Neighbouring
//       cubes split their common faces alike, so the surface is closed.
//   2D: every unit square contributes the segments joining the midpoints of its
//       sign-changing sides; a square with two diagonal inside corners cuts off
//       each inside corner (both pairings give the same length).
// All corners are lattice points, so the area inside a cube (the length inside a
// square) depends only on which of its 8 (4) corners are inside: a 256-entry
// (16-entry) table computed on the host from the construction above.  Per cube,
// each label present among its corners adds the table entry of its corner mask.
// Areas are summed in Q.32 fixed point (uint64), so results do not depend on the
// order of the atomics.
#include <math.h>

#include <mutex>

#include "lt_internal.h"

namespace lt {

constexpr double MESH_SCALE = 4294967296.0;     // Q.32
constexpr int MESH_TAB = 128;                   // labels per block table
constexpr int MESH_ZCHUNK = 64;                 // cube layers per block (3D); rows per block (2D)
constexpr int MESH_BY = 4;                      // cube rows per block (3D)

// ---------------------------------------------------------------- host tables

struct V3 {
    double x, y, z;
};
static V3 v3sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
static V3 v3mid(V3 a, V3 b) { return {(a.x + b.x) / 2, (a.y + b.y) / 2, (a.z + b.z) / 2}; }
static double v3cross_norm(V3 a, V3 b) {
    const double cx = a.y * b.z - a.z * b.y, cy = a.z * b.x - a.x * b.z, cz = a.x * b.y - a.y * b.x;
    return sqrt(cx * cx + cy * cy + cz * cz);
}

// Iso-surface area inside one tetrahedron with corners p[0..3], `in` = inside flags.
static double tet_area(const V3 p[4], const bool in[4]) {
    int n_in = 0;
    for (int i = 0; i < 4; ++i) n_in += in[i];
    if (n_in == 0 || n_in == 4) return 0.0;
    if (n_in == 1 || n_in == 3) {
        int lone = 0;                                   // the corner unlike the others
        for (int i = 0; i < 4; ++i)
            if (in[i] == (n_in == 1)) lone = i;
        V3 m[3];
        int k = 0;
        for (int i = 0; i < 4; ++i)
            if (i != lone) m[k++] = v3mid(p[lone], p[i]);
        return 0.5 * v3cross_norm(v3sub(m[1], m[0]), v3sub(m[2], m[0]));
    }
    int u = -1, v = -1, a = -1, b = -1;                 // inside u, v; outside a, b
    for (int i = 0; i < 4; ++i) {
        if (in[i]) (u < 0 ? u : v) = i;
        else (a < 0 ? a : b) = i;
    }
    // midpoints on u-a, u-b, v-b, v-a in cyclic order: a parallelogram
    const V3 mua = v3mid(p[u], p[a]), mub = v3mid(p[u], p[b]), mva = v3mid(p[v], p[a]);
    return v3cross_norm(v3sub(mub, mua), v3sub(mva, mua));
}

// Cube table: corner k of the unit cube is (dx, dy, dz) = (k & 1, (k >> 1) & 1, k >> 2);
// entry m is the area inside the cube when the corners with bit k of m set are inside.
static void build_cube_table(uint64_t* out) {
    static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (int m = 0; m < 256; ++m) {
        double area = 0.0;
        for (const auto& pr : perms) {
            int c[3] = {0, 0, 0};
            V3 p[4];
            bool in[4];
            for (int s = 0; s < 4; ++s) {
                if (s > 0) c[pr[s - 1]] = 1;             // walk e_a, then e_b, then e_c
                p[s] = {(double)c[0], (double)c[1], (double)c[2]};
                const int k = c[0] | (c[1] << 1) | (c[2] << 2);
                in[s] = (m >> k) & 1;
            }
            area += tet_area(p, in);
        }
        out[m] = (uint64_t)llround(area * MESH_SCALE);
    }
}

// Square table: corner k of the unit square is (dx, dy) = (k & 1, k >> 1).
static void build_square_table(uint64_t* out) {
    const double h = 0.5 * sqrt(2.0);                   // segment cutting off one corner
    for (int m = 0; m < 16; ++m) {
        const int n_in = __builtin_popcount(m);
        double len = 0.0;
        if (n_in == 1 || n_in == 3) len = h;
        else if (m == 0x3 || m == 0xc || m == 0x5 || m == 0xa) len = 1.0;   // one side inside
        else if (m == 0x9 || m == 0x6) len = 2.0 * h;   // diagonal pair: both corners cut off
        out[m] = (uint64_t)llround(len * MESH_SCALE);
    }
}

static std::once_flag g_mesh_once;
static uint64_t g_cube_tab[256], g_square_tab[16];

__constant__ uint64_t c_cube_tab[256];
__constant__ uint64_t c_square_tab[16];

// ---------------------------------------------------------------- device side

__global__ void mesh_zero(uint64_t* vol, uint64_t* area, uint32_t nlab) {
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < nlab) {
        vol[l] = 0;
        area[l] = 0;
    }
}

__device__ __forceinline__ void wave_lds_sync_mesh() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Running per-thread total of one label; merged into the block table when another
// label arrives (columns cross few objects, so merges are rare).
struct RunAcc {
    uint32_t l = 0;
    uint64_t s = 0;
};

struct MeshTable {
    uint32_t* key;
    unsigned long long* vol;
    unsigned long long* area;
};

__device__ __forceinline__ void mesh_merge(const MeshTable& t, uint64_t* gsum, bool is_area, uint32_t l,
                                           uint64_t s) {
    if (l == 0 || s == 0) return;
    const int slot = lds_slot<MESH_TAB>(t.key, l);
    if (slot >= 0) atomicAdd(is_area ? &t.area[slot] : &t.vol[slot], (unsigned long long)s);
    else atomicAdd((unsigned long long*)&gsum[l], (unsigned long long)s);
}

__device__ __forceinline__ void run_add(RunAcc& r, const MeshTable& t, uint64_t* gsum, bool is_area, uint32_t l,
                                        uint64_t s) {
    if (l != r.l) {
        mesh_merge(t, gsum, is_area, r.l, r.s);
        r.l = l;
        r.s = 0;
    }
    r.s += s;
}

// Per cube (corner labels c[0..NC-1]): every label present adds the table entry of
// its corner mask to its area run.
template <int NC>
__device__ __forceinline__ void cube_labels(const uint32_t (&c)[NC], const uint64_t* tab, RunAcc& ra,
                                            const MeshTable& t, uint64_t* garea) {
    bool uniform = true;
#pragma unroll
    for (int k = 1; k < NC; ++k) uniform &= c[k] == c[0];
    if (uniform) return;                                // inside one label or background: no surface
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        if (c[k] == 0u) continue;
        bool first = true;
#pragma unroll
        for (int j = 0; j < k; ++j) first &= c[j] != c[k];
        if (!first) continue;
        uint32_t m = 0;
#pragma unroll
        for (int j = 0; j < NC; ++j) m |= (c[j] == c[k] ? 1u : 0u) << j;
        run_add(ra, t, garea, true, c[k], tab[m]);
    }
}

// Per-lane area of a queued cube: each label present among the 8 corners adds the
// table entry of its corner mask (typically two labels: an object and background
// or a touching object).
__device__ __forceinline__ void cube_general(const uint32_t (&c)[8], RunAcc& ra, const MeshTable& t,
                                             uint64_t* garea) {
    uint32_t rem = 0xffu;
    while (rem) {
        const uint32_t k = (uint32_t)__builtin_ctz(rem);
        const uint32_t a0 = (k & 1u) ? c[1] : c[0], a1 = (k & 1u) ? c[3] : c[2];
        const uint32_t a2 = (k & 1u) ? c[5] : c[4], a3 = (k & 1u) ? c[7] : c[6];
        const uint32_t b0 = (k & 2u) ? a1 : a0, b1 = (k & 2u) ? a3 : a2;
        const uint32_t v = (k & 4u) ? b1 : b0;
        uint32_t m = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) m |= (c[j] == v ? 1u : 0u) << j;
        if (v) run_add(ra, t, garea, true, v, c_cube_tab[m]);
        rem &= ~m;
    }
}

constexpr int MQ_CAP = 128;                     // queued cubes per wave (two uint4 each)

// 3D: block = 64 (x) x MESH_BY (y) threads, one wave per cube row.  Lane i of wave
// ty loads the label column X = bx * 64 + i of rows Y - 1 and Y (Y = by * MESH_BY +
// ty) and owns the cube with corners x in {X - 1, X}, y in {Y - 1, Y} (the X - 1
// values come from lane i - 1 by a DPP lane shift; lane 0 loads them).  The lane
// with X = nx - 1 also owns the cube past the last column, the wave with Y = ny - 1
// the cubes past the last row (their outer corners are outside, i.e. 0), so cube
// origins cover -1..n-1 per axis (the zero padding).  A block walks cube layers
// cz in [bz * MESH_ZCHUNK - 1, ...), the last block through nz - 1, loading one plane
// ahead.  Uniform cubes (one label, or background) hold no surface; the others are
// appended to the wave's queue in LDS and processed 64 at a time, so the per-label
// work scales with the surface rather than the volume.  The voxel counted with a
// cube is its (1, 1, 1) corner, so every voxel of the image is counted once.
template <typename L>
__global__ void __launch_bounds__(64 * MESH_BY)
mesh_area3d(const L* __restrict__ lab, int nx, int ny, int nz, uint32_t max_label, uint64_t* __restrict__ gvol,
            uint64_t* __restrict__ garea, uint32_t* err) {
    __shared__ uint32_t s_key[MESH_TAB];
    __shared__ unsigned long long s_vol[MESH_TAB], s_area[MESH_TAB];
    __shared__ uint4 s_q[MESH_BY][MQ_CAP][2];
    const int lane = threadIdx.x;
    const int wy = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    const int tid = wy * 64 + lane;
    for (int q = tid; q < MESH_TAB; q += 64 * MESH_BY) {
        s_key[q] = 0u;
        s_vol[q] = s_area[q] = 0ull;
    }
    __syncthreads();
    const MeshTable t{s_key, s_vol, s_area};
    uint4 (*queue)[2] = s_q[wy];
    const int X = blockIdx.x * 64 + lane;
    const int Y = blockIdx.y * MESH_BY + wy;
    const int cz0 = blockIdx.z * MESH_ZCHUNK - 1;
    const int cz1 = blockIdx.z + 1 == gridDim.z ? nz : cz0 + MESH_ZCHUNK;   // cube layers [cz0, cz1)
    RunAcc rv, ra;
    if (Y < ny) {                                       // wave-uniform
        const size_t plane = (size_t)ny * nx;
        const bool xin = X < nx, xmin = X >= 1 && X - 1 < nx, y0in = Y >= 1;
        const bool extra_x = X == nx - 1, extra_y = Y == ny - 1;
        const size_t r0 = (size_t)(y0in ? Y - 1 : 0) * nx, r1 = (size_t)Y * nx;
        // raw loads of plane z: rows Y - 1, Y at column X (and X - 1 for lane 0); the
        // range check waits until the values are used, so the loads stay in flight
        // (as 32-bit words: negative int32 labels read as >= 2^31 > max_label)
        struct Raw {
            uint32_t a, b, am, bm;
        };
        bool bad = false;                               // a label above max_label (or negative)
        auto load = [&](int z) {
            Raw r{0u, 0u, 0u, 0u};
            if (z >= 0 && z < nz) {
                const L* base = lab + (size_t)z * plane;
                if (xin && y0in) r.a = (uint32_t)base[r0 + X];
                if (xin) r.b = (uint32_t)base[r1 + X];
                if (lane == 0 && xmin && y0in) r.am = (uint32_t)base[r0 + X - 1];
                if (lane == 0 && xmin) r.bm = (uint32_t)base[r1 + X - 1];
            }
            return r;
        };
        auto valid = [&](uint32_t v) -> uint32_t {
            const bool b = v > max_label;
            bad |= b;
            return b ? 0u : v;
        };
        // plane values: [0] (Y-1, X-1), [1] (Y-1, X), [2] (Y, X-1), [3] (Y, X)
        auto finish = [&](const Raw& r, uint32_t (&p)[4]) {
            p[1] = valid(r.a);
            p[3] = valid(r.b);
            const uint32_t am = valid(r.am), bm = valid(r.bm);
            p[0] = (uint32_t)__builtin_amdgcn_update_dpp((int)am, (int)p[1], 0x138, 0xf, 0xf, false);  // wave_shr:1
            p[2] = (uint32_t)__builtin_amdgcn_update_dpp((int)bm, (int)p[3], 0x138, 0xf, 0xf, false);
        };
        int head = 0, tail = 0;                         // wave-uniform queue counters
        auto drain = [&](int cnt) {
            wave_lds_sync_mesh();
            if (lane < cnt) {
                const int slot = (head + lane) & (MQ_CAP - 1);
                const uint4 lo = queue[slot][0], hi = queue[slot][1];
                const uint32_t c[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
                cube_general(c, ra, t, garea);
            }
            head += cnt;
            wave_lds_sync_mesh();
        };
        auto cube = [&](bool own, const uint32_t (&c)[8]) {
            bool uni = true;
#pragma unroll
            for (int k = 1; k < 8; ++k) uni &= c[k] == c[0];
            const bool q = own && !uni;
            const uint64_t m = __ballot(q);
            if (!m) return;
            if (q) {
                const int slot = (tail + __popcll(m & ((1ull << lane) - 1ull))) & (MQ_CAP - 1);
                queue[slot][0] = make_uint4(c[0], c[1], c[2], c[3]);
                queue[slot][1] = make_uint4(c[4], c[5], c[6], c[7]);
            }
            tail += __popcll(m);
            if (tail - head >= 64) drain(64);
        };
        uint32_t lo[4], hi[4];
        finish(load(cz0), lo);
        Raw nxt = load(cz0 + 1);
        for (int cz = cz0; cz < cz1; ++cz) {
            const Raw cur = nxt;
            if (cz + 2 <= cz1) nxt = load(cz + 2);
            finish(cur, hi);
            if (hi[3]) run_add(rv, t, gvol, false, hi[3], 1);
            const uint32_t c[8] = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
            cube(xin, c);
            if (__ballot(extra_x)) {                    // the cube past the last column
                const uint32_t e[8] = {lo[1], 0u, lo[3], 0u, hi[1], 0u, hi[3], 0u};
                cube(extra_x, e);
            }
            if (extra_y) {                              // the cubes past the last row
                const uint32_t e[8] = {lo[2], lo[3], 0u, 0u, hi[2], hi[3], 0u, 0u};
                cube(xin, e);
                const uint32_t f[8] = {lo[3], 0u, 0u, 0u, hi[3], 0u, 0u, 0u};
                cube(extra_x, f);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) lo[k] = hi[k];
        }
        if (tail > head) drain(tail - head);
        if (__ballot(bad) && lane == 0) atomicOr(err, ERR_LABEL);
    }
    mesh_merge(t, gvol, false, rv.l, rv.s);
    mesh_merge(t, garea, true, ra.l, ra.s);
    __syncthreads();
    for (int q = tid; q < MESH_TAB; q += 64 * MESH_BY) {
        const uint32_t l = s_key[q];
        if (l == 0u) continue;
        if (s_vol[q]) atomicAdd((unsigned long long*)&gvol[l], s_vol[q]);
        if (s_area[q]) atomicAdd((unsigned long long*)&garea[l], s_area[q]);
    }
}

// 2D: block = 256 threads along x; thread owns the column of squares with origin
// cx = blockIdx.x * 256 + tid - 1 over the square rows cy in [by * MESH_ZCHUNK - 1, ...).
template <typename L>
__global__ void __launch_bounds__(256)
mesh_len2d(const L* __restrict__ lab, int nx, int ny, uint32_t max_label, uint64_t* __restrict__ gvol,
           uint64_t* __restrict__ garea, uint32_t* err) {
    __shared__ uint32_t s_key[MESH_TAB];
    __shared__ unsigned long long s_vol[MESH_TAB], s_area[MESH_TAB];
    const int tid = threadIdx.x;
    for (int q = tid; q < MESH_TAB; q += 256) {
        s_key[q] = 0u;
        s_vol[q] = s_area[q] = 0ull;
    }
    __syncthreads();
    const MeshTable t{s_key, s_vol, s_area};
    const int cx = blockIdx.x * 256 + tid - 1;
    const int cy0 = blockIdx.y * MESH_ZCHUNK - 1;
    const int cy1 = min(ny, cy0 + MESH_ZCHUNK);
    RunAcc rv, ra;
    if (cx < nx) {
        const bool x0in = cx >= 0, x1in = cx + 1 < nx;
        const size_t xa = (size_t)(x0in ? cx : 0), xb = (size_t)(x1in ? cx + 1 : 0);
        bool bad = false;
        auto load_row = [&](int y, uint32_t (&p)[2]) {
            L v0 = L(0), v1 = L(0);
            if (y >= 0 && y < ny) {
                const L* base = lab + (size_t)y * nx;
                if (x0in) v0 = base[xa];
                if (x1in) v1 = base[xb];
            }
            const bool b0 = label_negative(v0) || (uint64_t)v0 > max_label;
            const bool b1 = label_negative(v1) || (uint64_t)v1 > max_label;
            bad |= b0 | b1;
            p[0] = b0 ? 0u : (uint32_t)v0;
            p[1] = b1 ? 0u : (uint32_t)v1;
        };
        uint32_t lo[2], hi[2];
        load_row(cy0, lo);
        for (int cy = cy0; cy < cy1; ++cy) {
            load_row(cy + 1, hi);
            const uint32_t c[4] = {lo[0], lo[1], hi[0], hi[1]};
            if (hi[1]) run_add(rv, t, gvol, false, hi[1], 1);
            cube_labels<4>(c, c_square_tab, ra, t, garea);
            lo[0] = hi[0];
            lo[1] = hi[1];
        }
        if (bad) atomicOr(err, ERR_LABEL);
    }
    mesh_merge(t, gvol, false, rv.l, rv.s);
    mesh_merge(t, garea, true, ra.l, ra.s);
    __syncthreads();
    for (int q = tid; q < MESH_TAB; q += 256) {
        const uint32_t l = s_key[q];
        if (l == 0u) continue;
        if (s_vol[q]) atomicAdd((unsigned long long*)&gvol[l], s_vol[q]);
        if (s_area[q]) atomicAdd((unsigned long long*)&garea[l], s_area[q]);
    }
}

// Per label: area (contour length in 2D) from the Q.32 sum and the mesh sphericity,
// 3D pi^(1/3) (6V)^(2/3) / A (Background, Eq. 1, with the mesh area), 2D
// 2 sqrt(pi V) / P (the perimeter sphericity with the contour length as P_o).
// V is the voxel (pixel) count; labels with V = 0 get area 0 and NaN.
__global__ void mesh_finish(const uint64_t* __restrict__ vol_acc, const uint64_t* __restrict__ area_acc,
                            uint32_t nlab, int ndim, uint64_t* __restrict__ volume, float* __restrict__ area,
                            float* __restrict__ sphericity) {
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nlab) return;
    const uint64_t v = vol_acc[l];
    const double a = (double)area_acc[l] * (1.0 / MESH_SCALE);
    if (volume) volume[l] = v;
    if (area) area[l] = (float)a;
    if (sphericity) {
        double s = __builtin_nan("");
        if (v > 0 && a > 0.0) {
            const double V = (double)v;
            s = ndim == 3 ? cbrt(M_PI) * pow(6.0 * V, 2.0 / 3.0) / a : 2.0 * sqrt(M_PI * V) / a;
        }
        sphericity[l] = (float)s;
    }
}

// ---------------------------------------------------------------- host side

size_t mesh_scratch_bytes(uint32_t max_label) {
    return 2 * (((size_t)max_label + 1) * sizeof(uint64_t) + 256);
}

static lt_status mesh_tables(lt_ctx* ctx) {
    std::call_once(g_mesh_once, [] {
        build_cube_table(g_cube_tab);
        build_square_table(g_square_tab);
    });
    (void)ctx;
    lt_status st = hip_check(hipMemcpyToSymbol(HIP_SYMBOL(c_cube_tab), g_cube_tab, sizeof(g_cube_tab)),
                             "copy cube table");
    if (!st) st = hip_check(hipMemcpyToSymbol(HIP_SYMBOL(c_square_tab), g_square_tab, sizeof(g_square_tab)),
                            "copy square table");
    return st;
}

lt_status mesh_table_host(int ndim, double* out) {
    std::call_once(g_mesh_once, [] {
        build_cube_table(g_cube_tab);
        build_square_table(g_square_tab);
    });
    const int n = ndim == 3 ? 256 : 16;
    const uint64_t* tab = ndim == 3 ? g_cube_tab : g_square_tab;
    for (int m = 0; m < n; ++m) out[m] = (double)tab[m] / MESH_SCALE;
    return LT_OK;
}

template <typename L>
static lt_status mesh_typed(lt_ctx* ctx, const L* lab, const Geom& g, uint32_t max_label, uint64_t* vol_acc,
                            uint64_t* area_acc, hipStream_t s) {
    if (g.ndim == 3) {
        dim3 grid((g.nx + 63) / 64, (g.ny + MESH_BY - 1) / MESH_BY, (g.nz + MESH_ZCHUNK - 1) / MESH_ZCHUNK);
        ProfScope p(ctx, s, "mesh_area3d");
        mesh_area3d<L><<<grid, dim3(64, MESH_BY), 0, s>>>(lab, g.nx, g.ny, g.nz, max_label, vol_acc, area_acc,
                                                           ctx->d_err);
    } else {
        dim3 grid((g.nx + 1 + 255) / 256, (g.ny + 1 + MESH_ZCHUNK - 1) / MESH_ZCHUNK);
        ProfScope p(ctx, s, "mesh_len2d");
        mesh_len2d<L><<<grid, 256, 0, s>>>(lab, g.nx, g.ny, max_label, vol_acc, area_acc, ctx->d_err);
    }
    return hip_check(hipGetLastError(), "mesh kernel launch");
}

lt_status launch_mesh(lt_ctx* ctx, const void* labels, lt_dtype dt, const Geom& g, uint32_t max_label,
                      uint64_t* volume, float* area, float* sphericity, void* scratch, hipStream_t s) {
    if (!ctx->mesh_ready) {
        lt_status st = mesh_tables(ctx);
        if (st) return st;
        ctx->mesh_ready = true;
    }
    const uint32_t nlab = max_label + 1;
    uint64_t* vol_acc = (uint64_t*)scratch;
    uint64_t* area_acc = (uint64_t*)((char*)scratch + (((size_t)nlab * sizeof(uint64_t) + 255) & ~size_t(255)));
    {
        ProfScope p(ctx, s, "mesh_zero");
        mesh_zero<<<(nlab + 255) / 256, 256, 0, s>>>(vol_acc, area_acc, nlab);
    }
    lt_status st = hip_check(hipGetLastError(), "mesh_zero launch");
    if (st) return st;
    if (g.n > 0) {
        switch (dt) {
            case LT_U16: st = mesh_typed(ctx, (const uint16_t*)labels, g, max_label, vol_acc, area_acc, s); break;
            case LT_I32: st = mesh_typed(ctx, (const int32_t*)labels, g, max_label, vol_acc, area_acc, s); break;
            case LT_U32: st = mesh_typed(ctx, (const uint32_t*)labels, g, max_label, vol_acc, area_acc, s); break;
        }
        if (st) return st;
    }
    {
        ProfScope p(ctx, s, "mesh_finish");
        mesh_finish<<<(nlab + 255) / 256, 256, 0, s>>>(vol_acc, area_acc, nlab, g.ndim, volume, area, sphericity);
    }
    return hip_check(hipGetLastError(), "mesh_finish launch");
}

}  // namespace lt
