// Per-label squared Euclidean distance transform, three separable passes.
//
// For an object voxel p of label l the nearest non-l lattice point (another label,
// background, or any position outside the image) is sought.  Along each line the
// voxels of l form runs; the run's end points act as zero-cost sites and a voxel of
// the same label in another run is never nearer than the non-l voxel between the
// runs, so every run is an independent 1D problem:
//   pass x:  g(p)  = distance along x to the first non-l position (1D transform);
//   pass y:  d2(p) = min over j in the y-run of p of (y_p - y_j)^2 + g(j)^2, and the
//            squared distance to the run's end sites;
//   pass z:  d(p)  = the same along z over d2 (3D only).
// Each pass searches outward from p and stops as soon as k^2 reaches the best value
// found, so the search is exact and costs O(sqrt(D)) loads per voxel.  Lanes of a
// wave hold consecutive x, so every load of a pass is a coalesced row access.
#include "lt_internal.h"

namespace lt {

template <typename L>
__global__ void __launch_bounds__(256)
edt_pass_x(const L* __restrict__ lab, uint16_t* __restrict__ g, int nx, int ny, uint32_t* err) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nx) return;
    const size_t row = (size_t)blockIdx.z * ny + blockIdx.y;
    const L* r = lab + row * nx;
    const L l = r[x];
    int out = 0;
    if (l != 0) {
        if (label_negative(l)) atomicOr(err, ERR_LABEL);
        int k = 1;
        for (;; ++k) {
            const int a = x - k, b = x + k;
            if (a < 0 || b >= nx) break;
            if (r[a] != l || r[b] != l) break;
        }
        out = k;
    }
    g[row * nx + x] = (uint16_t)out;
}

// One line pass along y (AXIS = 1, input g, squared here) or z (AXIS = 2, input d2).
template <typename L, int AXIS, typename F>
__global__ void __launch_bounds__(256)
edt_pass_line(const L* __restrict__ lab, const F* __restrict__ f, int32_t* __restrict__ out,
              int nx, int ny, int nz) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nx) return;
    const int y = blockIdx.y, z = blockIdx.z;
    const size_t i = ((size_t)z * ny + y) * nx + x;
    const L l = lab[i];
    if (l == 0) {
        out[i] = 0;
        return;
    }
    const ptrdiff_t stride = AXIS == 1 ? (ptrdiff_t)nx : (ptrdiff_t)nx * ny;
    const int pos = AXIS == 1 ? y : z;
    const int n = AXIS == 1 ? ny : nz;
    const int f0 = (int)f[i];
    int best = AXIS == 1 ? f0 * f0 : f0;
    bool lo = true, hi = true;
    for (int k = 1; k * k < best && (lo || hi); ++k) {
        const int kk = k * k;
        if (lo) {
            if (pos - k < 0 || lab[i - k * stride] != l) {
                best = min(best, kk);
                lo = false;
            } else {
                const int v = (int)f[i - k * stride];
                best = min(best, kk + (AXIS == 1 ? v * v : v));
            }
        }
        if (hi) {
            if (pos + k >= n || lab[i + k * stride] != l) {
                best = min(best, kk);
                hi = false;
            } else {
                const int v = (int)f[i + k * stride];
                best = min(best, kk + (AXIS == 1 ? v * v : v));
            }
        }
    }
    out[i] = best;
}

template <typename L>
static lt_status edt_typed(lt_ctx* ctx, const L* lab, const Geom& g, int32_t* dist, hipStream_t s) {
    // scratch: g (uint16) then d2 (int32, 3D only)
    const size_t gbytes = (g.n * sizeof(uint16_t) + 255) & ~size_t(255);
    const size_t need = gbytes + (g.ndim == 3 ? g.n * sizeof(int32_t) : 0);
    lt_status st = ensure_scratch(ctx, need);
    if (st) return st;
    uint16_t* gx = (uint16_t*)ctx->scratch.ptr;
    int32_t* d2 = (int32_t*)((char*)ctx->scratch.ptr + gbytes);
    const dim3 block(256);
    const dim3 grid((g.nx + 255) / 256, g.ny, g.nz);
    { ProfScope _p(ctx, s, "edt_pass_x");
    edt_pass_x<L><<<grid, block, 0, s>>>(lab, gx, g.nx, g.ny, ctx->d_err);
    }
    if (g.ndim == 2) {
        { ProfScope _p(ctx, s, "edt_pass_y");
        edt_pass_line<L, 1, uint16_t><<<grid, block, 0, s>>>(lab, gx, dist, g.nx, g.ny, g.nz);
        }
    } else {
        { ProfScope _p(ctx, s, "edt_pass_y");
        edt_pass_line<L, 1, uint16_t><<<grid, block, 0, s>>>(lab, gx, d2, g.nx, g.ny, g.nz);
        }
        { ProfScope _p(ctx, s, "edt_pass_z");
        edt_pass_line<L, 2, int32_t><<<grid, block, 0, s>>>(lab, d2, dist, g.nx, g.ny, g.nz);
        }
    }
    return hip_check(hipGetLastError(), "edt launch");
}

lt_status launch_edt(lt_ctx* ctx, const void* labels, lt_dtype dt, const Geom& g, int32_t* dist_sq,
                     hipStream_t s) {
    switch (dt) {
        case LT_U16: return edt_typed(ctx, (const uint16_t*)labels, g, dist_sq, s);
        case LT_I32: return edt_typed(ctx, (const int32_t*)labels, g, dist_sq, s);
        case LT_U32: return edt_typed(ctx, (const uint32_t*)labels, g, dist_sq, s);
    }
    return set_error(LT_E_DTYPE, "unknown dtype");
}

}  // namespace lt
