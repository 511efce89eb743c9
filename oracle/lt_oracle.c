/*
 * CPU oracle for local-thickness sphericity and roundness -- TEST INFRASTRUCTURE.
 *
 * Plain, slow and written to be checked by eye against the definitions.  It shares
 * no code, header, table or helper with the GPU library; only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg load it.  The product path never
 * calls it.
 *
 * Conventions (Method section: local thickness is the radius of the largest
 * inscribed circle/sphere containing the point):
 *   - lattice Z^d (d = 2 or 3), unit spacing, C order [z][y][x] (2D: [y][x]);
 *   - label 0 is background; every position outside the image is background;
 *   - distances are per label: for a voxel of label l, every voxel of another
 *     label is background (all objects are measured at once, each on its own);
 *   - distances are between voxel centres, balls are centred on lattice points and
 *     open: the ball of x holds every q with |q - x|^2 < D(x).
 *
 * Entry points (all arrays int64, C order, shape = {nz, ny, nx} or {ny, nx}):
 *   oracle_edt      squared per-label Euclidean distance transform D
 *   oracle_lt       squared local thickness LT (every object voxel scatters its ball)
 * Both take an optional `w` (NULL: unit spacing): ndim positive integer weights,
 * the squared voxel spacings along (z, y, x) or (y, x) in a common length unit.
 * Every squared distance is then the weighted sum w_z dz^2 + w_y dy^2 + w_x dx^2
 * (anisotropic spacing; the paper's volumes use unit spacing, which is w = 1).
 * Each returns 0 on success, -1 on a bad argument or allocation failure.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t dz, dy, dx;
    int64_t n2;
} lt_offset;

static int by_norm(const void* pa, const void* pb) {
    const lt_offset* a = (const lt_offset*)pa;
    const lt_offset* b = (const lt_offset*)pb;
    if (a->n2 != b->n2) return a->n2 < b->n2 ? -1 : 1;
    if (a->dz != b->dz) return a->dz < b->dz ? -1 : 1;
    if (a->dy != b->dy) return a->dy < b->dy ? -1 : 1;
    if (a->dx != b->dx) return a->dx < b->dx ? -1 : 1;
    return 0;
}

/* Largest k >= 0 with w k^2 <= b. */
static int64_t axis_reach(int64_t b, int64_t w) {
    int64_t k = 0;
    while (w * (k + 1) * (k + 1) <= b) ++k;
    return k;
}

/* Every lattice offset o with |o|_w^2 = wz dz^2 + wy dy^2 + wx dx^2 <= b (dz = 0 in
 * 2D), sorted by |o|_w^2.  wt = {wz, wy, wx}. */
static lt_offset* sorted_offsets(int ndim, int64_t b, const int64_t wt[3], int64_t* count) {
    int64_t rz = (ndim == 3) ? axis_reach(b, wt[0]) : 0;
    int64_t ry = axis_reach(b, wt[1]), rx = axis_reach(b, wt[2]);
    int64_t cap = (2 * rz + 1) * (2 * ry + 1) * (2 * rx + 1);
    lt_offset* o = (lt_offset*)malloc((size_t)cap * sizeof(lt_offset));
    if (!o) return NULL;
    int64_t n = 0;
    for (int64_t dz = -rz; dz <= rz; ++dz)
        for (int64_t dy = -ry; dy <= ry; ++dy)
            for (int64_t dx = -rx; dx <= rx; ++dx) {
                int64_t n2 = wt[0] * dz * dz + wt[1] * dy * dy + wt[2] * dx * dx;
                if (n2 > b) continue;
                o[n].dz = (int32_t)dz;
                o[n].dy = (int32_t)dy;
                o[n].dx = (int32_t)dx;
                o[n].n2 = n2;
                ++n;
            }
    qsort(o, (size_t)n, sizeof(lt_offset), by_norm);
    *count = n;
    return o;
}

static int unpack_shape(int ndim, const int64_t* shape, int64_t* nz, int64_t* ny, int64_t* nx) {
    if (ndim == 3) {
        *nz = shape[0]; *ny = shape[1]; *nx = shape[2];
    } else if (ndim == 2) {
        *nz = 1; *ny = shape[0]; *nx = shape[1];
    } else {
        return -1;
    }
    if (*nz < 0 || *ny < 0 || *nx < 0) return -1;
    return 0;
}

/* Weights {wz, wy, wx} from the optional argument (unit spacing when NULL);
 * -1 if one is not positive. */
static int unpack_weights(int ndim, const int64_t* w, int64_t wt[3]) {
    wt[0] = wt[1] = wt[2] = 1;
    if (!w) return 0;
    for (int i = 0; i < ndim; ++i) {
        if (w[i] < 1) return -1;
        wt[3 - ndim + i] = w[i];
    }
    return 0;
}

/* A squared distance that no D in the image can exceed: along each axis i the
 * image border is at most (n_i + 1) / 2 voxels away, so D(p) <= w_i ((n_i + 1) / 2)^2
 * for every i. */
static int64_t distance_bound(int ndim, int64_t nz, int64_t ny, int64_t nx, const int64_t wt[3]) {
    int64_t hz = (nz + 1) / 2 + 1, hy = (ny + 1) / 2 + 1, hx = (nx + 1) / 2 + 1;
    int64_t b = wt[1] * hy * hy;
    if (wt[2] * hx * hx < b) b = wt[2] * hx * hx;
    if (ndim == 3 && wt[0] * hz * hz < b) b = wt[0] * hz * hz;
    return b;
}

/* D(p) = 0 where L(p) = 0; otherwise the smallest |p - q|_w^2 over lattice points q
 * that lie outside the image or carry a label other than L(p).  The offsets are
 * visited in increasing |o|_w^2, so the first qualifying q gives the minimum. */
int oracle_edt(const int64_t* lab, int ndim, const int64_t* shape, const int64_t* w, int64_t* D) {
    int64_t nz, ny, nx, wt[3];
    if (!lab || !shape || !D || unpack_shape(ndim, shape, &nz, &ny, &nx) || unpack_weights(ndim, w, wt))
        return -1;
    int64_t n = nz * ny * nx;
    if (n == 0) return 0;
    int64_t cnt = 0;
    lt_offset* off = sorted_offsets(ndim, distance_bound(ndim, nz, ny, nx, wt), wt, &cnt);
    if (!off) return -1;
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                int64_t i = (z * ny + y) * nx + x;
                int64_t l = lab[i];
                if (l == 0) { D[i] = 0; continue; }
                int64_t best = -1;
                for (int64_t k = 1; k < cnt; ++k) {          /* k = 0 is o = 0 */
                    int64_t qz = z + off[k].dz, qy = y + off[k].dy, qx = x + off[k].dx;
                    int outside = qz < 0 || qz >= nz || qy < 0 || qy >= ny || qx < 0 || qx >= nx;
                    if (outside || lab[(qz * ny + qy) * nx + qx] != l) { best = off[k].n2; break; }
                }
                D[i] = best;                   /* the bound guarantees best >= 1 */
            }
    free(off);
    return 0;
}

/* LT(p) = max{ D(x) : D(x) > 0 and |p - x|_w^2 < D(x) } on object voxels, 0 on
 * background: every voxel x with D(x) > 0 writes D(x) into each lattice point of
 * its open ball, keeping the larger value.  No centre is skipped.  Labels are not
 * needed: a ball holds only voxels of its centre's label, since the nearest voxel
 * of any other label (or outside the image) is exactly D(x) away.
 * If work != NULL it receives the number of ball points visited. */
int oracle_lt(const int64_t* D, int ndim, const int64_t* shape, const int64_t* w, int64_t* LT, int64_t* work) {
    int64_t nz, ny, nx, wt[3];
    if (!D || !shape || !LT || unpack_shape(ndim, shape, &nz, &ny, &nx) || unpack_weights(ndim, w, wt))
        return -1;
    int64_t n = nz * ny * nx;
    if (work) *work = 0;
    if (n == 0) return 0;
    memset(LT, 0, (size_t)n * sizeof(int64_t));
    int64_t cnt = 0;
    lt_offset* off = sorted_offsets(ndim, distance_bound(ndim, nz, ny, nx, wt), wt, &cnt);
    if (!off) return -1;
    int64_t visited = 0;
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                int64_t d = D[(z * ny + y) * nx + x];
                if (d <= 0) continue;
                for (int64_t k = 0; k < cnt && off[k].n2 < d; ++k) {
                    int64_t pz = z + off[k].dz, py = y + off[k].dy, px = x + off[k].dx;
                    ++visited;
                    if (pz < 0 || pz >= nz || py < 0 || py >= ny || px < 0 || px >= nx) continue;
                    int64_t j = (pz * ny + py) * nx + px;
                    if (LT[j] < d) LT[j] = d;
                }
            }
    free(off);
    if (work) *work = visited;
    return 0;
}
