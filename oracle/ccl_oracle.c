/*
 * CPU oracle for connected-components labeling (test infrastructure only).
 *
 * This file is the checker that the GPU library is compared against.  Only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no code, header or helper with the GPU library.
 *
 * What it computes (the plain definition the paper's method reaches):
 *   The paper (Introduction) defines CCL as giving one unique ID to every
 *   connected region of a grid, with all members of a region sharing it.
 *   Its union-find always links a larger index under a smaller one (the
 *   atomicMin direction of the merge operation in Sec. II-A-3; the left and
 *   upper cells carry smaller initial labels, Sec. II-A-2), so each final
 *   root is the smallest raster index of its component.  The oracle writes
 *   that result out directly:
 *
 *     L[y*W + x] = 0                                     if I[y,x] == 0
 *     L[y*W + x] = 1 + min{ y'*W + x' : (y',x') ~ (y,x) } otherwise
 *
 *   where ~ is connectivity through foreground pixels using 4-neighbours
 *   (Manhattan distance 1, the paper's Kernel 1) or 8-neighbours (Chebyshev
 *   distance 1).  Raster indices use the image width W, never the row pitch.
 *
 * How: a raster-order scan; every unvisited foreground pixel p starts a
 * breadth-first flood fill that stamps 1 + p on everything it reaches.
 * Because the scan visits pixels in increasing raster order, the first
 * pixel of a component to be reached is its minimum-index pixel, so no
 * minimum tracking is needed.  Single threaded, O(H*W) time and memory.
 *
 * The equal-value variant follows the kernels' literal test ("same
 * property": a cell joins a neighbour whose image value is equal), so
 * every value class, background included, is labeled; there, a pixel of
 * any value gets 1 + the smallest raster index of its equal-valued
 * component.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL 1
#define ORACLE_ENOMEM 2

static int valid_conn2d(int conn) { return conn == 4 || conn == 8; }

/* Flood fill shared by the binary and the equal-value labelings.
 * mode 0: pixels join iff both are nonzero (binary foreground).
 * mode 1: pixels join iff their values are equal (every class labeled). */
static int flood_2d(const uint8_t *img, int64_t H, int64_t W, int64_t pitch,
                    int conn, int mode, uint32_t *out)
{
    if (!img || !out || H <= 0 || W <= 0 || pitch < W || !valid_conn2d(conn))
        return ORACLE_EINVAL;
    if (H * W > (int64_t)0xFFFFFFFFll)
        return ORACLE_EINVAL;
    const int64_t n = H * W;
    int64_t *queue = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!queue)
        return ORACLE_ENOMEM;
    memset(out, 0, (size_t)n * sizeof(uint32_t));

    /* neighbour offsets: the first four are the 4-neighbourhood */
    static const int dy[8] = {-1, 0, 0, 1, -1, -1, 1, 1};
    static const int dx[8] = {0, -1, 1, 0, -1, 1, -1, 1};
    const int nnb = conn;

    for (int64_t p = 0; p < n; ++p) {
        const int64_t py = p / W, px = p % W;
        const uint8_t v = img[py * pitch + px];
        if (out[p] != 0)
            continue;
        if (mode == 0 && v == 0)
            continue;
        const uint32_t lab = (uint32_t)(p + 1);
        int64_t head = 0, tail = 0;
        out[p] = lab;
        queue[tail++] = p;
        while (head < tail) {
            const int64_t q = queue[head++];
            const int64_t qy = q / W, qx = q % W;
            for (int k = 0; k < nnb; ++k) {
                const int64_t ny = qy + dy[k], nx = qx + dx[k];
                if (ny < 0 || ny >= H || nx < 0 || nx >= W)
                    continue;
                const int64_t r = ny * W + nx;
                if (out[r] != 0)
                    continue;
                const uint8_t w = img[ny * pitch + nx];
                const int joins = (mode == 0) ? (w != 0) : (w == v);
                if (!joins)
                    continue;
                out[r] = lab;
                queue[tail++] = r;
            }
        }
    }
    free(queue);
    return ORACLE_OK;
}

/* Binary labeling: nonzero is foreground, background gets 0. */
int oracle_label_2d(const uint8_t *img, int64_t H, int64_t W, int64_t pitch,
                    int conn, uint32_t *out)
{
    return flood_2d(img, H, W, pitch, conn, 0, out);
}

/* Equal-value labeling of every value class, background included. */
int oracle_label_2d_equal(const uint8_t *img, int64_t H, int64_t W,
                          int64_t pitch, int conn, uint32_t *out)
{
    return flood_2d(img, H, W, pitch, conn, 1, out);
}

/* Per-component statistics of the labeling (the applications' quantities:
 * size and location of each component).  One record per component, in
 * increasing label order:
 *   label = 1 + smallest raster index of the component
 *   area  = number of pixels
 *   x_min, y_min, x_max, y_max = bounding box (inclusive)
 *   sum_x, sum_y = sums of the pixels' column and row indices (centroid =
 *                  sum / area)
 * mode 0 = binary foreground components, mode 1 = equal-value components.
 * Labels are computed by the flood fill above; a second raster pass then
 * visits the components' pixels.  Because a label is the raster index of its
 * component's first pixel, the components appear in increasing label order
 * the first time each is met, which gives every component its record index.
 * Records beyond `capacity` are counted in *n but not written. */
typedef struct oracle_component {
    uint32_t label, area, x_min, y_min, x_max, y_max;
    uint64_t sum_x, sum_y;
} oracle_component;

int oracle_stats_2d(const uint8_t *img, int64_t H, int64_t W, int64_t pitch, int conn,
                    int mode, oracle_component *out, int64_t capacity, int64_t *n)
{
    if (!n || capacity < 0 || (capacity > 0 && !out) || (mode != 0 && mode != 1))
        return ORACLE_EINVAL;
    if (H <= 0 || W <= 0 || H * W > (int64_t)0xFFFFFFFFll)
        return ORACLE_EINVAL;
    const int64_t npx = H * W;
    uint32_t *lab = (uint32_t *)malloc((size_t)npx * sizeof(uint32_t));
    uint32_t *rec = (uint32_t *)malloc((size_t)npx * sizeof(uint32_t));
    if (!lab || !rec) {
        free(lab);
        free(rec);
        return ORACLE_ENOMEM;
    }
    int rc = flood_2d(img, H, W, pitch, conn, mode, lab);
    int64_t count = 0;
    for (int64_t p = 0; rc == ORACLE_OK && p < npx; ++p) {
        const uint32_t L = lab[p];
        if (L == 0)
            continue;
        const uint32_t root = L - 1;
        if (root == (uint32_t)p)
            rec[p] = (uint32_t)count++;  /* first pixel of a new component */
        const uint32_t c = rec[root];
        if ((int64_t)c >= capacity)
            continue;
        const uint32_t x = (uint32_t)(p % W), y = (uint32_t)(p / W);
        oracle_component *s = &out[c];
        if (root == (uint32_t)p) {
            s->label = L;
            s->area = 0;
            s->x_min = s->x_max = x;
            s->y_min = s->y_max = y;
            s->sum_x = s->sum_y = 0;
        }
        s->area += 1;
        if (x < s->x_min) s->x_min = x;
        if (x > s->x_max) s->x_max = x;
        if (y < s->y_min) s->y_min = y;
        if (y > s->y_max) s->y_max = y;
        s->sum_x += x;
        s->sum_y += y;
    }
    free(lab);
    free(rec);
    *n = count;
    return rc;
}

/* 3D labeling of a binary volume (D slices of H rows of W voxels; voxel
 * (z, y, x) at vol[z * pitch_z + y * pitch_y + x], nonzero = foreground).
 * Neighbours: conn 6 = the face neighbours, 18 = faces and edges, 26 =
 * faces, edges and corners.  label = 1 + the smallest raster index
 * z*H*W + y*W + x of the voxel's component, 0 for background; the same
 * raster-order flood fill as in 2D. */
int oracle_label_3d(const uint8_t *vol, int64_t D, int64_t H, int64_t W, int64_t pitch_y,
                    int64_t pitch_z, int conn, uint32_t *out)
{
    if (!vol || !out || D <= 0 || H <= 0 || W <= 0 || pitch_y < W || pitch_z < H * pitch_y)
        return ORACLE_EINVAL;
    if (conn != 6 && conn != 18 && conn != 26)
        return ORACLE_EINVAL;
    const int64_t n = D * H * W;
    if (n > (int64_t)0xFFFFFFFFll)
        return ORACLE_EINVAL;
    int dz[26], dy[26], dx[26], nnb = 0;
    for (int a = -1; a <= 1; ++a)
        for (int b = -1; b <= 1; ++b)
            for (int c = -1; c <= 1; ++c) {
                const int steps = (a != 0) + (b != 0) + (c != 0);
                if (steps == 0 || (conn == 6 && steps > 1) || (conn == 18 && steps > 2))
                    continue;
                dz[nnb] = a;
                dy[nnb] = b;
                dx[nnb] = c;
                ++nnb;
            }
    int64_t *queue = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!queue)
        return ORACLE_ENOMEM;
    memset(out, 0, (size_t)n * sizeof(uint32_t));
    const int64_t HW = H * W;
    for (int64_t p = 0; p < n; ++p) {
        const int64_t pz = p / HW, py = (p / W) % H, px = p % W;
        if (out[p] != 0 || vol[pz * pitch_z + py * pitch_y + px] == 0)
            continue;
        const uint32_t lab = (uint32_t)p + 1u;
        int64_t head = 0, tail = 0;
        out[p] = lab;
        queue[tail++] = p;
        while (head < tail) {
            const int64_t q = queue[head++];
            const int64_t qz = q / HW, qy = (q / W) % H, qx = q % W;
            for (int k = 0; k < nnb; ++k) {
                const int64_t nz = qz + dz[k], ny = qy + dy[k], nx = qx + dx[k];
                if (nz < 0 || nz >= D || ny < 0 || ny >= H || nx < 0 || nx >= W)
                    continue;
                const int64_t r = nz * HW + ny * W + nx;
                if (out[r] != 0 || vol[nz * pitch_z + ny * pitch_y + nx] == 0)
                    continue;
                out[r] = lab;
                queue[tail++] = r;
            }
        }
    }
    free(queue);
    return ORACLE_OK;
}
