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
