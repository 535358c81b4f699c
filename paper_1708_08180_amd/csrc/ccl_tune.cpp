// Tile-configuration choice for the single-image path.
#include "ccl_internal.h"

namespace ccl {

void default_config(int H, int W, int conn, int *th, int *nw) {
    (void)H;
    (void)W;
    (void)conn;
    *th = 32;
    *nw = 2;
}

}  // namespace ccl
