// Fused 2D cell kernel, tile height 8.
#define CELL_ROWS 8
#include "cell2d_rows.hpp"
