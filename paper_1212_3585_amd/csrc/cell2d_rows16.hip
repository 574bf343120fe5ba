// Fused 2D cell kernel, tile height 16.
#define CELL_ROWS 16
#include "cell2d_rows.hpp"
