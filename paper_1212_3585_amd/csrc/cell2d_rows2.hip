// Fused 2D cell kernel, tile height 2.
#define CELL_ROWS 2
#include "cell2d_rows.hpp"
