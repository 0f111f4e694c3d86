// Tile edge of the plan's grid layout (host only, no device code).
#pragma once
#include <cstddef>
#include <string>

namespace sbd {

// Choose the tile edge T (grid cells) from the requested edge T_req (0 selects 32):
//  * T is a power of two in [8, 256];
//  * T >= 2 PL with PL = (w + 1) / 2, so a grid cell is covered by at most 2 x 2 padded tiles;
//  * T h >= delta_min, so the fine near-field cells (at most one per tile edge, the 3 x 3
//    cell search of the neighbour kernels) are at least delta_min wide and no close pair
//    is missed;
//  * one padded tile (T + 2 PL)^2 fits the LDS of a workgroup for the spread (32-bit or
//    64-bit accumulators, complex capacity) and for the interpolation (grid window plus
//    unit_points rows of 20 bytes).
// Returns 0 and sets *T_out; -1 for a bad request, -6 when no tile meets every rule
// (msg says which).
int choose_tile(int T_req, int w, double h, double delta_min, int precision, size_t max_lds, int unit_points,
                int* T_out, std::string& msg);

// LDS bytes of the spread and interpolation kernels for a tile edge T.
size_t spread_lds_bytes(int T, int w, int precision);
size_t interp_lds_bytes(int T, int w, int precision, int unit_points);

}  // namespace sbd
