#include "layout.h"

#include <algorithm>

namespace sbd {

size_t spread_lds_bytes(int T, int w, int precision) {
  const size_t SG = (size_t)T + 2 * (size_t)((w + 1) / 2);
  return SG * SG * (precision ? 8 : 4) * 2;  // complex f is accepted by every plan
}

size_t interp_lds_bytes(int T, int w, int precision, int unit_points) {
  const size_t SG = (size_t)T + 2 * (size_t)((w + 1) / 2);
  return SG * SG * (precision ? 8 : 4) * 2 + (size_t)unit_points * 20 + 16;
}

int choose_tile(int T_req, int w, double h, double delta_min, int precision, size_t max_lds, int unit_points,
                int* T_out, std::string& msg) {
  int T = T_req > 0 ? T_req : 32;
  if (T < 8 || T > 256 || (T & (T - 1))) {
    msg = "tile must be a power of two in [8, 256]";
    return -1;
  }
  if (!(h > 0) || !(delta_min > 0) || w < 1) {
    msg = "layout needs h > 0, delta_min > 0, w >= 1";
    return -1;
  }
  const int PL = (w + 1) / 2;
  while (T < 2 * PL && T < 256) T *= 2;
  while ((double)T * h < delta_min * (1.0 + 1e-9) && T < 256) T *= 2;
  if (T < 2 * PL || (double)T * h < delta_min * (1.0 + 1e-9)) {
    msg = "delta_min spans more than 256 grid cells (tile edge limit)";
    return -6;
  }
  if (std::max(spread_lds_bytes(T, w, precision), interp_lds_bytes(T, w, precision, unit_points)) > max_lds) {
    msg = "tile too large for the LDS of one workgroup (choose a smaller tile)";
    return -6;
  }
  *T_out = T;
  return 0;
}

}  // namespace sbd
