// Test driver: runs the library's tile-edge choice and prints the result as JSON.
// usage: layout_driver T_req w h delta_min precision max_lds unit_points
#include <cstdio>
#include <cstdlib>
#include <string>

#include "../paper_1711_07877_amd/csrc/host/layout.h"

int main(int argc, char** argv) {
  if (argc != 8) return 2;
  int T = 0;
  std::string msg;
  const int w = atoi(argv[2]), prec = atoi(argv[5]), up = atoi(argv[7]);
  int rc = sbd::choose_tile(atoi(argv[1]), w, atof(argv[3]), atof(argv[4]), prec, (size_t)atoll(argv[6]), up, &T, msg);
  if (rc) {
    printf("{\"rc\": %d, \"msg\": \"%s\"}\n", rc, msg.c_str());
    return 0;
  }
  printf("{\"rc\": 0, \"T\": %d, \"spread_lds\": %zu, \"interp_lds\": %zu}\n", T, sbd::spread_lds_bytes(T, w, prec),
         sbd::interp_lds_bytes(T, w, prec, up));
  return 0;
}
