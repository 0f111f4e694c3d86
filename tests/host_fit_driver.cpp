// Test driver: runs the library's host SBD fit and prints its result as JSON.
// usage: host_fit_driver kind a eps kappa
#include <cstdio>
#include <cstdlib>
#include <string>

#include "../paper_1711_07877_amd/csrc/host/sbd_fit.h"

int main(int argc, char** argv) {
  if (argc != 5) return 2;
  sbd::FitResult fit;
  std::string msg;
  int rc = sbd::sbd_fit(atoi(argv[1]), atof(argv[2]), atof(argv[3]), atof(argv[4]), 0, 4, fit, msg);
  if (rc) {
    printf("{\"rc\": %d}\n", rc);
    return 0;
  }
  printf("{\"rc\": 0, \"P\": %d, \"err\": %.17g, \"lam\": %.17g, \"kappa_p\": %.17g, \"robin_H\": %.17g, \"a\": %.17g,",
         fit.P, fit.err, fit.lam, fit.kappa_p, fit.robin_H, fit.a);
  printf(" \"radii\": [");
  for (int p = 0; p < fit.P; ++p) printf("%s%.17g", p ? ", " : "", fit.radii[p]);
  printf("], \"coef\": [");
  for (int p = 0; p < fit.P; ++p) printf("%s%.17g", p ? ", " : "", fit.coef[p]);
  printf("], \"M\": [");
  for (int p = 0; p < fit.P; ++p) printf("%s%lld", p ? ", " : "", (long long)fit.M[p]);
  printf("]}\n");
  return 0;
}
