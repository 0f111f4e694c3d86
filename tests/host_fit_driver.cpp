// Test driver: runs the library's host SBD fit and prints its result as JSON.
// usage: host_fit_driver kind a eps kappa
//        host_fit_driver general delta_max a eps c_log enforce [m w a b]...
#include <cstdio>
#include <cstdlib>
#include <string>

#include "../paper_1711_07877_amd/csrc/host/sbd_fit.h"

int main(int argc, char** argv) {
  sbd::FitResult fit;
  std::string msg;
  int rc;
  if (argc >= 7 && std::string(argv[1]) == "general") {
    sbd::GeneralKernel g;
    g.c_log = atof(argv[5]);
    g.enforce = atoi(argv[6]);
    if ((argc - 7) % 4) return 2;
    for (int i = 7; i < argc; i += 4)
      g.terms.push_back(sbd::TrigTerm{atoi(argv[i]), atof(argv[i + 1]), atof(argv[i + 2]), atof(argv[i + 3])});
    rc = sbd::sbd_fit_general(g, atof(argv[2]), atof(argv[3]), atof(argv[4]), 4, fit, msg);
  } else {
    if (argc != 5) return 2;
    rc = sbd::sbd_fit(atoi(argv[1]), atof(argv[2]), atof(argv[3]), atof(argv[4]), 0, 4, fit, msg);
  }
  if (rc) {
    printf("{\"rc\": %d}\n", rc);
    return 0;
  }
  printf("{\"rc\": 0, \"P\": %d, \"n_enforced\": %d, \"constant\": %.17g, \"err\": %.17g, \"lam\": %.17g, \"kappa_p\": %.17g, \"robin_H\": %.17g, \"a\": %.17g,",
         fit.P, fit.n_enforced, fit.constant, fit.err, fit.lam, fit.kappa_p, fit.robin_H, fit.a);
  printf(" \"radii\": [");
  for (int p = 0; p < fit.P; ++p) printf("%s%.17g", p ? ", " : "", fit.radii[p]);
  printf("], \"coef\": [");
  for (int p = 0; p < fit.P; ++p) printf("%s%.17g", p ? ", " : "", fit.coef[p]);
  printf("], \"M\": [");
  for (int p = 0; p < fit.P; ++p) printf("%s%lld", p ? ", " : "", (long long)fit.M[p]);
  printf("]}\n");
  return 0;
}
