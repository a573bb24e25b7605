// Builds the host model tables (velocity set, moment matrix, inverse,
// symmetry blocks) for regular and singular parameter sets; built with
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitizers.py.
#include <cstdio>
#include <cstring>
#include <string>
#include "dbm.h"
#include "dbm_internal.hpp"
namespace dbm { int build_species(const dbm_species &in, const dbm_config &cfg, SpeciesDev &sp, std::string &err); }
int main() {
  dbm_config c; std::memset(&c, 0, sizeof c);
  c.nx = 8; c.ny = 8; c.dx = c.dy = 1e-3; c.dt = 1e-5; c.nspecies = 1;
  double vs[][8] = {{1.5,0.8,2.2,2.6,2.5,0,0,0}, {1,1,1,1,1,1,1,1}, {1.5,0.8,2.2,0.8,2.5,0,0,0}, {0,0,0,0,0,0,0,0}};
  for (auto &v : vs) for (double m : {1.0, 2.0, 32.0}) {
    dbm_species s; std::memset(&s, 0, sizeof s); s.m = m; s.I = 3; s.tau = 2e-5;
    for (int g = 0; g < 4; ++g) { s.v[g] = v[g]; s.eta[g] = v[4 + g]; }
    dbm::SpeciesDev sp; std::string err;
    int rc = dbm::build_species(s, c, sp, err);
    std::printf("m=%g v0=%g rc=%d %s\n", m, v[0], rc, err.c_str());
  }
  return 0;
}
