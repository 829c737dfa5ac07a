// Host-side check of the projector-geometry builder (build_tables_host),
// built with the address and undefined-behaviour sanitizers on the host
// code (test infrastructure; no device call is made). For periodic, Bloch,
// self-overlapping, ragged and zero-boundary geometries it checks the
// tables' invariants: the atom-major ranges partition the entries, every
// entry's grid index lies on the grid, the point-major counts add up to the
// entry count, the covered points are the points with entries, in
// increasing order; and that out-of-range descriptors are rejected.
#include <cstdio>
#include <string>
#include <vector>

#include "internal.h"

// the library's error reporting lives in its ABI layer, not built here
namespace gfd {
int fail(int code, const std::string &msg) {
  std::fprintf(stderr, "rejected (%d): %s\n", code, msg.c_str());
  return code;
}
int hip_fail(hipError_t e, const char *what) {
  std::fprintf(stderr, "HIP error %d in %s\n", static_cast<int>(e), what);
  return GPAW_EHIP;
}
}  // namespace gfd

namespace {

int check_case(const char *name, int n0, int n1, int n2, double h, double k0, int natoms,
               double rc, int boundary, unsigned seed) {
  std::vector<gpaw_channel> ch = {{0, rc / 3, rc}, {0, rc / 5, rc}, {1, rc / 3, rc},
                                  {1, rc / 5, rc}, {2, rc / 3, rc}};
  std::vector<double> pos(3 * natoms);
  unsigned x = seed;
  const double L[3] = {n0 * h, n1 * h, n2 * h};
  for (int a = 0; a < 3 * natoms; ++a) {
    x = x * 1664525u + 1013904223u;
    pos[a] = (x >> 8) * (1.0 / 16777216.0) * L[a % 3];
  }
  gpaw_sys_desc d{};
  d.n[0] = n0;
  d.n[1] = n1;
  d.n[2] = n2;
  d.h[0] = d.h[1] = d.h[2] = h;
  d.k[0] = k0;
  d.dtype = k0 != 0.0 ? GPAW_C128 : GPAW_F64;
  d.natoms = natoms;
  d.pos = pos.data();
  d.nchan = static_cast<int32_t>(ch.size());
  d.chan = ch.data();
  d.max_bands = 1;
  d.boundary = boundary;
  gpaw_sys s;
  s.n[0] = n0;
  s.n[1] = n1;
  s.n[2] = n2;
  s.ng = static_cast<int64_t>(n0) * n1 * n2;
  s.natoms = natoms;
  s.zbc = boundary;
  gfd::HostTables ht;
  const int rc_build = gfd::build_tables_host(&d, &s, ht);
  if (rc_build != GPAW_OK) {
    std::printf("%s: build failed (%d)\n", name, rc_build);
    return 1;
  }
  const int64_t nent = s.tab.nent;
  int bad = 0;
  if (static_cast<int64_t>(ht.a_start.size()) != natoms + 1 || ht.a_start[0] != 0 ||
      ht.a_start[natoms] != nent)
    ++bad;
  for (int a = 0; a < natoms; ++a)
    if (ht.a_start[a] > ht.a_start[a + 1]) ++bad;
  for (int64_t e = 0; e < nent; ++e)
    if (ht.e_g[e] < 0 || ht.e_g[e] >= s.ng) ++bad;
  int64_t total = 0, covered = 0, prev = -1;
  for (int64_t g = 0; g < s.ng; ++g) {
    const int cnt = static_cast<int>(static_cast<unsigned>(ht.pinfo[g].w) >> 24);
    total += cnt;
    if (cnt > 0) {
      if (covered >= static_cast<int64_t>(ht.cov.size()) || ht.cov[covered] != g) ++bad;
      if (g <= prev) ++bad;
      prev = g;
      ++covered;
      const int first = ht.pinfo[g].w & 0xFFFFFF;
      for (int j = 0; j < cnt; ++j)
        if ((ht.pm_code[first + j] >> 12) >= natoms) ++bad;
    }
  }
  if (total != nent || covered != s.tab.ncov || static_cast<int64_t>(ht.cov.size()) != covered)
    ++bad;
  std::printf("%s: %lld entries, %lld covered points, %d violations\n", name,
              static_cast<long long>(nent), static_cast<long long>(covered), bad);
  return bad ? 1 : 0;
}

int check_rejected() {
  std::vector<gpaw_channel> ch(9, gpaw_channel{0, 0.5, 2.0});
  double pos[3] = {0.0, 0.0, 0.0};
  gpaw_sys_desc d{};
  d.n[0] = d.n[1] = d.n[2] = 8;
  d.h[0] = d.h[1] = d.h[2] = 0.2;
  d.natoms = 1;
  d.pos = pos;
  d.nchan = 9;  // more channels than the layout holds
  d.chan = ch.data();
  d.max_bands = 1;
  gpaw_sys s;
  s.ng = 512;
  gfd::HostTables ht;
  const int rc = gfd::build_tables_host(&d, &s, ht);
  std::printf("too many channels: status %d\n", rc);
  return rc == GPAW_OK ? 1 : 0;
}

}  // namespace

int main() {
  int bad = 0;
  bad += check_case("periodic 24^3", 24, 24, 24, 0.2, 0.0, 4, 2.0, 0, 1);
  bad += check_case("Bloch ragged 13x17x11", 13, 17, 11, 0.21, 0.37, 3, 1.6, 0, 2);
  bad += check_case("self-overlapping 16^3", 16, 16, 16, 0.2, 0.25, 3, 2.0, 0, 3);
  bad += check_case("zero boundary 20x18x24", 20, 18, 24, 0.2, 0.0, 5, 2.0, 1, 4);
  bad += check_case("tiny 3x4x5", 3, 4, 5, 0.3, 0.0, 2, 2.0, 0, 5);
  bad += check_case("no atoms", 9, 10, 8, 0.2, 0.0, 0, 2.0, 0, 6);
  bad += check_rejected();
  std::printf(bad ? "FAILED\n" : "all checks passed\n");
  return bad ? 1 : 0;
}
