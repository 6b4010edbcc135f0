// Host check of the pass kernels' workgroup-to-work maps (block_maps.hpp) over
// every shape the library accepts: n1, n2 <= 32, circulant lengths M3 = 2^k <=
// 4096, both precisions, every pencil count the launchers and the tuner use.
// Each map must be a bijection onto the work items of its launch, and every
// write a kernel derives from its item must land inside the buffer it writes.
#include <cstdio>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "../../include/vie.h"
#include "block_maps.hpp"
#include "vie_internal.hpp"

namespace {

using vie::PencilBlock;

struct Checker {
  std::string err;
  long checked = 0;
  bool fail(const std::string& m) {
    if (err.empty()) err = m;
    return false;
  }
};

// map: a permutation of [0, nblocks) whose images, decoded by pencil_block, cover
// every pencil (c, i2, i1) exactly once, inside the grid
bool check_pencil_map(Checker& ck, int n1, int n2, int P, const std::function<int(int, int)>& map,
                      const char* name) {
  const int nb = vie::pencil_blocks(n1, n2, P);
  std::vector<char> seen(nb, 0), cov(3L * n1 * n2, 0);
  char where[160];
  std::snprintf(where, sizeof where, "%s n1=%d n2=%d P=%d", name, n1, n2, P);
  for (int b = 0; b < nb; ++b) {
    const int m = map(b, nb);
    if (m < 0 || m >= nb) return ck.fail(std::string(where) + ": image out of range");
    if (seen[m]++) return ck.fail(std::string(where) + ": not injective");
    const PencilBlock pb = vie::pencil_block(m, n1, n2, P);
    if (pb.c < 0 || pb.c >= 3 || pb.i2 < 0 || pb.i2 >= n2 || pb.i1_0 < 0 || pb.np < 1 || pb.np > P ||
        pb.i1_0 + pb.np > n1)
      return ck.fail(std::string(where) + ": pencil block outside the grid");
    for (int p = 0; p < pb.np; ++p) {
      const long id = ((long)pb.c * n2 + pb.i2) * n1 + pb.i1_0 + p;
      if (cov[id]++) return ck.fail(std::string(where) + ": pencil covered twice");
    }
  }
  for (char c : cov)
    if (c != 1) return ck.fail(std::string(where) + ": pencil not covered");
  ++ck.checked;
  return true;
}

// writes of a pencil block, as the z passes compute them: the kz-plane-major
// intermediate at (c n2 + i2) n1 + i1 + kz 3 n1 n2, kz < M3, and the vector at
// c N + (i1 n2 + i2) n3 + n, n < n3
bool check_pencil_writes(Checker& ck, int n1, int n2, int n3, int M3, int P) {
  const long plane = 3L * n1 * n2, N = (long)n1 * n2 * n3;
  const int nb = vie::pencil_blocks(n1, n2, P);
  for (int b = 0; b < nb; ++b) {
    const PencilBlock pb = vie::pencil_block(b, n1, n2, P);
    const long u_last = (long)(M3 - 1) * plane + ((long)pb.c * n2 + pb.i2) * n1 + pb.i1_0 + pb.np - 1;
    const long y_last = (long)pb.c * N + ((long)(pb.i1_0 + pb.np - 1) * n2 + pb.i2) * n3 + n3 - 1;
    if (u_last >= plane * M3 || y_last >= 3 * N) {
      char m[160];
      std::snprintf(m, sizeof m, "pencil writes n=(%d,%d,%d) M3=%d P=%d block %d leave the buffer", n1, n2, n3, M3,
                    P, b);
      return ck.fail(m);
    }
  }
  ++ck.checked;
  return true;
}

// cross-section passes: M3 workgroups, one plane each (paired_plane), or M3 / 2
// plane pairs (pair_planes; one plane when M3 = 1): every plane exactly once
bool check_planes(Checker& ck, int M3) {
  char where[96];
  std::snprintf(where, sizeof where, "planes M3=%d", M3);
  std::vector<char> seen(M3, 0);
  for (int b = 0; b < M3; ++b) {
    const int kz = vie::paired_plane(b, M3);
    if (kz < 0 || kz >= M3 || seen[kz]++) return ck.fail(std::string(where) + ": paired_plane not a bijection");
  }
  std::fill(seen.begin(), seen.end(), 0);
  const int pairs = M3 == 1 ? 1 : M3 / 2;
  for (int p = 0; p < pairs; ++p) {
    int a, b;
    vie::pair_planes(p, M3, &a, &b);
    const int np = M3 == 1 ? 1 : 2;
    const int kz[2] = {a, b};
    for (int i = 0; i < np; ++i)
      if (kz[i] < 0 || kz[i] >= M3 || seen[kz[i]]++) return ck.fail(std::string(where) + ": pair_planes overlap");
  }
  for (char c : seen)
    if (c != 1) return ck.fail(std::string(where) + ": plane not covered");
  ck.checked += 2;
  return true;
}

int pow2_at_least(int v) {
  int m = 1;
  while (m < v) m <<= 1;
  return m;
}

bool run_all(Checker& ck) {
  for (int M3 = 1; M3 <= 4096; M3 <<= 1)
    if (!check_planes(ck, M3)) return false;
  for (int n1 = 1; n1 <= 32; ++n1)
    for (int n2 = 1; n2 <= 32; ++n2) {
      // generic z passes: P = tp in {1, 2, 4, 8, 16}
      for (int tp = 1; tp <= 16; tp <<= 1)
        if (!check_pencil_map(ck, n1, n2, tp, [](int b, int nb) { return vie::xcd_group8(b, nb); }, "generic z"))
          return false;
      // four-step z passes: every pencil count of each precision
      for (int M3 = 512; M3 <= 4096; M3 <<= 1) {
        for (int vb : {8, 16}) {
          int opts[8];
          const int n = vb == 16 ? vie::z4_pencil_options<double>(M3, opts, 8)
                                 : vie::z4_pencil_options<float>(M3, opts, 8);
          for (int i = 0; i < n; ++i) {
            const int P = opts[i];
            if (!check_pencil_map(ck, n1, n2, P,
                                  [P, vb](int b, int nb) { return vie::xcd_group(b, nb, P, vb); }, "four-step z"))
              return false;
          }
        }
      }
    }
  // write extents for every n3 <= 2048 at its circulant length, a few n1, n2
  for (int n3 = 1; n3 <= 2048; ++n3) {
    const int M3 = pow2_at_least(2 * n3 - 1);
    if (M3 > 1 && 2 * n3 > M3) return ck.fail("n3 above half its circulant length (four-step padding)");
    for (int n1 : {1, 7, 20, 32})
      for (int n2 : {1, 9, 32})
        for (int P : {1, 2, 4, 8, 16})
          if (!check_pencil_writes(ck, n1, n2, n3, M3, P)) return false;
  }
  return true;
}

}  // namespace

extern "C" int vie_check_block_maps(char* msg, size_t cap, int planted) {
  Checker ck;
  bool ok;
  if (planted) {
    // a map that drops the last workgroup of every full group of 64 onto its
    // neighbour: the checker must refuse it
    ok = check_pencil_map(ck, 32, 32, 1,
                          [](int b, int nb) {
                            const int m = vie::xcd_group8(b, nb);
                            return (m % 64 == 63 && m + 1 <= nb) ? m - 1 : m;
                          },
                          "planted");
  } else {
    ok = run_all(ck);
  }
  std::string out = ok ? "ok: " + std::to_string(ck.checked) + " maps and extents checked" : ck.err;
  if (msg && cap) {
    std::strncpy(msg, out.c_str(), cap - 1);
    msg[cap - 1] = 0;
  }
  return ok ? VIE_OK : VIE_EINVAL;
}
