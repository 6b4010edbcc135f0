// Host check of the pass kernels' workgroup-to-work maps (block_maps.hpp) over
// every shape the library accepts: n1, n2 <= 32, circulant lengths M3 = 2^k <=
// 4096, both precisions, every pencil count the launchers and the tuner use.
// Each map must be a bijection onto the work items of its launch, and every
// write a kernel derives from its item must land inside the buffer it writes.
// The LDS maps of the 64 x 32 cross-section pass (xy6432_maps.hpp) must be
// bijections inside their areas and, lane by lane over each access of one LDS
// pass (256 bytes), free of bank conflicts where the kernel's comment says so.
#include <cstdio>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "../../include/vie.h"
#include "block_maps.hpp"
#include "vie_internal.hpp"
#include "xy6432_maps.hpp"

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

// LDS maps of the 64 x 32 pass.  hand: the hand-off map (the planted check passes
// a wrong one).  One LDS pass serves 256 bytes: 256 / vb lanes of vb-byte values,
// each value vb / 4 of the 64 four-byte banks, so the lanes of a pass conflict
// unless their indices differ modulo 256 / vb.
bool check_xy6432(Checker& ck, const std::function<int(int, int, int)>& hand) {
  const int H = vie::kXy32HandVals;
  std::vector<char> seen(H, 0);
  for (int c = 0; c < 3; ++c)
    for (int y = 0; y < 16; ++y)
      for (int kx = 0; kx < 64; ++kx) {
        const int h = hand(c, y, kx);
        if (h < 0 || h >= H || h / 64 != c * 16 + y) return ck.fail("xy6432 hand-off entry outside its row");
        if (seen[h]++) return ck.fail("xy6432 hand-off map not injective");
      }
  for (int f = 0; f < 4; ++f) {
    std::vector<char> s64(64, 0);
    for (int i = 0; i < 8; ++i)
      for (int j = 0; j < 8; ++j) {
        const int r = vie::xy32_rowx(i, j, f);
        if (r < 0 || r >= 64 || s64[r]++) return ck.fail("xy6432 row exchange not a bijection");
      }
  }
  for (int r = 0; r < 4; ++r) {
    std::vector<char> s32(32, 0);
    for (int a = 0; a < 4; ++a)
      for (int k = 0; k < 8; ++k) {
        const int x = vie::xy32_colx(a, k, r);
        if (x < 0 || x >= vie::kXy32ColX || s32[x]++) return ck.fail("xy6432 column exchange not a bijection");
      }
  }
  for (int kx = 0; kx < 64; ++kx) {
    std::vector<int> used;
    for (int a = 0; a < 4; ++a)
      for (int k = 0; k < 8; ++k) {
        const int x = vie::xy32_cslot(a, k, kx);
        const int row = x / 64, c = row / 16, y = row % 16;
        if (x < 0 || c >= 2 || vie::xy32_hand(c, y, kx) != x)
          return ck.fail("xy6432 compact exchange outside the column's entries of components 0 and 1");
        for (int u : used)
          if (u == x) return ck.fail("xy6432 compact exchange not injective");
        used.push_back(x);
      }
  }
  ck.checked += 4;
  for (int vb : {16, 8}) {
    const int lanes = 256 / vb, mod = 256 / vb;
    char where[96];
    auto pass_ok = [&](const std::vector<int>& idx, const char* what) {
      std::vector<char> slot(mod, 0);
      for (int e : idx)
        if (slot[((e % mod) + mod) % mod]++) {
          std::snprintf(where, sizeof where, "xy6432 bank conflict: %s, %d-byte values", what, vb);
          return ck.fail(where);
        }
      return true;
    };
    std::vector<int> idx, idx2;
    // column groups of 4 lanes: lane l -> column kx0 + l / 4, lane a = l % 4
    for (int kx0 = 0; kx0 < 64; kx0 += lanes / 4) {
      for (int c = 0; c < 3; ++c)
        for (int b = 0; b < 4; ++b) {
          idx.clear();
          for (int l = 0; l < lanes; ++l) idx.push_back(hand(c, (l & 3) + 4 * b, kx0 + (l >> 2)));
          if (!pass_ok(idx, "column loads and stores")) return false;
        }
      for (int k = 0; k < 8; ++k) {
        idx.clear();
        idx2.clear();
        for (int l = 0; l < lanes; ++l) {
          const int kx = kx0 + (l >> 2);
          idx.push_back(vie::xy32_cslot(l & 3, k, kx));
          idx2.push_back(H + kx * vie::kXy32ColX + vie::xy32_colx(l & 3, k, kx & 3));
        }
        if (!pass_ok(idx, "compact column exchange writes")) return false;
        if (vb == 16 && !pass_ok(idx2, "column exchange writes")) return false;
      }
      for (int s = 0; s < 4; ++s)
        for (int e = 0; e < 2; ++e) {
          idx.clear();
          idx2.clear();
          for (int l = 0; l < lanes; ++l) {
            const int kx = kx0 + (l >> 2), k = 2 * (l & 3) + e;
            idx.push_back(vie::xy32_cslot(s, k, kx));
            idx2.push_back(H + kx * vie::kXy32ColX + vie::xy32_colx(s, k, kx & 3));
          }
          if (!pass_ok(idx, "compact column exchange reads")) return false;
          if (vb == 16 && !pass_ok(idx2, "column exchange reads")) return false;
        }
    }
    // row groups of 8 lanes: lane l -> group q0 + l / 8, lane a = l % 8
    for (int q0 = 0; q0 < 32; q0 += lanes / 8)
      for (int i = 0; i < 2; ++i)
        for (int m = 0; m < 8; ++m) {
          idx.clear();
          idx2.clear();
          std::vector<int> idx3;
          for (int l = 0; l < lanes; ++l) {
            const int q = q0 + (l >> 3), a = l & 7;
            if (i == 1 && q >= 16) continue;
            int c, y;
            vie::xy32_row_task(q, i, &c, &y);
            idx.push_back(hand(c, y, a + 8 * m));
            idx2.push_back((c * 16 + y) * 64 + vie::xy32_rowx(m, a, q & 3));
            idx3.push_back((c * 16 + y) * 64 + vie::xy32_rowx(a, m, q & 3));
          }
          if (!pass_ok(idx, "row stores and loads")) return false;
          if (!pass_ok(idx2, "row exchange writes") || !pass_ok(idx3, "row exchange reads")) return false;
        }
    ck.checked += 1;
  }
  return true;
}

int pow2_at_least(int v) {
  int m = 1;
  while (m < v) m <<= 1;
  return m;
}

bool run_all(Checker& ck) {
  if (!check_xy6432(ck, [](int c, int y, int kx) { return vie::xy32_hand(c, y, kx); })) return false;
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
  if (planted == 2) {
    // a hand-off swizzle by (y & 3) 8: a bijection, but the column loads of one
    // LDS pass then share banks; the checker must refuse it
    ok = check_xy6432(ck, [](int c, int y, int kx) { return (c * 16 + y) * 64 + (kx ^ ((y & 3) * 8)); });
  } else if (planted) {
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
