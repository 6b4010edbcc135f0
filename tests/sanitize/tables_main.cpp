// Driver for the sanitizer test of the host Green tables (green_table.cpp):
// computes the Toeplitz table N and the curl table K for one grid with several
// threads and writes them, raw complex128, to the given file (N first, then K).
// Built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_sanitize.py; any report makes the run fail.
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <vector>

namespace vie {
int green_table(const int n[3], double kappa, std::complex<double>* out, int nthreads);
int curl_table(const int n[3], double kappa, std::complex<double>* out, int nthreads);
}  // namespace vie

int main(int argc, char** argv) {
  if (argc != 7) {
    std::fprintf(stderr, "usage: %s n1 n2 n3 kappa threads out\n", argv[0]);
    return 2;
  }
  const int n[3] = {std::atoi(argv[1]), std::atoi(argv[2]), std::atoi(argv[3])};
  const double kappa = std::atof(argv[4]);
  const int threads = std::atoi(argv[5]);
  const long N = (long)n[0] * n[1] * n[2];
  std::vector<std::complex<double>> tn(6 * N), tk(3 * N);
  if (vie::green_table(n, kappa, tn.data(), threads) != 0) return 3;
  if (vie::curl_table(n, kappa, tk.data(), threads) != 0) return 4;
  FILE* f = std::fopen(argv[6], "wb");
  if (!f) return 5;
  const bool ok = std::fwrite(tn.data(), sizeof(tn[0]), tn.size(), f) == tn.size() &&
                  std::fwrite(tk.data(), sizeof(tk[0]), tk.size(), f) == tk.size();
  std::fclose(f);
  return ok ? 0 : 6;
}
