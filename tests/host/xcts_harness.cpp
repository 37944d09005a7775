// Host harness for the library's XCTS solver: csrc/xcts.hip built with g++
// against the HIP stand-in in hip_shim/, called the way grmhd_xcts_solve calls
// it (grid nodes and map widths from build_operators, a work buffer of the
// context's scratch size, the diagnostics partials).
//
//   xcts_harness nr nth nph r_in r_out th_min th_max max_iter in.bin out.bin
//
// in.bin: E then the initial guess psi (P doubles each, [phi][theta][r]);
// out.bin: int32 return code, int32 iterations, double last change, psi.
#include <algorithm>
#include <barrier>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "grmhd_internal.h"

dim3 blockIdx, blockDim, gridDim;
thread_local dim3 threadIdx;

namespace hipshim {
namespace {
// A pool of host threads, one per GPU thread of a block, started once.
struct Pool {
  unsigned n = 0;
  std::vector<std::thread> workers;
  std::barrier<>* start = nullptr;  // main thread + workers
  std::barrier<>* done = nullptr;
  std::barrier<>* sync = nullptr;   // workers only (__syncthreads)
  const std::function<void()>* body = nullptr;
  bool quit = false;
  void grow(unsigned want) {
    if (want == n) return;
    stop();
    n = want;
    start = new std::barrier<>(n + 1);
    done = new std::barrier<>(n + 1);
    sync = new std::barrier<>(n);
    for (unsigned t = 0; t < n; ++t)
      workers.emplace_back([this, t] {
        threadIdx = dim3(t, 0, 0);
        for (;;) {
          start->arrive_and_wait();
          if (quit) return;
          (*body)();
          done->arrive_and_wait();
        }
      });
  }
  void stop() {
    if (!n) return;
    quit = true;
    start->arrive_and_wait();
    for (auto& w : workers) w.join();
    workers.clear();
    delete start;
    delete done;
    delete sync;
    quit = false;
    n = 0;
  }
  ~Pool() { stop(); }
};
Pool pool;
}  // namespace

void run_block(const std::function<void()>& body) {
  pool.grow(blockDim.x);
  pool.body = &body;
  pool.start->arrive_and_wait();
  pool.done->arrive_and_wait();
}

void syncthreads() { pool.sync->arrive_and_wait(); }
}  // namespace hipshim

int main(int argc, char** argv) {
  if (argc != 11) {
    fprintf(stderr, "usage: xcts_harness nr nth nph r_in r_out th_min th_max max_iter in.bin out.bin\n");
    return 2;
  }
  grmhd_grid grid{};
  grid.nr = atoi(argv[1]);
  grid.nth = atoi(argv[2]);
  grid.nph = atoi(argv[3]);
  grid.r_in = atof(argv[4]);
  grid.r_out = atof(argv[5]);
  grid.th_min = atof(argv[6]);
  grid.th_max = atof(argv[7]);
  grid.filt_alpha = 36.0;
  grid.filt_order = 16;
  grid.filter_on = 1;
  grid.dealias = 0;
  const int max_iter = atoi(argv[8]);
  grmhd::Operators ops;
  grmhd::build_operators(grid, 0.25, &ops);
  const long long P = (long long)grid.nr * grid.nth * grid.nph;
  // the context's scratch buffer and diagnostics partials, as grmhd_xcts_solve passes them
  std::vector<double> work((size_t)grmhd::SC_NFIELDS * P);
  const int dblocks = (int)std::min<long long>((P + 255) / 256, 1024);
  std::vector<double> partials((size_t)dblocks * grmhd::DIAG_Q);
  if (5 * (size_t)P + grmhd::xcts_operator_doubles(grid.nr, grid.nth, grid.nph) > work.size()) return 3;
  std::vector<double> E(P), psi(P);
  FILE* f = fopen(argv[9], "rb");
  if (!f || fread(E.data(), 8, P, f) != (size_t)P || fread(psi.data(), 8, P, f) != (size_t)P) return 4;
  fclose(f);
  grmhd::XctsGrid g{grid.nr, grid.nth, grid.nph, ops.Lh, ops.Th, ops.r.data(), ops.th.data()};
  int it = 0;
  double ch = 0.0;
  std::string err;
  const int rc = grmhd::xcts_solve(g, work.data(), partials.data(), dblocks * grmhd::DIAG_Q / 2, nullptr, E.data(),
                                   psi.data(), max_iter, 1e-11, &it, &ch, &err);
  if (rc) fprintf(stderr, "%s\n", err.c_str());
  FILE* o = fopen(argv[10], "wb");
  if (!o) return 5;
  const int32_t hdr[2] = {rc, it};
  fwrite(hdr, 4, 2, o);
  fwrite(&ch, 8, 1, o);
  fwrite(psi.data(), 8, P, o);
  fclose(o);
  hipshim::pool.stop();
  return 0;
}
