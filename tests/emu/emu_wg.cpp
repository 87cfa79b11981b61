// CPU emulation of the LDS-window simulation launch and the whole-lattice
// re-run launch of sim_kernel<EMU_BLOCK, table mode, one-step burns>: each
// workgroup is EMU_BLOCK OS threads, several workgroups run at once and take
// simulations from the shared work counter, buffers are sized exactly (built
// with AddressSanitizer, any access outside them is reported), and a
// watchdog reports a barrier that never completes with the line every thread
// waits at.
//
// usage: emu_wg CASE_DIR W H WINDOW QUEUE_CAP WORKGROUPS SEED [global]
// With `global`, the re-run launch keeps each workgroup's whole-lattice
// bitset in global memory (the form for lattices whose bitset does not fit
// LDS) and its LDS holds the queues only.
// CASE_DIR holds the landscape layers veg.bin (uint8), elev.bin, slope.bin,
// aspect.bin, wind.bin (float32, row-major H x W), which the kernel source's
// own preprocess_kernel turns into cell records, table.bin (an Eq. 1 table,
// H x W x 8 uint32) and sims.bin (fire_sim records); the results go to
// CASE_DIR/emu_results.bin (fire_result records).
#include "kernel.inc"
#include <chrono>
#include <fstream>
#include <string>
#include <thread>
#ifndef EMU_BLOCK
#define EMU_BLOCK 1024
#endif
thread_local Dim3 threadIdx, blockIdx;
Dim3 blockDim, gridDim;
thread_local uint32_t *g_lds;
thread_local WgCtx *g_wg;
thread_local int *g_where;
std::atomic<long> g_progress{0};
std::mutex g_atomic_mu;
using namespace firegpu;
constexpr int BLOCK = EMU_BLOCK;

template <class T> std::vector<T> load(const std::string &path) {
  std::ifstream f(path, std::ios::binary | std::ios::ate);
  if (!f) { fprintf(stderr, "missing %s\n", path.c_str()); exit(2); }
  const size_t bytes = f.tellg();
  f.seekg(0);
  std::vector<T> v(bytes / sizeof(T));
  f.read(reinterpret_cast<char *>(v.data()), bytes);
  return v;
}

template <bool WIN, bool GB = false>
void run_workgroup(const SimArgs &a, int b, size_t lds_words) {
  std::vector<uint32_t> lds(lds_words, 0xDEADBEEFu);
  WgCtx ctx;
  Barrier block(BLOCK);
  ctx.block = &block;
  for (int w = 0; w < BLOCK / 64; ++w) ctx.wave.push_back(new Barrier(64));
  for (int p = 0; p < BLOCK / 2; ++p) ctx.pair.push_back(new Barrier(2));
  std::vector<int> where(BLOCK, 0);
  std::atomic<bool> done{false};
  std::thread watchdog([&] {
    long last = -1;
    int still = 0;
    while (!done.load()) {
      std::this_thread::sleep_for(std::chrono::seconds(1));
      const long p = g_progress.load();
      if (p != last) { still = 0; last = p; continue; }
      if (++still < 120) continue;
      fprintf(stderr, "no barrier completed for 120 s (workgroup %d); thread:line\n", b);
      for (int t = 0; t < BLOCK; ++t)
        fprintf(stderr, "%d:%d%s", t, where[t], t % 16 == 15 ? "\n" : " ");
      fflush(stderr);
      _exit(3);
    }
  });
  std::vector<std::thread> th;
  for (int t = 0; t < BLOCK; ++t)
    th.emplace_back([&, t] {
      threadIdx.x = t;
      blockIdx.x = b;
      g_wg = &ctx;
      g_lds = lds.data();
      g_where = &where[t];
      sim_kernel<BLOCK, true, false, WIN, GB>(a);
      where[t] = 999999;
      block.arrive_and_drop();
    });
  for (auto &x : th) x.join();
  done = true;
  watchdog.join();
  for (auto *p : ctx.wave) delete p;
  for (auto *p : ctx.pair) delete p;
}

int main(int argc, char **argv) {
  if (argc != 8 && argc != 9) {
    fprintf(stderr, "usage: emu_wg CASE_DIR W H WINDOW QUEUE_CAP WORKGROUPS SEED [global]\n");
    return 2;
  }
  const bool global_bits = argc == 9 && std::string(argv[8]) == "global";
  const std::string d = argv[1];
  const int W = atoi(argv[2]), H = atoi(argv[3]), win = atoi(argv[4]), cap = atoi(argv[5]);
  const int groups = atoi(argv[6]);
  const uint64_t seed = strtoull(argv[7], nullptr, 0);
  auto veg = load<uint8_t>(d + "/veg.bin");
  auto elev = load<float>(d + "/elev.bin");
  auto slope = load<float>(d + "/slope.bin");
  auto aspect = load<float>(d + "/aspect.bin");
  auto wind = load<float>(d + "/wind.bin");
  auto table = load<uint32_t>(d + "/table.bin");
  auto simb = load<uint8_t>(d + "/sims.bin");
  const int n_sims = (int)(simb.size() / sizeof(fire_sim));
  const int64_t n = (int64_t)W * H;
  const int stride = (W + 31) / 32;
  if ((int64_t)veg.size() != n || (int64_t)elev.size() != n || (int64_t)slope.size() != n ||
      (int64_t)aspect.size() != n || (int64_t)wind.size() != n ||
      (int64_t)table.size() != n * 8) {
    fprintf(stderr, "case files do not match %d x %d\n", W, H);
    return 2;
  }
  // the landscape records, by the kernel source's preprocessing (one thread
  // covers the grid-stride loops)
  std::vector<uint4> rec(n);
  std::vector<double> ps(2 * n), omega(8 * n);
  std::vector<uint32_t> blocked((size_t)H * stride);
  threadIdx.x = 0; blockIdx.x = 0; blockDim.x = 1; gridDim.x = 1;
  preprocess_kernel(veg.data(), elev.data(), slope.data(), aspect.data(), wind.data(), W, H,
                    stride, rec.data(), ps.data(), omega.data(), blocked.data());
  std::vector<LandscapeDev> lsd(1);
  LandscapeDev &L = lsd[0];
  L.W = W; L.H = H; L.stride = stride; L.valid = 1; L.rec = rec.data(); L.ps = ps.data();
  L.omega = omega.data(); L.blocked = blocked.data(); L.burn_steps = nullptr; L.forest_class = 1;
  const double beta_unused[5] = {0, 0, 0, 0, 0};
  std::vector<fire_result> out(n_sims);
  std::vector<uint32_t> work(2, 0), err(1, 0), retry(1 + n_sims, 0);
  const int64_t ovf_cap = std::max<int64_t>(1, n - cap);
  std::vector<uint32_t> spill((size_t)groups * 2 * ovf_cap);
  SimArgs a{};
  a.ls = lsd.data(); a.n_ls = 1; a.tg = nullptr; a.n_tg = 0;
  a.betas = beta_unused; a.n_params = 1;
  a.sims = reinterpret_cast<const fire_sim *>(simb.data()); a.order = nullptr; a.n_sims = n_sims;
  a.key0 = (uint32_t)seed; a.key1 = (uint32_t)(seed >> 32);
  a.tables = table.data(); a.table_stride = (int64_t)W * H * 8; a.table_ls = 0;
  a.out = out.data(); a.maps = nullptr; a.map_words = 0;
  a.work = &work[0]; a.error_flag = err.data(); a.ovf = spill.data(); a.ovf_life = nullptr;
  a.ovf_cap = ovf_cap; a.queue_cap = cap;
  const int bw = std::min(win, H) * std::min(win / 32, stride);
  a.bitset_words = bw; a.win = win; a.retry = retry.data(); a.n_dev = nullptr; a.stat_out = nullptr;
  a.times = nullptr; a.times_cap = 0;
  blockDim.x = BLOCK;
  gridDim.x = groups;
  {
    std::vector<std::thread> wgs;
    for (int b = 0; b < groups; ++b)
      wgs.emplace_back([&, b] { run_workgroup<true>(a, b, (size_t)bw + 2 * cap + 16); });
    for (auto &x : wgs) x.join();
  }
  printf("window launch: error flag %u, re-runs %u of %d\n", err[0], retry[0], n_sims);
  fflush(stdout);
  SimArgs b2 = a;
  b2.work = &work[1]; b2.order = retry.data() + 1; b2.n_dev = retry.data(); b2.win = 0;
  b2.bitset_words = H * stride;
  std::vector<uint32_t> gbits(global_bits ? (size_t)groups * H * stride : 0, 0xDEADBEEFu);
  b2.gbits = global_bits ? gbits.data() : nullptr;
  {
    std::vector<std::thread> wgs;
    for (int b = 0; b < groups; ++b)
      wgs.emplace_back([&, b] {
        if (global_bits) run_workgroup<false, true>(b2, b, (size_t)2 * cap + 16);
        else run_workgroup<false>(b2, b, (size_t)H * stride + 2 * cap + 16);
      });
    for (auto &x : wgs) x.join();
  }
  std::ofstream o(d + "/emu_results.bin", std::ios::binary);
  o.write(reinterpret_cast<const char *>(out.data()), sizeof(fire_result) * n_sims);
  printf("re-run launch done: error flag %u\n", err[0]);
  return err[0] != 0;
}
