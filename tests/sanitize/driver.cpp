// Host-code driver for the sanitizer builds (AddressSanitizer + UBSan, and
// ThreadSanitizer): exercises the planner, the light-cone sets, the plan
// records and the serving loop through the C-ABI on host-only contexts
// (device -1: the executor is simulated), including error paths and
// concurrent submit / poll / cancel / shutdown.  Exits 0 when every call
// returned what it should; a sanitizer report makes the run fail.
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "qsim.h"

namespace {

int failures = 0;
#define EXPECT(cond)                                                   \
  do {                                                                 \
    if (!(cond)) {                                                     \
      std::fprintf(stderr, "%s:%d: expected %s\n", __FILE__, __LINE__, #cond); \
      ++failures;                                                      \
    }                                                                  \
  } while (0)

struct Circ {
  int n = 0, np = 0;
  std::vector<qsim_gate> g;
  std::vector<std::vector<double>> mats;  // U1 matrices (stable storage)
  qsim_circuit c() const { return qsim_circuit{n, (int32_t)g.size(), np, 0, g.data()}; }
};

qsim_gate gate(int kind, int q0, int q1 = -1, int param = -1, double angle = 0.0, const double* mat = nullptr) {
  qsim_gate x{};
  x.kind = (uint8_t)kind;
  x.q0 = q0;
  x.q1 = q1;
  x.param = param;
  x.angle = angle;
  x.mat = mat;
  return x;
}

// RY and RZ on every qubit, then CNOTs on even pairs and on odd pairs.
Circ brickwork(int n, int depth) {
  Circ c;
  c.n = n;
  for (int l = 0; l < depth; ++l) {
    for (int q = 0; q < n; ++q) c.g.push_back(gate(QSIM_RY, q, -1, c.np++));
    for (int q = 0; q < n; ++q) c.g.push_back(gate(QSIM_RZ, q, -1, c.np++));
    for (int q = 0; q + 1 < n; q += 2) c.g.push_back(gate(QSIM_CNOT, q, q + 1));
    for (int q = 1; q + 1 < n; q += 2) c.g.push_back(gate(QSIM_CNOT, q, q + 1));
  }
  return c;
}

// RY on every qubit, then CZ on (i, i+1) for i of the layer's parity.
Circ ry_cz(int n, int depth) {
  Circ c;
  c.n = n;
  for (int l = 0; l < depth; ++l) {
    for (int q = 0; q < n; ++q) c.g.push_back(gate(QSIM_RY, q, -1, c.np++));
    for (int q = l % 2; q + 1 < n; q += 2) c.g.push_back(gate(QSIM_CZ, q, q + 1));
  }
  return c;
}

// A unitary RZ(a) RY(b) RZ(c) as a row-major complex matrix.
std::vector<double> unitary(double a, double b, double c) {
  const double cb = std::cos(b / 2), sb = std::sin(b / 2);
  // entries e^{-i(a+c)/2} cb, -e^{-i(a-c)/2} sb, e^{i(a-c)/2} sb, e^{i(a+c)/2} cb
  const double p = (a + c) / 2, m = (a - c) / 2;
  return {std::cos(p) * cb, -std::sin(p) * cb, -std::cos(m) * sb, std::sin(m) * sb,
          std::cos(m) * sb, std::sin(m) * sb,  std::cos(p) * cb, std::sin(p) * cb};
}

Circ random_circ(int n, int ng, std::mt19937_64& rng) {
  Circ c;
  c.n = n;
  std::uniform_int_distribution<int> kind(0, 5), qd(0, n - 1);
  std::uniform_real_distribution<double> ang(-M_PI, M_PI);
  c.mats.reserve(ng);
  for (int k = 0; k < ng; ++k) {
    int kd = kind(rng), q0 = qd(rng), q1 = qd(rng);
    if ((kd == QSIM_CZ || kd == QSIM_CNOT) && (n < 2 || q0 == q1)) kd = QSIM_RX;
    if (kd == QSIM_CZ || kd == QSIM_CNOT) c.g.push_back(gate(kd, q0, q1));
    else if (kd == QSIM_U1) {
      c.mats.push_back(unitary(ang(rng), ang(rng), ang(rng)));
      c.g.push_back(gate(kd, q0, -1, -1, 0.0, c.mats.back().data()));
    } else {
      c.g.push_back(gate(kd, q0, -1, (k % 5 == 0) ? -1 : c.np++, ang(rng)));
    }
  }
  return c;
}

struct Ham {
  std::vector<double> coeff;
  std::vector<int32_t> off{0}, qubits;
  std::vector<uint8_t> paulis;
  void add(double c, const std::vector<std::pair<int, char>>& ops) {
    coeff.push_back(c);
    for (auto& o : ops) {
      qubits.push_back(o.first);
      paulis.push_back((uint8_t)o.second);
    }
    off.push_back((int32_t)qubits.size());
  }
  qsim_hamiltonian h() const {
    return qsim_hamiltonian{(int32_t)coeff.size(), 0, coeff.data(), off.data(), qubits.data(), paulis.data()};
  }
};

Ham tfim(int n, double hx) {
  Ham H;
  for (int q = 0; q < n; ++q) H.add(1.0, {{q, 'Z'}, {(q + 1) % n, 'Z'}});
  for (int q = 0; q < n; ++q) H.add(hx, {{q, 'X'}});
  return H;
}

Ham random_ham(int n, int T, std::mt19937_64& rng) {
  Ham H;
  std::uniform_int_distribution<int> qd(0, n - 1), pd(0, 2), wd(1, std::min(n, 3));
  std::uniform_real_distribution<double> cd(-1, 1);
  for (int t = 0; t < T; ++t) {
    std::vector<std::pair<int, char>> ops;
    const int w = wd(rng);
    for (int k = 0; k < w; ++k) {
      const int q = qd(rng);
      bool dup = false;
      for (auto& o : ops) dup |= o.first == q;
      if (!dup) ops.push_back({q, "XYZ"[pd(rng)]});
    }
    H.add(cd(rng), ops);
  }
  return H;
}

void host_planning() {
  // dense plan of the n=30 workload and its gate order
  Circ b = brickwork(30, 20);
  Ham H = tfim(30, 1.0);
  qsim_circuit cc = b.c();
  qsim_hamiltonian hh = H.h();
  int64_t info[4] = {0, 0, 0, 0};
  std::vector<int32_t> order(4 * b.g.size());
  EXPECT(qsim_plan_dense(&cc, &hh, QSIM_C64, info, order.data(), (int)b.g.size()) == QSIM_OK);
  EXPECT(info[0] > 0 && info[1] >= info[0]);
  EXPECT(qsim_plan_dense(&cc, &hh, QSIM_C128, info, nullptr, 0) == QSIM_OK);
  // light-cone sets of a 500-qubit RY+CZ brickwork, ring plus chord terms
  Circ lc = ry_cz(500, 4);
  Ham M;
  for (int q = 0; q < 500; ++q) M.add(1.0, {{q, 'Z'}, {(q + 1) % 500, 'Z'}});
  for (int q = 0; q < 250; ++q) M.add(1.0, {{q, 'Z'}, {q + 250, 'Z'}});
  qsim_circuit lcc = lc.c();
  qsim_hamiltonian mh = M.h();
  std::vector<int32_t> off(M.coeff.size() + 1), qs(M.coeff.size() * 40);
  EXPECT(qsim_lightcone_sets(&lcc, &mh, off.data(), qs.data(), (int)qs.size()) == QSIM_OK);
  EXPECT(qsim_lightcone_sets(&lcc, &mh, off.data(), qs.data(), 10) == QSIM_ETOOBIG);
  // random circuits of every kind, every dtype, with and without plan records
  std::mt19937_64 rng(7);
  qsim_options o{};
  o.device = -1;
  qsim_ctx* ctx = nullptr;
  EXPECT(qsim_init(&ctx, &o) == QSIM_OK && ctx);
  for (int k = 0; k < 40; ++k) {
    const int n = 1 + (int)(rng() % 24);
    Circ c = random_circ(n, 20 + (int)(rng() % 120), rng);
    Ham R = random_ham(n, 1 + (int)(rng() % 12), rng);
    qsim_circuit rc = c.c();
    qsim_hamiltonian rh = R.h();
    std::vector<int32_t> ord(4 * c.g.size() + 4);
    EXPECT(qsim_plan_dense(&rc, &rh, k % 2 ? QSIM_C128 : QSIM_C64, info, ord.data(), (int)c.g.size() + 1) == QSIM_OK);
    int count = 0;
    std::vector<int32_t> rec(8 * 64);
    const int r = qsim_plan_passes(ctx, &rc, &rh, QSIM_C64, k % 3 == 0, rec.data(), 64, &count);
    EXPECT(r == QSIM_OK || (r == QSIM_ETOOBIG && count > 64));
    std::vector<int32_t> loff(R.coeff.size() + 1), lq(R.coeff.size() * (n + 1));
    EXPECT(qsim_lightcone_sets(&rc, &rh, loff.data(), lq.data(), (int)lq.size()) == QSIM_OK);
  }
  // invalid input
  {
    Circ c = brickwork(4, 1);
    c.g[0].q0 = 9;  // qubit out of range
    qsim_circuit bc = c.c();
    Ham h4 = tfim(4, 0.5);
    qsim_hamiltonian hh4 = h4.h();
    EXPECT(qsim_plan_dense(&bc, &hh4, QSIM_C64, info, nullptr, 0) == QSIM_EINVAL);
    Circ d = brickwork(4, 1);
    d.g.push_back(gate(QSIM_CNOT, 2, 2));  // duplicate qubit
    qsim_circuit dc = d.c();
    EXPECT(qsim_plan_dense(&dc, &hh4, QSIM_C64, info, nullptr, 0) == QSIM_EINVAL);
    std::vector<double> bad = {1, 0, 1, 0, 0, 0, 1, 0};  // not unitary
    Circ u = brickwork(4, 1);
    u.g.push_back(gate(QSIM_U1, 1, -1, -1, 0.0, bad.data()));
    qsim_circuit uc = u.c();
    EXPECT(qsim_plan_dense(&uc, &hh4, QSIM_C64, info, nullptr, 0) == QSIM_EINVAL);
    Ham badh;
    badh.add(1.0, {{0, 'Q'}});
    qsim_hamiltonian bh = badh.h();
    qsim_circuit ok = brickwork(4, 1).c();
    Circ okc = brickwork(4, 1);
    ok = okc.c();
    EXPECT(qsim_plan_dense(&ok, &bh, QSIM_C64, info, nullptr, 0) == QSIM_EINVAL);
  }
  qsim_finalize(ctx);
}

void serving() {
  // simulated executor: each scheduler step takes 2 ms, so requests queue
  setenv("QSIM_TEST_MOCK_STEP_MS", "2", 1);
  qsim_options o{};
  o.device = -1;
  o.max_queue = 48;
  o.hbm_budget_bytes = 1ull << 26;  // 64 MiB of state memory in flight
  qsim_ctx* ctx = nullptr;
  EXPECT(qsim_init(&ctx, &o) == QSIM_OK && ctx);
  struct Req {
    Circ c;
    Ham H;
    std::vector<double> th;
    int grad;
  };
  const int kThreads = 4, kPer = 12;
  std::vector<std::vector<Req>> reqs(kThreads);
  for (int t = 0; t < kThreads; ++t) {
    std::mt19937_64 rng(100 + t);
    for (int k = 0; k < kPer; ++k) {
      const int n = 12 + (int)(rng() % 9), depth = 4 + (int)(rng() % 5);
      Req r{ry_cz(n, depth), tfim(n, 0.5), {}, (int)(k % 2)};
      r.th.resize(r.c.np);
      for (double& x : r.th) x = std::uniform_real_distribution<double>(-M_PI, M_PI)(rng);
      reqs[t].push_back(std::move(r));
    }
  }
  std::atomic<int> done{0}, cancelled{0}, rejected{0};
  std::vector<std::thread> th;
  for (int t = 0; t < kThreads; ++t)
    th.emplace_back([&, t] {
      std::vector<uint64_t> tickets;
      std::vector<int> np;
      for (Req& r : reqs[t]) {
        qsim_circuit cc = r.c.c();
        qsim_hamiltonian hh = r.H.h();
        qsim_request q{&cc, r.th.data(), &hh, r.grad, 0};
        uint64_t tk = 0;
        const int rc = qsim_submit(ctx, &q, &tk);
        if (rc == QSIM_EAGAIN) {
          ++rejected;
          continue;
        }
        EXPECT(rc == QSIM_OK);
        tickets.push_back(tk);
        np.push_back(r.grad ? r.c.np : 0);
      }
      if (!tickets.empty()) {
        const int rc = qsim_cancel(ctx, tickets.back());
        EXPECT(rc == QSIM_OK || rc == QSIM_ENOTFOUND);
      }
      for (size_t k = 0; k < tickets.size(); ++k) {
        std::vector<double> g(std::max(1, np[k]));
        double E = 0, times[3];
        for (;;) {
          const int rc = qsim_poll_timed(ctx, tickets[k], &E, g.data(), times);
          if (rc == QSIM_PENDING) {
            std::this_thread::sleep_for(std::chrono::microseconds(200));
            continue;
          }
          if (rc == QSIM_OK) ++done;
          else if (rc == QSIM_ECANCELED) ++cancelled;
          else EXPECT(rc == QSIM_OK);
          break;
        }
      }
    });
  std::thread stats([&] {
    for (int k = 0; k < 50; ++k) {
      qsim_server_stats s{};
      EXPECT(qsim_server_stats_get(ctx, &s) == QSIM_OK);
      std::this_thread::sleep_for(std::chrono::milliseconds(1));
    }
  });
  for (auto& x : th) x.join();
  stats.join();
  EXPECT(done + cancelled + rejected == kThreads * kPer);
  EXPECT(done > 0);
  std::printf("serving: %d completed, %d cancelled, %d rejected\n", done.load(), cancelled.load(), rejected.load());
  // shutdown with requests pending: their tickets end, nothing leaks or hangs
  for (int k = 0; k < 6; ++k) {
    Req& r = reqs[0][k];
    qsim_circuit cc = r.c.c();
    qsim_hamiltonian hh = r.H.h();
    qsim_request q{&cc, r.th.data(), &hh, 1, 0};
    uint64_t tk = 0;
    const int rc = qsim_submit(ctx, &q, &tk);
    EXPECT(rc == QSIM_OK || rc == QSIM_EAGAIN);
  }
  qsim_finalize(ctx);
}

}  // namespace

int main(int argc, char** argv) {
  const bool plan = argc < 2 || std::string(argv[1]) != "serving";
  const bool serve = argc < 2 || std::string(argv[1]) != "planning";
  if (plan) host_planning();
  if (serve) serving();
  std::printf("driver: %d failures\n", failures);
  return failures ? 1 : 0;
}
