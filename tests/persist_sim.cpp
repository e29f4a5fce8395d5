// Host-side simulation of the persistent factorisation's task protocol
// (paper_1805_00569_amd/csrc/persist_plan.hpp): workers take tasks from the
// queues in order (their own queue first, then the others), wait until their
// system has finished `need` tasks, run for a random time and count the task
// done.  With one queue per XCD, worker w runs on XCD w % X (X XCDs hold
// workers, drawn from the seed) and a queue is served only by the XCD that
// claimed it first.  Checks, for ragged batches: every task is taken once,
// no worker ever waits forever (the simulation would stall), a task starts
// only after every task of its system's earlier stages, every system's
// tasks run on one XCD, and each system's tasks cover its factorisation
// exactly (every tile below the diagonal solved once, every diagonal block
// factored once, every trailing tile updated once per panel).
//
// Usage: persist_sim <seed> <workers> <mode 0|1|2> <Wp> <T_0> <T_1> ...  (mode 2: column pairs)
// (Wp = 0: every system draws its own panel width in [1, 24])
// Prints "OK <tasks> <makespan> <queues>" or "FAIL <reason>".
#include <cstdio>
#include <cstdlib>
#include <map>
#include <queue>
#include <random>
#include <set>
#include <tuple>
#include <vector>

#include "../paper_1805_00569_amd/csrc/persist_plan.hpp"

using namespace krr;

static int fail(const char* m, long a = 0, long b = 0) {
  std::printf("FAIL %s %ld %ld\n", m, a, b);
  return 1;
}

int main(int argc, char** argv) {
  if (argc < 6) return fail("usage");
  const unsigned seed = (unsigned)std::atoi(argv[1]);
  const int W = std::atoi(argv[2]);
  const int mode = std::atoi(argv[3]);   // 0 matrix-core path, 1 packed, 2 packed with column pairs
  const bool packed = mode != 0;
  const int Wp = std::atoi(argv[4]);
  std::vector<int> T, act;
  for (int i = 5; i < argc; ++i) {
    T.push_back(std::atoi(argv[i]));
    act.push_back(1);
  }
  const int n = (int)T.size();
  std::mt19937 wrng(seed * 7919u + 1u);
  std::vector<int> Wps(n, Wp);
  for (int s = 0; s < n; ++s)
    if (Wp == 0) Wps[s] = 1 + (int)(wrng() % 24u);
  const PPlan P = build_plan(T, act, Wps, packed, 8, mode == 2);
  const int nt = (int)P.tasks.size();
  // coverage of each system's tasks
  for (int s = 0; s < n; ++s) {
    const int Ts = T[s];
    std::map<std::pair<int, int>, int> solved;           // tile (i, k), i > k
    std::vector<int> diag(Ts > 0 ? Ts : 0, 0);
    std::map<std::tuple<int, int, int>, int> updated;    // (panel start, i, j) of trailing updates
    int cnt = 0;
    for (const PTask& t : P.tasks) {
      if (t.s != s) continue;
      ++cnt;
      if (t.kind == PT_DIAG) diag[t.a]++;
      if (t.kind == PT_PCOL) {
        for (int w = 0; w < 4; ++w) {
          const int i = t.a + 1 + 4 * t.b + w;
          if (i < Ts) solved[{i, t.a}]++;
        }
        if (t.flags & PF_DIAG_NEXT) diag[t.a + 1]++;
      }
      if (t.kind == PT_PHEAD) {
        const int K0 = t.a, kend = std::min(K0 + Wps[s], Ts);
        diag[K0]++;
        if (K0 + 1 < kend) {
          solved[{K0 + 1, K0}]++;
          diag[K0 + 1]++;
        }
      }
      if (t.kind == PT_PPAIR) {
        const int c = t.a, g = t.b, K0 = t.c, kend = std::min(K0 + Wps[s], Ts);
        const int r0 = g == 0 ? c + 2 : c + 4 * g, nr = g == 0 ? 2 : 4;
        for (int w = 0; w < nr; ++w) {
          const int i = r0 + w;
          if (i < Ts) {
            solved[{i, c}]++;
            solved[{i, c + 1}]++;
          }
        }
        if (g == 0 && c + 2 < kend) diag[c + 2]++;
        if (g == 0 && c + 3 < kend) {
          solved[{c + 3, c + 2}]++;
          diag[c + 3]++;
        }
      }
      if (t.kind == PT_TRSM) solved[{t.a, t.b}]++;
      if (t.kind == PT_PTRAIL) {
        // super-tile b of the trailing region rows [K1, Ts): decode as the device does (band order)
        const int R = Ts - t.c, NS = (R + 1) / 2;
        int bx = t.b, lo = 0, hi = std::min(NS, 8), I = -1, J = -1;
        for (;;) {
          const int c = (hi * (hi + 1) - lo * (lo + 1)) / 2;
          if (bx < c) break;
          bx -= c;
          lo = hi;
          hi = std::min(NS, lo + 8);
        }
        const int h = hi - lo;
        if (bx < lo * h) {
          J = bx / h;
          I = lo + bx % h;
        } else {
          bx -= lo * h;
          J = lo;
          while (bx >= hi - J) {
            bx -= hi - J;
            ++J;
          }
          I = J + bx;
        }
        for (int w = 0; w < 4; ++w) {
          const int i = t.c + 2 * I + (w & 1), j = t.c + 2 * J + (w >> 1);
          if (i < Ts && j <= i) updated[{t.a, i, j}]++;
        }
      }
      if (t.kind == PT_TRI) {
        int ii = 0;
        while ((ii + 1) * (ii + 2) / 2 <= t.a) ++ii;
        const int jj = t.a - ii * (ii + 1) / 2;
        updated[{t.b, t.c + ii, t.c + jj}]++;
      }
    }
    if (cnt != P.total[s]) return fail("total", s, cnt);
    for (int k = 0; k < Ts; ++k)
      if (diag[k] != 1) return fail("diag", s, k);
    for (int i = 0; i < Ts; ++i)
      for (int k = 0; k < i; ++k)
        if (solved[{i, k}] != 1) return fail("solve", s, i * 100000 + k);
    const int Wq = Wps[s];
    for (int K0 = 0; K0 < Ts; K0 += Wq) {
      const int K1 = std::min(K0 + Wq, Ts);
      for (int i = K1; i < Ts; ++i)
        for (int j = K1; j <= i; ++j)
          if (updated[{K0, i, j}] != 1) return fail("trail", s, i * 100000 + j);
    }
    long expect_upd = 0;
    for (int K0 = 0; K0 < Ts; K0 += Wq) {
      const long R = Ts - std::min(K0 + Wq, Ts);
      expect_upd += R * (R + 1) / 2;
    }
    long got_upd = 0;
    for (auto& kv : updated) got_upd += kv.second;
    if (got_upd != expect_upd) return fail("trail_count", s, got_upd);
  }
  // need = tasks of the system in earlier stages: non-decreasing along a
  // system's tasks in queue order, and the tasks of one stage share it
  std::vector<int> last_need(n, -1), seen(n, 0);
  for (int q = 0; q < P.nq; ++q) {
    std::vector<int> sq(n, 0);
    for (int x = P.qoff[q]; x < P.qoff[q + 1]; ++x) {
      const PTask& t = P.tasks[x];
      if (t.need < last_need[t.s]) return fail("need_order", t.s, x);
      if (t.need > seen[t.s]) return fail("need_ahead", t.s, x);   // a predecessor would sit later
      last_need[t.s] = t.need;
      seen[t.s]++;
    }
  }
  // event simulation
  std::mt19937 rng(seed);
  std::uniform_int_distribution<int> dur(1, 20);
  std::vector<int> head(P.nq, 0), done(n, 0);
  std::vector<char> taken(nt, 0);
  struct Wk {
    int task = -1;
    long until = 0;   // running: finish time; waiting: -1
    bool finished = false;
  };
  std::vector<Wk> wk(W);
  const bool local = P.nq == 8;
  const int nxcd = local ? 1 + (int)(seed % 8u) : 1;   // XCDs that hold workers
  std::vector<int> owner(P.nq, -1), sys_xcd(n, -1);
  auto take = [&](int w) {
    const int xcd = w % nxcd;
    const int home = local ? xcd % P.nq : w % P.nq;
    for (int u = 0; u < P.nq; ++u) {
      const int q = (home + u) % P.nq;
      if (local) {
        if (owner[q] < 0) owner[q] = xcd;   // claim
        if (owner[q] != xcd) continue;
      }
      if (head[q] < P.qoff[q + 1] - P.qoff[q]) {
        const int x = P.qoff[q] + head[q]++;
        if (taken[x]) return -2;
        taken[x] = 1;
        if (local) {
          const int sy = P.tasks[x].s;
          if (sys_xcd[sy] >= 0 && sys_xcd[sy] != xcd) return -3;
          sys_xcd[sy] = xcd;
        }
        return x;
      }
    }
    return -1;
  };
  long now = 0;
  int left = nt;
  // start order of workers is shuffled every round
  std::vector<int> ord(W);
  for (int i = 0; i < W; ++i) ord[i] = i;
  while (left > 0) {
    bool progress = false;
    std::shuffle(ord.begin(), ord.end(), rng);
    for (int w : ord) {
      Wk& k = wk[w];
      if (k.finished) continue;
      if (k.task >= 0 && k.until > 0 && k.until <= now) {   // finish
        const PTask& t = P.tasks[k.task];
        done[t.s]++;
        --left;
        k.task = -1;
        k.until = 0;
        progress = true;
      }
      if (k.task < 0) {
        const int x = take(w);
        if (x == -2) return fail("double_take", w);
        if (x == -3) return fail("system_on_two_xcds", w);
        if (x < 0) {
          k.finished = true;
          continue;
        }
        k.task = x;
        k.until = -1;
        progress = true;
      }
      if (k.until < 0) {   // waiting
        const PTask& t = P.tasks[k.task];
        if (done[t.s] >= t.need) {
          if (done[t.s] > P.total[t.s]) return fail("overcount", t.s);
          k.until = now + dur(rng);
          progress = true;
        }
      }
    }
    // advance time to the next finish
    long nxt = -1;
    for (const Wk& k : wk)
      if (k.task >= 0 && k.until > 0 && (nxt < 0 || k.until < nxt)) nxt = k.until;
    if (nxt < 0) {
      if (!progress && left > 0) return fail("deadlock", left);
      continue;
    }
    now = std::max(now + 1, nxt);
  }
  for (int s = 0; s < n; ++s)
    if (done[s] != P.total[s]) return fail("incomplete", s, done[s]);
  std::printf("OK %d %ld %d\n", nt, now, P.nq);
  return 0;
}
