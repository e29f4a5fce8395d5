// Task plan of the persistent batched Cholesky factorisation (host code, no
// HIP dependency: the CPU tests build it with a plain C++ compiler).
//
// The blocked right-looking factorisation of every system is a sequence of
// stages (one per launch of the multi-launch sequence: a diagonal block, a
// panel column, a trailing update, ...); the tasks of one stage are
// independent (one workgroup each), and a stage may start once every task of
// the system's earlier stages is done.  A system's stages therefore need no
// barrier with other systems: the persistent kernel runs the stages of all
// systems of a ragged batch from device queues, so that small systems fill the
// machine while the large ones work through their longer sequences, and no
// launch boundary idles the device.
//
// Queues: with 8 or more systems there is one queue per XCD, and systems are
// spread over them by longest-processing-time on their estimated work (the
// tasks of a system then share one L2); with fewer systems there is a single
// queue.  Inside a queue the stages of its systems are ordered by the work
// their system has left (most first, ties by system, then stage), so the
// largest systems' stages come first; a system's own stages keep their order
// (its remaining work strictly decreases).  A workgroup takes the next task
// of its own queue and, once that queue is empty, of the others in turn.
//
// Deadlock freedom: a task only waits for tasks of its own system's earlier
// stages, which sit earlier in the same queue; tasks leave a queue in order,
// and a workgroup finishes its task before it takes another, so the earliest
// unfinished task of any queue has all its predecessors done and makes
// progress.
#pragma once

#include <algorithm>
#include <cstdint>
#include <numeric>
#include <vector>

namespace krr {

enum PTaskKind : int32_t {
  PT_DIAG = 0,    // diagonal block a = k (packed path: panel start b = K0; with its column update)
  PT_PCOL = 1,    // packed panel column a = k, tile-row group b = g (rows k+1+4g .. +3), panel start c = K0
  PT_PTRAIL = 2,  // packed trailing update: panel start a = K0, super-tile b, first trailing row c = K1
  PT_COL = 3,     // column update of tile (a = i, b = k) over the panel columns [c = K0, k)
  PT_TRSM = 4,    // panel solve of tile (a = i, b = k)
  PT_TRI = 5,     // trailing update: triangle index a, panel [b = K0, c = K1)
  PT_PHEAD = 6,   // packed panel head (column pairs): diagonal block a = K0, tile (K0+1, K0), diagonal block K0 + 1
  PT_PPAIR = 7    // packed column pair a = c, c + 1, tile-row group b = g (0: rows c+2, c+3 and the diagonal
                  // chain two columns ahead; g > 0: rows c+4g .. +3), panel start c = K0
};

enum PTaskFlags : int32_t {
  PF_PACK = 1,       // PT_PCOL: write the BF16 operand fragments of the column (PT_PPAIR: of column c + 1)
  PF_DIAG_NEXT = 2   // PT_PCOL, group 0: then factor diagonal block k + 1
};

struct PTask {
  int32_t kind, s;   // kind, system index in the batch
  int32_t a, b, c;   // kind-specific (see PTaskKind)
  int32_t flags;
  int32_t need;      // tasks of system s in its earlier stages (all must be done first)
  int32_t pad;
};

struct PPlan {
  std::vector<PTask> tasks;      // queue q holds tasks[qoff[q], qoff[q + 1])
  std::vector<int32_t> qoff;     // nq + 1
  std::vector<int32_t> total;    // tasks per system
  int nq = 1;
};

// Stages of one system with T tile rows, panel width Wp.  packed: the BF16
// packed path (diagonal block, then one stage per panel column with the next
// diagonal block carried by group 0, then the packed trailing update; with
// `pairs`, a panel of two or more columns runs as its head, one stage per
// pair of columns and, for an odd width, its last column on its own -- the
// stages of the launch sequence with column pairs);
// otherwise the matrix-core path (per column: column update, diagonal block,
// panel solve; then the trailing triangle).  `work` receives a relative work
// estimate per stage.
inline void plan_stages(int s, int T, int Wp, bool packed, std::vector<std::vector<PTask>>& stages,
                        std::vector<double>& work, bool pairs = false) {
  auto add = [&](std::vector<PTask>&& st, double w) {
    stages.push_back(std::move(st));
    work.push_back(w);
  };
  const double tile3 = 64.0 * 64.0 * 64.0;
  for (int K0 = 0; K0 < T; K0 += Wp) {
    const int K1 = std::min(K0 + Wp, T);
    if (packed && pairs && K1 - K0 >= 2) {
      add({PTask{PT_PHEAD, s, K0, 0, 0, 0, 0, 0}}, tile3 * 3.0);
      for (int c = K0; c + 1 < K1 && c + 2 < T; c += 2) {
        const int ng = 1 + std::max(0, (T - c - 4 + 3) / 4);
        const int32_t fl = (c + 2 < K1 || K1 < T) ? PF_PACK : 0;
        std::vector<PTask> st;
        for (int g = 0; g < ng; ++g) st.push_back(PTask{PT_PPAIR, s, c, g, K0, fl, 0, 0});
        add(std::move(st), tile3 * (double)(T - c - 2) * (2.0 + 2.0 * (c - K0)));
      }
      if ((K1 - K0) % 2 == 1 && K1 < T) {
        const int k = K1 - 1, ng = (T - k - 1 + 3) / 4;
        std::vector<PTask> st;
        for (int g = 0; g < ng; ++g) st.push_back(PTask{PT_PCOL, s, k, g, K0, PF_PACK, 0, 0});
        add(std::move(st), tile3 * (double)(T - k - 1) * (1.0 + 2.0 * (k - K0)));
      }
      if (K1 < T) {
        const int R = T - K1, NS = (R + 1) / 2, ntri = NS * (NS + 1) / 2;
        std::vector<PTask> st;
        for (int b = 0; b < ntri; ++b) st.push_back(PTask{PT_PTRAIL, s, K0, b, K1, 0, 0, 0});
        add(std::move(st), tile3 * 2.0 * (K1 - K0) * (double)R * (R + 1) / 2.0);
      }
    } else if (packed) {
      add({PTask{PT_DIAG, s, K0, K0, 0, 0, 0, 0}}, tile3);
      for (int k = K0; k < K1; ++k) {
        if (k + 1 >= T) continue;
        const int ng = (T - k - 1 + 3) / 4;
        const int32_t fl = ((k + 1 < K1 || K1 < T) ? PF_PACK : 0);
        std::vector<PTask> st;
        for (int g = 0; g < ng; ++g)
          st.push_back(PTask{PT_PCOL, s, k, g, K0, fl | ((g == 0 && k + 1 < K1) ? PF_DIAG_NEXT : 0), 0, 0});
        add(std::move(st), tile3 * (double)(T - k - 1) * (1.0 + 2.0 * (k - K0)));
      }
      if (K1 < T) {
        const int R = T - K1, NS = (R + 1) / 2, ntri = NS * (NS + 1) / 2;
        std::vector<PTask> st;
        for (int b = 0; b < ntri; ++b) st.push_back(PTask{PT_PTRAIL, s, K0, b, K1, 0, 0, 0});
        add(std::move(st), tile3 * 2.0 * (K1 - K0) * (double)R * (R + 1) / 2.0);
      }
    } else {
      for (int k = K0; k < K1; ++k) {
        if (k > K0) {
          std::vector<PTask> st;
          for (int i = k; i < T; ++i) st.push_back(PTask{PT_COL, s, i, k, K0, 0, 0, 0});
          add(std::move(st), tile3 * 2.0 * (k - K0) * (T - k));
        }
        add({PTask{PT_DIAG, s, k, K0, 0, 0, 0, 0}}, tile3);
        if (k + 1 < T) {
          std::vector<PTask> st;
          for (int i = k + 1; i < T; ++i) st.push_back(PTask{PT_TRSM, s, i, k, 0, 0, 0, 0});
          add(std::move(st), tile3 * (T - k - 1));
        }
      }
      if (K1 < T) {
        const int R = T - K1;
        std::vector<PTask> st;
        for (int bx = 0; bx < R * (R + 1) / 2; ++bx) st.push_back(PTask{PT_TRI, s, bx, K0, K1, 0, 0, 0});
        add(std::move(st), tile3 * 2.0 * (K1 - K0) * (double)R * (R + 1) / 2.0);
      }
    }
  }
}

// Plan for the systems with T[s] > 0 and active[s] != 0 (the others get no
// task); system s takes panels of Wp[s] tiles.  nq_max: 8 (one queue per
// XCD) or 1.  pairs: the packed path's column-pair stages.
inline PPlan build_plan(const std::vector<int>& T, const std::vector<int>& active, const std::vector<int>& Wp,
                        bool packed, int nq_max, bool pairs = false) {
  const int n = (int)T.size();
  PPlan P;
  P.total.assign(n, 0);
  struct Stage {
    int s, idx;
    double left;   // the system's work from this stage on
    std::vector<PTask> tasks;
  };
  std::vector<std::vector<Stage>> per(n);
  std::vector<double> tot(n, 0.0);
  int n_act = 0;
  for (int s = 0; s < n; ++s) {
    if (T[s] <= 0 || !active[s]) continue;
    ++n_act;
    std::vector<std::vector<PTask>> st;
    std::vector<double> w;
    plan_stages(s, T[s], Wp[s], packed, st, w, pairs);
    double left = std::accumulate(w.begin(), w.end(), 0.0);
    tot[s] = left;
    int need = 0;
    for (size_t j = 0; j < st.size(); ++j) {
      for (PTask& t : st[j]) t.need = need;
      need += (int)st[j].size();
      per[s].push_back(Stage{s, (int)j, left, std::move(st[j])});
      left -= w[j];
    }
    P.total[s] = need;
  }
  P.nq = (n_act >= nq_max) ? nq_max : 1;
  // systems to queues: longest processing time first
  std::vector<int> order;
  for (int s = 0; s < n; ++s)
    if (!per[s].empty()) order.push_back(s);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return tot[x] > tot[y]; });
  std::vector<double> load(P.nq, 0.0);
  std::vector<std::vector<int>> qsys(P.nq);
  for (int s : order) {
    const int q = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[q] += tot[s];
    qsys[q].push_back(s);
  }
  P.qoff.assign(P.nq + 1, 0);
  for (int q = 0; q < P.nq; ++q) {
    std::vector<const Stage*> sts;
    for (int s : qsys[q])
      for (const Stage& g : per[s]) sts.push_back(&g);
    std::stable_sort(sts.begin(), sts.end(), [](const Stage* x, const Stage* y) {
      if (x->left != y->left) return x->left > y->left;
      if (x->s != y->s) return x->s < y->s;
      return x->idx < y->idx;
    });
    for (const Stage* g : sts) P.tasks.insert(P.tasks.end(), g->tasks.begin(), g->tasks.end());
    P.qoff[q + 1] = (int32_t)P.tasks.size();
  }
  return P;
}

}  // namespace krr
