// Internal declarations of libabcore (device layout, launch helpers).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

#include "abcore.h"

namespace abc {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
// Per-wave local queue (LDS) used to batch frontier pushes, Sec. IV-A's
// warp-local queue sized for a 64-lane wavefront.
constexpr int kLocalQueue = 512;

// GCC+ class encoding in the working degree array (Sec. IV-B, Lemma 1):
// certain members are never decremented, certain non-members never counted.
constexpr int32_t kDegIn = 0x7FFFFFFF;
constexpr int32_t kDegOut = -1;
// Largest usable threshold: kDegIn must stay above every threshold.
constexpr int32_t kMaxThreshold = 0x7FFFFFFE;

// Peel bookkeeping shared by every multi-round computation.  One instance
// lives in device memory per handle.  The queue Q is append-only for the
// whole computation (each vertex enters it at most once), so a round is the
// index range [lo, hi) of Q; the last workgroup of a round launch advances
// the range to the items appended during that round.
struct PeelState {
  int32_t tail;       // append cursor into Q (atomic)
  int32_t lo, hi;     // current round = Q[lo, hi)
  int32_t rounds;     // non-empty rounds executed
  uint32_t finished;  // workgroups done in the current launch
  int32_t k;          // core decomposition: current level
  int32_t next_k;     // core decomposition: level of the next scan
  int32_t alive_cur;  // core decomposition: entries in the current alive list
  int32_t alive_next; // core decomposition: entries written to the next list
  int32_t alive_sel;  // which alive buffer is current (0/1)
  int32_t min_alive;  // smallest degree among kept vertices of the last scan
  int32_t done;       // computation finished
  int32_t max_core;   // largest level with removals
  int32_t status;     // device-side status for updates (0 ok)
  int32_t aux0, aux1; // small results (uncertain count, labels, answer bits)
  int32_t first;      // size of the initial frontier (scan phase)
  int64_t entries;    // adjacency entries read by peel rounds
  int64_t launches;   // round/step launches that did work
};

// Dynamic edge storage for updates after the build (Sec. V).  Deleted CSR
// entries are tombstoned in place as ~col (negative, order-preserving after
// decoding); inserted edges live in per-vertex singly linked lists of
// half-edges.  Half-edge 2j is the entry of pair j in the upper row, 2j+1 in
// the lower row; a deleted half-edge stores ~other.
struct Delta {
  int32_t *head = nullptr;   // n, -1 = empty list
  int32_t *next = nullptr;   // 2*cap
  int32_t *other = nullptr;  // 2*cap: neighbour id (negative = deleted)
  int64_t cap = 0;
  int64_t count = 0;         // pairs used
};

struct Graph {
  int device = 0;
  int32_t nU = 0, nL = 0;
  int64_t n = 0;
  int64_t m = 0;      // current distinct edges
  int64_t m_csr = 0;  // pairs stored in the CSR at build
  int64_t *off = nullptr;   // n+1
  int32_t *cols = nullptr;  // 2*m_csr
  int32_t *deg0 = nullptr;  // current degree of every vertex
  int32_t *deg = nullptr;   // working degree (per computation)
  int32_t *queue = nullptr; // n + padding
  int32_t *list = nullptr;  // n: scratch vertex list (uncertain set, alive lists)
  int32_t *list2 = nullptr; // n: second alive list
  PeelState *state = nullptr;
  PeelState *h_state = nullptr;  // pinned host mirror
  int32_t *core = nullptr;  // cached core numbers
  bool core_valid = false;
  int32_t max_core = 0;
  int32_t *comp = nullptr;  // component labels
  bool comp_valid = false;
  int32_t *parent = nullptr; // union-find scratch
  bool has_tombstones = false;
  Delta delta;
  int version = 0;
  // options
  int peel_mode = 1;
  int grid = 0;            // 0 = derived from the device
  int rounds_per_sync = 16;
  int cu_count = 256;
  // peel-kernel timing (ABCORE_OPT_TIMING)
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;  // recorded pairs
  std::vector<hipEvent_t> event_pool;
  int64_t timed_launches = 0;
};

// Peel flavours.
enum PeelKind : int { kGCC = 0, kGCCPlus = 1, kKCore = 2 };

// Parameters of a peel round, passed by value to kernels.
struct PeelArgs {
  const int64_t *off;
  const int32_t *cols;
  int32_t *deg;
  int32_t *queue;
  PeelState *st;
  const int32_t *ins_head;  // nullable
  const int32_t *ins_next;
  const int32_t *ins_other;
  int32_t *core;            // kKCore: output core numbers
  int32_t nU;
  int32_t thrU, thrL;       // thresholds (kKCore: k + 1 read from st)
};

void set_error(const char *fmt, ...);

// Launchers (defined in the .hip files).
hipError_t launch_init_state(PeelState *st, hipStream_t s);
hipError_t launch_scan_gcc(Graph &g, int32_t thrU, int32_t thrL, hipStream_t s);
hipError_t launch_scan_component_of(Graph &g, int32_t thrU, int32_t thrL, int32_t x,
                                    int32_t y, hipStream_t s);
hipError_t launch_peel_rounds(Graph &g, PeelKind kind, int32_t thrU, int32_t thrL,
                              int rounds, hipStream_t s);
hipError_t launch_pack(Graph &g, int32_t thrU, int32_t thrL, uint32_t *bits,
                       hipStream_t s);
hipError_t launch_pack_from_core(Graph &g, int32_t k, uint32_t *bits, hipStream_t s);
hipError_t launch_classify(Graph &g, int32_t thrU, int32_t thrL, int32_t dl, int32_t dq,
                           hipStream_t s);
hipError_t launch_restricted_init(Graph &g, int32_t thrU, int32_t thrL, int32_t dl,
                                  hipStream_t s);
hipError_t launch_kcore_init(Graph &g, hipStream_t s);
hipError_t launch_kcore_steps(Graph &g, int steps, hipStream_t s);
hipError_t launch_cc(Graph &g, int32_t only_label, hipStream_t s);

int peel_grid(const Graph &g);

}  // namespace abc
