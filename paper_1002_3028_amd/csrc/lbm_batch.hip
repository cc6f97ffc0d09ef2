// lbm_batch.hip -- many resident jets advanced by persistent launches.
// Population buffers are carved out of one device arena (the HBM budget) by
// a first-fit allocator.  Active jets are grouped into cohorts whose buffers
// together fit the Infinity Cache; a run of k steps advances cohort after
// cohort, each with one launch per step over a flat tile list covering the
// cohort's jets, so every cohort's working set stays cache-resident for its
// k steps.  Each cohort has fixed device arrays (descriptors, tile prefix
// sums, header) and the launch configuration never changes with the set of
// jets, so the captured graph of k steps of a cohort is replayed as jets come
// and go.
//
// A batch holds jets of several storage forms (the batch's own unless a
// jet's configuration names another); each cohort holds one form, so that
// a serving loop can route some requests to another form without a second
// batch, whose groups would double the launches per group.
//
// Runs only enqueue, so that a serving loop can queue the next group before
// it retires and admits jets: the cohort lists exist twice (a rebuild writes
// the copy that the groups in flight do not read), every group records an
// event, profiles are extracted on a stream of their own after the group in
// which the jet finished, and admission and retirement do not wait for the
// batch's stream (each slot keeps its block for the property table and inlet
// rows from one jet to the next, so admission allocates only when a jet
// needs more than any earlier jet of its slot).
#include <algorithm>
#include <cstring>
#include <map>
#include <tuple>

#include "lbm_runtime.hpp"

using namespace lbmx;

namespace {

struct Slot {
  bool used = false;
  int prec = LBM_PREC_FP32;  // the jet's storage form
  int shape = 0;             // tile shape of its cohort (set by rebuild)
  lbm_config cfg{};
  std::vector<double> nu_tab, al_tab;
  JetDesc desc{};
  size_t off = 0, bytes = 0;
  float4 *d_table = nullptr;  // both inside the slot's block `aux`
  float4 *d_inlet = nullptr;
  int64_t step = 0, target = 0;
  int32_t flip = 0;       // state after s steps in buf[(s + flip) & 1]
  int64_t done_seq = -1;  // the group in which the jet reached its target
};

// Device block of a slot for its jet's property table and inlet rows; kept
// from one jet to the next, so that admission needs no allocation.  The
// first kPoolSlots slots take kBlockBytes each from one pool allocated with
// the batch; a jet that needs more gets a larger block of its own, and the
// block it replaces is freed only with the batch (freeing device memory
// would wait for the device, stalling a pipelined loop).
constexpr size_t kBlockBytes = size_t(64) << 10;  // the table and 7 inlet rows of 512 nodes
constexpr int32_t kPoolSlots = 512;
struct SlotBlock {
  void *p = nullptr;  // device
  void *h = nullptr;  // pinned host staging of the same size (the upload is
                      // then an asynchronous copy in stream order)
  size_t cap = 0;
  bool own = false;   // allocated for this slot (else a part of the pool)
};

// First-fit free list over [0, size) with 256-byte granules.
struct Arena {
  std::map<size_t, size_t> free_;  // offset -> size
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t *off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, noff = it->first + bytes;
        free_.erase(it);
        if (rest) free_[noff] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
};

}  // namespace

struct lbm_batch {
  int device = 0;
  int prec = LBM_PREC_FP32;
  int layout = LBM_LAYOUT_TWO_BUFFERS;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  size_t budget = 0, used = 0;
  void *arena_mem = nullptr;
  Arena arena;
  std::vector<Slot> slots;
  std::vector<SlotBlock> blocks;   // per slot
  void *pool_d = nullptr, *pool_h = nullptr;  // the first slots' blocks
  std::vector<std::pair<void *, void *>> replaced;  // blocks freed with the batch
  // cohort lists, two copies (index `copy`): per cohort the compact list of
  // its jets, the tile prefix sums and the header
  JetDesc *d_jets = nullptr;
  JetDesc *d_slot_desc = nullptr;  // per slot, for the single-jet helper kernels
  int32_t *d_tiles = nullptr;
  BatchHdr *d_hdr = nullptr;
  int32_t max_cohorts = 0;
  int32_t n_cohorts = 0;
  int32_t copy = 1;                // the copy the last rebuild wrote
  int32_t copy_cohorts[2] = {0, 0};  // headers written in each copy
  bool copy_used[2] = {false, false};
  hipEvent_t copy_done[2] = {};    // after the last group that read each copy
  // group completion: group n records done[n % RING] after its launches
  static constexpr int RING = 16;
  int64_t seq = 0;                 // groups enqueued
  hipEvent_t done[RING] = {};
  // device time of the groups: start[n % RING] before group n's launches;
  // summed up to group `timed` - 1 when waits find them complete
  hipEvent_t start[RING] = {};
  int64_t timed = 0, timed_groups = 0;
  double device_ms = 0.0;
  hipStream_t io = nullptr;        // profile and moment extraction
  hipStream_t cap = nullptr;       // graph capture (never holds work)
  hipEvent_t mark = nullptr;       // "everything enqueued so far" on `stream`
  JetDesc *h_slot = nullptr;       // pinned staging of each slot's descriptor
  int32_t *h_zero = nullptr;       // pinned 0 (a slot's instability flag)
  // 0: one cohort.  Two cohorts run at once (two streams), and together they
  // fill the 256 MiB Infinity Cache.
  size_t cohort_bytes = size_t(128) << 20;
  int32_t *d_flags = nullptr;
  // pinned staging of what rebuild uploads (cohort after cohort, compact), so
  // that the uploads are asynchronous copies ordered before the launches; two
  // copies, as the device lists
  JetDesc *h_jets = nullptr;   // 2 x max_slots descriptors
  int32_t *h_tiles = nullptr;  // 2 x (max_slots + max_cohorts) tile prefix sums
  BatchHdr *h_hdr = nullptr;   // 2 x max_cohorts
  Scratch scratch;
  std::vector<int32_t> active;  // slots in the compact list, in order
  bool dirty = true;
  int shape = -1;       // -1: auto
  int32_t wg = 0;       // 0: auto
  // storage form, tile shape and grid of each cohort of each copy of the
  // lists (set by rebuild)
  struct Cohort {
    int prec = LBM_PREC_FP32, shape = 0;
    int32_t grid = 0;
  };
  std::vector<Cohort> cohorts[2];
  // (k, shape, grid, cohort, copy, storage form)
  std::map<std::tuple<int, int, int, int, int, int>, hipGraphExec_t> graphs;
  // cohorts alternate between the batch's stream and a second one, so that
  // one cohort's launches fill the device while the other's start or drain
  static constexpr int MAX_STREAMS = 4;
  int32_t nstreams = 2;
  hipStream_t side[MAX_STREAMS - 1] = {};  // streams 1.. (stream 0 is `stream`)
  hipEvent_t fork = nullptr;
  hipEvent_t join[MAX_STREAMS - 1] = {};
};

namespace {

// The requested (or default) shape for a storage form.
int pick_shape(const lbm_batch *b, int prec) {
  if (b->layout == LBM_LAYOUT_SINGLE) return 0;  // the in-place kernel's tiles
  return b->shape >= 0 ? b->shape : default_tile_shape(prec);
}

bool storage_form(int prec) {
  return prec == LBM_PREC_FP32 || prec == LBM_PREC_FP16DEV || prec == LBM_PREC_BF16DEV ||
         prec == LBM_PREC_FP16SR;
}

// A jet's storage form: its configuration's, or the batch's for 0.
int jet_prec(const lbm_batch *b, const lbm_config *cfg) {
  return cfg->precision == 0 ? b->prec : cfg->precision;
}

void drop_graphs(lbm_batch *b) {
  for (auto &kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  b->graphs.clear();
}

// Pointers of copy `cp` of the cohort lists and of their staging.
struct Lists {
  JetDesc *dj, *hj;
  int32_t *dt, *ht;
  BatchHdr *dh, *hh;
};
Lists lists_of(const lbm_batch *b, int32_t cp) {
  const size_t ms = b->slots.size(), mc = (size_t)b->max_cohorts;
  return {b->d_jets + cp * mc * ms, b->h_jets + cp * ms,
          b->d_tiles + cp * mc * (ms + 1), b->h_tiles + cp * (ms + mc),
          b->d_hdr + cp * mc, b->h_hdr + cp * mc};
}

// Rebuild and upload the cohorts: active jets by storage form (the batch's
// first), in slot order within a form; a new cohort at every change of form
// and whenever the next jet's buffers would take the cohort past
// cohort_bytes.  Written into the copy of the lists that the groups in
// flight do not read.
int rebuild(lbm_batch *b) {
  const int32_t ms = (int32_t)b->slots.size();
  std::vector<int32_t> order;
  for (int32_t s = 0; s < ms; ++s)
    if (b->slots[s].used && b->slots[s].step < b->slots[s].target) order.push_back(s);
  // by storage form, the batch's first; slot order within a form
  const auto form_key = [&](int32_t s) {
    const int p = b->slots[s].prec;
    return std::make_pair(p != b->prec, p);
  };
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t x, int32_t y) { return form_key(x) < form_key(y); });
  // storage forms after each position's own (cohorts kept for them: a form
  // change always opens a cohort; max_cohorts >= the forms present, since it
  // is at least min(max_slots, 64))
  std::vector<int32_t> later(order.size(), 0);
  for (size_t q = order.size(); q-- > 1;)
    later[q - 1] = later[q] + (b->slots[order[q]].prec != b->slots[order[q - 1]].prec ? 1 : 0);
  std::vector<std::vector<JetDesc>> jets(1);
  std::vector<std::vector<int32_t>> start(1, std::vector<int32_t>(1, 0));
  std::vector<size_t> bytes(1, 0);
  std::vector<lbm_batch::Cohort> meta(1);
  b->active.clear();
  for (size_t q = 0; q < order.size(); ++q) {
    const int32_t s = order[q];
    Slot &sl = b->slots[s];
    const bool other_form = !jets.back().empty() && meta.back().prec != sl.prec;
    const bool full = b->cohort_bytes && !jets.back().empty() &&
                      bytes.back() + sl.bytes > b->cohort_bytes &&
                      (int32_t)jets.size() + later[q] < b->max_cohorts;
    if (other_form || full) {
      jets.emplace_back();
      start.emplace_back(1, 0);
      bytes.push_back(0);
      meta.emplace_back();
    }
    if (jets.back().empty()) {
      meta.back().prec = sl.prec;
      meta.back().shape = pick_shape(b, sl.prec);
    }
    const int shape = meta.back().shape;
    sl.shape = shape;
    int32_t tx;
    const int nt = tiles_of(&sl.cfg, shape, &tx);
    sl.desc.tiles_x = tx;
    sl.desc.step0 = sl.step;
    sl.desc.flip = sl.flip;
    jets.back().push_back(sl.desc);
    start.back().push_back(start.back().back() + nt);
    bytes.back() += sl.bytes;
    b->active.push_back(s);
  }
  // the groups that read this copy last, and the uploads from its staging
  // queued before them, must be done before either is rewritten
  const int32_t cp = 1 - b->copy;
  if (b->copy_used[cp]) LBM_HIP(hipEventSynchronize(b->copy_done[cp]));
  const Lists L = lists_of(b, cp);
  b->n_cohorts = jets.back().empty() && jets.size() == 1 ? 0 : (int32_t)jets.size();
  // cohorts that emptied keep an empty tile list
  const int32_t nh = std::max(b->copy_cohorts[cp], b->n_cohorts);
  size_t jo = 0, to = 0;  // staging offsets
  for (int32_t c = 0; c < nh; ++c) {
    const int32_t n = c < b->n_cohorts ? (int32_t)jets[c].size() : 0;
    L.hh[c] = BatchHdr{n, {0, 0, 0}};
    if (n > 0) std::memcpy(L.hj + jo, jets[c].data(), n * sizeof(JetDesc));
    if (n > 0) std::memcpy(L.ht + to, start[c].data(), (n + 1) * sizeof(int32_t));
    else L.ht[to] = 0;
    if (n > 0)
      LBM_HIP(hipMemcpyAsync(L.dj + (size_t)c * ms, L.hj + jo, n * sizeof(JetDesc),
                             hipMemcpyHostToDevice, b->stream));
    LBM_HIP(hipMemcpyAsync(L.dt + (size_t)c * (ms + 1), L.ht + to, (n + 1) * sizeof(int32_t),
                           hipMemcpyHostToDevice, b->stream));
    jo += n;
    to += n + 1;
  }
  if (nh > 0)
    LBM_HIP(hipMemcpyAsync(L.dh, L.hh, nh * sizeof(BatchHdr), hipMemcpyHostToDevice,
                           b->stream));
  b->copy_cohorts[cp] = b->n_cohorts;
  b->copy = cp;
  // persistent grid of fixed size per cohort (graphs stay valid as jets come
  // and go): by default the workgroups the device holds at once
  for (lbm_batch::Cohort &m : meta) {
    int32_t g = b->wg > 0 ? b->wg
                          : resident_workgroups(m.shape, m.prec, b->layout == LBM_LAYOUT_SINGLE);
    m.grid = (g + 7) / 8 * 8;
  }
  b->cohorts[cp] = meta;
  b->dirty = false;
  return LBM_OK;
}

// Launch group k of cohort c on stream st (capturing its graph on the
// capture stream the first time).
int run_group(lbm_batch *b, int32_t k, int32_t c, hipStream_t st) {
  const lbm_batch::Cohort &m = b->cohorts[b->copy][c];
  const int shape = m.shape, prec = m.prec;
  const int32_t grid = m.grid;
  int nsh;
  const int32_t np = tile_shapes(&nsh)[shape].steps == 2 ? k / 2 : 0;
  const int32_t ms = (int32_t)b->slots.size();
  auto key = std::make_tuple((int)k, shape, (int)grid, (int)c, (int)b->copy, prec);
  auto it = b->graphs.find(key);
  if (it == b->graphs.end()) {
    const Lists L = lists_of(b, b->copy);
    JetDesc *jets = L.dj + (size_t)c * ms;
    const int32_t *tiles = L.dt + (size_t)c * (ms + 1);
    const BatchHdr *hdr = L.dh + c;
    hipStream_t cs = b->cap;
    hipGraph_t g;
    LBM_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    int rc = LBM_OK;
    // k / 2 pair launches with a two-step shape (one single step if k is
    // odd), else k single steps
    for (int32_t q = 0; q < np && !rc; ++q)
      rc = launch_step(shape, prec, grid, cs, jets, tiles, hdr, 2 * q, q & 1, 2, b->d_flags);
    for (int32_t q = 2 * np; q < k && !rc; ++q)
      rc = b->layout == LBM_LAYOUT_SINGLE
               ? launch_aa_step(prec, grid, cs, jets, tiles, hdr, q, b->d_flags)
               : launch_step(shape, prec, grid, cs, jets, tiles, hdr, q, np & 1, 1, b->d_flags);
    if (!rc) rc = launch_advance(cs, jets, hdr, ms, k, np);
    const hipError_t e = hipStreamEndCapture(cs, &g);
    if (rc || e != hipSuccess) return rc ? rc : LBM_EDEVICE;
    hipGraphExec_t ex;
    const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return LBM_EDEVICE;
    it = b->graphs.emplace(key, ex).first;
  }
  LBM_HIP(hipGraphLaunch(it->second, st));
  return LBM_OK;
}

// Make the extraction stream wait until the slot's state is final: the group
// in which its jet reached its target, or, for a jet still running, all the
// work enqueued so far.
int io_after(lbm_batch *b, const Slot &sl) {
  if (sl.done_seq >= 0) {
    LBM_HIP(hipStreamWaitEvent(b->io, b->done[sl.done_seq % lbm_batch::RING], 0));
  } else {
    LBM_HIP(hipEventRecord(b->mark, b->stream));
    LBM_HIP(hipStreamWaitEvent(b->io, b->mark, 0));
  }
  return LBM_OK;
}

Slot *slot_of(lbm_batch *b, int32_t s) {
  if (!b || s < 0 || s >= (int32_t)b->slots.size() || !b->slots[s].used) return nullptr;
  return &b->slots[s];
}

}  // namespace

extern "C" {

int lbm_batch_create(size_t budget_bytes, int32_t max_slots, int32_t precision,
                     void *hip_stream, lbm_batch **out) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  if (max_slots < 1 || max_slots > 65536 || budget_bytes < 256) return LBM_EINVAL;
  if (precision != LBM_PREC_FP32 && precision != LBM_PREC_FP16DEV &&
      precision != LBM_PREC_BF16DEV && precision != LBM_PREC_FP16SR)
    return LBM_EINVAL;
  lbm_batch *b = new (std::nothrow) lbm_batch();
  if (!b) return LBM_ENOMEM;
  b->prec = precision;
  b->budget = budget_bytes & ~size_t(255);
  b->slots.resize(max_slots);
  b->blocks.resize(max_slots);
  b->max_cohorts = std::min<int32_t>(max_slots, 64);
  (void)hipGetDevice(&b->device);
  const size_t mc = (size_t)b->max_cohorts;
  bool ok = hipMalloc(&b->arena_mem, b->budget) == hipSuccess &&
            hipMalloc(&b->d_jets, 2 * mc * max_slots * sizeof(JetDesc)) == hipSuccess &&
            hipMalloc(&b->d_slot_desc, max_slots * sizeof(JetDesc)) == hipSuccess &&
            hipMalloc(&b->d_tiles, 2 * mc * (max_slots + 1) * sizeof(int32_t)) == hipSuccess &&
            hipMalloc(&b->d_hdr, 2 * mc * sizeof(BatchHdr)) == hipSuccess &&
            hipMalloc(&b->d_flags, max_slots * sizeof(int32_t)) == hipSuccess &&
            hipHostMalloc(&b->h_jets, 2 * max_slots * sizeof(JetDesc), hipHostMallocDefault) ==
                hipSuccess &&
            hipHostMalloc(&b->h_tiles, 2 * (max_slots + mc) * sizeof(int32_t),
                          hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc(&b->h_hdr, 2 * mc * sizeof(BatchHdr), hipHostMallocDefault) ==
                hipSuccess &&
            hipHostMalloc(&b->h_slot, max_slots * sizeof(JetDesc), hipHostMallocDefault) ==
                hipSuccess &&
            hipHostMalloc(&b->h_zero, sizeof(int32_t), hipHostMallocDefault) == hipSuccess;
  const size_t pooled = (size_t)std::min(max_slots, kPoolSlots);
  ok = ok && hipMalloc(&b->pool_d, pooled * kBlockBytes) == hipSuccess &&
       hipHostMalloc(&b->pool_h, pooled * kBlockBytes, hipHostMallocDefault) == hipSuccess;
  for (size_t q = 0; ok && q < pooled; ++q)
    b->blocks[q] = SlotBlock{(char *)b->pool_d + q * kBlockBytes,
                             (char *)b->pool_h + q * kBlockBytes, kBlockBytes, false};
  // The runtime spreads a process's streams over a few hardware queues (four
  // by default), and work on streams that share a queue runs in submission
  // order.  The batch's own streams are created back to back -- the cohort
  // streams first, then extraction and capture -- so that they land on
  // distinct queues: with a caller's stream, or with other streams created in
  // between, the second cohort stream shared the first one's queue in one
  // batch out of two, and the cohorts ran one after the other.
  if (ok && hip_stream) {
    b->stream = (hipStream_t)hip_stream;
  } else if (ok) {
    ok = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) == hipSuccess;
    b->own_stream = ok;
  }
  // the second cohort stream of the default two; one stream if it cannot be had
  if (ok && lbm_batch_set_streams(b, 2) != LBM_OK) b->nstreams = 1;
  ok = ok && hipStreamCreateWithFlags(&b->io, hipStreamNonBlocking) == hipSuccess &&
       hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) == hipSuccess &&
       hipEventCreateWithFlags(&b->mark, hipEventDisableTiming) == hipSuccess;
  for (int q = 0; ok && q < 2; ++q)
    ok = hipEventCreateWithFlags(&b->copy_done[q], hipEventDisableTiming) == hipSuccess;
  for (int q = 0; ok && q < lbm_batch::RING; ++q)
    ok = hipEventCreateWithFlags(&b->done[q], hipEventDefault) == hipSuccess &&
         hipEventCreateWithFlags(&b->start[q], hipEventDefault) == hipSuccess;
  if (ok) {
    *b->h_zero = 0;
    std::vector<int32_t> zeros(max_slots, 0);
    std::vector<BatchHdr> hz(2 * mc, BatchHdr{0, {0, 0, 0}});
    std::vector<int32_t> tz(2 * mc * (max_slots + 1), 0);
    ok = hipMemcpy(b->d_flags, zeros.data(), max_slots * sizeof(int32_t),
                   hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(b->d_hdr, hz.data(), hz.size() * sizeof(BatchHdr), hipMemcpyHostToDevice) ==
             hipSuccess &&
         hipMemcpy(b->d_tiles, tz.data(), tz.size() * sizeof(int32_t), hipMemcpyHostToDevice) ==
             hipSuccess;
  }
  if (!ok) {
    lbm_batch_destroy(b);
    return LBM_ENOMEM;
  }
  b->arena.reset(b->budget);
  *out = b;
  return LBM_OK;
}

int lbm_batch_jet_bytes(const lbm_batch *b, const lbm_config *cfg, size_t *bytes) {
  if (!b || !cfg || !bytes) return LBM_EINVAL;
  const int rc = validate_config(cfg, false);
  if (rc) return rc;
  const int prec = jet_prec(b, cfg);
  if (!storage_form(prec)) return LBM_EINVAL;
  *bytes = n_buffers(b->layout) * buffer_bytes(cfg, prec);
  return LBM_OK;
}

int lbm_batch_set_layout(lbm_batch *b, int32_t layout) {
  if (!b || (layout != LBM_LAYOUT_TWO_BUFFERS && layout != LBM_LAYOUT_SINGLE)) return LBM_EINVAL;
  for (const Slot &s : b->slots)
    if (s.used) return LBM_ESTATE;
  LBM_HIP(hipStreamSynchronize(b->stream));
  b->layout = layout;
  b->dirty = true;
  drop_graphs(b);
  return LBM_OK;
}

int lbm_batch_admit(lbm_batch *b, const lbm_config *cfg, int32_t n_t, const double *ux,
                    const double *ur, const double *T, int64_t target_steps, int32_t *slot) {
  if (!b || !cfg || !slot || target_steps < 0) return LBM_EINVAL;
  *slot = -1;
  int rc = validate_config(cfg, false);
  if (rc) return rc;
  int32_t s = -1;
  for (int32_t q = 0; q < (int32_t)b->slots.size(); ++q)
    if (!b->slots[q].used) {
      s = q;
      break;
    }
  if (s < 0) return LBM_ENOMEM;
  const int prec = jet_prec(b, cfg);
  if (!storage_form(prec)) return LBM_EINVAL;
  const size_t one = buffer_bytes(cfg, prec);
  const size_t need = n_buffers(b->layout) * one;
  size_t off;
  if (!b->arena.alloc(need, &off)) return LBM_ENOMEM;
  Slot &sl = b->slots[s];
  sl = Slot();
  sl.cfg = *cfg;
  sl.prec = prec;
  sl.cfg.precision = prec;
  sl.cfg.layout = b->layout;
  if (cfg->table_n > 0) {
    sl.nu_tab.assign(cfg->nu_mult, cfg->nu_mult + cfg->table_n);
    sl.al_tab.assign(cfg->alpha_mult, cfg->alpha_mult + cfg->table_n);
    sl.cfg.nu_mult = sl.nu_tab.data();
    sl.cfg.alpha_mult = sl.al_tab.data();
  }
  std::vector<float4> rows;
  if ((rc = make_inlet(&sl.cfg, n_t, ux, ur, T, rows))) {
    b->arena.release(off, need);
    return rc;
  }
  std::vector<float4> table = make_table(&sl.cfg);
  // the slot's block holds the table and the inlet rows; a jet that needs
  // more than the block holds gets a larger one (at least twice the size),
  // and the old one waits for the batch's end
  const size_t tb = align256(table.size() * sizeof(float4));
  const size_t ib = align256(rows.size() * sizeof(float4));
  SlotBlock &blk = b->blocks[s];
  if (blk.cap < tb + ib) {
    const size_t cap = std::max({tb + ib, 2 * blk.cap, kBlockBytes});
    SlotBlock nb{nullptr, nullptr, cap, true};
    if (hipMalloc(&nb.p, cap) != hipSuccess ||
        hipHostMalloc(&nb.h, cap, hipHostMallocDefault) != hipSuccess) {
      if (nb.p) (void)hipFree(nb.p);
      b->arena.release(off, need);
      sl = Slot();
      return LBM_ENOMEM;
    }
    if (blk.own) b->replaced.emplace_back(blk.p, blk.h);
    blk = nb;
  }
  sl.d_table = (float4 *)blk.p;
  sl.d_inlet = (float4 *)((char *)blk.p + tb);
  sl.used = true;
  sl.off = off;
  sl.bytes = need;
  sl.step = 0;
  sl.target = target_steps;
  JetDesc &d = sl.desc;
  fill_desc(d, &sl.cfg);
  d.buf[0] = (char *)b->arena_mem + off;
  d.buf[1] = b->layout == LBM_LAYOUT_SINGLE ? d.buf[0] : (char *)b->arena_mem + off + one;
  d.table = sl.d_table;
  d.inlet = sl.d_inlet;
  d.n_t = n_t == 0 ? 1 : n_t;
  d.target = target_steps;
  d.step0 = 0;
  d.slot = s;
  int32_t tx;
  tiles_of(&sl.cfg, pick_shape(b, prec), &tx);
  d.tiles_x = tx;
  // Uploads and initialisation are queued on the batch's stream, behind the
  // groups in flight.  Those no longer touch this slot's memory: the jet it
  // held last was retired only once its last group had finished, and later
  // groups skip it (its step count is at its target).
  // (the staging of this slot is free: its last upload preceded the groups
  // of the jet retired from the slot)
  b->h_slot[s] = d;
  std::memcpy(blk.h, table.data(), table.size() * sizeof(float4));
  std::memcpy((char *)blk.h + tb, rows.data(), rows.size() * sizeof(float4));
  LBM_HIP(hipMemcpyAsync(blk.p, blk.h, tb + ib, hipMemcpyHostToDevice, b->stream));
  LBM_HIP(hipMemcpyAsync(b->d_slot_desc + s, b->h_slot + s, sizeof(JetDesc),
                         hipMemcpyHostToDevice, b->stream));
  LBM_HIP(hipMemcpyAsync(b->d_flags + s, b->h_zero, sizeof(int32_t), hipMemcpyHostToDevice,
                         b->stream));
  const float4 u0 =
      make_float4((float)cfg->rho0, (float)cfg->ux0, (float)cfg->ur0, (float)cfg->T0);
  for (int64_t q = n_buffers(b->layout) - 1; q >= 0 && !rc; --q) {
    const int32_t v = state_view_of(b->layout, q, 0);
    rc = launch_init(prec, b->stream, b->d_slot_desc + s, &sl.cfg, q, v, nullptr, u0);
    if (!rc) rc = launch_ghost_fill(prec, b->stream, b->d_slot_desc + s, &sl.cfg, q, v);
  }
  if (rc) return rc;
  b->used += sl.bytes;
  b->dirty = true;
  *slot = s;
  return LBM_OK;
}

int lbm_batch_run(lbm_batch *b, int32_t k_steps) {
  if (!b || k_steps < 0) return LBM_EINVAL;
  if (k_steps == 0) return LBM_OK;
  int rc;
  if (b->dirty && (rc = rebuild(b))) return rc;
  if (b->active.empty()) return LBM_OK;
  LBM_HIP(hipEventRecord(b->start[b->seq % lbm_batch::RING], b->stream));
  const int32_t ns = std::max(1, std::min(b->nstreams, b->n_cohorts));
  if (ns > 1) {
    // the other streams start after everything queued so far
    LBM_HIP(hipEventRecord(b->fork, b->stream));
    for (int32_t q = 0; q + 1 < ns; ++q) LBM_HIP(hipStreamWaitEvent(b->side[q], b->fork, 0));
  }
  for (int32_t c = 0; c < b->n_cohorts; ++c)
    if ((rc = run_group(b, k_steps, c, c % ns ? b->side[c % ns - 1] : b->stream))) return rc;
  // and everything queued later on the batch's stream waits for them
  for (int32_t q = 0; q + 1 < ns; ++q) {
    LBM_HIP(hipEventRecord(b->join[q], b->side[q]));
    LBM_HIP(hipStreamWaitEvent(b->stream, b->join[q], 0));
  }
  // the group's completion, which is also the last use (so far) of the copy
  // of the lists it read
  LBM_HIP(hipEventRecord(b->done[b->seq % lbm_batch::RING], b->stream));
  LBM_HIP(hipEventRecord(b->copy_done[b->copy], b->stream));
  b->copy_used[b->copy] = true;
  // mirror of the advance kernel: every pair a jet took in full toggled its flip
  int nsh;
  const TileShape *shapes = tile_shapes(&nsh);
  bool finished = false;
  for (int32_t s : b->active) {
    Slot &sl = b->slots[s];
    const int64_t np = shapes[sl.shape].steps == 2 ? k_steps / 2 : 0;
    if (sl.step >= sl.target) continue;
    if (np > 0 && sl.target - sl.step >= 2)
      sl.flip ^= (int32_t)(std::min<int64_t>(np, (sl.target - sl.step) / 2) & 1);
    sl.step = std::min<int64_t>(sl.step + k_steps, sl.target);
    if (sl.step >= sl.target) {
      sl.done_seq = b->seq;
      finished = true;
    }
  }
  ++b->seq;
  if (finished) b->dirty = true;  // drop finished jets from the tile list
  return LBM_OK;
}

// Add the device time of the complete groups up to `newest` (their events
// are still in the ring unless more than RING groups were queued since).
static int collect_times(lbm_batch *b, int64_t newest) {
  for (int64_t g = std::max(b->timed, b->seq - lbm_batch::RING); g <= newest; ++g) {
    float ms = 0.0f;
    LBM_HIP(hipEventElapsedTime(&ms, b->start[g % lbm_batch::RING],
                                b->done[g % lbm_batch::RING]));
    b->device_ms += ms;
    ++b->timed_groups;
  }
  b->timed = std::max(b->timed, newest + 1);
  return LBM_OK;
}

int lbm_batch_wait(lbm_batch *b, int32_t in_flight) {
  if (!b || in_flight < 0 || in_flight >= lbm_batch::RING) return LBM_EINVAL;
  const int64_t g = b->seq - 1 - in_flight;  // the newest group that must be done
  if (g < 0) return LBM_OK;
  LBM_HIP(hipEventSynchronize(b->done[g % lbm_batch::RING]));
  LBM_HIP(hipGetLastError());
  return collect_times(b, g);
}

int lbm_batch_device_time(lbm_batch *b, double *ms, int64_t *groups) {
  if (!b || !ms) return LBM_EINVAL;
  *ms = b->device_ms;
  if (groups) *groups = b->timed_groups;
  return LBM_OK;
}

int lbm_batch_poll(lbm_batch *b, int32_t slot, int64_t *steps_done) {
  Slot *sl = slot_of(b, slot);
  if (!sl || !steps_done) return LBM_EINVAL;
  *steps_done = sl->step;
  return LBM_OK;
}

// Extraction of one jet's results runs on the batch's extraction stream after
// the group in which the jet finished (io_after), so that it waits neither
// for the groups queued since nor holds them up: the helper kernel, then the
// jet's instability flag and the result back to the host.
static int extract(lbm_batch *b, int32_t slot, void *dev, size_t bytes, void *host,
                   int32_t *flag) {
  LBM_HIP(hipMemcpyAsync(flag, b->d_flags + slot, sizeof(int32_t), hipMemcpyDeviceToHost,
                         b->io));
  LBM_HIP(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, b->io));
  LBM_HIP(hipStreamSynchronize(b->io));
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

int lbm_batch_profiles(lbm_batch *b, int32_t slot, double *ux_axis, double *T_axis,
                       double *ux_exit, double *T_exit) {
  Slot *sl = slot_of(b, slot);
  if (!sl) return LBM_EINVAL;
  const int n = sl->cfg.nx + sl->cfg.nr;
  void *p;
  int rc = b->scratch.get(n * sizeof(float2), &p);
  if (rc) return rc;
  if ((rc = io_after(b, *sl))) return rc;
  if ((rc = launch_profiles(sl->prec, b->io, b->d_slot_desc + slot, &sl->cfg, sl->step,
                            state_view_of(b->layout, sl->step, sl->flip), (float2 *)p)))
    return rc;
  std::vector<float2> v(n);
  int32_t flag = 0;
  if ((rc = extract(b, slot, p, n * sizeof(float2), v.data(), &flag))) return rc;
  for (int i = 0; i < sl->cfg.nx; ++i) {
    if (ux_axis) ux_axis[i] = v[i].x;
    if (T_axis) T_axis[i] = v[i].y;
  }
  for (int j = 0; j < sl->cfg.nr; ++j) {
    if (ux_exit) ux_exit[j] = v[sl->cfg.nx + j].x;
    if (T_exit) T_exit[j] = v[sl->cfg.nx + j].y;
  }
  return flag ? LBM_EUNSTABLE : LBM_OK;
}

int lbm_batch_moments(lbm_batch *b, int32_t slot, double *rho, double *ux, double *ur,
                      double *T) {
  Slot *sl = slot_of(b, slot);
  if (!sl) return LBM_EINVAL;
  const int64_t nodes = (int64_t)sl->cfg.nx * sl->cfg.nr;
  void *p;
  int rc = b->scratch.get(nodes * sizeof(float4), &p);
  if (rc) return rc;
  if ((rc = io_after(b, *sl))) return rc;
  if ((rc = launch_moments(sl->prec, b->io, b->d_slot_desc + slot, &sl->cfg, sl->step,
                           state_view_of(b->layout, sl->step, sl->flip), (float4 *)p)))
    return rc;
  std::vector<float4> m((size_t)nodes);
  int32_t flag = 0;
  if ((rc = extract(b, slot, p, nodes * sizeof(float4), m.data(), &flag))) return rc;
  for (int64_t n = 0; n < nodes; ++n) {
    if (rho) rho[n] = m[n].x;
    if (ux) ux[n] = m[n].y;
    if (ur) ur[n] = m[n].z;
    if (T) T[n] = m[n].w;
  }
  return flag ? LBM_EUNSTABLE : LBM_OK;
}

int lbm_batch_retire(lbm_batch *b, int32_t slot) {
  Slot *sl = slot_of(b, slot);
  if (!sl) return LBM_EINVAL;
  // no group may still use the jet's memory: wait for the group in which it
  // finished (later groups skip it), or for all queued work if it had not
  if (sl->done_seq >= 0)
    LBM_HIP(hipEventSynchronize(b->done[sl->done_seq % lbm_batch::RING]));
  else
    LBM_HIP(hipStreamSynchronize(b->stream));
  b->arena.release(sl->off, sl->bytes);
  b->used -= sl->bytes;
  *sl = Slot();
  b->dirty = true;
  return LBM_OK;
}

int lbm_batch_sync(lbm_batch *b) {
  if (!b) return LBM_EINVAL;
  LBM_HIP(hipStreamSynchronize(b->stream));
  LBM_HIP(hipGetLastError());
  if (b->seq > 0) {
    const int rc = collect_times(b, b->seq - 1);
    if (rc) return rc;
  }
  return LBM_OK;
}

int lbm_batch_active(const lbm_batch *b, int32_t *n_active, size_t *bytes_used) {
  if (!b) return LBM_EINVAL;
  int32_t n = 0;
  for (const Slot &s : b->slots) n += s.used ? 1 : 0;
  if (n_active) *n_active = n;
  if (bytes_used) *bytes_used = b->used;
  return LBM_OK;
}

int lbm_batch_set_cohort_bytes(lbm_batch *b, size_t bytes) {
  if (!b) return LBM_EINVAL;
  LBM_HIP(hipStreamSynchronize(b->stream));
  b->cohort_bytes = bytes;
  b->dirty = true;
  return LBM_OK;
}

int lbm_batch_set_launch(lbm_batch *b, int32_t tile_shape, int32_t workgroups) {
  if (!b || workgroups < 0) return LBM_EINVAL;
  int n;
  tile_shapes(&n);
  if (tile_shape < -1 || tile_shape >= n) return LBM_EINVAL;
  LBM_HIP(hipStreamSynchronize(b->stream));
  b->shape = tile_shape;
  b->wg = workgroups;
  b->dirty = true;
  drop_graphs(b);
  return LBM_OK;
}

int lbm_batch_set_streams(lbm_batch *b, int32_t n) {
  if (!b || n < 1 || n > lbm_batch::MAX_STREAMS) return LBM_EINVAL;
  LBM_HIP(hipStreamSynchronize(b->stream));
  for (hipStream_t s : b->side)
    if (s) LBM_HIP(hipStreamSynchronize(s));
  bool ok = b->fork || hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess;
  for (int32_t q = 0; ok && q + 1 < n; ++q) {
    if (!b->side[q] && hipStreamCreateWithFlags(&b->side[q], hipStreamNonBlocking) != hipSuccess)
      b->side[q] = nullptr, ok = false;
    if (ok && !b->join[q] && hipEventCreateWithFlags(&b->join[q], hipEventDisableTiming) != hipSuccess)
      b->join[q] = nullptr, ok = false;
  }
  if (!ok) {
    b->nstreams = 1;
    return LBM_EDEVICE;
  }
  b->nstreams = n;
  return LBM_OK;
}

void lbm_batch_destroy(lbm_batch *b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  for (hipStream_t st : b->side)
    if (st) (void)hipStreamSynchronize(st);
  if (b->io) (void)hipStreamSynchronize(b->io);
  drop_graphs(b);
  for (SlotBlock &k : b->blocks) {
    if (k.own && k.p) (void)hipFree(k.p);
    if (k.own && k.h) (void)hipHostFree(k.h);
  }
  for (auto &k : b->replaced) {
    (void)hipFree(k.first);
    (void)hipHostFree(k.second);
  }
  if (b->pool_d) (void)hipFree(b->pool_d);
  if (b->pool_h) (void)hipHostFree(b->pool_h);
  b->scratch.release();
  if (b->arena_mem) (void)hipFree(b->arena_mem);
  if (b->d_jets) (void)hipFree(b->d_jets);
  if (b->d_slot_desc) (void)hipFree(b->d_slot_desc);
  if (b->d_tiles) (void)hipFree(b->d_tiles);
  if (b->d_hdr) (void)hipFree(b->d_hdr);
  if (b->d_flags) (void)hipFree(b->d_flags);
  if (b->h_jets) (void)hipHostFree(b->h_jets);
  if (b->h_tiles) (void)hipHostFree(b->h_tiles);
  if (b->h_hdr) (void)hipHostFree(b->h_hdr);
  if (b->h_slot) (void)hipHostFree(b->h_slot);
  if (b->h_zero) (void)hipHostFree(b->h_zero);
  if (b->io) (void)hipStreamDestroy(b->io);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->mark) (void)hipEventDestroy(b->mark);
  for (hipEvent_t e : b->copy_done)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : b->done)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : b->start)
    if (e) (void)hipEventDestroy(e);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (int q = 0; q + 1 < lbm_batch::MAX_STREAMS; ++q) {
    if (b->join[q]) (void)hipEventDestroy(b->join[q]);
    if (b->side[q]) (void)hipStreamDestroy(b->side[q]);
  }
  delete b;
}

}  // extern "C"
