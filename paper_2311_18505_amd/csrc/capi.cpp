// C ABI of libstringfdtd: batch handles, device memory, uploads and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/stringfdtd.h"
#include "planner.h"
#include "sfd_types.h"

namespace sfd {
hipError_t launch_kernel(int precision, int kernel, int variant, const LaunchArgs &a, int blocks, hipStream_t st);
hipError_t launch_zero(int32_t *c, int n, hipStream_t st);
int max_blocks_per_cu(int precision, int kernel, int variant);
hipError_t launch_delay(uint64_t ticks, hipStream_t st);
hipError_t launch_rewind(int precision, const Desc *desc, Status *status, const Status *status0, int first, int count,
                         hipStream_t st);
hipError_t launch_scatter(const void *src, const UploadSeg *segs, int n, hipStream_t st);
hipError_t launch_gather(int precision, const Desc *desc, const Status *status, const int32_t *slots,
                         const int64_t *offs, int n, int64_t count, void *dst, int64_t *row_done, int32_t *row_flags,
                         hipStream_t st);
hipError_t launch_plain(const Desc *d_desc, Status *d_status, int slot, int64_t n_steps, size_t lds_bytes,
                        hipStream_t st);
hipError_t static_scratch_ptr(int device, void **ptr);
}  // namespace sfd

using namespace sfd;

namespace {

std::string g_create_error;

// Chunked first-fit allocator over large device allocations.
class Arena {
 public:
  ~Arena() { clear(); }
  void clear() {
    for (auto &c : chunks_) (void)hipFree(c.base);
    chunks_.clear();
  }
  void *alloc(size_t n) {
    n = (n + 255) & ~size_t(255);
    for (auto &c : chunks_) {
      for (auto it = c.free.begin(); it != c.free.end(); ++it) {
        if (it->second >= n) {
          size_t off = it->first, sz = it->second;
          c.free.erase(it);
          if (sz > n) c.free[off + n] = sz - n;
          return c.base + off;
        }
      }
    }
    size_t csz = std::max(n, (size_t)256 << 20);
    void *p = nullptr;
    if (hipMalloc(&p, csz) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    chunks_.push_back(Chunk{(char *)p, csz, {}});
    Chunk &c = chunks_.back();
    if (csz > n) c.free[n] = csz - n;
    return c.base;
  }
  void release(void *p, size_t n) {
    if (!p) return;
    n = (n + 255) & ~size_t(255);
    for (auto &c : chunks_) {
      char *q = (char *)p;
      if (q < c.base || q >= c.base + c.size) continue;
      size_t off = (size_t)(q - c.base);
      auto it = c.free.emplace(off, n).first;
      auto nx = std::next(it);
      if (nx != c.free.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        c.free.erase(nx);
      }
      if (it != c.free.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
          pv->second += it->second;
          c.free.erase(it);
        }
      }
      return;
    }
  }

 private:
  struct Chunk {
    char *base;
    size_t size;
    std::map<size_t, size_t> free;
  };
  std::vector<Chunk> chunks_;
};

struct Slot {
  bool planned = false, excited = false;
  Plan plan;
  char *dmem = nullptr;
  size_t dsize = 0;
  int64_t samples_host = 0;   // samples expected after the launches issued so far
  bool flagged = false;       // a flag was observed on the device
  bool restruck = false;      // re-excited since string_batch_excite (no rewind)
  int64_t gen = 0;            // excitation generation (excite or restrike), names the slot's tables
};

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

}  // namespace

struct sb_batch {
  int capacity = 0, precision = 0;
  size_t esz = 8;
  hipStream_t stream = nullptr;
  // size classes run concurrently on streams of their own, forked from and
  // joined back into `stream` through events (default priority)
  hipStream_t unit_stream[kNumUnits] = {};
  hipEvent_t ev_fork = nullptr;
  uint64_t delay_ticks = 0;      // head start of the large-class launches (wall-clock ticks, ~20 us)
  hipEvent_t ev_join[kNumUnits] = {};
  hipEvent_t ev_t0[kNumUnits] = {}, ev_t1[kNumUnits] = {};   // timing of each launch
  int32_t unit_strings[kNumUnits] = {};                       // strings of the last launch
  std::string err;
  std::vector<Slot> slots;
  Arena arena;
  Desc *d_desc = nullptr;
  Status *d_status = nullptr;
  Status *d_status0 = nullptr;   // status right after excitation (for rewind)
  int32_t *d_work = nullptr;     // wavefront tasks: 64/G slot indices each (-1: empty group)
  int32_t *d_counters = nullptr;
  void *d_trash = nullptr;        // write target of empty groups and unused slots
  Status *d_trash_status = nullptr;
  // streaming readout: slot list, offsets and the gathered rows (grown on demand)
  // bulk uploads of excite: staging buffer and segment list (grown on demand)
  char *d_stage = nullptr;
  size_t stage_bytes = 0;
  UploadSeg *d_segs = nullptr;
  size_t segs_cap = 0;
  int32_t *d_gslots = nullptr;
  int64_t *d_goffs = nullptr;
  int64_t *d_gdone = nullptr;     // per gathered row: the slot's samples_done and flags
  int32_t *d_gflags = nullptr;
  void *d_scratch = nullptr;      // this device's copy of the library's fixed scratch (allocation-free calls)
  void *d_gbuf = nullptr;
  size_t gbuf_bytes = 0;
  std::vector<int32_t> h_work;
  std::vector<int32_t> h_plain;   // plain path: slots in launch order
  bool work_dirty = true;
  int64_t epoch = 0;               // bumped whenever slots change (invalidates a captured graph)
  int64_t next_gen = 0;            // last excitation generation handed to a slot
  int blocks_per_cu[kNumUnits] = {};   // persistent blocks per CU per launch (0: occupancy limit)
  // captured launches (string_batch_graph_capture)
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int64_t graph_steps = 0, graph_epoch = -1;
  std::vector<int> graph_members;
  int mon_period = 480;
  double mon_tol = 1e-9;
  double tol = 1e-13;
  int max_sweeps = 64;
  int num_cu = 256;
};

static int fail(sb_batch *b, int code, const std::string &msg) {
  if (b) b->err = msg;
  return code;
}

static int hip_fail(sb_batch *b, hipError_t e, const char *where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  (void)hipGetLastError();
  return fail(b, SB_EDEVICE, m);
}

static_assert(kNumUnits == SB_NUM_LAUNCHES, "launch units of the C ABI");

static size_t work_capacity(int capacity);
static void graph_release(sb_batch *b);

extern "C" int string_batch_create(int capacity, int precision, void *hip_stream, sb_batch **out) {
  g_create_error.clear();
  if (!out || capacity < 1 || (precision != SB_FP64 && precision != SB_FP32C && precision != SB_FP64_PLAIN)) {
    g_create_error = "bad capacity, precision or output pointer";
    return SB_EINVAL;
  }
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    g_create_error = "no HIP device";
    return SB_EDEVICE;
  }
  sb_batch *b = new (std::nothrow) sb_batch();
  if (!b) return SB_ENOMEM;
  b->capacity = capacity;
  b->precision = precision;
  b->esz = precision == SB_FP32C ? 4 : 8;
  b->stream = (hipStream_t)hip_stream;
  b->mon_tol = precision == SB_FP32C ? 1e-4 : 1e-9;
  b->tol = precision == SB_FP32C ? 1e-7 : 1e-13;
  b->slots.resize(capacity);
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    b->num_cu = prop.multiProcessorCount;
  hipError_t e;
  if ((e = hipMalloc(&b->d_desc, sizeof(Desc) * capacity)) != hipSuccess ||
      (e = hipMalloc(&b->d_status, sizeof(Status) * capacity)) != hipSuccess ||
      (e = hipMalloc(&b->d_status0, sizeof(Status) * capacity)) != hipSuccess ||
      (e = hipMalloc(&b->d_work, sizeof(int32_t) * work_capacity(capacity))) != hipSuccess ||
      (e = hipMalloc(&b->d_counters, sizeof(int32_t) * kNumVariants * kNumClasses)) != hipSuccess ||
      (e = hipMalloc(&b->d_trash, kMaxTrash)) != hipSuccess ||
      (e = hipMalloc(&b->d_trash_status, sizeof(Status))) != hipSuccess) {
    g_create_error = std::string("hipMalloc: ") + hipGetErrorString(e);
    (void)hipGetLastError();
    hipFree(b->d_desc);
    hipFree(b->d_status);
    hipFree(b->d_status0);
    hipFree(b->d_work);
    hipFree(b->d_counters);
    hipFree(b->d_trash);
    hipFree(b->d_trash_status);
    delete b;
    return SB_ENOMEM;
  }
  // zeroed descriptors: a slot without an excitation has null state pointers
  if ((e = hipMemset(b->d_desc, 0, sizeof(Desc) * capacity)) != hipSuccess ||
      (e = hipMemset(b->d_status, 0, sizeof(Status) * capacity)) != hipSuccess) {
    g_create_error = std::string("hipMemset: ") + hipGetErrorString(e);
    delete b;
    return SB_EDEVICE;
  }
  for (int c = 0; c < kNumUnits && e == hipSuccess; ++c) {
    e = hipStreamCreateWithFlags(&b->unit_stream[c], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_join[c], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreate(&b->ev_t0[c]);
    if (e == hipSuccess) e = hipEventCreate(&b->ev_t1[c]);
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
  // the device address of the fixed scratch on this (current) device
  if (e == hipSuccess) e = static_scratch_ptr(dev, &b->d_scratch);
  if (e == hipSuccess) {
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) khz = 100000;
    b->delay_ticks = (uint64_t)khz / 50;   // 20 us
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    g_create_error = std::string("stream/event creation: ") + hipGetErrorString(e);
    (void)hipGetLastError();
    string_batch_destroy(b);
    return SB_EDEVICE;
  }
  *out = b;
  return SB_OK;
}

extern "C" int string_batch_destroy(sb_batch *b) {
  if (!b) return SB_EINVAL;
  (void)hipStreamSynchronize(b->stream);
  for (int c = 0; c < kNumUnits; ++c) {
    if (b->unit_stream[c]) {
      (void)hipStreamSynchronize(b->unit_stream[c]);
      (void)hipStreamDestroy(b->unit_stream[c]);
    }
    if (b->ev_join[c]) (void)hipEventDestroy(b->ev_join[c]);
    if (b->ev_t0[c]) (void)hipEventDestroy(b->ev_t0[c]);
    if (b->ev_t1[c]) (void)hipEventDestroy(b->ev_t1[c]);
  }
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  graph_release(b);
  if (b->cap_stream) {
    (void)hipStreamSynchronize(b->cap_stream);
    (void)hipStreamDestroy(b->cap_stream);
  }
  b->arena.clear();
  hipFree(b->d_desc);
  hipFree(b->d_status);
  hipFree(b->d_status0);
  hipFree(b->d_work);
  hipFree(b->d_counters);
  hipFree(b->d_trash);
  hipFree(b->d_trash_status);
  hipFree(b->d_gslots);
  hipFree(b->d_goffs);
  hipFree(b->d_gdone);
  hipFree(b->d_gflags);
  hipFree(b->d_gbuf);
  hipFree(b->d_stage);
  hipFree(b->d_segs);
  delete b;
  return SB_OK;
}

extern "C" const char *string_batch_last_error(const sb_batch *b) {
  return b ? b->err.c_str() : g_create_error.c_str();
}

// Entries of the task array: every class pads its last task with at most 64/G - 1 empty groups.
static_assert(kNumUnits == SB_NUM_LAUNCHES, "launch units of the C ABI");

// task lists (strings, padded per class to whole tasks) and the ticket map of
// the merged launch (at most one ticket per string)
// every string once in a task list (each list padded to whole wavefronts),
// and at most one ticket per task
static size_t work_capacity(int capacity) {
  return 2 * (size_t)capacity + (size_t)kNumVariants * kNumParts * (kWave + 1);
}

static bool range_ok(const sb_batch *b, int first, int count) {
  return first >= 0 && count >= 0 && (int64_t)first + count <= b->capacity;
}

// Device region of one slot: state | initial state | real tables | output | integer tables.
// State and tables are lane-major over the G lanes of the string's class; the
// output has 64 samples of padding that absorb the stores of idle lanes.
static size_t region_size(const sb_batch *b, const Desc &D, size_t *off_st0, size_t *off_tabf, size_t *off_out,
                          size_t *off_tab) {
  if (b->precision == SB_FP64_PLAIN) {
    // natural order: u^n | u^{n-1} | zeta^n | zeta^{n-1}; weights per t-half; position tables
    const size_t st = align256(8 * 2 * (size_t)(D.nt + D.nl));
    const size_t tf = align256(8 * (size_t)D.Nt);
    const size_t ou = align256(8 * (size_t)(D.n_samples + kWave));
    const size_t tb = align256(4 * ((size_t)D.nt + D.nl + D.Nt + 2 * (size_t)D.Nl));
    *off_st0 = st;
    *off_tabf = 2 * st;
    *off_out = 2 * st + tf;
    *off_tab = 2 * st + tf + ou;
    return 2 * st + tf + ou + tb;
  }
  const size_t G = (size_t)kClassLanes[D.cls];
  const bool cubic = D.grid_interp == 3;   // three more weights per t-slot, two more ranges per l-slot
  const size_t st = align256(b->esz * G * 4 * (D.mt + D.ml));
  const size_t tf = align256(b->esz * G * (3 * D.mt + D.ml + (cubic ? 3 * D.mt : 0)));
  const size_t ou = align256(b->esz * (size_t)(D.n_samples + kWave));
  const size_t tb = align256(sizeof(uint32_t) * G * (D.mt + 2 * D.ml + (cubic ? 2 * D.ml : 0)));
  *off_st0 = st;
  *off_tabf = 2 * st;
  *off_out = 2 * st + tf;
  *off_tab = 2 * st + tf + ou;
  // the zeta channel, when asked for, follows with the output's size
  return 2 * st + tf + ou + tb + (D.zeta_out ? ou : 0);
}

// Offset of the zeta channel in a slot's region (batched paths).
static size_t zeta_out_offset(const sb_batch *b, const Desc &D) {
  size_t a0, a, o, t;
  return region_size(b, D, &a0, &a, &o, &t) - align256(b->esz * (size_t)(D.n_samples + kWave));
}

extern "C" int string_batch_set_params(sb_batch *b, int first, int count, const sb_string_params *p) {
  if (!b) return SB_EINVAL;
  if (!p || !range_ok(b, first, count)) return fail(b, SB_EINVAL, "bad slot range or null params");
  std::vector<Plan> plans(count);
  for (int i = 0; i < count; ++i) {
    std::string err;
    int st = plan_string(p[i], plans[i], err, b->precision == SB_FP32C);
    if (st) return fail(b, st, "slot " + std::to_string(first + i) + ": " + err);
    if (b->precision == SB_FP64_PLAIN && p[i].readout_zeta)
      return fail(b, SB_EINVAL, "slot " + std::to_string(first + i) + ": the zeta channel needs a batched precision");
  }
  // queued launches may still read the memory released below
  hipError_t es = hipStreamSynchronize(b->stream);
  if (es != hipSuccess) return hip_fail(b, es, "sync");
  for (int i = 0; i < count; ++i) {
    Slot &s = b->slots[first + i];
    if (s.dmem) {
      b->arena.release(s.dmem, s.dsize);
      s.dmem = nullptr;
    }
    size_t a0, a, o, t;
    s.plan = std::move(plans[i]);
    s.dsize = region_size(b, s.plan.desc, &a0, &a, &o, &t);
    s.dmem = (char *)b->arena.alloc(s.dsize);
    if (!s.dmem) {
      s.planned = false;
      return fail(b, SB_ENOMEM, "device memory exhausted");
    }
    s.planned = true;
    s.excited = false;
    s.flagged = false;
    s.samples_host = 0;
  }
  b->work_dirty = true;
  ++b->epoch;
  // mark the slots idle on the device until they are excited
  std::vector<Status> zs(count);
  for (auto &z : zs) {
    std::memset(&z, 0, sizeof(z));
    z.H_step = -1;
  }
  // and null descriptors (the previous state memory of these slots is released)
  std::vector<Desc> zd(count);
  std::memset(zd.data(), 0, sizeof(Desc) * count);
  hipError_t e = hipMemcpyAsync(b->d_status + first, zs.data(), sizeof(Status) * count, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_desc + first, zd.data(), sizeof(Desc) * count, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hip_fail(b, e, "set_params upload");
  return SB_OK;
}

template <typename T>
static void to_prec(const std::vector<double> &src, std::vector<char> &dst) {
  dst.resize(src.size() * sizeof(T));
  T *d = (T *)dst.data();
  for (size_t i = 0; i < src.size(); ++i) d[i] = (T)src[i];
}

extern "C" int string_batch_excite(sb_batch *b, int first, int count, const sb_excitation *e) {
  if (!b) return SB_EINVAL;
  if (!e || !range_ok(b, first, count)) return fail(b, SB_EINVAL, "bad slot range or null excitation");
  for (int i = 0; i < count; ++i)
    if (!b->slots[first + i].planned) return fail(b, SB_ESTATE, "slot " + std::to_string(first + i) + " has no parameters");
  // validate everything before touching any slot
  for (int i = 0; i < count; ++i) {
    Plan tmp = b->slots[first + i].plan;
    std::string err;
    int st = plan_excitation(e[i], tmp, err);
    if (!st && b->precision == SB_FP64_PLAIN) st = plan_plain(tmp, err);
    if (st) return fail(b, st, "slot " + std::to_string(first + i) + ": " + err);
  }
  // queued launches may still step these slots
  hipError_t es = hipStreamSynchronize(b->stream);
  if (es != hipSuccess) return hip_fail(b, es, "sync");
  // every string's state, tables and first samples go into one staging
  // buffer: one copy and one scatter kernel instead of five copies a string
  std::vector<char> stage;
  std::vector<UploadSeg> segs;
  auto put = [&](const void *src, size_t bytes, void *dst) {
    const size_t off = (stage.size() + 15) & ~size_t(15);
    stage.resize(off + bytes);
    std::memcpy(stage.data() + off, src, bytes);
    segs.push_back(UploadSeg{off, dst, bytes});
    return off;
  };
  std::vector<char> bs, bt, bh;
  std::vector<Desc> descs(count);
  std::vector<Status> stats(count);
  hipError_t err = hipSuccess;
  for (int i = 0; i < count && err == hipSuccess; ++i) {
    Slot &s = b->slots[first + i];
    std::string msg;
    plan_excitation(e[i], s.plan, msg);
    if (b->precision == SB_FP64_PLAIN) plan_plain(s.plan, msg);
    Desc &D = s.plan.desc;
    size_t ost0, otf, oout, otab;
    region_size(b, D, &ost0, &otf, &oout, &otab);
    D.st = s.dmem;
    D.st0 = s.dmem + ost0;
    const bool plain = b->precision == SB_FP64_PLAIN;
    const int G = kClassLanes[D.cls];
    D.st_elems = plain ? 2 * (D.nt + D.nl) : G * 4 * (D.mt + D.ml);
    D.tabf = s.dmem + otf;
    D.out = s.dmem + oout;
    D.out_z = (!plain && D.zeta_out) ? s.dmem + zeta_out_offset(b, D) : nullptr;
    D.tab = (const uint32_t *)(s.dmem + otab);
    // initial state, lane-major: u, v, cu, cv (transverse), same for zeta
    std::vector<double> u0;
    double uH0, uH1;
    initial_state(e[i], s.plan, u0, uH0, uH1);
    std::vector<double> state((size_t)D.st_elems, 0.0);
    if (plain) {
      for (int i = 1; i <= D.nt; ++i) state[i - 1] = state[D.nt + i - 1] = u0[i];   // u^1 = u^0
      D.ptab = (const int32_t *)(s.dmem + otab);
      D.pw = (const double *)(s.dmem + otf);
    } else {
      for (int lane = 0; lane < G; ++lane)
        for (int r = 0; r < D.mt; ++r) {
          const int node = lane * D.mt + r + 1;
          if (node <= D.nt) state[(size_t)r * G + lane] = u0[node];
        }
    }
    double y0 = 0.0;
    if (D.on0) y0 += D.ow0 * u0[D.on0];
    if (D.on1) y0 += D.ow1 * u0[D.on1];
    std::vector<double> head = {y0, y0};   // y^0 = y^1 (w^1 = w^0)
    if (plain) {
      to_prec<double>(state, bs);
      to_prec<double>(s.plan.pw, bt);
      to_prec<double>(head, bh);
    } else if (b->precision == SB_FP32C) {
      to_prec<float>(state, bs);
      to_prec<float>(s.plan.tabf, bt);
      to_prec<float>(head, bh);
    } else {
      to_prec<double>(state, bs);
      to_prec<double>(s.plan.tabf, bt);
      to_prec<double>(head, bh);
    }
    put(bs.data(), bs.size(), s.dmem);
    put(bs.data(), bs.size(), s.dmem + ost0);
    put(bt.data(), bt.size(), s.dmem + otf);
    put(bh.data(), bh.size(), s.dmem + oout);
    if (!plain && D.zeta_out) {
      // zeta^0 = zeta^1 = 0 for every excitation (on the plain path out_z
      // shares its storage with the position tables: never test it there)
      const std::vector<char> zero(bh.size(), 0);
      put(zero.data(), zero.size(), D.out_z);
    }
    if (plain)
      put(s.plan.ptab.data(), s.plan.ptab.size() * sizeof(int32_t), s.dmem + otab);
    else
      put(s.plan.tab.data(), s.plan.tab.size() * sizeof(uint32_t), s.dmem + otab);
    descs[i] = D;
    Status &S = stats[i];
    std::memset(&S, 0, sizeof(S));
    S.samples_done = std::min<int64_t>(2, D.n_samples);
    S.H_step = -1;
    S.uH_n = uH1;
    S.uH_nm1 = uH0;
    S.eta_nm1 = uH0;   // eta^0 = u_H^0 - I u^0, the string starts at rest under the hammer
    s.excited = true;
    s.restruck = false;
    s.flagged = false;
    s.samples_host = S.samples_done;
    s.gen = ++b->next_gen;
  }
  // staging buffers of the batch (the previous upload has completed: the
  // stream was synchronised above)
  if (err == hipSuccess && stage.size() > b->stage_bytes) {
    err = hipFree(b->d_stage);
    b->d_stage = nullptr;
    b->stage_bytes = 0;
    if (err == hipSuccess) err = hipMalloc(&b->d_stage, stage.size());
    if (err == hipSuccess) b->stage_bytes = stage.size();
  }
  if (err == hipSuccess && segs.size() > b->segs_cap) {
    err = hipFree(b->d_segs);
    b->d_segs = nullptr;
    b->segs_cap = 0;
    if (err == hipSuccess) err = hipMalloc(&b->d_segs, sizeof(UploadSeg) * segs.size());
    if (err == hipSuccess) b->segs_cap = segs.size();
  }
  if (err == hipSuccess && !stage.empty())
    err = hipMemcpyAsync(b->d_stage, stage.data(), stage.size(), hipMemcpyHostToDevice, b->stream);
  if (err == hipSuccess && !segs.empty())
    err = hipMemcpyAsync(b->d_segs, segs.data(), sizeof(UploadSeg) * segs.size(), hipMemcpyHostToDevice, b->stream);
  if (err == hipSuccess) err = launch_scatter(b->d_stage, b->d_segs, (int)segs.size(), b->stream);
  if (err == hipSuccess)
    err = hipMemcpyAsync(b->d_desc + first, descs.data(), sizeof(Desc) * count, hipMemcpyHostToDevice, b->stream);
  if (err == hipSuccess)
    err = hipMemcpyAsync(b->d_status + first, stats.data(), sizeof(Status) * count, hipMemcpyHostToDevice, b->stream);
  if (err == hipSuccess)
    err = hipMemcpyAsync(b->d_status0 + first, stats.data(), sizeof(Status) * count, hipMemcpyHostToDevice, b->stream);
  if (err == hipSuccess) err = hipStreamSynchronize(b->stream);
  if (err != hipSuccess) return hip_fail(b, err, "excite upload");
  b->work_dirty = true;
  ++b->epoch;
  return SB_OK;
}

// Work lists of one launch: active slots per size class, packed into
// wavefront tasks of 64/G strings with similar remaining work side by side (a
// wavefront runs as long as its longest string), longest tasks first; the
// device copy is refreshed when it changes.
// Variant 1 holds the tasks with bowed strings: they run in kernels of their
// own, which keeps the bow's code and registers out of every other task.
struct WorkPlan {
  int off[kNumVariants][kNumParts + 1] = {};      // per variant, start of each part's tasks
  // ticket maps of the merged launch (parts of classes 0..4, index 0) and of
  // each large class's launch (its shapes, index 1 + class - kNumSmall)
  static constexpr int kTicketLists = 1 + kNumClasses - kNumSmall;
  int tickets_off[kNumVariants][kTicketLists] = {}, n_tickets[kNumVariants][kTicketLists] = {};
  std::vector<int> members;   // slots stepped
};

static int part_lanes(int part) { return kClassLanes[part / kNumShapes]; }

// Estimated cost of one step of a wavefront task of a part (VALU
// instructions, roughly: the per-lane scans and bookkeeping plus the
// per-slot work of both grids), for ordering tickets only.
static double part_step_cost(int part) {
  const int c = part / kNumShapes, s = part % kNumShapes;
  return 300.0 + 60.0 * (shape_mt(c, s) + shape_ml(c, s));
}
// the most expensive part's tickets are dealt over the first 1 - kTailSpan of
// the sequence, a part of no cost over all of it
constexpr double kTailSpan = 0.6;

static int build_work(sb_batch *b, int first, int count, int64_t n_steps, WorkPlan &wp) {
  // per part: (steps, cost, slot) of each string
  struct Item {
    int64_t steps;
    double cost;
    int slot;
  };
  std::vector<Item> parts[kNumVariants][kNumParts];
  bool any = false;
  for (int i = first; i < first + count; ++i) {
    Slot &s = b->slots[i];
    if (!s.excited) continue;
    any = true;
    if (s.flagged || s.samples_host >= s.plan.desc.n_samples) continue;
    const int64_t st = std::min<int64_t>(n_steps, s.plan.desc.n_samples - s.samples_host);
    const double cost = (double)st * (double)(s.plan.desc.nt + s.plan.desc.nl + 8);
    const Desc &d = s.plan.desc;
    const int part = b->precision == SB_FP64_PLAIN ? 0 : d.cls * kNumShapes + d.shape;
    // bowed and clamped strings, the zeta channel and cubic hammers run in
    // the instantiation that carries their code, strings with the cubic grid
    // interpolant in the one that adds it
    const bool cubic_hammer = d.ham_on && (d.hn2 || d.hn3);
    const int v = d.grid_interp == 3 ? kVarCubic
                                     : ((d.bow_on || d.clamped || d.zeta_out || cubic_hammer) ? kVarBow : kVarPlain);
    parts[v][part].push_back({st, cost, i});
  }
  if (!any) return fail(b, SB_ESTATE, "no excited slot");
  std::vector<int32_t> work;
  for (int v = 0; v < kNumVariants; ++v) {
    for (int q = 0; q < kNumParts; ++q) {
      auto &L = parts[v][q];
      // longest first by steps: the strings of a part cost the same per
      // step (one layout), and a wavefront steps as long as its longest
      // group, so the groups of a task should have equal steps (the cost
      // breaks ties and orders the plain path's one-string launches)
      std::stable_sort(L.begin(), L.end(), [](const Item &x, const Item &y) {
        return x.steps != y.steps ? x.steps > y.steps : x.cost > y.cost;
      });
      wp.off[v][q] = (int)work.size();
      const int groups = b->precision == SB_FP64_PLAIN ? 1 : kWave / part_lanes(q);
      for (size_t i = 0; i < L.size(); i += groups)
        for (int g = 0; g < groups; ++g) work.push_back(i + g < L.size() ? L[i + g].slot : -1);
      for (auto &w : L) wp.members.push_back(w.slot);
    }
    wp.off[v][kNumParts] = (int)work.size();
    if (b->precision != SB_FP64_PLAIN) {
      // tickets of the merged launch and of each large class's launch: the
      // tasks of their parts dealt out in proportion to their counts, each
      // part longest first, over a span of the ticket sequence that shrinks
      // with the part's cost per step (task t of a part of n tasks at
      // (t / n) (1 - kTailSpan cost / largest cost)).  The mix of parts on
      // the CUs stays broad over the launch, which runs faster than one part
      // after another (their bottlenecks differ), while the tail holds the
      // cheapest tasks (with chunked stepping every task has the same steps,
      // and an expensive task started last would set the chunk's end).  A
      // ticket is part << 24 | task (a large class: its shape).
      for (int u = 0; u < WorkPlan::kTicketLists; ++u) {
        const int q_lo = u == 0 ? 0 : (kNumSmall + u - 1) * kNumShapes;
        const int q_hi = u == 0 ? kNumSmall * kNumShapes : q_lo + kNumShapes;
        std::vector<std::pair<double, int32_t>> tk;
        double cmax = 0.0;
        for (int q = q_lo; q < q_hi; ++q)
          if (!parts[v][q].empty()) cmax = std::max(cmax, part_step_cost(q));
        for (int q = q_lo; q < q_hi; ++q) {
          const int groups = kWave / part_lanes(q);
          const int nt = (int)((parts[v][q].size() + groups - 1) / groups);
          const double span = 1.0 - kTailSpan * part_step_cost(q) / std::max(cmax, 1.0);
          for (int t = 0; t < nt; ++t)
            tk.push_back({-(double)t / (double)nt * span, (int32_t)(((q - q_lo) << 24) | t)});
        }
        std::stable_sort(tk.begin(), tk.end(), [](const std::pair<double, int32_t> &x, const std::pair<double, int32_t> &y) {
          return x.first > y.first;
        });
        wp.tickets_off[v][u] = (int)work.size();
        wp.n_tickets[v][u] = (int)tk.size();
        for (auto &t : tk) work.push_back(t.second);
      }
    }
  }
  if (work.empty() || b->precision == SB_FP64_PLAIN) {
    b->h_plain = std::move(work);
    return SB_OK;
  }
  if (work != b->h_work || b->work_dirty) {
    // the previous upload may still be read by queued launches: order the
    // host buffer's reuse after them
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e == hipSuccess && b->cap_stream) e = hipStreamSynchronize(b->cap_stream);
    if (e != hipSuccess) return hip_fail(b, e, "sync");
    b->h_work = work;
    e = hipMemcpyAsync(b->d_work, b->h_work.data(), sizeof(int32_t) * work.size(), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(b, e, "work upload");
    b->work_dirty = false;
  }
  return SB_OK;
}

// One step launch on `st`: counters cleared by a kernel (no memset nodes
// under capture), the three launches (classes 0..4 merged, class 5, classes 6 and 7)
// forked onto their own streams and joined back.  Issues no synchronisation
// and no copy, so it can be captured.
static int enqueue_step(sb_batch *b, hipStream_t st, const WorkPlan &wp, int64_t n_steps) {
  hipError_t e = launch_zero(b->d_counters, kNumVariants * kNumClasses, st);
  if (e == hipSuccess) e = hipEventRecord(b->ev_fork, st);
  if (e != hipSuccess) return hip_fail(b, e, "fork");
  // largest strings first: their launches hold the longest per-step latency
  bool big_launched = false;
  for (int u = kNumUnits - 1; u >= 0; --u) {
    hipStream_t cs = b->unit_stream[u];
    b->unit_strings[u] = 0;
    bool forked = false;
    // the unit's classes one after the other (unit 0: the merged launch of
    // classes 0..4); the bow-family variants follow the plain one on the same stream
    const int c_lo = u == 0 ? 0 : (u == 1 ? kNumSmall : kNumSmall + 1);
    const int c_hi = u == 0 ? 1 : (u == 1 ? kNumSmall + 1 : kNumClasses);
    for (int c = c_lo; c < c_hi; ++c) {
      const int kernel = u == 0 ? 0 : kernel_of_class(c);
      for (int v = 0; v < kNumVariants; ++v) {
        LaunchArgs a;
        a.desc = b->d_desc;
        a.status = b->d_status;
        int lo, hi;
        for (int p = 0; p < kNumSmall * kNumShapes; ++p) a.part_work[p] = nullptr;
        a.tickets = nullptr;
        {
          // ticketed launches: the merged one over the parts of classes
          // 0..4, a large class's over its shapes
          const int tl = u == 0 ? 0 : 1 + c - kNumSmall;
          const int q0 = u == 0 ? 0 : c * kNumShapes;
          const int nq = u == 0 ? kNumSmall * kNumShapes : kNumShapes;
          for (int p = 0; p < nq; ++p) a.part_work[p] = b->d_work + wp.off[v][q0 + p];
          a.tickets = b->d_work + wp.tickets_off[v][tl];
          a.work = a.part_work[0];
          a.n_work = wp.n_tickets[v][tl];
          lo = wp.off[v][q0];
          hi = wp.off[v][q0 + nq];
        }
        for (int k = lo; k < hi; ++k) b->unit_strings[u] += b->h_work[k] >= 0 ? 1 : 0;
        if (a.n_work == 0) continue;
        a.counter = b->d_counters + kNumVariants * c + v;
        a.n_steps = n_steps;
        a.mon_period = b->mon_period;
        a.max_sweeps = b->max_sweeps;
        a.tol = b->tol;
        a.mon_tol = b->mon_tol;
        a.trash_st = b->d_trash;
        a.trash_status = b->d_trash_status;
        int per_cu = b->blocks_per_cu[u];
        const int occ = std::max(1, max_blocks_per_cu(b->precision, kernel, v));
        per_cu = per_cu > 0 ? std::min(per_cu, occ) : occ;
        const int blocks = std::min(a.n_work, b->num_cu * per_cu);
        if (!forked) {
          e = hipStreamWaitEvent(cs, b->ev_fork, 0);
          // the merged launch starts a little after the large classes (their
          // wavefronts need whole SIMDs; the merged one's would fill them first)
          if (e == hipSuccess && u == 0 && big_launched) e = launch_delay(b->delay_ticks, cs);
          if (e == hipSuccess) e = hipEventRecord(b->ev_t0[u], cs);
          forked = true;
        }
        if (e == hipSuccess) e = launch_kernel(b->precision, kernel, v, a, blocks, cs);
        if (e != hipSuccess) return hip_fail(b, e, "step launch");
      }
    }
    if (!forked) continue;
    big_launched = big_launched || u > 0;
    e = hipEventRecord(b->ev_t1[u], cs);
    if (e == hipSuccess) e = hipEventRecord(b->ev_join[u], cs);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, b->ev_join[u], 0);
    if (e != hipSuccess) return hip_fail(b, e, "step launch");
  }
  return SB_OK;
}

static void advance_host(sb_batch *b, const std::vector<int> &members, int64_t n_steps) {
  for (int i : members) {
    Slot &s = b->slots[i];
    s.samples_host = std::min<int64_t>(s.samples_host + n_steps, s.plan.desc.n_samples);
  }
}

static int do_step(sb_batch *b, int first, int count, int64_t n_steps) {
  if (n_steps < 0) return fail(b, SB_EINVAL, "n_steps < 0");
  if (!range_ok(b, first, count)) return fail(b, SB_EINVAL, "bad slot range");
  if (n_steps == 0) return SB_OK;
  WorkPlan wp;
  int st = build_work(b, first, count, n_steps, wp);
  if (st) return st;
  if (wp.members.empty()) return SB_OK;
  if (b->precision == SB_FP64_PLAIN) {
    // one string per launch, in order
    for (int32_t i : b->h_plain) {
      if (i < 0) continue;
      hipError_t e = launch_plain(b->d_desc, b->d_status, i, n_steps, plain_lds_bytes(b->slots[i].plan.desc), b->stream);
      if (e != hipSuccess) return hip_fail(b, e, "plain launch");
    }
  } else {
    st = enqueue_step(b, b->stream, wp, n_steps);
    if (st) return st;
  }
  advance_host(b, wp.members, n_steps);
  return SB_OK;
}

static void graph_release(sb_batch *b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
  b->graph_members.clear();
}

extern "C" int string_batch_graph_capture(sb_batch *b, int64_t steps_per_launch, int n_launches) {
  if (!b) return SB_EINVAL;
  if (b->precision == SB_FP64_PLAIN) return fail(b, SB_EINVAL, "the plain path launches one string at a time");
  if (steps_per_launch < 1 || n_launches < 1 || n_launches > 100000) return fail(b, SB_EINVAL, "bad launch shape");
  WorkPlan wp;
  int st = build_work(b, 0, b->capacity, steps_per_launch * n_launches, wp);
  if (st) return st;
  if (wp.members.empty()) return fail(b, SB_ESTATE, "no slot left to step");
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hip_fail(b, e, "sync");
  graph_release(b);
  e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return hip_fail(b, e, "begin capture");
  for (int l = 0; l < n_launches && st == SB_OK; ++l) st = enqueue_step(b, b->cap_stream, wp, steps_per_launch);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(b->cap_stream, &g);
  if (st != SB_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return st != SB_OK ? st : hip_fail(b, e, "end capture");
  }
  e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    b->gexec = nullptr;
    return hip_fail(b, e, "instantiate");
  }
  b->graph = g;
  b->graph_steps = steps_per_launch * n_launches;
  b->graph_members = wp.members;
  b->graph_epoch = b->epoch;
  return SB_OK;
}

// Autotuner: the persistent blocks per CU of the three launches, chosen
// jointly.  A probe is one whole step launch (all three forked and joined)
// of probe_steps steps from the excited state: every task runs probe_steps
// steps, so the probe is the run in miniature, with the contention between
// the launches.  Coordinate descent over the launches, largest strings first,
// keeps for each the candidate (1, 2, 4, 6 or 8 blocks per CU, up to its
// occupancy limit) with the shortest probe.  Every slot is rewound to its
// excitation before and after.
extern "C" int string_batch_autotune(sb_batch *b, int64_t probe_steps, int32_t *chosen) {
  if (!b) return SB_EINVAL;
  if (b->precision == SB_FP64_PLAIN) return fail(b, SB_EINVAL, "the plain path has nothing to tune");
  if (probe_steps < 1) return fail(b, SB_EINVAL, "probe_steps < 1");
  int st = string_batch_rewind(b, 0, b->capacity);
  if (st) return st;
  WorkPlan wp;
  st = build_work(b, 0, b->capacity, probe_steps, wp);
  if (st) return st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  auto probe = [&](float &ms) -> int {
    int r = string_batch_rewind(b, 0, b->capacity);
    if (r) return r;
    hipError_t x = hipEventRecord(e0, b->stream);
    if (x != hipSuccess) return hip_fail(b, x, "autotune");
    r = enqueue_step(b, b->stream, wp, probe_steps);
    if (r) return r;
    x = hipEventRecord(e1, b->stream);
    if (x == hipSuccess) x = hipEventSynchronize(e1);
    if (x == hipSuccess) x = hipEventElapsedTime(&ms, e0, e1);
    return x == hipSuccess ? SB_OK : hip_fail(b, x, "autotune");
  };
  int occ[kNumUnits], nw[kNumUnits] = {};
  for (int v = 0; v < kNumVariants; ++v)
    for (int q = 0; q < kNumParts; ++q)
      nw[unit_of_class(q / kNumShapes)] += (wp.off[v][q + 1] - wp.off[v][q]) / (kWave / part_lanes(q));
  for (int u = 0; u < kNumUnits; ++u) {
    occ[u] = 1;
    for (int c = 0; c < kNumClasses; ++c)
      if (unit_of_class(c) == u) occ[u] = std::max(occ[u], max_blocks_per_cu(b->precision, kernel_of_class(c), kVarPlain));
    b->blocks_per_cu[u] = occ[u];
    if (chosen) chosen[u] = 0;
  }
  float best_ms = 1e30f;
  if (e == hipSuccess) {
    float ms = 0.f;
    (void)probe(ms);        // first launch of every kernel: not timed
    st = probe(best_ms);
  }
  for (int c = kNumUnits - 1; c >= 0 && e == hipSuccess && st == SB_OK; --c) {
    if (nw[c] == 0) continue;
    int best = b->blocks_per_cu[c];
    for (int cand : {1, 2, 4, 6, 8}) {
      if (cand > occ[c] || cand == best) continue;
      b->blocks_per_cu[c] = cand;
      float ms = 0.f;
      st = probe(ms);
      if (st) break;
      if (ms < best_ms) {
        best_ms = ms;
        best = cand;
      }
    }
    b->blocks_per_cu[c] = best;
  }
  for (int c = 0; c < kNumUnits && chosen; ++c) chosen[c] = nw[c] ? b->blocks_per_cu[c] : 0;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st) return st;
  if (e != hipSuccess) return hip_fail(b, e, "autotune");
  return string_batch_rewind(b, 0, b->capacity);
}

extern "C" int string_batch_set_blocks_per_cu(sb_batch *b, const int32_t *blocks) {
  if (!b) return SB_EINVAL;
  if (!blocks) return fail(b, SB_EINVAL, "null blocks");
  for (int c = 0; c < kNumUnits; ++c)
    if (blocks[c] < 0 || blocks[c] > 64) return fail(b, SB_EINVAL, "blocks per CU outside 0..64");
  for (int c = 0; c < kNumUnits; ++c) b->blocks_per_cu[c] = blocks[c];
  return SB_OK;
}

extern "C" int string_batch_launch_times(sb_batch *b, float *ms, int32_t *strings) {
  if (!b) return SB_EINVAL;
  if (!ms || !strings) return fail(b, SB_EINVAL, "null output");
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hip_fail(b, e, "sync");
  for (int c = 0; c < kNumUnits; ++c) {
    ms[c] = 0.f;
    strings[c] = b->unit_strings[c];
    if (!strings[c]) continue;
    e = hipEventElapsedTime(&ms[c], b->ev_t0[c], b->ev_t1[c]);
    if (e != hipSuccess) return hip_fail(b, e, "launch timing");
  }
  return SB_OK;
}

extern "C" int string_batch_graph_launch(sb_batch *b) {
  if (!b) return SB_EINVAL;
  if (!b->gexec) return fail(b, SB_ESTATE, "no captured graph");
  if (b->graph_epoch != b->epoch) return fail(b, SB_ESTATE, "slots changed since the capture");
  hipError_t e = hipGraphLaunch(b->gexec, b->stream);
  if (e != hipSuccess) return hip_fail(b, e, "graph launch");
  advance_host(b, b->graph_members, b->graph_steps);
  return SB_OK;
}

extern "C" int string_batch_step(sb_batch *b, int64_t n_steps) {
  if (!b) return SB_EINVAL;
  return do_step(b, 0, b->capacity, n_steps);
}

extern "C" int string_batch_step_range(sb_batch *b, int first, int count, int64_t n_steps) {
  if (!b) return SB_EINVAL;
  return do_step(b, first, count, n_steps);
}

static int read_status(sb_batch *b, int idx, Status *S);

// Describes the flagged slots among n (for last_error) and returns SB_EUNSTABLE.
static int unstable(sb_batch *b, const std::vector<int> &bad) {
  std::string m = "flagged by the energy monitor or the solver (output stops at samples_done): slot";
  for (size_t i = 0; i < bad.size() && i < 16; ++i) m += " " + std::to_string(bad[i]);
  if (bad.size() > 16) m += " ... (" + std::to_string(bad.size()) + " slots)";
  return fail(b, SB_EUNSTABLE, m);
}

// Samples offset.. of one output channel of slot idx (u, or zeta) into dst.
// Host destinations get zeros for the samples the slot has not produced, and
// SB_EUNSTABLE when the slot is flagged.
static int read_channel(sb_batch *b, int idx, int64_t offset, int64_t count, void *dst, int dst_is_device, bool zeta) {
  if (!b) return SB_EINVAL;
  if (idx < 0 || idx >= b->capacity || !dst || offset < 0 || count < 0) return fail(b, SB_EINVAL, "bad arguments");
  Slot &s = b->slots[idx];
  if (!s.excited) return fail(b, SB_ESTATE, "slot not excited");
  // (on the plain path out_z shares its storage with the position tables)
  if (zeta && (b->precision == SB_FP64_PLAIN || !s.plan.desc.zeta_out || !s.plan.desc.out_z))
    return fail(b, SB_ESTATE, "slot set without the zeta channel");
  if (offset + count > s.plan.desc.n_samples) return fail(b, SB_EINVAL, "range beyond n_samples");
  if (count == 0) return SB_OK;
  const char *src = (const char *)(zeta ? s.plan.desc.out_z : s.plan.desc.out) + offset * b->esz;
  if (dst_is_device) {
    hipError_t e = hipMemcpyAsync(dst, src, count * b->esz, hipMemcpyDeviceToDevice, b->stream);
    if (e != hipSuccess) return hip_fail(b, e, zeta ? "read_output_zeta" : "read_output");
    return SB_OK;
  }
  Status S;
  int st = read_status(b, idx, &S);    // synchronises the stream
  if (st) return st;
  const int64_t have = std::max<int64_t>(0, std::min<int64_t>(count, S.samples_done - offset));
  if (have > 0) {
    hipError_t e = hipMemcpy(dst, src, have * b->esz, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(b, e, zeta ? "read_output_zeta" : "read_output");
  }
  std::memset((char *)dst + have * b->esz, 0, (count - have) * b->esz);
  if (S.flags) return unstable(b, {idx});
  return SB_OK;
}

extern "C" int string_batch_read_output(sb_batch *b, int idx, int64_t offset, int64_t count, void *dst, int dst_is_device) {
  return read_channel(b, idx, offset, count, dst, dst_is_device, false);
}

extern "C" int string_batch_read_output_zeta(sb_batch *b, int idx, int64_t offset, int64_t count, void *dst,
                                             int dst_is_device) {
  return read_channel(b, idx, offset, count, dst, dst_is_device, true);
}

extern "C" int string_batch_gather_output(sb_batch *b, int n, const int32_t *slots, const int64_t *offsets,
                                          int64_t count, void *dst, int dst_is_device, int64_t *samples_done,
                                          int32_t *flags) {
  if (!b) return SB_EINVAL;
  if (n < 0 || n > b->capacity || count < 0 || (n > 0 && (!slots || !offsets || !dst)))
    return fail(b, SB_EINVAL, "bad arguments");
  if (n == 0) return SB_OK;
  for (int i = 0; i < n; ++i) {
    if (slots[i] < 0 || slots[i] >= b->capacity) return fail(b, SB_EINVAL, "bad slot");
    const Slot &s = b->slots[slots[i]];
    if (!s.excited) return fail(b, SB_ESTATE, "slot " + std::to_string(slots[i]) + " not excited");
    if (offsets[i] < 0 || offsets[i] >= s.plan.desc.n_samples) return fail(b, SB_EINVAL, "offset outside the output");
  }
  hipError_t e = hipSuccess;
  if (!b->d_gslots) {
    e = hipMalloc(&b->d_gslots, sizeof(int32_t) * b->capacity);
    if (e == hipSuccess) e = hipMalloc(&b->d_goffs, sizeof(int64_t) * b->capacity);
    if (e == hipSuccess) e = hipMalloc(&b->d_gdone, sizeof(int64_t) * b->capacity);
    if (e == hipSuccess) e = hipMalloc(&b->d_gflags, sizeof(int32_t) * b->capacity);
    if (e != hipSuccess) return hip_fail(b, e, "gather buffers");
  }
  const size_t bytes = (size_t)n * (size_t)count * b->esz;
  void *rows = dst;
  if (!dst_is_device && bytes > 0) {
    if (bytes > b->gbuf_bytes) {
      // the previous buffer may still be read by queued copies
      e = hipStreamSynchronize(b->stream);
      if (e == hipSuccess) e = hipFree(b->d_gbuf);
      b->d_gbuf = nullptr;
      b->gbuf_bytes = 0;
      if (e == hipSuccess) e = hipMalloc(&b->d_gbuf, bytes);
      if (e != hipSuccess) return hip_fail(b, e, "gather buffer");
      b->gbuf_bytes = bytes;
    }
    rows = b->d_gbuf;
  }
  // the index arrays of a previous call may still be read by its kernel
  e = hipStreamSynchronize(b->stream);
  if (e == hipSuccess) e = hipMemcpy(b->d_gslots, slots, sizeof(int32_t) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_goffs, offsets, sizeof(int64_t) * n, hipMemcpyHostToDevice);
  // (with count 0 the kernel only records progress and flags: rows is never touched)
  if (e == hipSuccess)
    e = launch_gather(b->precision, b->d_desc, b->d_status, b->d_gslots, b->d_goffs, n, count, rows, b->d_gdone,
                      b->d_gflags, b->stream);
  if (e == hipSuccess && !dst_is_device && bytes > 0)
    e = hipMemcpyAsync(dst, rows, bytes, hipMemcpyDeviceToHost, b->stream);
  const bool want_status = !dst_is_device || samples_done || flags;
  if (!want_status) {
    if (e != hipSuccess) return hip_fail(b, e, "gather_output");
    return SB_OK;
  }
  // progress and flags of the listed slots
  std::vector<int64_t> hd(n);
  std::vector<int32_t> hf(n);
  if (e == hipSuccess) e = hipMemcpyAsync(hd.data(), b->d_gdone, sizeof(int64_t) * n, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(hf.data(), b->d_gflags, sizeof(int32_t) * n, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hip_fail(b, e, "gather_output");
  std::vector<int> bad;
  for (int i = 0; i < n; ++i) {
    if (samples_done) samples_done[i] = hd[i];
    if (flags) flags[i] = hf[i];
    if (hf[i]) {
      bad.push_back(slots[i]);
      b->slots[slots[i]].flagged = true;
    }
  }
  if (!bad.empty()) return unstable(b, bad);
  return SB_OK;
}

static_assert(kNoAllocMaxRows == SB_NOALLOC_MAX_ROWS, "row limit of the allocation-free gather");

// string_batch_gather_output into a device destination with the index
// arrays and per-row status in the library's fixed scratch instead of the
// batch's own buffers (which the first gather allocates): no allocation at
// all.  Synchronous with the batch stream (the scratch of the previous call
// is free once the stream has drained).
extern "C" int string_batch_gather_output_noalloc(sb_batch *b, int n, const int32_t *slots, const int64_t *offsets,
                                                  int64_t count, void *dst, int64_t *samples_done, int32_t *flags) {
  if (!b) return SB_EINVAL;
  // the size limit first: it is the one error a caller of this entry point must expect
  if (n > kNoAllocMaxRows || n > b->capacity)
    return fail(b, SB_EINVAL, "n = " + std::to_string(n) + " rows exceeds the allocation-free gather's maximum of " +
                                  std::to_string(std::min(kNoAllocMaxRows, b->capacity)));
  if (n < 0 || count < 0 || (n > 0 && (!slots || !offsets || (count > 0 && !dst))))
    return fail(b, SB_EINVAL, "bad arguments");
  if (n == 0) return SB_OK;
  for (int i = 0; i < n; ++i) {
    if (slots[i] < 0 || slots[i] >= b->capacity) return fail(b, SB_EINVAL, "bad slot");
    const Slot &s = b->slots[slots[i]];
    if (!s.excited) return fail(b, SB_ESTATE, "slot " + std::to_string(slots[i]) + " not excited");
    if (offsets[i] < 0 || offsets[i] >= s.plan.desc.n_samples) return fail(b, SB_EINVAL, "offset outside the output");
  }
  if (!b->d_scratch) return fail(b, SB_EDEVICE, "no fixed scratch on this device");
  char *base = (char *)b->d_scratch;
  int32_t *d_slots = (int32_t *)(base + kScratchSlotsOff);
  int64_t *d_offs = (int64_t *)(base + kScratchOffsOff);
  int64_t *d_done = (int64_t *)(base + kScratchDoneOff);
  int32_t *d_flags = (int32_t *)(base + kScratchFlagsOff);
  // earlier work on the stream (a previous call's gather reads the scratch)
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e == hipSuccess) e = hipMemcpy(d_slots, slots, sizeof(int32_t) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_offs, offsets, sizeof(int64_t) * n, hipMemcpyHostToDevice);
  // (with count 0 the kernel only records progress and flags)
  if (e == hipSuccess)
    e = launch_gather(b->precision, b->d_desc, b->d_status, d_slots, d_offs, n, count, dst, d_done, d_flags, b->stream);
  std::vector<int64_t> hd(n);
  std::vector<int32_t> hf(n);
  if (e == hipSuccess) e = hipMemcpyAsync(hd.data(), d_done, sizeof(int64_t) * n, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(hf.data(), d_flags, sizeof(int32_t) * n, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hip_fail(b, e, "gather_output_noalloc");
  std::vector<int> bad;
  for (int i = 0; i < n; ++i) {
    if (samples_done) samples_done[i] = hd[i];
    if (flags) flags[i] = hf[i];
    if (hf[i]) {
      bad.push_back(slots[i]);
      b->slots[slots[i]].flagged = true;
    }
  }
  if (!bad.empty()) return unstable(b, bad);
  return SB_OK;
}

extern "C" int string_batch_output_ptr(sb_batch *b, int idx, void **dev_ptr) {
  if (!b) return SB_EINVAL;
  if (idx < 0 || idx >= b->capacity || !dev_ptr) return fail(b, SB_EINVAL, "bad arguments");
  if (!b->slots[idx].excited) return fail(b, SB_ESTATE, "slot not excited");
  *dev_ptr = b->slots[idx].plan.desc.out;
  return SB_OK;
}

static int read_status(sb_batch *b, int idx, Status *S) {
  if (idx < 0 || idx >= b->capacity) return fail(b, SB_EINVAL, "bad slot");
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e == hipSuccess) e = hipMemcpy(S, b->d_status + idx, sizeof(Status), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(b, e, "status read");
  if (S->flags) b->slots[idx].flagged = true;
  return SB_OK;
}

extern "C" int string_batch_read_energy(sb_batch *b, int idx, double *H_latest, int64_t *step_of_H) {
  if (!b) return SB_EINVAL;
  Status S;
  int st = read_status(b, idx, &S);
  if (st) return st;
  if (H_latest) *H_latest = S.H_latest;
  if (step_of_H) *step_of_H = S.H_step;
  return SB_OK;
}

extern "C" int string_batch_info(sb_batch *b, int idx, sb_string_info *info) {
  if (!b) return SB_EINVAL;
  if (!info) return fail(b, SB_EINVAL, "null info");
  if (idx < 0 || idx >= b->capacity) return fail(b, SB_EINVAL, "bad slot");
  Slot &s = b->slots[idx];
  std::memset(info, 0, sizeof(*info));
  if (!s.planned) return fail(b, SB_ESTATE, "slot has no parameters");
  info->N_t = s.plan.desc.Nt;
  info->N_l = s.plan.desc.Nl;
  info->size_class = s.plan.desc.cls;
  info->lanes = kClassLanes[s.plan.desc.cls];
  info->slots_t = b->precision == SB_FP64_PLAIN ? 0 : s.plan.desc.mt;
  info->slots_l = b->precision == SB_FP64_PLAIN ? 0 : s.plan.desc.ml;
  info->n_samples = s.plan.desc.n_samples;
  if (!s.excited) return SB_OK;
  Status S;
  int st = read_status(b, idx, &S);
  if (st) return st;
  info->samples_done = S.samples_done;
  info->flags = S.flags;
  info->max_sweeps = S.max_sweeps;
  info->total_sweeps = S.total_sweeps;
  s.samples_host = S.samples_done;
  return SB_OK;
}

extern "C" int string_batch_set_monitor(sb_batch *b, int period, double growth_tol) {
  if (!b) return SB_EINVAL;
  if (period < 0 || !(growth_tol >= 0) || !std::isfinite(growth_tol)) return fail(b, SB_EINVAL, "bad monitor settings");
  b->mon_period = period;
  b->mon_tol = growth_tol;
  return SB_OK;
}

extern "C" int string_batch_set_solver(sb_batch *b, double tol, int max_sweeps) {
  if (!b) return SB_EINVAL;
  if (!(tol >= 0) || !std::isfinite(tol) || max_sweeps < 1 || max_sweeps > 100000)
    return fail(b, SB_EINVAL, "bad solver settings");
  b->tol = tol;
  b->max_sweeps = max_sweeps;
  return SB_OK;
}

// A new hammer or bow on sounding strings (several excitations per note).
// The state stays; the slot's plan takes the new excitation; a hammer
// arrives touching the string at level n-1 (the level before the next step
// n) with velocity v_H, a bow's controls restart from level n-1.  All slots
// of one call share two synchronisations: one after reading their status
// (and, for hammers, their state), one after writing plans and status.
extern "C" int string_batch_restrike_list(sb_batch *b, int count, const int32_t *slots, const sb_excitation *e) {
  if (!b) return SB_EINVAL;
  if (count < 0 || (count > 0 && (!e || !slots))) return fail(b, SB_EINVAL, "null slots or excitations");
  if (b->precision == SB_FP64_PLAIN) return fail(b, SB_EINVAL, "the plain path takes excitations only at the start");
  std::vector<Plan> plans(count);
  for (int i = 0; i < count; ++i) {
    const int k = slots[i];
    if (k < 0 || k >= b->capacity) return fail(b, SB_EINVAL, "slot index out of range");
    for (int j = 0; j < i; ++j)
      if (slots[j] == k) return fail(b, SB_EINVAL, "slot " + std::to_string(k) + " listed twice");
    Slot &s = b->slots[k];
    if (!s.excited) return fail(b, SB_ESTATE, "slot " + std::to_string(k) + " is not excited");
    if (e[i].type != SB_EXC_HAMMER && e[i].type != SB_EXC_BOW)
      return fail(b, SB_EINVAL, "slot " + std::to_string(k) + ": a new excitation is a hammer or a bow");
    if (s.samples_host >= s.plan.desc.n_samples) return fail(b, SB_ESTATE, "slot " + std::to_string(k) + " has finished");
    plans[i] = s.plan;
    std::string err;
    const int st = plan_excitation(e[i], plans[i], err);
    if (st) return fail(b, st, "slot " + std::to_string(k) + ": " + err);
  }
  if (count == 0) return SB_OK;
  // the state must be current: queued launches finish first
  hipError_t he = hipStreamSynchronize(b->stream);
  if (he == hipSuccess && b->cap_stream) he = hipStreamSynchronize(b->cap_stream);
  if (he != hipSuccess) return hip_fail(b, he, "sync");
  // read status (and the state of hammered slots)
  std::vector<Status> S(count);
  std::vector<std::vector<char>> raw(count);
  for (int i = 0; i < count && he == hipSuccess; ++i) {
    he = hipMemcpyAsync(&S[i], b->d_status + slots[i], sizeof(Status), hipMemcpyDeviceToHost, b->stream);
    if (he == hipSuccess && e[i].type == SB_EXC_HAMMER) {
      const Desc &D = plans[i].desc;
      raw[i].resize((size_t)4 * D.mt * kClassLanes[D.cls] * b->esz);
      he = hipMemcpyAsync(raw[i].data(), D.st, raw[i].size(), hipMemcpyDeviceToHost, b->stream);
    }
  }
  if (he == hipSuccess) he = hipStreamSynchronize(b->stream);
  if (he != hipSuccess) return hip_fail(b, he, "restrike read");
  std::vector<std::vector<char>> tabs(count);
  for (int i = 0; i < count; ++i) {
    Desc &D = plans[i].desc;
    const int64_t n = S[i].samples_done - 1;   // the next step computes w^{n+1}
    if (e[i].type == SB_EXC_BOW) {
      D.bt0 = (double)(n - 1) / D.fs;
      D.bT = (double)(D.n_samples - (n - 1)) / D.fs;
    } else {
      // u_H^{n-1} = I_H u^{n-1}, u_H^n = u_H^{n-1} + k v_H, from the state
      // (u^n and v^{n-1/2} = u^n - u^{n-1}, each as value minus compensation)
      const int G = kClassLanes[D.cls], mt = D.mt;
      auto at = [&](int a, int r, int lane) {
        const size_t idx = ((size_t)a * mt + r) * G + lane;
        return b->precision == SB_FP32C ? (double)((const float *)raw[i].data())[idx]
                                        : ((const double *)raw[i].data())[idx];
      };
      auto prev = [&](int node) {   // u^{n-1} at a node (1-based)
        if (node <= 0) return 0.0;
        const int lane = (node - 1) / mt, r = (node - 1) % mt;
        return (at(0, r, lane) - at(2, r, lane)) - (at(1, r, lane) - at(3, r, lane));
      };
      const double uHm = D.hw0 * prev(D.hn0) + D.hw1 * prev(D.hn1) + D.hw2 * prev(D.hn2) + D.hw3 * prev(D.hn3);
      S[i].uH_nm1 = uHm;
      S[i].uH_n = uHm + D.k * e[i].v_H;
      S[i].eta_nm1 = 0.0;
      S[i].touched = 0;
    }
    if (b->precision == SB_FP32C)
      to_prec<float>(plans[i].tabf, tabs[i]);
    else
      to_prec<double>(plans[i].tabf, tabs[i]);
  }
  for (int i = 0; i < count && he == hipSuccess; ++i) {
    const Desc &D = plans[i].desc;
    he = hipMemcpyAsync(const_cast<void *>(D.tabf), tabs[i].data(), tabs[i].size(), hipMemcpyHostToDevice, b->stream);
    if (he == hipSuccess)
      he = hipMemcpyAsync(b->d_desc + slots[i], &plans[i].desc, sizeof(Desc), hipMemcpyHostToDevice, b->stream);
    if (he == hipSuccess) he = hipMemcpyAsync(b->d_status + slots[i], &S[i], sizeof(Status), hipMemcpyHostToDevice, b->stream);
  }
  if (he == hipSuccess) he = hipStreamSynchronize(b->stream);   // host buffers are released after this
  if (he != hipSuccess) return hip_fail(b, he, "restrike upload");
  for (int i = 0; i < count; ++i) {
    Slot &s = b->slots[slots[i]];
    s.plan = plans[i];
    s.restruck = true;
    s.gen = ++b->next_gen;
  }
  ++b->epoch;
  b->work_dirty = true;
  return SB_OK;
}

extern "C" int string_batch_restrike(sb_batch *b, int first, int count, const sb_excitation *e) {
  if (!b) return SB_EINVAL;
  if (!range_ok(b, first, count)) return fail(b, SB_EINVAL, "bad slot range");
  std::vector<int32_t> slots(count);
  for (int i = 0; i < count; ++i) slots[i] = first + i;
  return string_batch_restrike_list(b, count, slots.data(), e);
}

extern "C" int string_batch_rewind(sb_batch *b, int first, int count) {
  if (!b) return SB_EINVAL;
  if (!range_ok(b, first, count)) return fail(b, SB_EINVAL, "bad slot range");
  for (int i = first; i < first + count; ++i)
    if (b->slots[i].restruck) return fail(b, SB_ESTATE, "slot " + std::to_string(i) + " was re-excited; excite it again");
  for (int i = first; i < first + count; ++i) {
    Slot &s = b->slots[i];
    if (!s.excited) continue;
    s.samples_host = std::min<int64_t>(2, s.plan.desc.n_samples);
    s.flagged = false;
  }
  hipError_t e = launch_rewind(b->precision, b->d_desc, b->d_status, b->d_status0, first, count, b->stream);
  if (e != hipSuccess) return hip_fail(b, e, "rewind");
  return SB_OK;
}

// Snapshot of one slot: this header, the slot's Status at kSnapStatusOff and
// its state block (both grids, velocities and compensations, in the batch's
// precision and layout) at kSnapStateOff.
namespace {
struct SnapHeader {
  char magic[8];
  int32_t precision, slot, cls, esz;
  int64_t gen, st_elems, n_samples, bytes;
  int32_t nt, nl;
};
constexpr char kSnapMagic[8] = {'S', 'B', 'S', 'N', 'A', 'P', '1', 0};
constexpr int64_t kSnapStatusOff = 128, kSnapStateOff = 256;
static_assert(sizeof(SnapHeader) <= (size_t)kSnapStatusOff, "snapshot header");
static_assert(kSnapStatusOff + (int64_t)sizeof(Status) <= kSnapStateOff, "snapshot status");

SnapHeader snap_header(const sb_batch *b, int idx) {
  const Slot &s = b->slots[idx];
  const Desc &D = s.plan.desc;
  SnapHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, kSnapMagic, sizeof(h.magic));
  h.precision = b->precision;
  h.slot = idx;
  h.cls = D.cls;
  h.esz = (int32_t)b->esz;
  h.gen = s.gen;
  h.st_elems = D.st_elems;
  h.n_samples = D.n_samples;
  h.bytes = kSnapStateOff + (int64_t)D.st_elems * (int64_t)b->esz;
  h.nt = D.nt;
  h.nl = D.nl;
  return h;
}

// Queued launches and copies of the batch finish first.
hipError_t sync_batch(sb_batch *b) {
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e == hipSuccess && b->cap_stream) e = hipStreamSynchronize(b->cap_stream);
  return e;
}
}  // namespace

extern "C" int string_batch_snapshot_bytes(sb_batch *b, int idx, int64_t *bytes) {
  if (!b) return SB_EINVAL;
  if (!bytes || idx < 0 || idx >= b->capacity) return fail(b, SB_EINVAL, "bad arguments");
  if (!b->slots[idx].excited) return fail(b, SB_ESTATE, "slot not excited");
  *bytes = snap_header(b, idx).bytes;
  return SB_OK;
}

extern "C" int string_batch_snapshot(sb_batch *b, int idx, void *dst, int64_t bytes, int dst_is_device) {
  if (!b) return SB_EINVAL;
  if (!dst || idx < 0 || idx >= b->capacity) return fail(b, SB_EINVAL, "bad arguments");
  const Slot &s = b->slots[idx];
  if (!s.excited) return fail(b, SB_ESTATE, "slot not excited");
  const SnapHeader h = snap_header(b, idx);
  if (bytes < h.bytes) return fail(b, SB_EINVAL, "buffer smaller than the snapshot (" + std::to_string(h.bytes) + " bytes)");
  char head[kSnapStatusOff];
  std::memset(head, 0, sizeof(head));
  std::memcpy(head, &h, sizeof(h));
  char *d = (char *)dst;
  const hipMemcpyKind out = dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  hipError_t e = sync_batch(b);
  if (e == hipSuccess) {
    if (dst_is_device)
      e = hipMemcpyAsync(d, head, sizeof(head), hipMemcpyHostToDevice, b->stream);
    else
      std::memcpy(d, head, sizeof(head));
  }
  if (e == hipSuccess) e = hipMemcpyAsync(d + kSnapStatusOff, b->d_status + idx, sizeof(Status), out, b->stream);
  if (e == hipSuccess && !dst_is_device)
    std::memset(d + kSnapStatusOff + sizeof(Status), 0, kSnapStateOff - kSnapStatusOff - sizeof(Status));
  if (e == hipSuccess)
    e = hipMemcpyAsync(d + kSnapStateOff, s.plan.desc.st, (size_t)(h.bytes - kSnapStateOff), out, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);   // `head` is released after this
  if (e != hipSuccess) return hip_fail(b, e, "snapshot");
  return SB_OK;
}

extern "C" int string_batch_restore(sb_batch *b, int idx, const void *src, int64_t bytes, int src_is_device) {
  if (!b) return SB_EINVAL;
  if (!src || idx < 0 || idx >= b->capacity) return fail(b, SB_EINVAL, "bad arguments");
  Slot &s = b->slots[idx];
  if (!s.excited) return fail(b, SB_ESTATE, "slot not excited");
  const SnapHeader want = snap_header(b, idx);
  if (bytes < kSnapStateOff) return fail(b, SB_EINVAL, "not a snapshot (too short)");
  const char *p = (const char *)src;
  SnapHeader h;
  Status S;
  hipError_t e = hipSuccess;
  if (src_is_device) {
    e = hipMemcpy(&h, p, sizeof(h), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&S, p + kSnapStatusOff, sizeof(S), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(b, e, "restore read");
  } else {
    std::memcpy(&h, p, sizeof(h));
    std::memcpy(&S, p + kSnapStatusOff, sizeof(S));
  }
  if (std::memcmp(h.magic, kSnapMagic, sizeof(h.magic)) != 0) return fail(b, SB_EINVAL, "not a snapshot");
  if (h.bytes != bytes || h.bytes != want.bytes || h.precision != want.precision || h.esz != want.esz ||
      h.st_elems != want.st_elems || h.cls != want.cls || h.nt != want.nt || h.nl != want.nl ||
      h.n_samples != want.n_samples)
    return fail(b, SB_EINVAL, "the snapshot does not fit this slot's string");
  if (h.slot != idx) return fail(b, SB_EINVAL, "the snapshot was taken from slot " + std::to_string(h.slot));
  if (h.gen != s.gen) return fail(b, SB_ESTATE, "the slot was excited or re-excited since the snapshot");
  const int64_t n = want.n_samples;
  if (S.samples_done < std::min<int64_t>(2, n) || S.samples_done > n) return fail(b, SB_EINVAL, "corrupt snapshot");
  const hipMemcpyKind in = src_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  e = sync_batch(b);
  if (e == hipSuccess) e = hipMemcpyAsync(b->d_status + idx, &S, sizeof(Status), hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s.plan.desc.st, p + kSnapStateOff, (size_t)(h.bytes - kSnapStateOff), in, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);   // `S` is released after this
  if (e != hipSuccess) return hip_fail(b, e, "restore");
  s.samples_host = S.samples_done;
  s.flagged = S.flags != 0;
  b->work_dirty = true;
  ++b->epoch;
  return SB_OK;
}
