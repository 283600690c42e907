// Host runtime of libvlp: contexts, keysets, elementwise calls, programs
// (level-scheduled netlists) and the C ABI declared in include/vlp.h.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <list>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/vlp.h"
#include "internal.h"
#include "netlist.h"

using namespace vlp;

struct vlp_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  size_t budget = 0, used = 0;
  std::string err;
  uint4* tw_fwd = nullptr;  // device twiddle table
  int num_cus = 256;
  vlp_tuning tune{4, 1, 512, 0};
  // Grow-only scratch for the elementwise calls.
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  // This device's fixed scratch for vlp_gate_noalloc (device address).
  void* noalloc = nullptr;
  // Bytes of merged work items that vlp_step may need: the sum over live
  // programs of their largest level's items; the scratch is kept at least
  // this large from program creation on, so vlp_step never allocates.
  size_t step_reserve = 0;
  int live_keysets = 0, live_programs = 0;
  std::list<vlp_program*> eval_cache;  // programs made by vlp_evaluate, most recent first
  // Kernel timing (vlp_profile_enable).
  bool prof = false;
  struct Mark { hipEvent_t e0, e1; int kind; uint64_t items; };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> event_pool;
};

struct vlp_keyset {
  vlp_ctx* ctx;
  uint32_t* bk_ntt;
  uint32_t* ksk;
  int users;  // live programs made with it
};

// A program's per-level work, in device arrays.
struct Level {
  uint32_t br_first, br_count;  // range in the program's BR item array
  uint32_t ks_first, ks_count;  // range in the KS item array
};

struct vlp_program {
  vlp_ctx* ctx;
  vlp_keyset* ks;
  vlp_shape shape;
  vlp_circuit circuit;
  uint64_t gates = 0, brs = 0, kss = 0;
  std::vector<Level> levels;
  uint32_t next_level = 0;
  BrItem* br_items = nullptr;
  KsItem* ks_items = nullptr;
  uint32_t* gate_buf = nullptr;   // internal gate outputs [n_internal][631]
  uint32_t* ext_buf = nullptr;    // LWE_N slots [max BR per level][1025]
  const uint32_t** more_buf = nullptr;  // operand lists of k-input XOR items
  uint32_t* dig_buf = nullptr;    // key-switching digits of one launch
  size_t bytes = 0;
  size_t step_bytes = 0;  // its share of the context's step reserve
  uint32_t max_br_level = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  vlp_tuning graph_tune{};  // launch shape the graph was captured with
  // arguments, for the vlp_evaluate cache
  const uint32_t *q, *loc, *pay;
  uint32_t *R, *v;
};

namespace {

vlp_status fail(vlp_ctx* ctx, vlp_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (ctx) ctx->err = buf;
  return st;
}

std::string g_create_err;

#define HIPCHECK(ctx, expr)                                                                          \
  do {                                                                                               \
    hipError_t e_ = (expr);                                                                          \
    if (e_ != hipSuccess) return fail((ctx), VLP_EHIP, "%s: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

#define LAUNCHCHECK(ctx, expr)                                                                       \
  do {                                                                                               \
    int e_ = (expr);                                                                                 \
    if (e_ != 0) return fail((ctx), VLP_EHIP, "%s: %s", #expr, hipGetErrorString((hipError_t)e_)); \
  } while (0)

vlp_status dev_alloc(vlp_ctx* ctx, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) return VLP_OK;
  if (ctx->used + bytes > ctx->budget)
    return fail(ctx, VLP_EBUDGET, "allocation of %zu bytes exceeds the budget (%zu of %zu in use)", bytes, ctx->used,
                ctx->budget);
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(ctx, e == hipErrorOutOfMemory ? VLP_EBUDGET : VLP_EHIP, "hipMalloc(%zu): %s", bytes,
                hipGetErrorString(e));
  }
  ctx->used += bytes;
  return VLP_OK;
}

void dev_free(vlp_ctx* ctx, void* p, size_t bytes) {
  if (!p) return;
  (void)hipFree(p);
  ctx->used -= bytes;
}

vlp_status ensure_scratch(vlp_ctx* ctx, size_t bytes) {
  if (ctx->scratch_bytes >= bytes) return VLP_OK;
  HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
  dev_free(ctx, ctx->scratch, ctx->scratch_bytes);
  ctx->scratch = nullptr;
  ctx->scratch_bytes = 0;
  size_t want = std::max(bytes, (size_t)1 << 20);
  vlp_status st = dev_alloc(ctx, &ctx->scratch, want);
  if (st != VLP_OK) return st;
  ctx->scratch_bytes = want;
  return VLP_OK;
}

// Device addresses of the fixed no-allocation scratch, one per device, looked
// up once (with that device current) by the first context made on it.
std::mutex g_noalloc_mu;
std::vector<void*> g_noalloc_addr;

hipError_t noalloc_address_for(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if ((size_t)device >= g_noalloc_addr.size()) g_noalloc_addr.resize((size_t)device + 1, nullptr);
  if (!g_noalloc_addr[(size_t)device]) {
    void* p = nullptr;
    const hipError_t e = (hipError_t)noalloc_scratch_address(&p);
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_noalloc_addr[(size_t)device] = p;
  }
  *out = g_noalloc_addr[(size_t)device];
  return hipSuccess;
}

bool params_ok(const vlp_params* p) {
  return p && p->n == (uint32_t)LWE_n && p->N == (uint32_t)RING_N && p->k == 1 && p->bg_bit == (uint32_t)BG_BIT &&
         p->ell == (uint32_t)ELL && p->ks_basebit == (uint32_t)KS_BASEBIT && p->ks_t == (uint32_t)KS_T;
}

bool ranges_overlap(const void* a, size_t an, const void* b, size_t bn) {
  if (!a || !b) return false;
  const char *pa = (const char*)a, *pb = (const char*)b;
  return pa < pb + bn && pb < pa + an;
}


int mark_begin(vlp_ctx* ctx);
void mark_end(vlp_ctx* ctx, int id, int kind, uint64_t items);

// Blind rotations are launched in rounds that the device holds at once
// (CUs x workgroups per CU x rotations per workgroup): rotations that start
// together walk the key in step, so each key row reaches L2 once for many of
// them (a persistent loop over many rounds let them drift apart and re-fetch
// the key: up to ~36 MB instead of ~0.5 MB of key traffic per rotation).
// Automatic mode: a round of at most 2 rotations per CU runs on the
// four-wavefront kernel (half the latency), larger rounds on the
// two-wavefront kernel.
int timed_br(vlp_ctx* ctx, const BrItem* items, uint32_t count) {
  const uint32_t mode = ctx->tune.br_waves_per_rotation, bpc = ctx->tune.br_blocks_per_cu;
  const uint32_t rpb = ctx->tune.br_rotations_per_block, cus = (uint32_t)ctx->num_cus;
  const uint32_t small = cus * 2;  // rotations one round of the four-wavefront kernel holds
  for (uint32_t first = 0; first < count;) {
    const uint32_t rem = count - first;
    uint32_t n;
    int e;
    const int m = mark_begin(ctx);
    if (mode == 4 || (mode == 0 && rem <= small)) {
      const uint32_t blocks = mode == 4 ? cus * bpc : small;
      n = std::min(blocks, rem);
      e = launch_br4(items + first, n, ctx->tw_fwd, blocks, ctx->stream);
    } else if (mode == 1) {
      const uint32_t blocks = cus * bpc;
      n = std::min(blocks * rpb, rem);
      e = launch_br(items + first, n, ctx->tw_fwd, rpb, blocks, ctx->stream);
    } else {
      const uint32_t blocks = cus * bpc;
      n = std::min(blocks * rpb, rem);
      e = launch_br2(items + first, n, ctx->tw_fwd, rpb, blocks, ctx->stream);
    }
    mark_end(ctx, m, 0, n);
    if (e != 0) return e;
    first += n;
  }
  return 0;
}

int timed_ks(vlp_ctx* ctx, const KsItem* items, uint32_t count, const uint32_t* ksk, uint32_t* dig) {
  if (count == 0) return 0;
  const int m = mark_begin(ctx);
  const int e =
      launch_ks_group(items, count, ksk, dig, ctx->tune.ks_gates_per_block, (uint32_t)ctx->num_cus, ctx->stream);
  mark_end(ctx, m, 1, count);
  return e;
}

hipEvent_t take_event(vlp_ctx* ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

bool capturing(vlp_ctx* ctx) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(ctx->stream, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

// Opens a timed region around one kernel launch (kind 0 = blind rotation, 1 = key switch).
int mark_begin(vlp_ctx* ctx) {
  if (!ctx->prof || capturing(ctx)) return -1;
  vlp_ctx::Mark m{take_event(ctx), take_event(ctx), 0, 0};
  if (!m.e0 || !m.e1) return -1;
  (void)hipEventRecord(m.e0, ctx->stream);
  ctx->marks.push_back(m);
  return (int)ctx->marks.size() - 1;
}

void mark_end(vlp_ctx* ctx, int id, int kind, uint64_t items) {
  if (id < 0) return;
  vlp_ctx::Mark& m = ctx->marks[(size_t)id];
  m.kind = kind;
  m.items = items;
  (void)hipEventRecord(m.e1, ctx->stream);
}

// Gate pre-combination coefficients (Section 2.2 construction).
void gate_coeffs(uint8_t op, int32_t* ca, int32_t* cb, uint32_t* cst) {
  switch (op) {
    case VLP_AND: *ca = 1; *cb = 1; *cst = 0u - MU; break;
    case VLP_OR: *ca = 1; *cb = 1; *cst = MU; break;
    case VLP_NAND: *ca = -1; *cb = -1; *cst = MU; break;
    case VLP_XOR: *ca = 2; *cb = 2; *cst = 2 * MU; break;
    case VLP_XNOR: *ca = -2; *cb = -2; *cst = 0u - 2 * MU; break;
    default: *ca = 1; *cb = 1; *cst = 0u - MU; break;  // MUX first unit
  }
}

uint32_t encode_bit(uint32_t bit) { return bit ? MU : 0u - MU; }

}  // namespace

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
extern "C" const char* vlp_version(void) { return "vlp 0.3 (gfx950, two-prime NTT)"; }

extern "C" void vlp_default_params(vlp_params* p) {
  if (!p) return;
  p->n = LWE_n;
  p->N = RING_N;
  p->k = 1;
  p->bg_bit = BG_BIT;
  p->ell = ELL;
  p->ks_basebit = KS_BASEBIT;
  p->ks_t = KS_T;
}

extern "C" const char* vlp_last_error(const vlp_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

extern "C" vlp_status vlp_ctx_create(vlp_ctx** out, const vlp_params* p, int device, void* hip_stream, size_t hbm_budget) {
  if (!out) {
    g_create_err = "out is NULL";
    return VLP_EINVAL;
  }
  *out = nullptr;
  if (!params_ok(p)) {
    g_create_err = "parameters differ from the supported set {630, 1024, 1, 7, 3, 2, 8}";
    return VLP_EPARAM;
  }
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || device < 0 || device >= ndev) {
    g_create_err = std::string("no such HIP device: ") + (e != hipSuccess ? hipGetErrorString(e) : "index out of range");
    return VLP_EHIP;
  }
  vlp_ctx* ctx = new vlp_ctx();
  ctx->device = device;
  e = hipSetDevice(device);
  if (e == hipSuccess) {
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e == hipSuccess) {
      ctx->num_cus = prop.multiProcessorCount;
      size_t total = prop.totalGlobalMem;
      ctx->budget = hbm_budget ? hbm_budget : total / 10 * 9;
    }
  }
  if (e == hipSuccess) {
    if (hip_stream) {
      ctx->stream = (hipStream_t)hip_stream;
    } else {
      e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking);
      ctx->own_stream = e == hipSuccess;
    }
  }
  if (e == hipSuccess) {
    e = noalloc_address_for(device, &ctx->noalloc);
    if (e != hipSuccess && ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  }
  if (e != hipSuccess) {
    g_create_err = std::string("HIP set-up failed: ") + hipGetErrorString(e);
    delete ctx;
    return VLP_EHIP;
  }
  std::vector<uint32_t> tf(4 * RING_N);
  make_twiddles(tf.data());
  vlp_status st = dev_alloc(ctx, (void**)&ctx->tw_fwd, RING_N * 16);
  if (st == VLP_OK) {
    e = hipMemcpy(ctx->tw_fwd, tf.data(), RING_N * 16, hipMemcpyHostToDevice);
    if (e != hipSuccess) st = fail(ctx, VLP_EHIP, "twiddle upload: %s", hipGetErrorString(e));
  }
  if (st != VLP_OK) {
    g_create_err = ctx->err;
    dev_free(ctx, ctx->tw_fwd, RING_N * 16);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return st;
  }
  *out = ctx;
  return VLP_OK;
}

static void program_free(vlp_program* prog);

extern "C" vlp_status vlp_ctx_destroy(vlp_ctx* ctx) {
  if (!ctx) return VLP_EINVAL;
  (void)hipStreamSynchronize(ctx->stream);
  for (vlp_program* p : ctx->eval_cache) program_free(p);
  ctx->eval_cache.clear();
  if (ctx->live_keysets || ctx->live_programs)
    return fail(ctx, VLP_EBUSY, "%d keysets and %d programs still alive", ctx->live_keysets, ctx->live_programs);
  for (const auto& m : ctx->marks) {
    ctx->event_pool.push_back(m.e0);
    ctx->event_pool.push_back(m.e1);
  }
  for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
  dev_free(ctx, ctx->scratch, ctx->scratch_bytes);
  dev_free(ctx, ctx->tw_fwd, RING_N * 16);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return VLP_OK;
}

extern "C" vlp_status vlp_mem_info(const vlp_ctx* ctx, size_t* used, size_t* budget) {
  if (!ctx) return VLP_EINVAL;
  if (used) *used = ctx->used;
  if (budget) *budget = ctx->budget;
  return VLP_OK;
}

extern "C" vlp_status vlp_sync(vlp_ctx* ctx) {
  if (!ctx) return VLP_EINVAL;
  HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
  return VLP_OK;
}

extern "C" vlp_status vlp_get_tuning(const vlp_ctx* ctx, vlp_tuning* t) {
  if (!ctx || !t) return VLP_EINVAL;
  *t = ctx->tune;
  return VLP_OK;
}

extern "C" vlp_status vlp_set_tuning(vlp_ctx* ctx, const vlp_tuning* t) {
  if (!ctx || !t) return VLP_EINVAL;
  const uint32_t rpb = t->br_rotations_per_block, g = t->ks_gates_per_block, r = t->br_waves_per_rotation;
  if (!(r == 0 || r == 1 || r == 2 || r == 4)) return fail(ctx, VLP_EINVAL, "br_waves_per_rotation must be 0, 1, 2 or 4");
  const bool rpb_ok = r == 1 ? (rpb == 1 || rpb == 2 || rpb == 4 || rpb == 8)
                             : (r == 4 ? rpb == 1 : (rpb == 1 || rpb == 2 || rpb == 4));
  if (!rpb_ok) return fail(ctx, VLP_EINVAL, "br_rotations_per_block %u not available with %u wavefronts per rotation", rpb, r);
  if (t->br_blocks_per_cu < 1 || t->br_blocks_per_cu > 64) return fail(ctx, VLP_EINVAL, "br_blocks_per_cu out of [1, 64]");
  if (!(g == 128 || g == 256 || g == 512)) return fail(ctx, VLP_EINVAL, "ks_gates_per_block must be 128, 256 or 512");
  ctx->tune = *t;
  return VLP_OK;
}

// ---------------------------------------------------------------------------
// Keysets
// ---------------------------------------------------------------------------
extern "C" vlp_status vlp_keyset_load(vlp_ctx* ctx, const uint32_t* bk_dev, const uint32_t* ksk_dev, vlp_keyset** out) {
  if (!ctx) return VLP_EINVAL;
  if (!bk_dev || !ksk_dev || !out) return fail(ctx, VLP_EINVAL, "null argument");
  *out = nullptr;
  vlp_keyset* ks = new vlp_keyset{ctx, nullptr, nullptr, 0};
  vlp_status st = dev_alloc(ctx, (void**)&ks->bk_ntt, BK_NTT_WORDS * 4);
  if (st == VLP_OK) st = dev_alloc(ctx, (void**)&ks->ksk, KSK_WORDS * 4);
  if (st != VLP_OK) {
    dev_free(ctx, ks->bk_ntt, BK_NTT_WORDS * 4);
    delete ks;
    return st;
  }
  int e = launch_bk_transform(bk_dev, ks->bk_ntt, ctx->tw_fwd, ctx->stream);
  if (e == 0) e = launch_ksk_relayout(ksk_dev, ks->ksk, ctx->stream);
  if (e != 0) {
    dev_free(ctx, ks->bk_ntt, BK_NTT_WORDS * 4);
    dev_free(ctx, ks->ksk, KSK_WORDS * 4);
    delete ks;
    return fail(ctx, VLP_EHIP, "key preparation launch: %s", hipGetErrorString((hipError_t)e));
  }
  ctx->live_keysets++;
  *out = ks;
  return VLP_OK;
}

extern "C" vlp_status vlp_keyset_destroy(vlp_keyset* ks) {
  if (!ks) return VLP_EINVAL;
  vlp_ctx* ctx = ks->ctx;
  // Programs cached by vlp_evaluate for this keyset go first.
  for (auto it = ctx->eval_cache.begin(); it != ctx->eval_cache.end();) {
    if ((*it)->ks == ks) {
      (void)hipStreamSynchronize(ctx->stream);
      program_free(*it);
      it = ctx->eval_cache.erase(it);
    } else {
      ++it;
    }
  }
  if (ks->users) return fail(ctx, VLP_EBUSY, "keyset still used by %d programs", ks->users);
  (void)hipStreamSynchronize(ctx->stream);
  dev_free(ctx, ks->bk_ntt, BK_NTT_WORDS * 4);
  dev_free(ctx, ks->ksk, KSK_WORDS * 4);
  ctx->live_keysets--;
  delete ks;
  return VLP_OK;
}

// ---------------------------------------------------------------------------
// Elementwise calls
// ---------------------------------------------------------------------------
extern "C" vlp_status vlp_bootstrap(vlp_ctx* ctx, const vlp_keyset* ks, const uint32_t* in_dev, uint32_t* out_dev,
                                    uint32_t mu, size_t B) {
  if (!ctx) return VLP_EINVAL;
  if (B == 0) return VLP_OK;
  if (!ks || ks->ctx != ctx || !in_dev || !out_dev) return fail(ctx, VLP_EINVAL, "null or foreign argument");
  if (B > (1u << 26)) return fail(ctx, VLP_EINVAL, "B too large");
  if (ranges_overlap(in_dev, B * CT_n * 4, out_dev, B * CT_N * 4)) return fail(ctx, VLP_EINVAL, "in and out overlap");
  vlp_status st = ensure_scratch(ctx, B * sizeof(BrItem));
  if (st != VLP_OK) return st;
  BrItem* items = (BrItem*)ctx->scratch;
  LAUNCHCHECK(ctx, launch_make_br_items(items, (uint32_t)B, in_dev, nullptr, 1, 0, 0, mu, out_dev, ks->bk_ntt, ctx->stream));
  LAUNCHCHECK(ctx, timed_br(ctx, items, (uint32_t)B));
  return VLP_OK;
}

extern "C" vlp_status vlp_keyswitch(vlp_ctx* ctx, const vlp_keyset* ks, const uint32_t* in_dev, uint32_t* out_dev,
                                    size_t B) {
  if (!ctx) return VLP_EINVAL;
  if (B == 0) return VLP_OK;
  if (!ks || ks->ctx != ctx || !in_dev || !out_dev) return fail(ctx, VLP_EINVAL, "null or foreign argument");
  if (B > (1u << 26)) return fail(ctx, VLP_EINVAL, "B too large");
  if (ranges_overlap(in_dev, B * CT_N * 4, out_dev, B * CT_n * 4)) return fail(ctx, VLP_EINVAL, "in and out overlap");
  const size_t item_bytes = (B * sizeof(KsItem) + 255) & ~(size_t)255;
  vlp_status st = ensure_scratch(ctx, item_bytes + ks_digit_bytes(B));
  if (st != VLP_OK) return st;
  KsItem* items = (KsItem*)ctx->scratch;
  uint32_t* dig = (uint32_t*)((char*)ctx->scratch + item_bytes);
  LAUNCHCHECK(ctx, launch_make_ks_items(items, (uint32_t)B, in_dev, nullptr, 0, out_dev, ks->ksk, ctx->stream));
  LAUNCHCHECK(ctx, timed_ks(ctx, items, (uint32_t)B, ks->ksk, dig));
  return VLP_OK;
}

namespace {

// Argument checks shared by the two gate calls; VLP_OK when the call may run.
vlp_status gate_args(vlp_ctx* ctx, const vlp_keyset* ks, vlp_gate_op op, const uint32_t* a_dev, const uint32_t* b_dev,
                     const uint32_t* c_dev, uint32_t* out_dev, size_t B) {
  if (op < VLP_AND || op > VLP_MUX) return fail(ctx, VLP_EINVAL, "unknown gate op %d", (int)op);
  if (B == 0) return VLP_OK;
  if (!ks || ks->ctx != ctx || !a_dev || !out_dev) return fail(ctx, VLP_EINVAL, "null or foreign argument");
  if (op != VLP_NOT && !b_dev) return fail(ctx, VLP_EINVAL, "b is NULL");
  if ((op == VLP_MUX) != (c_dev != nullptr)) return fail(ctx, VLP_EINVAL, "c must be given for MUX only");
  if (B > (1u << 26)) return fail(ctx, VLP_EINVAL, "B too large");
  const size_t nb = B * CT_n * 4;
  if (ranges_overlap(a_dev, nb, out_dev, nb) || ranges_overlap(b_dev, nb, out_dev, nb) ||
      ranges_overlap(c_dev, nb, out_dev, nb))
    return fail(ctx, VLP_EINVAL, "output overlaps an input");
  return VLP_OK;
}

// Bytes of scratch a bootstrapped gate call over B gates lays out from `base`:
// sample-extracted outputs (one or two per gate), then the blind-rotation and
// key-switching items, then the key-switching digits.
constexpr size_t gate_scratch_bytes(vlp_gate_op op, size_t B) {
  return (((op == VLP_MUX ? 2 * B : B) * CT_N * 4 + 255) & ~(size_t)255) + (op == VLP_MUX ? 2 * B : B) * sizeof(BrItem) +
         B * sizeof(KsItem) + ks_digit_bytes(B);
}
static_assert(gate_scratch_bytes(VLP_MUX, NOALLOC_MAX_GATES) <= NOALLOC_BYTES, "fixed scratch too small");

// Enqueues B bootstrapped gates (op != NOT) with their scratch at `base`.
// Kernel timing (vlp_profile_enable) only when `timed`.
vlp_status gate_run(vlp_ctx* ctx, const vlp_keyset* ks, vlp_gate_op op, const uint32_t* a_dev, const uint32_t* b_dev,
                    const uint32_t* c_dev, uint32_t* out_dev, size_t B, void* base, bool timed) {
  const size_t units = op == VLP_MUX ? 2 * B : B;
  const size_t ext_bytes = (units * CT_N * 4 + 255) & ~(size_t)255;
  uint32_t* ext = (uint32_t*)base;
  BrItem* bri = (BrItem*)((char*)base + ext_bytes);
  KsItem* ksi = (KsItem*)((char*)bri + units * sizeof(BrItem));
  uint32_t* dig = (uint32_t*)((char*)ksi + B * sizeof(KsItem));
  int32_t ca, cb;
  uint32_t cst;
  gate_coeffs((uint8_t)op, &ca, &cb, &cst);
  LAUNCHCHECK(ctx, launch_make_br_items(bri, (uint32_t)B, a_dev, b_dev, ca, cb, cst, MU, ext, ks->bk_ntt, ctx->stream));
  if (op == VLP_MUX)
    LAUNCHCHECK(ctx, launch_make_br_items(bri + B, (uint32_t)B, a_dev, c_dev, -1, 1, 0u - MU, MU, ext + B * CT_N,
                                          ks->bk_ntt, ctx->stream));
  const bool prof = ctx->prof;
  ctx->prof = prof && timed;
  int e = timed_br(ctx, bri, (uint32_t)units);
  if (e == 0)
    e = launch_make_ks_items(ksi, (uint32_t)B, ext, op == VLP_MUX ? ext + B * CT_N : nullptr, op == VLP_MUX ? MU : 0u,
                             out_dev, ks->ksk, ctx->stream);
  if (e == 0) e = timed_ks(ctx, ksi, (uint32_t)B, ks->ksk, dig);
  ctx->prof = prof;
  if (e != 0) return fail(ctx, VLP_EHIP, "gate launch: %s", hipGetErrorString((hipError_t)e));
  return VLP_OK;
}

}  // namespace

extern "C" vlp_status vlp_gate(vlp_ctx* ctx, const vlp_keyset* ks, vlp_gate_op op, const uint32_t* a_dev,
                               const uint32_t* b_dev, const uint32_t* c_dev, uint32_t* out_dev, size_t B) {
  if (!ctx) return VLP_EINVAL;
  vlp_status st = gate_args(ctx, ks, op, a_dev, b_dev, c_dev, out_dev, B);
  if (st != VLP_OK || B == 0) return st;
  if (op == VLP_NOT) {
    LAUNCHCHECK(ctx, launch_negate(a_dev, out_dev, B * CT_n, ctx->stream));
    return VLP_OK;
  }
  st = ensure_scratch(ctx, gate_scratch_bytes(op, B) + 256);
  if (st != VLP_OK) return st;
  return gate_run(ctx, ks, op, a_dev, b_dev, c_dev, out_dev, B, ctx->scratch, true);
}

extern "C" vlp_status vlp_gate_noalloc(vlp_ctx* ctx, const vlp_keyset* ks, vlp_gate_op op, const uint32_t* a_dev,
                                       const uint32_t* b_dev, const uint32_t* c_dev, uint32_t* out_dev, size_t B) {
  if (!ctx) return VLP_EINVAL;
  vlp_status st = gate_args(ctx, ks, op, a_dev, b_dev, c_dev, out_dev, B);
  if (st != VLP_OK || B == 0) return st;
  if (B > NOALLOC_MAX_GATES)
    return fail(ctx, VLP_EINVAL, "B = %zu exceeds the %zu gates the fixed scratch holds", B, NOALLOC_MAX_GATES);
  if (op == VLP_NOT) {
    LAUNCHCHECK(ctx, launch_negate(a_dev, out_dev, B * CT_n, ctx->stream));
    return VLP_OK;
  }
  if (!ctx->noalloc) return fail(ctx, VLP_EHIP, "no fixed scratch on device %d", ctx->device);
  return gate_run(ctx, ks, op, a_dev, b_dev, c_dev, out_dev, B, ctx->noalloc, false);
}

// ---------------------------------------------------------------------------
// Programs
// ---------------------------------------------------------------------------
static void program_free(vlp_program* prog) {
  vlp_ctx* ctx = prog->ctx;
  if (prog->graph_exec) (void)hipGraphExecDestroy(prog->graph_exec);
  if (prog->graph) (void)hipGraphDestroy(prog->graph);
  dev_free(ctx, prog->br_items, 0);
  dev_free(ctx, prog->ks_items, 0);
  dev_free(ctx, prog->gate_buf, 0);
  dev_free(ctx, prog->ext_buf, 0);
  dev_free(ctx, prog->more_buf, 0);
  dev_free(ctx, prog->dig_buf, 0);
  ctx->used -= prog->bytes;
  ctx->step_reserve -= prog->step_bytes;
  prog->ks->users--;
  ctx->live_programs--;
  delete prog;
}

static vlp_status shape_words(const vlp_shape* sh, size_t* q, size_t* loc, size_t* pay) {
  const size_t M = sh->M, l = sh->l_I, d = sh->mode == VLP_IDM ? 1 : sh->d;
  *q = d * l;
  *loc = sh->mode == VLP_INTV ? M * d * 2 * l : M * d * l;
  *pay = M * sh->l_S;
  return VLP_OK;
}

extern "C" vlp_status vlp_server_encrypt(vlp_ctx* ctx, const vlp_shape* shape, const uint32_t* pk_loc,
                                         const uint32_t* pk_pay, const int64_t* loc, const uint8_t* pay,
                                         uint32_t* out_loc, uint32_t* out_pay) {
  if (!ctx) return VLP_EINVAL;
  if (!shape) return fail(ctx, VLP_EINVAL, "shape is NULL");
  const char* why = "";
  if (!shape_valid(*shape, &why)) return fail(ctx, VLP_EINVAL, "bad shape: %s", why);
  size_t wq, n_loc, n_pay;
  shape_words(shape, &wq, &n_loc, &n_pay);
  if (!pk_loc || !loc || !out_loc) return fail(ctx, VLP_EINVAL, "pk_loc, loc and out_loc are required");
  if (n_pay && (!pk_pay || !pay || !out_pay)) return fail(ctx, VLP_EINVAL, "l_S > 0 needs pk_pay, pay and out_pay");
  const size_t b_loc = n_loc * CT_n * 4, b_pay = n_pay * CT_n * 4;
  const size_t b_vals = n_loc / shape->l_I * sizeof(int64_t), b_bits = n_pay;
  // Each output either is its own public key (in place) or overlaps nothing.
  if (out_loc != pk_loc && ranges_overlap(out_loc, b_loc, pk_loc, b_loc))
    return fail(ctx, VLP_EINVAL, "out_loc partly overlaps pk_loc");
  if (n_pay && out_pay != pk_pay && ranges_overlap(out_pay, b_pay, pk_pay, b_pay))
    return fail(ctx, VLP_EINVAL, "out_pay partly overlaps pk_pay");
  if (ranges_overlap(out_loc, b_loc, loc, b_vals) || (n_pay && ranges_overlap(out_loc, b_loc, pk_pay, b_pay)) ||
      (n_pay && ranges_overlap(out_loc, b_loc, pay, b_bits)))
    return fail(ctx, VLP_EINVAL, "out_loc overlaps another argument");
  if (n_pay && (ranges_overlap(out_pay, b_pay, pk_loc, b_loc) || ranges_overlap(out_pay, b_pay, out_loc, b_loc) ||
                ranges_overlap(out_pay, b_pay, loc, b_vals) || ranges_overlap(out_pay, b_pay, pay, b_bits)))
    return fail(ctx, VLP_EINVAL, "out_pay overlaps another argument");
  LAUNCHCHECK(ctx, launch_server_enc(pk_loc, out_loc, n_loc, loc, nullptr, shape->l_I, ctx->stream));
  if (n_pay) LAUNCHCHECK(ctx, launch_server_enc(pk_pay, out_pay, n_pay, nullptr, pay, 1, ctx->stream));
  return VLP_OK;
}

// Device memory of a program: work items, internal gate outputs, extraction
// slots of its widest level, k-input XOR operand lists, key-switching digits,
// and its share of the merged-step scratch.
struct ProgramSizes {
  std::vector<int32_t> slot;        // gate -> user output slot (v_out[i] = i, R[j] = M + j) or -1
  std::vector<uint32_t> internal;   // gate -> internal buffer index (if slot < 0)
  uint32_t n_internal = 0, max_br = 0, max_ks = 0;
  uint64_t n_br = 0, n_ks = 0;
  size_t n_more = 0;
  size_t b_items = 0, k_items = 0, b_gate = 0, b_ext = 0, b_more = 0, b_dig = 0, total = 0, step = 0;
};

static const char* program_sizes(const Netlist& nl, bool with_v_out, ProgramSizes& z) {
  const size_t M = nl.M, lS = nl.l_S;
  z.slot.assign(nl.gates.size(), -1);
  if (with_v_out)
    for (size_t i = 0; i < M; ++i)
      if (nl.v_of_record[i].src == Src::Gate) z.slot[nl.v_of_record[i].index] = (int32_t)i;
  for (size_t j = 0; j < lS; ++j) {
    const Operand& r = nl.result[j];
    if (r.src != Src::Gate || z.slot[r.index] >= 0) return "a result bit is not a distinct gate";
    z.slot[r.index] = (int32_t)(M + j);
  }
  z.internal.assign(nl.gates.size(), 0);
  for (size_t g = 0; g < nl.gates.size(); ++g)
    if (z.slot[g] < 0) z.internal[g] = z.n_internal++;
  std::vector<uint32_t> nbr(nl.levels + 1, 0), nks(nl.levels + 1, 0);
  for (const Gate& G : nl.gates) {
    nbr[G.level] += G.op == VLP_MUX ? 2 : 1;
    nks[G.level] += 1;
  }
  for (uint32_t L = 1; L <= nl.levels; ++L) {
    z.max_br = std::max(z.max_br, nbr[L]);
    z.max_ks = std::max(z.max_ks, nks[L]);
  }
  z.n_br = nl.blind_rotations();
  z.n_ks = nl.key_switches();
  // Operand-list entries of the k-input XORs: the non-trivial operands past the first two.
  for (const Gate& G : nl.gates) {
    if (G.op != OP_XORK) continue;
    size_t live = (G.a.is_const() ? 0 : 1) + (G.b.is_const() ? 0 : 1);
    for (uint32_t t = 0; t < G.xk_count; ++t) live += nl.xk_ops[G.xk_first + t].is_const() ? 0 : 1;
    z.n_more += live > 2 ? live - 2 : 0;
  }
  z.b_items = z.n_br * sizeof(BrItem);
  z.k_items = z.n_ks * sizeof(KsItem);
  z.b_gate = (size_t)z.n_internal * CT_n * 4;
  z.b_ext = (size_t)z.max_br * CT_N * 4;
  z.b_more = z.n_more * sizeof(const uint32_t*);
  z.b_dig = ks_digit_bytes(z.max_ks);
  z.total = z.b_items + z.k_items + z.b_gate + z.b_ext + z.b_more + z.b_dig;
  z.step = (((size_t)z.max_br * sizeof(BrItem) + 255) & ~(size_t)255) + (size_t)z.max_ks * sizeof(KsItem) + 256;
  return nullptr;
}

// The circuits of the calls without a circuit argument (and of a NULL one).
static const vlp_circuit DEFAULT_CIRCUIT = {1, 0};
static const vlp_circuit& circuit_or_default(const vlp_circuit* c) { return c ? *c : DEFAULT_CIRCUIT; }

extern "C" vlp_status vlp_plan_bytes(const vlp_shape* shape, int with_v_out, size_t* bytes) {
  return vlp_plan_bytes_ex(shape, nullptr, with_v_out, bytes);
}

extern "C" vlp_status vlp_plan_bytes_ex(const vlp_shape* shape, const vlp_circuit* circuit, int with_v_out,
                                        size_t* bytes) {
  if (!shape || !bytes) return VLP_EINVAL;
  Netlist nl;
  const char* why = "";
  if (!build_netlist(*shape, circuit_or_default(circuit), nl, &why)) return VLP_EINVAL;
  ProgramSizes z;
  if (program_sizes(nl, with_v_out != 0, z)) return VLP_EINVAL;
  *bytes = z.total + z.step;
  return VLP_OK;
}

extern "C" vlp_status vlp_plan_counts(const vlp_shape* shape, uint64_t* gates, uint64_t* brs, uint64_t* kss,
                                      uint32_t* levels) {
  return vlp_plan_counts_ex(shape, nullptr, gates, brs, kss, levels);
}

extern "C" vlp_status vlp_plan_counts_ex(const vlp_shape* shape, const vlp_circuit* circuit, uint64_t* gates,
                                         uint64_t* brs, uint64_t* kss, uint32_t* levels) {
  if (!shape) return VLP_EINVAL;
  Netlist nl;
  const char* why = "";
  if (!build_netlist(*shape, circuit_or_default(circuit), nl, &why)) return VLP_EINVAL;
  if (gates) *gates = nl.gates.size();
  if (brs) *brs = nl.blind_rotations();
  if (kss) *kss = nl.key_switches();
  if (levels) *levels = nl.levels;
  return VLP_OK;
}

extern "C" vlp_status vlp_program_create(vlp_ctx* ctx, const vlp_keyset* ks_c, const vlp_shape* shape,
                                         const uint32_t* query_dev, const uint32_t* db_loc_dev,
                                         const uint32_t* db_pay_dev, uint32_t* R_dev, uint32_t* v_out_dev,
                                         vlp_program** out) {
  return vlp_program_create_ex(ctx, ks_c, shape, nullptr, query_dev, db_loc_dev, db_pay_dev, R_dev, v_out_dev, out);
}

extern "C" vlp_status vlp_program_create_ex(vlp_ctx* ctx, const vlp_keyset* ks_c, const vlp_shape* shape,
                                            const vlp_circuit* circuit_arg, const uint32_t* query_dev,
                                            const uint32_t* db_loc_dev, const uint32_t* db_pay_dev, uint32_t* R_dev,
                                            uint32_t* v_out_dev, vlp_program** out) {
  if (!ctx) return VLP_EINVAL;
  const vlp_circuit& circuit = circuit_or_default(circuit_arg);
  vlp_keyset* ks = const_cast<vlp_keyset*>(ks_c);
  if (!ks || ks->ctx != ctx || !shape || !out || !query_dev || !db_loc_dev)
    return fail(ctx, VLP_EINVAL, "null or foreign argument");
  *out = nullptr;
  if (shape->l_S > 0 && (!db_pay_dev || !R_dev)) return fail(ctx, VLP_EINVAL, "l_S > 0 needs db_pay and R");
  Netlist nl;
  const char* why = "";
  if (!build_netlist(*shape, circuit, nl, &why)) return fail(ctx, VLP_EINVAL, "bad shape: %s", why);
  size_t wq, wl, wp;
  shape_words(shape, &wq, &wl, &wp);
  const size_t M = nl.M, lS = nl.l_S;
  if (ranges_overlap(R_dev, lS * CT_n * 4, v_out_dev, M * CT_n * 4))
    return fail(ctx, VLP_EINVAL, "R and v_out overlap");
  for (const void* in : {(const void*)query_dev, (const void*)db_loc_dev, (const void*)db_pay_dev}) {
    const size_t inb = in == query_dev ? wq * CT_n * 4 : (in == db_loc_dev ? wl * CT_n * 4 : wp * CT_n * 4);
    if (ranges_overlap(in, inb, R_dev, lS * CT_n * 4) || ranges_overlap(in, inb, v_out_dev, M * CT_n * 4))
      return fail(ctx, VLP_EINVAL, "an output overlaps an input");
  }

  // Output slots: v of record i -> v_out[i] (if given); R[j] -> R[j]; other gates internal.
  ProgramSizes z;
  if (const char* bad = program_sizes(nl, v_out_dev != nullptr, z))
    return fail(ctx, VLP_EINVAL, "unsupported shape: %s", bad);
  const std::vector<int32_t>& slot = z.slot;
  const std::vector<uint32_t>& internal = z.internal;
  std::vector<std::vector<uint32_t>> by_level(nl.levels + 1);
  for (size_t g = 0; g < nl.gates.size(); ++g) by_level[nl.gates[g].level].push_back((uint32_t)g);
  const uint64_t n_br = z.n_br, n_ks = z.n_ks;
  const size_t n_more = z.n_more;
  const size_t b_items = z.b_items, k_items = z.k_items, b_gate = z.b_gate, b_ext = z.b_ext, b_more = z.b_more,
               b_dig = z.b_dig, total = z.total;
  // The merged-step scratch grows with the reserve at creation (vlp_step never allocates).
  const size_t new_reserve = ctx->step_reserve + z.step;
  const size_t grow = new_reserve > ctx->scratch_bytes ? new_reserve : 0;
  if (ctx->used + total + (grow ? grow - ctx->scratch_bytes : 0) > ctx->budget)
    return fail(ctx, VLP_EBUDGET, "program needs %zu bytes (+%zu of step scratch); %zu of %zu in use", total,
                grow ? grow - ctx->scratch_bytes : 0, ctx->used, ctx->budget);
  if (grow) {
    vlp_status gst = ensure_scratch(ctx, grow);
    if (gst != VLP_OK) return gst;
  }
  const uint32_t max_br = z.max_br;

  vlp_program* prog = new vlp_program();
  prog->ctx = ctx;
  prog->ks = ks;
  prog->shape = *shape;
  prog->circuit = circuit;
  prog->gates = nl.gates.size();
  prog->brs = n_br;
  prog->kss = n_ks;
  prog->max_br_level = max_br;
  prog->q = query_dev;
  prog->loc = db_loc_dev;
  prog->pay = db_pay_dev;
  prog->R = R_dev;
  prog->v = v_out_dev;
  hipError_t e = hipSuccess;
  if (b_items) e = hipMalloc((void**)&prog->br_items, b_items);
  if (e == hipSuccess && k_items) e = hipMalloc((void**)&prog->ks_items, k_items);
  if (e == hipSuccess && b_gate) e = hipMalloc((void**)&prog->gate_buf, b_gate);
  if (e == hipSuccess && b_ext) e = hipMalloc((void**)&prog->ext_buf, b_ext);
  if (e == hipSuccess && b_more) e = hipMalloc((void**)&prog->more_buf, b_more);
  if (e == hipSuccess && b_dig) e = hipMalloc((void**)&prog->dig_buf, b_dig);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(prog->br_items);
    (void)hipFree(prog->ks_items);
    (void)hipFree(prog->gate_buf);
    (void)hipFree(prog->ext_buf);
    (void)hipFree(prog->more_buf);
    (void)hipFree(prog->dig_buf);
    delete prog;
    return fail(ctx, e == hipErrorOutOfMemory ? VLP_EBUDGET : VLP_EHIP, "program allocation: %s",
                hipGetErrorString(e));
  }
  prog->bytes = total;
  prog->step_bytes = z.step;
  ctx->used += total;
  ctx->step_reserve += z.step;
  ks->users++;
  ctx->live_programs++;

  // Resolve operands to device pointers.
  auto ptr = [&](const Operand& o) -> const uint32_t* {
    switch (o.src) {
      case Src::Query: return query_dev + (size_t)o.index * CT_n;
      case Src::DbLoc: return db_loc_dev + (size_t)o.index * CT_n;
      case Src::DbPay: return db_pay_dev + (size_t)o.index * CT_n;
      case Src::Gate: {
        const int32_t s = slot[o.index];
        if (s < 0) return prog->gate_buf + (size_t)internal[o.index] * CT_n;
        if ((size_t)s < M) return v_out_dev + (size_t)s * CT_n;
        return R_dev + (size_t)(s - M) * CT_n;
      }
      default: return nullptr;
    }
  };
  // A BR unit: (0, cst) + ca * x + cb * y, with trivial operands folded into cst.
  auto unit = [&](int32_t ca, Operand x, int32_t cb, Operand y, uint32_t cst, uint32_t* out) {
    BrItem it{};
    if (x.is_const()) {
      cst += (uint32_t)ca * encode_bit(x.index);
      ca = 0;
    }
    if (y.is_const()) {
      cst += (uint32_t)cb * encode_bit(y.index);
      cb = 0;
    }
    const uint32_t* px = ca ? ptr(x) : nullptr;
    const uint32_t* py = cb ? ptr(y) : nullptr;
    if (!px) {  // the kernel needs the first operand
      px = py;
      ca = cb;
      py = nullptr;
      cb = 0;
    }
    if (!px) {  // trivial operands only (a MUX rotation with a trivial select): any ciphertext times 0
      px = query_dev;
      ca = 0;
    }
    it.a = px;
    it.b = py;
    it.ca = ca;
    it.cb = cb;
    it.cst = cst;
    it.mu = MU;
    it.out = out;
    it.bk = ks->bk_ntt;
    return it;
  };
  std::vector<const uint32_t*> hm;  // operand lists of k-input XOR items
  hm.reserve(n_more);
  // A k-input XOR unit: (0, (k-1)/4) + 2 * (sum of the operands), trivial ones folded.
  auto xork_unit = [&](const Gate& G, uint32_t* out) {
    std::vector<Operand> ops{G.a, G.b};
    for (uint32_t t = 0; t < G.xk_count; ++t) ops.push_back(nl.xk_ops[G.xk_first + t]);
    uint32_t cst = (uint32_t)(ops.size() - 1) << 30;
    std::vector<const uint32_t*> live;
    for (const Operand& o : ops) {
      if (o.is_const()) cst += 2u * encode_bit(o.index);
      else live.push_back(ptr(o));
    }
    BrItem it{};
    it.a = live[0];
    it.ca = 2;
    it.b = live.size() > 1 ? live[1] : nullptr;
    it.cb = live.size() > 1 ? 2 : 0;
    if (live.size() > 2) {
      it.more = prog->more_buf + hm.size();
      it.n_more = (uint32_t)(live.size() - 2);
      it.cm = 2;
      for (size_t t = 2; t < live.size(); ++t) hm.push_back(live[t]);
    }
    it.cst = cst;
    it.mu = MU;
    it.out = out;
    it.bk = ks->bk_ntt;
    return it;
  };
  std::vector<BrItem> hb;
  std::vector<KsItem> hk;
  hb.reserve(n_br);
  hk.reserve(n_ks);
  for (uint32_t L = 1; L <= nl.levels; ++L) {
    Level lv{(uint32_t)hb.size(), 0, (uint32_t)hk.size(), 0};
    uint32_t e_slot = 0;
    for (uint32_t g : by_level[L]) {
      const Gate& G = nl.gates[g];
      uint32_t* gout = const_cast<uint32_t*>(ptr(Operand::gate(g)));
      KsItem k{};
      k.out = gout;
      k.ksk = ks->ksk;
      if (G.op == VLP_MUX) {
        uint32_t* u1 = prog->ext_buf + (size_t)e_slot++ * CT_N;
        uint32_t* u2 = prog->ext_buf + (size_t)e_slot++ * CT_N;
        hb.push_back(unit(1, G.a, 1, G.b, 0u - MU, u1));
        hb.push_back(unit(-1, G.a, 1, G.c, 0u - MU, u2));
        k.u1 = u1;
        k.u2 = u2;
        k.cst = MU;
      } else if (G.op == OP_XORK) {
        uint32_t* u1 = prog->ext_buf + (size_t)e_slot++ * CT_N;
        hb.push_back(xork_unit(G, u1));
        k.u1 = u1;
        k.u2 = nullptr;
        k.cst = 0;
      } else {
        int32_t ca, cb;
        uint32_t cst;
        gate_coeffs(G.op, &ca, &cb, &cst);
        uint32_t* u1 = prog->ext_buf + (size_t)e_slot++ * CT_N;
        hb.push_back(unit(ca, G.a, cb, G.b, cst, u1));
        k.u1 = u1;
        k.u2 = nullptr;
        k.cst = 0;
      }
      hk.push_back(k);
    }
    lv.br_count = (uint32_t)hb.size() - lv.br_first;
    lv.ks_count = (uint32_t)hk.size() - lv.ks_first;
    prog->levels.push_back(lv);
  }
  if (b_items) e = hipMemcpy(prog->br_items, hb.data(), b_items, hipMemcpyHostToDevice);
  if (e == hipSuccess && k_items) e = hipMemcpy(prog->ks_items, hk.data(), k_items, hipMemcpyHostToDevice);
  if (e == hipSuccess && b_more) e = hipMemcpy(prog->more_buf, hm.data(), b_more, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    program_free(prog);
    return fail(ctx, VLP_EHIP, "program upload: %s", hipGetErrorString(e));
  }
  *out = prog;
  return VLP_OK;
}

extern "C" vlp_status vlp_program_reset(vlp_program* prog) {
  if (!prog) return VLP_EINVAL;
  prog->next_level = 0;
  return VLP_OK;
}

extern "C" vlp_status vlp_program_counts(const vlp_program* prog, uint64_t* gates, uint64_t* brs, uint64_t* kss,
                                         uint32_t* levels) {
  if (!prog) return VLP_EINVAL;
  if (gates) *gates = prog->gates;
  if (brs) *brs = prog->brs;
  if (kss) *kss = prog->kss;
  if (levels) *levels = (uint32_t)prog->levels.size();
  return VLP_OK;
}

extern "C" vlp_status vlp_program_level_counts(const vlp_program* prog, uint32_t level, uint64_t* blind_rotations,
                                               uint64_t* key_switches) {
  if (!prog || level >= prog->levels.size()) return VLP_EINVAL;
  if (blind_rotations) *blind_rotations = prog->levels[level].br_count;
  if (key_switches) *key_switches = prog->levels[level].ks_count;
  return VLP_OK;
}

extern "C" vlp_status vlp_program_destroy(vlp_program* prog) {
  if (!prog) return VLP_EINVAL;
  vlp_ctx* ctx = prog->ctx;
  HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
  program_free(prog);
  return VLP_OK;
}

static vlp_status run_level(vlp_ctx* ctx, vlp_program* prog, uint32_t L) {
  const Level& lv = prog->levels[L];
  LAUNCHCHECK(ctx, timed_br(ctx, prog->br_items + lv.br_first, lv.br_count));
  LAUNCHCHECK(ctx, timed_ks(ctx, prog->ks_items + lv.ks_first, lv.ks_count, prog->ks->ksk, prog->dig_buf));
  return VLP_OK;
}

extern "C" vlp_status vlp_step(vlp_ctx* ctx, vlp_program* const* progs, size_t n, size_t* remaining) {
  if (!ctx) return VLP_EINVAL;
  if (n && !progs) return fail(ctx, VLP_EINVAL, "progs is NULL");
  // A program listed twice would have its level's items batched twice (and
  // its level advanced twice): rejected before any work is enqueued.
  {
    std::vector<const vlp_program*> sorted(progs, progs + n);
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
      return fail(ctx, VLP_EINVAL, "a program appears more than once in progs");
  }
  // Gather this step's BR and KS items of every unfinished program into one batch.
  size_t nbr = 0, nks = 0, left = 0;
  for (size_t p = 0; p < n; ++p) {
    vlp_program* pr = progs[p];
    if (!pr || pr->ctx != ctx) return fail(ctx, VLP_EINVAL, "null or foreign program");
    if (pr->next_level < pr->levels.size()) {
      nbr += pr->levels[pr->next_level].br_count;
      nks += pr->levels[pr->next_level].ks_count;
    }
  }
  if (nbr) {
    const size_t bytes = nbr * sizeof(BrItem) + nks * sizeof(KsItem) + 256;
    vlp_status st = ensure_scratch(ctx, bytes);
    if (st != VLP_OK) return st;
    BrItem* bri = (BrItem*)ctx->scratch;
    KsItem* ksi = (KsItem*)((char*)ctx->scratch + ((nbr * sizeof(BrItem) + 255) & ~(size_t)255));
    size_t ob = 0, ok = 0;
    std::vector<std::pair<size_t, size_t>> ks_groups;  // (first, count) per program
    for (size_t p = 0; p < n; ++p) {
      vlp_program* pr = progs[p];
      if (pr->next_level >= pr->levels.size()) continue;
      const Level& lv = pr->levels[pr->next_level];
      HIPCHECK(ctx, hipMemcpyAsync(bri + ob, pr->br_items + lv.br_first, lv.br_count * sizeof(BrItem),
                                   hipMemcpyDeviceToDevice, ctx->stream));
      HIPCHECK(ctx, hipMemcpyAsync(ksi + ok, pr->ks_items + lv.ks_first, lv.ks_count * sizeof(KsItem),
                                   hipMemcpyDeviceToDevice, ctx->stream));
      ks_groups.push_back({ok, lv.ks_count});
      ob += lv.br_count;
      ok += lv.ks_count;
    }
    LAUNCHCHECK(ctx, timed_br(ctx, bri, (uint32_t)nbr));
    size_t gi = 0;
    for (size_t p = 0; p < n; ++p) {
      vlp_program* pr = progs[p];
      if (pr->next_level >= pr->levels.size()) continue;
      LAUNCHCHECK(ctx,
                  timed_ks(ctx, ksi + ks_groups[gi].first, (uint32_t)ks_groups[gi].second, pr->ks->ksk, pr->dig_buf));
      gi++;
    }
  }
  for (size_t p = 0; p < n; ++p) {
    vlp_program* pr = progs[p];
    if (pr->next_level < pr->levels.size()) pr->next_level++;
    if (pr->next_level < pr->levels.size()) left++;
  }
  if (remaining) *remaining = left;
  return VLP_OK;
}

extern "C" vlp_status vlp_program_run(vlp_ctx* ctx, vlp_program* prog, int use_graph) {
  if (!ctx || !prog || prog->ctx != ctx) return ctx ? fail(ctx, VLP_EINVAL, "null or foreign program") : VLP_EINVAL;
  // The graph holds every level: a program part-way through (vlp_step) runs
  // its remaining levels without it.
  if (!use_graph || prog->next_level != 0) {
    for (uint32_t L = prog->next_level; L < prog->levels.size(); ++L) {
      vlp_status st = run_level(ctx, prog, L);
      if (st != VLP_OK) return st;
    }
    prog->next_level = (uint32_t)prog->levels.size();
    return VLP_OK;
  }
  if (prog->graph_exec && memcmp(&prog->graph_tune, &ctx->tune, sizeof(vlp_tuning)) != 0) {
    // Captured with another launch shape: capture again with the current one.
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    (void)hipGraphExecDestroy(prog->graph_exec);
    (void)hipGraphDestroy(prog->graph);
    prog->graph_exec = nullptr;
    prog->graph = nullptr;
  }
  if (!prog->graph_exec) {
    prog->graph_tune = ctx->tune;
    HIPCHECK(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    vlp_status st = VLP_OK;
    for (uint32_t L = 0; L < prog->levels.size() && st == VLP_OK; ++L) st = run_level(ctx, prog, L);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(ctx->stream, &g);
    if (st != VLP_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return fail(ctx, VLP_EHIP, "graph capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&prog->graph_exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      return fail(ctx, VLP_EHIP, "graph instantiate: %s", hipGetErrorString(e));
    }
    prog->graph = g;
  }
  HIPCHECK(ctx, hipGraphLaunch(prog->graph_exec, ctx->stream));
  prog->next_level = (uint32_t)prog->levels.size();
  return VLP_OK;
}

extern "C" vlp_status vlp_evaluate(vlp_ctx* ctx, const vlp_keyset* ks, const vlp_shape* shape,
                                   const uint32_t* query_dev, const uint32_t* db_loc_dev, const uint32_t* db_pay_dev,
                                   uint32_t* R_dev, uint32_t* v_out_dev) {
  return vlp_evaluate_ex(ctx, ks, shape, nullptr, query_dev, db_loc_dev, db_pay_dev, R_dev, v_out_dev);
}

extern "C" vlp_status vlp_evaluate_ex(vlp_ctx* ctx, const vlp_keyset* ks, const vlp_shape* shape,
                                      const vlp_circuit* circuit_arg, const uint32_t* query_dev,
                                      const uint32_t* db_loc_dev, const uint32_t* db_pay_dev, uint32_t* R_dev,
                                      uint32_t* v_out_dev) {
  if (!ctx) return VLP_EINVAL;
  if (!shape) return fail(ctx, VLP_EINVAL, "shape is NULL");
  const vlp_circuit& circuit = circuit_or_default(circuit_arg);
  vlp_program* prog = nullptr;
  for (auto it = ctx->eval_cache.begin(); it != ctx->eval_cache.end(); ++it) {
    vlp_program* p = *it;
    if (p->ks == ks && memcmp(&p->shape, shape, sizeof(vlp_shape)) == 0 &&
        p->circuit.optimized == circuit.optimized && p->circuit.agg_k == circuit.agg_k && p->q == query_dev &&
        p->loc == db_loc_dev && p->pay == db_pay_dev && p->R == R_dev && p->v == v_out_dev) {
      prog = p;
      ctx->eval_cache.erase(it);
      break;
    }
  }
  if (!prog) {
    vlp_status st =
        vlp_program_create_ex(ctx, ks, shape, &circuit, query_dev, db_loc_dev, db_pay_dev, R_dev, v_out_dev, &prog);
    if (st == VLP_EBUDGET && !ctx->eval_cache.empty()) {
      // Make room by dropping cached programs, then retry once.
      (void)hipStreamSynchronize(ctx->stream);
      for (vlp_program* p : ctx->eval_cache) program_free(p);
      ctx->eval_cache.clear();
      st = vlp_program_create_ex(ctx, ks, shape, &circuit, query_dev, db_loc_dev, db_pay_dev, R_dev, v_out_dev, &prog);
    }
    if (st != VLP_OK) return st;
  }
  ctx->eval_cache.push_front(prog);
  while (ctx->eval_cache.size() > 8) {
    (void)hipStreamSynchronize(ctx->stream);
    program_free(ctx->eval_cache.back());
    ctx->eval_cache.pop_back();
  }
  prog->next_level = 0;
  return vlp_program_run(ctx, prog, 1);
}

extern "C" vlp_status vlp_profile_enable(vlp_ctx* ctx, int enable) {
  if (!ctx) return VLP_EINVAL;
  ctx->prof = enable != 0;
  return VLP_OK;
}

extern "C" vlp_status vlp_profile_read(vlp_ctx* ctx, vlp_kernel_stats* br, vlp_kernel_stats* ks) {
  if (!ctx) return VLP_EINVAL;
  HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
  vlp_kernel_stats acc[2] = {{0, 0, 0.0}, {0, 0, 0.0}};
  for (const auto& m : ctx->marks) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, m.e0, m.e1) == hipSuccess) {
      acc[m.kind].launches++;
      acc[m.kind].items += m.items;
      acc[m.kind].ms += ms;
    }
    ctx->event_pool.push_back(m.e0);
    ctx->event_pool.push_back(m.e1);
  }
  ctx->marks.clear();
  if (br) *br = acc[0];
  if (ks) *ks = acc[1];
  return VLP_OK;
}
