// C ABI of spvgpu: argument checks, workspace layout and launch order.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <utility>
#include <vector>

#include "spv_checks.h"
#include "spv_internal.h"

// Scratch of spv_validate_noalloc: one copy per GPU, held until the process
// ends.  Host code never uses this name as an address: the device address of
// each GPU's copy is resolved once per device (spv_create) and kept below.
static __device__ __align__(256) unsigned char scratch[SPV_NOALLOC_SCRATCH_BYTES];

struct spv_ctx {
  int device;
  int n_cu;
  int blocks_per_cu;   // persistent grid of the decode/validate kernels
  int occupancy;       // resident blocks per CU of the main kernel
  int chain_occ;       // resident blocks per CU of the chain pass
  int walk_occ;        // resident blocks per CU of the resolved walk
  int encode_block;    // records per encode block
  int enc_count_occ;   // resident blocks per CU of the encoder's count pass
  int enc_scatter_occ; // resident blocks per CU of the encoder's scatter pass
  hipError_t last;
  char msg[256];
  bool timing;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;  // created events
  size_t ev_used;                                          // pairs recorded since the last read
  void* scratch;       // this device's copy of the no-allocation scratch (nullptr if unresolved)
};

namespace spv {
int main_occupancy();
int chain_occupancy();
int walk_occupancy();
int encode_occupancy(int pass);
}

namespace {

// Device address of each GPU's scratch copy, resolved once per device.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// (with `dev` current)
void* resolve_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[dev] == nullptr) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch[dev] = ptr;
  }
  return g_scratch[dev];
}

struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) {
      ok = false;
      return;
    }
    if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

int fail_hip(spv_ctx* ctx, hipError_t e) {
  if (ctx) {
    ctx->last = e;
    snprintf(ctx->msg, sizeof(ctx->msg), "%s", hipGetErrorString(e));
  }
  return SPV_ERR_HIP;
}

int check_launch(spv_ctx* ctx) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail_hip(ctx, e);
  return SPV_SUCCESS;
}

// Option bits of spv_validate: the three known ones, the rules only with the
// semantic stage.
bool flags_ok(uint32_t f) {
  if (f & ~(SPV_OPT_NO_SEMANTIC | SPV_OPT_MODULE_RULES | SPV_OPT_DEBUG_CHECKS | SPV_OPT_SEM_OFFSETS |
            SPV_OPT_DEF_BEFORE_USE))
    return false;
  return !((f & SPV_OPT_NO_SEMANTIC) && (f & (SPV_OPT_MODULE_RULES | SPV_OPT_SEM_OFFSETS | SPV_OPT_DEF_BEFORE_USE)));
}

// SPV_OPT_DEBUG_CHECKS: the device check of the module offsets.  status[0]
// collects a violation bit; a single block clears it first.
__global__ void k_dbg_clear(uint32_t* status) { status[0] = 0; }

__global__ __launch_bounds__(256) void k_dbg_offsets(const int64_t* mod_off, int64_t M, int64_t W,
                                                      uint32_t* status) {
  const int64_t gtid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nth = int64_t(gridDim.x) * blockDim.x;
  bool bad = false;
  if (gtid == 0) bad = !spv::offsets_ends_ok(mod_off[0], mod_off[M], W);
  for (int64_t i = gtid; i < M; i += nth) bad |= !spv::offsets_pair_ok(mod_off[i], mod_off[i + 1]);
  if (bad) atomicOr(status, 1u);
}

// Runs the offset check and reads its verdict (synchronises the stream).
int debug_check_offsets(spv_ctx* ctx, const int64_t* mod_off, int64_t M, int64_t W, uint32_t* status,
                        hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) return fail_hip(ctx, hipGetLastError());
  if (cs != hipStreamCaptureStatusNone) return SPV_ERR_INVALID_ARG;  // a read-back cannot be captured
  hipLaunchKernelGGL(k_dbg_clear, dim3(1), dim3(1), 0, s, status);
  const int64_t g = M / 256 + 1;
  hipLaunchKernelGGL(k_dbg_offsets, dim3(int(g > 4096 ? 4096 : g)), dim3(256), 0, s, mod_off, M, W, status);
  uint32_t h = 0;
  hipError_t e = hipMemcpyAsync(&h, status, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail_hip(ctx, e);
  return h ? SPV_ERR_INVALID_ARG : SPV_SUCCESS;
}

int run_validate(spv_ctx* ctx, const uint32_t* words, const int64_t* mod_off, int64_t n_modules, int64_t n_words,
                 uint32_t* idx_off, uint16_t* idx_op, int64_t idx_cap, spv_result* results, int semantic, void* ws,
                 size_t ws_bytes, void* stream, bool allow_timing = true, bool rules = false, bool debug = false,
                 uint32_t diag_flags = 0) {
  if (!ctx) return SPV_ERR_INVALID_ARG;
  if (n_modules < 0 || n_words < 0) return SPV_ERR_INVALID_ARG;
  if (n_modules >= (int64_t(1) << 31) - 1) return SPV_ERR_LIMIT;
  if (n_modules == 0) return n_words == 0 ? SPV_SUCCESS : SPV_ERR_INVALID_ARG;
  if (!mod_off || !results) return SPV_ERR_INVALID_ARG;
  if (n_words > 0 && (!words || (reinterpret_cast<uintptr_t>(words) & 15u))) return SPV_ERR_INVALID_ARG;
  bool index = idx_off != nullptr || idx_op != nullptr;
  if (index && (!idx_off || !idx_op)) return SPV_ERR_INVALID_ARG;
  if (index && idx_cap < n_words) return SPV_ERR_CAPACITY;
  if (diag_flags && !index) return SPV_ERR_INVALID_ARG;  // the positions are found through the index
  spv::Layout L = spv::make_layout(n_modules, n_words);
  if (!ws || ws_bytes < L.total) return SPV_ERR_WORKSPACE;
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail_hip(ctx, hipErrorInvalidDevice);
  char* base = static_cast<char*>(ws);
  if (debug) {
    const int rc = debug_check_offsets(ctx, mod_off, n_modules, n_words,
                                       reinterpret_cast<uint32_t*>(base + L.ctrl) + spv::kCtlDebug,
                                       static_cast<hipStream_t>(stream));
    if (rc != SPV_SUCCESS) return rc;
  }
  spv::VParams p;
  p.words = words;
  p.mod_off = mod_off;
  p.M = n_modules;
  p.W = n_words;
  p.n_tiles = (n_words + spv::kTileWords - 1) / spv::kTileWords;
  p.idx_off = idx_off;
  p.idx_op = idx_op;
  p.results = results;
  p.ctrl = reinterpret_cast<uint32_t*>(base + L.ctrl);
  p.tileA = reinterpret_cast<unsigned long long*>(base + L.tileA);
  p.tileB = reinterpret_cast<unsigned long long*>(base + L.tileB);
  p.tfm = reinterpret_cast<int32_t*>(base + L.tfm);
  p.mods = reinterpret_cast<spv::ModState*>(base + L.mods);
  p.idmap = reinterpret_cast<unsigned long long*>(base + L.idmap);
  p.tsum = reinterpret_cast<uint32_t*>(base + L.tsum);
  p.lst = reinterpret_cast<uint32_t*>(base + L.lst);
  p.tres = reinterpret_cast<uint32_t*>(base + L.tres);
  p.rstate = reinterpret_cast<unsigned long long*>(base + L.rstate);
  p.p2list = reinterpret_cast<uint32_t*>(base + L.p2list);
  p.semantic = semantic;
  p.index = index ? 1 : 0;
  p.sched_static = 0;
  // small batches (a module per thread of one block): the second pass decides
  // its own work and writes the results (no finalize launch)
  p.p1_inline = (semantic && n_modules <= spv::kBlock && p.n_tiles > 0) ? 1 : 0;
  p.rules = rules ? 1 : 0;
  p.diag = reinterpret_cast<uint4*>(base + L.diag);
  p.sem_offsets = (diag_flags & SPV_OPT_SEM_OFFSETS) ? 1 : 0;
  p.before_use = (diag_flags & SPV_OPT_DEF_BEFORE_USE) ? 1 : 0;
  hipStream_t s = static_cast<hipStream_t>(stream);

  int64_t plan_units = n_modules > p.n_tiles ? n_modules : p.n_tiles;
  int64_t pg = plan_units / 256 + 1;
  int64_t chunks = n_words / 16384 + 1;
  if (semantic && chunks > pg) pg = chunks;
  int plan_grid = int(pg > 4096 ? 4096 : pg);
  spv::launch_plan(p, plan_grid, s);
  int r = check_launch(ctx);
  if (r) return r;
  int64_t grid = int64_t(ctx->n_cu) * ctx->blocks_per_cu;
  if (grid > p.n_tiles) grid = p.n_tiles;
  if (grid > 0) {
    std::pair<hipEvent_t, hipEvent_t>* ev = nullptr;
    if (ctx->timing && allow_timing) {
      if (ctx->ev_used == ctx->ev_pool.size()) {
        std::pair<hipEvent_t, hipEvent_t> e;
        hipError_t he = hipEventCreate(&e.first);
        if (he == hipSuccess) he = hipEventCreate(&e.second);
        if (he != hipSuccess) return fail_hip(ctx, he);
        ctx->ev_pool.push_back(e);
      }
      ev = &ctx->ev_pool[ctx->ev_used++];
      hipError_t he = hipEventRecord(ev->first, s);
      if (he != hipSuccess) return fail_hip(ctx, he);
    }
    // chain pass and resolve pass: entries and count prefixes of all tiles
    int64_t cgrid = int64_t(ctx->n_cu) * ctx->chain_occ;
    if (cgrid > p.n_tiles) cgrid = p.n_tiles;
    spv::launch_chain(p, int(cgrid), s);
    if ((r = check_launch(ctx))) return r;
    spv::launch_resolve(p, s);
    if ((r = check_launch(ctx))) return r;
    // resolved walk (returns at once when the resolve pass left the batch to
    // the single-pass walk, which is launched next and returns at once
    // otherwise)
    int64_t wgrid = int64_t(ctx->n_cu) * ctx->walk_occ;
    if (wgrid > p.n_tiles) wgrid = p.n_tiles;
    spv::launch_walk(p, int(wgrid), s);
    if ((r = check_launch(ctx))) return r;
    // the single-pass walk (returns at once when the resolved walk ran):
    // tiles are claimed in order from a counter, so a tile's predecessors
    // are always held by running blocks, whatever the residency
    p.sched_static = 0;
    hipError_t he = spv::launch_main(p, int(grid), s);
    if (he != hipSuccess) return fail_hip(ctx, he);
    if ((r = check_launch(ctx))) return r;
    if (ev) {
      hipError_t he = hipEventRecord(ev->second, s);
      if (he != hipSuccess) return fail_hip(ctx, he);
    }
  }
  if (semantic) {
    if (!p.p1_inline) {
      spv::launch_finalize(p, 1, s);
      if ((r = check_launch(ctx))) return r;
    }
    int64_t g2 = int64_t(ctx->n_cu) * 2;
    if (g2 > p.n_tiles) g2 = p.n_tiles;
    if (g2 > 0) {
      spv::launch_pass2(p, int(g2), s);
      if ((r = check_launch(ctx))) return r;
    }
  }
  // (small batches: the second pass's last block wrote the results)
  if (!p.p1_inline) spv::launch_finalize(p, 2, s);
  if (semantic && diag_flags) {
    if ((r = check_launch(ctx))) return r;
    spv::launch_diag(p, s);
  }
  return check_launch(ctx);
}

}  // namespace

extern "C" {

int spv_create(spv_ctx** out, int hip_device) {
  if (!out) return SPV_ERR_INVALID_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) return SPV_ERR_HIP;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) return SPV_ERR_HIP;
  spv_ctx* c = new spv_ctx;
  c->device = hip_device;
  c->n_cu = prop.multiProcessorCount;
  {
    DeviceGuard g(hip_device);
    int occ = spv::main_occupancy();
    c->occupancy = occ;
    int cocc = spv::chain_occupancy();
    c->chain_occ = cocc > 0 ? cocc : 2;
    int wocc = spv::walk_occupancy();
    c->walk_occ = wocc > 0 ? wocc : 2;
    c->blocks_per_cu = occ > 0 ? (occ < 8 ? occ : 8) : 2;
    c->scratch = resolve_scratch(hip_device);
    int eo = spv::encode_occupancy(0);
    c->enc_count_occ = eo > 0 ? eo : 2;
    eo = spv::encode_occupancy(1);
    c->enc_scatter_occ = eo > 0 ? eo : 2;
  }
  c->encode_block = 4096;
  c->last = hipSuccess;
  c->msg[0] = '\0';
  c->timing = false;
  c->ev_used = 0;
  *out = c;
  return SPV_SUCCESS;
}

int spv_destroy(spv_ctx* ctx) {
  if (ctx) {
    for (auto& e : ctx->ev_pool) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
  }
  delete ctx;
  return SPV_SUCCESS;
}

int spv_set_timing(spv_ctx* ctx, int enable) {
  if (!ctx) return SPV_ERR_INVALID_ARG;
  ctx->timing = enable != 0;
  ctx->ev_used = 0;
  return SPV_SUCCESS;
}

int spv_read_timing(spv_ctx* ctx, double* total_ms, int64_t* n_launches) {
  if (!ctx || !total_ms || !n_launches) return SPV_ERR_INVALID_ARG;
  DeviceGuard g(ctx->device);
  double sum = 0.0;
  for (size_t i = 0; i < ctx->ev_used; ++i) {
    hipError_t he = hipEventSynchronize(ctx->ev_pool[i].second);
    float ms = 0.0f;
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, ctx->ev_pool[i].first, ctx->ev_pool[i].second);
    if (he != hipSuccess) return fail_hip(ctx, he);
    sum += ms;
  }
  *total_ms = sum;
  *n_launches = int64_t(ctx->ev_used);
  ctx->ev_used = 0;
  return SPV_SUCCESS;
}

const char* spv_last_hip_error(spv_ctx* ctx) { return ctx ? ctx->msg : "no context"; }

int spv_set_tuning(spv_ctx* ctx, int blocks_per_cu, int encode_block) {
  if (!ctx || blocks_per_cu < 0 || encode_block < 0 || (encode_block % 256) != 0 || encode_block > 4096)
    return SPV_ERR_INVALID_ARG;
  if (blocks_per_cu > 0) ctx->blocks_per_cu = blocks_per_cu;
  if (encode_block > 0) ctx->encode_block = encode_block;
  return SPV_SUCCESS;
}

int spv_set_grids(spv_ctx* ctx, int chain_blocks_per_cu, int walk_blocks_per_cu) {
  if (!ctx || chain_blocks_per_cu < 0 || chain_blocks_per_cu > 64 || walk_blocks_per_cu < 0 ||
      walk_blocks_per_cu > 64)
    return SPV_ERR_INVALID_ARG;
  if (chain_blocks_per_cu > 0) ctx->chain_occ = chain_blocks_per_cu;
  if (walk_blocks_per_cu > 0) ctx->walk_occ = walk_blocks_per_cu;
  return SPV_SUCCESS;
}

int spv_get_grids(spv_ctx* ctx, int* chain_blocks_per_cu, int* walk_blocks_per_cu) {
  if (!ctx || !chain_blocks_per_cu || !walk_blocks_per_cu) return SPV_ERR_INVALID_ARG;
  *chain_blocks_per_cu = ctx->chain_occ;
  *walk_blocks_per_cu = ctx->walk_occ;
  return SPV_SUCCESS;
}

int spv_get_tuning(spv_ctx* ctx, int* blocks_per_cu, int* encode_block) {
  if (!ctx || !blocks_per_cu || !encode_block) return SPV_ERR_INVALID_ARG;
  *blocks_per_cu = ctx->blocks_per_cu;
  *encode_block = ctx->encode_block;
  return SPV_SUCCESS;
}

int spv_workspace_size(spv_ctx* ctx, int64_t n_modules, int64_t n_words, size_t* bytes) {
  if (!ctx || !bytes || n_modules < 0 || n_words < 0) return SPV_ERR_INVALID_ARG;
  *bytes = spv::make_layout(n_modules, n_words).total;
  return SPV_SUCCESS;
}

int spv_decode(spv_ctx* ctx, const uint32_t* words, const int64_t* mod_off, int64_t n_modules, int64_t n_words,
               uint32_t* idx_off, uint16_t* idx_op, int64_t idx_cap, spv_result* results, void* ws,
               size_t ws_bytes, void* stream) {
  return run_validate(ctx, words, mod_off, n_modules, n_words, idx_off, idx_op, idx_cap, results, 0, ws, ws_bytes,
                      stream);
}

int spv_validate(spv_ctx* ctx, const uint32_t* words, const int64_t* mod_off, int64_t n_modules, int64_t n_words,
                 uint32_t* idx_off, uint16_t* idx_op, int64_t idx_cap, spv_result* results, uint32_t option_flags,
                 void* ws, size_t ws_bytes, void* stream) {
  if (!flags_ok(option_flags)) return SPV_ERR_INVALID_ARG;
  return run_validate(ctx, words, mod_off, n_modules, n_words, idx_off, idx_op, idx_cap, results,
                      (option_flags & SPV_OPT_NO_SEMANTIC) ? 0 : 1, ws, ws_bytes, stream, true,
                      (option_flags & SPV_OPT_MODULE_RULES) != 0, (option_flags & SPV_OPT_DEBUG_CHECKS) != 0,
                      option_flags & (SPV_OPT_SEM_OFFSETS | SPV_OPT_DEF_BEFORE_USE));
}

int spv_validate_noalloc(spv_ctx* ctx, const uint32_t* words, const int64_t* mod_off, int64_t n_modules,
                         int64_t n_words, uint32_t* idx_off, uint16_t* idx_op, int64_t idx_cap, spv_result* results,
                         uint32_t option_flags, void* stream) {
  if (!ctx || n_modules < 0 || n_words < 0) return SPV_ERR_INVALID_ARG;
  if (!flags_ok(option_flags)) return SPV_ERR_INVALID_ARG;
  if (spv::make_layout(n_modules, n_words).total > size_t(SPV_NOALLOC_SCRATCH_BYTES)) return SPV_ERR_WORKSPACE;
  if (ctx->scratch == nullptr) return fail_hip(ctx, hipErrorInvalidSymbol);
  // no event recording on this path (nothing is created or allocated)
  return run_validate(ctx, words, mod_off, n_modules, n_words, idx_off, idx_op, idx_cap, results,
                      (option_flags & SPV_OPT_NO_SEMANTIC) ? 0 : 1, ctx->scratch, size_t(SPV_NOALLOC_SCRATCH_BYTES),
                      stream, false, (option_flags & SPV_OPT_MODULE_RULES) != 0,
                      (option_flags & SPV_OPT_DEBUG_CHECKS) != 0,
                      option_flags & (SPV_OPT_SEM_OFFSETS | SPV_OPT_DEF_BEFORE_USE));
}

int spv_encode_bound(int64_t n_modules, int64_t n_records, int64_t n_opnd_words, int64_t n_string_records,
                     int64_t n_chars, int64_t* max_words) {
  if (!max_words || n_modules < 0 || n_records < 0 || n_opnd_words < 0 || n_string_records < 0 || n_chars < 0)
    return SPV_ERR_INVALID_ARG;
  *max_words = 5 * n_modules + n_records + n_opnd_words + n_string_records + n_chars / 4;
  return SPV_SUCCESS;
}

int spv_records_workspace_size(spv_ctx* ctx, int64_t n_modules, int64_t n_words, size_t* bytes) {
  if (!ctx || !bytes || n_modules < 0 || n_words < 0) return SPV_ERR_INVALID_ARG;
  *bytes = spv::make_rlayout(n_modules, n_words).total;
  return SPV_SUCCESS;
}

int spv_decode_records(spv_ctx* ctx, const uint32_t* words, const int64_t* mod_off, int64_t n_modules,
                       int64_t n_words, const uint32_t* idx_off, const spv_result* results, uint16_t* op,
                       int32_t* opnd_off, uint32_t* opnd, int32_t* str_off, uint8_t* chars, int64_t* rec_mod_off,
                       void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || n_modules < 0 || n_words < 0) return SPV_ERR_INVALID_ARG;
  if (n_words >= (int64_t(1) << 29)) return SPV_ERR_LIMIT;  // int32 string offsets: 4 bytes per word
  if (n_modules >= (int64_t(1) << 31) - 1) return SPV_ERR_LIMIT;
  if (n_modules == 0) return n_words == 0 ? SPV_SUCCESS : SPV_ERR_INVALID_ARG;
  if (!mod_off || !results || !rec_mod_off || !opnd_off || !str_off) return SPV_ERR_INVALID_ARG;
  if (n_words > 0 && (!words || !idx_off || !op || !opnd || !chars)) return SPV_ERR_INVALID_ARG;
  spv::RLayout L = spv::make_rlayout(n_modules, n_words);
  if (!ws || ws_bytes < L.total) return SPV_ERR_WORKSPACE;
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail_hip(ctx, hipErrorInvalidDevice);
  char* base = static_cast<char*>(ws);
  spv::RParams p;
  p.words = words;
  p.mod_off = mod_off;
  p.M = n_modules;
  p.cap_records = n_words;
  p.idx_off = idx_off;
  p.results = results;
  p.op = op;
  p.opnd_off = opnd_off;
  p.opnd = opnd;
  p.str_off = str_off;
  p.chars = chars;
  p.rec_mod_off = rec_mod_off;
  p.ctrl = reinterpret_cast<uint32_t*>(base + L.ctrl);
  p.mscan = reinterpret_cast<unsigned long long*>(base + L.mscan);
  p.mstate = reinterpret_cast<unsigned long long*>(base + L.mstate);
  p.rscan = reinterpret_cast<unsigned long long*>(base + L.rscan);
  p.btot = reinterpret_cast<unsigned long long*>(base + L.btot);
  p.rstate = reinterpret_cast<unsigned long long*>(base + L.rstate);
  spv::launch_records(p, static_cast<hipStream_t>(stream));
  return check_launch(ctx);
}

int spv_text_workspace_size(spv_ctx* ctx, int64_t n_modules, int64_t n_words, uint32_t options, size_t* bytes) {
  if (!ctx || !bytes || n_modules < 0 || n_words < 0 || (options & ~31u)) return SPV_ERR_INVALID_ARG;
  *bytes = spv::make_tlayout(n_modules, n_words, options).total;
  return SPV_SUCCESS;
}

int spv_decode_text(spv_ctx* ctx, const uint32_t* words, const int64_t* mod_off, int64_t n_modules, int64_t n_words,
                    const uint32_t* idx_off, const spv_result* results, uint32_t options, uint8_t* text,
                    int64_t text_cap, int64_t* text_mod_off, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || n_modules < 0 || n_words < 0 || text_cap < 0 || (options & ~31u)) return SPV_ERR_INVALID_ARG;
  if (n_words >= (int64_t(1) << 29)) return SPV_ERR_LIMIT;     // instruction counts fit 29 bits
  if (n_modules >= (int64_t(1) << 26)) return SPV_ERR_LIMIT;   // header bytes of all modules fit 33 bits
  if (n_modules == 0) return n_words == 0 ? SPV_SUCCESS : SPV_ERR_INVALID_ARG;
  if (!mod_off || !results || !text_mod_off) return SPV_ERR_INVALID_ARG;
  if (n_words > 0 && (!words || !idx_off)) return SPV_ERR_INVALID_ARG;
  if (text_cap > 0 && (!text || (reinterpret_cast<uintptr_t>(text) & 3u))) return SPV_ERR_INVALID_ARG;
  spv::TLayout L = spv::make_tlayout(n_modules, n_words, options);
  if (!ws || ws_bytes < L.total) return SPV_ERR_WORKSPACE;
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail_hip(ctx, hipErrorInvalidDevice);
  char* base = static_cast<char*>(ws);
  spv::TParams p;
  p.words = words;
  p.mod_off = mod_off;
  p.M = n_modules;
  p.cap_inst = n_words;
  p.idx_off = idx_off;
  p.results = results;
  p.options = options;
  p.text = text;
  p.text_cap = text_cap;
  p.text_mod_off = text_mod_off;
  p.ctrl = reinterpret_cast<uint32_t*>(base + L.ctrl);
  p.mscan = reinterpret_cast<unsigned long long*>(base + L.mscan);
  p.mstate = reinterpret_cast<unsigned long long*>(base + L.mstate);
  p.lens = reinterpret_cast<uint32_t*>(base + L.lens);
  p.lpos = reinterpret_cast<uint32_t*>(base + L.lpos);
  p.btot = reinterpret_cast<unsigned long long*>(base + L.btot);
  p.bstate = reinterpret_cast<unsigned long long*>(base + L.bstate);
  p.slots = reinterpret_cast<spv::TxtSlot*>(base + L.slots);
  p.slot_cap = L.slot_cap;
  p.nlist = reinterpret_cast<uint2*>(base + L.nlist);
  p.bcount = reinterpret_cast<uint32_t*>(base + L.bcount);
  p.nfilter = reinterpret_cast<uint32_t*>(base + L.nfilter);
  spv::launch_text(p, static_cast<hipStream_t>(stream));
  return check_launch(ctx);
}

int spv_encode_workspace_size(spv_ctx* ctx, int64_t n_modules, int64_t n_records, size_t* bytes) {
  if (!ctx || !bytes || n_modules < 0 || n_records < 0) return SPV_ERR_INVALID_ARG;
  *bytes = spv::make_elayout(n_modules, n_records, ctx->encode_block).total;
  return SPV_SUCCESS;
}

int spv_encode(spv_ctx* ctx, const uint16_t* op, const int32_t* opnd_off, const uint32_t* opnd,
               const int32_t* str_off, const uint8_t* chars, const int64_t* rec_mod_off, int64_t n_modules,
               int64_t n_records, uint32_t version_word, uint32_t generator_word, uint32_t* words_out,
               int64_t* word_mod_off, int64_t words_cap, uint32_t* enc_code, int64_t* enc_bad_record, void* ws,
               size_t ws_bytes, void* stream) {
  if (!ctx || n_modules < 0 || n_records < 0 || words_cap < 0) return SPV_ERR_INVALID_ARG;
  if (n_modules == 0) return n_records == 0 ? SPV_SUCCESS : SPV_ERR_INVALID_ARG;
  if (!rec_mod_off || !word_mod_off || !enc_code || !enc_bad_record || !opnd_off || !str_off)
    return SPV_ERR_INVALID_ARG;
  if (n_records > 0 && !op) return SPV_ERR_INVALID_ARG;
  if (words_cap < 5 * n_modules + n_records) return SPV_ERR_CAPACITY;
  if (words_cap > 0 && !words_out) return SPV_ERR_INVALID_ARG;
  spv::ELayout L = spv::make_elayout(n_modules, n_records, ctx->encode_block);
  if (!ws || ws_bytes < L.total) return SPV_ERR_WORKSPACE;
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail_hip(ctx, hipErrorInvalidDevice);
  char* base = static_cast<char*>(ws);
  spv::EParams p;
  p.op = op;
  p.opnd_off = opnd_off;
  p.opnd = opnd;
  p.str_off = str_off;
  p.chars = chars;
  p.rec_mod_off = rec_mod_off;
  p.M = n_modules;
  p.N = n_records;
  p.version_word = version_word;
  p.generator_word = generator_word;
  p.words_out = words_out;
  p.word_mod_off = word_mod_off;
  p.words_cap = words_cap;
  p.enc_code = enc_code;
  p.enc_bad = enc_bad_record;
  p.ctrl = reinterpret_cast<uint32_t*>(base + L.ctrl);
  p.blk = reinterpret_cast<unsigned long long*>(base + L.blk);
  p.blkx = reinterpret_cast<unsigned long long*>(base + L.blkx);
  p.sstate = reinterpret_cast<unsigned long long*>(base + L.sstate);
  p.bmod = reinterpret_cast<int64_t*>(base + L.bmod);
  p.mod_bad = reinterpret_cast<unsigned long long*>(base + L.mod_bad);
  p.mod_maxid = reinterpret_cast<uint32_t*>(base + L.mod_maxid);
  p.mod_words = reinterpret_cast<int64_t*>(base + L.mod_words);
  p.stage = nullptr;
  p.block_records = ctx->encode_block;
  p.n_blocks = (n_records + ctx->encode_block - 1) / ctx->encode_block;
  // persistent grids of exactly the resident blocks: every block takes the
  // same share of record blocks, with no second partial round
  int64_t gc = int64_t(ctx->n_cu) * ctx->enc_count_occ, gs = int64_t(ctx->n_cu) * ctx->enc_scatter_occ;
  if (gc > p.n_blocks) gc = p.n_blocks;
  if (gs > p.n_blocks) gs = p.n_blocks;
  spv::launch_encode(p, int(gc > 0 ? gc : 1), int(gs > 0 ? gs : 1), static_cast<hipStream_t>(stream));
  return check_launch(ctx);
}

}  // extern "C"
