// Host runtime of libiqcc: the C ABI declared in include/iqcc.h.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/iqcc.h"
#include "iqcc_internal.h"

using namespace iqcc;

struct iqcc_ctx {
  int device = 0;
  int n_cu = 1;
  size_t lds_per_block = 65536;
  size_t lds_per_cu = 65536;
  std::string err;
  // tuning knobs
  int64_t load_bucket_terms = 256;
  int64_t split_bucket_terms = 768;
  int64_t anti_cap = 1024;
  int64_t grid_per_cu = 2;
  int64_t batch_split_bucket_terms = 384;   // many small Hamiltonians: more, smaller pairs
  int64_t batch_anti_cap = 512;
  int64_t batch_unit_pairs = 8;             // bucket pairs per work unit of a batch
  int64_t energy_grid_per_cu = 16;         // stand-alone energy kernel
  int64_t fuse_energy = 1;
  int64_t dis_tile = 256;
  int64_t dis_bucket_ranges = 0;           // 0: about 8 workgroups per CU in total
  int64_t inplace_bucket_terms = 256;      // mean bucket of an in-place store at max_terms
  int64_t inplace_item_terms = 0;          // 0: from the stash capacity
  int64_t inplace_cap = 0;                 // 0: as many stash entries as the LDS holds
  int64_t inplace_region_rows = 0;         // 0: regions share the arena minus the pool
  // device scratch
  double* lut = nullptr;        // 8192: 3-qubit (4 x 22 x 64) or 4-qubit (2 x 16 x 256) tables
  double* partial = nullptr;    // n_partial
  int64_t n_partial = 0;
  int64_t* scratch = nullptr;   // n_scratch
  int64_t n_scratch = 0;
};

struct iqcc_batch {
  int n = 0, W = 0;
  BatchItem* d_items = nullptr;
  BatchPlan* d_plan = nullptr;
  int64_t* d_queue = nullptr;
  DressConfig cfg{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap_stream = nullptr;
};

struct iqcc_store {
  int nq = 0, W = 0;
  int64_t max_terms = 0;
  uint32_t flags = 0;
  StoreDev d{};
  void* mem = nullptr;    // the store's device memory (header, bucket table, arena)
  bool owned = false;     // true: allocated by iqcc_store_create*, freed by destroy
  double floor = 0.0;     // every live |c| is >= floor (0: unknown)
  bool regions = false;   // contents laid out in bucket regions (in-place dressing allowed)
  int region_m = -1;      // their bucket bits (fixed while the layout lasts)
};

namespace {

int fail(iqcc_ctx* ctx, int code, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return code;
}

#define HIP_TRY(ctx, call)                                                              \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail((ctx), IQCC_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

#define LAUNCH_CHECK(ctx)                                                                  \
  do {                                                                                     \
    hipError_t e_ = hipGetLastError();                                                     \
    if (e_ != hipSuccess)                                                                  \
      return fail((ctx), IQCC_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e_)); \
  } while (0)

hipStream_t as_stream(void* s) { return (hipStream_t)s; }

int ensure_scratch(iqcc_ctx* ctx, int64_t n) {
  if (n <= ctx->n_scratch) return IQCC_OK;
  HIP_TRY(ctx, hipDeviceSynchronize());
  if (ctx->scratch) HIP_TRY(ctx, hipFree(ctx->scratch));
  ctx->scratch = nullptr;
  ctx->n_scratch = 0;
  HIP_TRY(ctx, hipMalloc(&ctx->scratch, sizeof(int64_t) * n));
  ctx->n_scratch = n;
  return IQCC_OK;
}

int ensure_partial(iqcc_ctx* ctx, int64_t n) {
  if (n <= ctx->n_partial) return IQCC_OK;
  HIP_TRY(ctx, hipDeviceSynchronize());
  if (ctx->partial) HIP_TRY(ctx, hipFree(ctx->partial));
  ctx->partial = nullptr;
  ctx->n_partial = 0;
  HIP_TRY(ctx, hipMalloc(&ctx->partial, sizeof(double) * n));
  ctx->n_partial = n;
  return IQCC_OK;
}

// Persistent dressing grid: grid_per_cu workgroups per CU, but no more than
// fit in one CU's LDS at once (pairs are dealt out statically, so a workgroup
// that is not resident would start late and finish last).
static int dress_grid(const iqcc_ctx* ctx, size_t lds_bytes) {
  int64_t per_cu = ctx->grid_per_cu;
  const int64_t fit = lds_bytes ? (int64_t)(ctx->lds_per_cu / lds_bytes) : per_cu;
  if (fit < per_cu) per_cu = fit > 0 ? fit : 1;
  return (int)(ctx->n_cu * per_cu);
}

bool padding_clear(int nq, int W, const uint64_t* x, const uint64_t* z) {
  for (int w = 0; w < W; ++w) {
    int lo = 64 * w;
    uint64_t valid = nq - lo >= 64 ? ~0ull : (nq - lo <= 0 ? 0ull : ((1ull << (nq - lo)) - 1));
    if ((x[w] & ~valid) || (z[w] & ~valid)) return false;
  }
  return true;
}

// Debug check of rows about to be loaded (synchronising, host side): no bit
// set at a qubit >= nq, and no key twice.
int validate_rows(iqcc_ctx* ctx, int nq, int W, const uint64_t* x, const uint64_t* z, int64_t n,
                  int64_t ld, hipStream_t s) {
  if (n <= 0) return IQCC_OK;
  std::vector<uint64_t> hx((size_t)W * n), hz((size_t)W * n);
  for (int w = 0; w < W; ++w) {
    HIP_TRY(ctx, hipMemcpyAsync(hx.data() + (size_t)w * n, x + (size_t)w * ld, 8 * (size_t)n,
                                hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(hz.data() + (size_t)w * n, z + (size_t)w * ld, 8 * (size_t)n,
                                hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(ctx, hipStreamSynchronize(s));
  std::vector<int64_t> order(n);
  for (int64_t i = 0; i < n; ++i) {
    uint64_t kx[kMaxWords], kz[kMaxWords];
    for (int w = 0; w < W; ++w) {
      kx[w] = hx[(size_t)w * n + i];
      kz[w] = hz[(size_t)w * n + i];
    }
    if (!padding_clear(nq, W, kx, kz))
      return fail(ctx, IQCC_ERR_INVALID_ARG, "row %lld has a bit beyond n_qubits", (long long)i);
    order[i] = i;
  }
  auto word = [&](int64_t r, int q) {   // x words, then z words
    return q < W ? hx[(size_t)q * n + r] : hz[(size_t)(q - W) * n + r];
  };
  std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    for (int q = 0; q < 2 * W; ++q)
      if (word(a, q) != word(b, q)) return word(a, q) < word(b, q);
    return false;
  });
  for (int64_t i = 1; i < n; ++i) {
    bool same = true;
    for (int q = 0; q < 2 * W && same; ++q) same = word(order[i - 1], q) == word(order[i], q);
    if (same)
      return fail(ctx, IQCC_ERR_INVALID_ARG, "rows %lld and %lld have the same key",
                  (long long)order[i - 1], (long long)order[i]);
  }
  return IQCC_OK;
}

int check_ctx(iqcc_ctx* ctx) {
  if (!ctx) return IQCC_ERR_INVALID_ARG;
  ctx->err.clear();
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return fail(ctx, IQCC_ERR_HIP, "hipSetDevice: %s", hipGetErrorString(e));
  return IQCC_OK;
}

Entangler make_entangler(int W, const uint64_t* px, const uint64_t* pz) {
  Entangler P{};
  for (int w = 0; w < W; ++w) {
    P.px[w] = px[w];
    P.pz[w] = pz[w];
  }
  P.hp = bucket_hash_host(W, P.px, P.pz);
  P.piv_word = 0;
  P.piv_in_x = 1;
  P.piv_mask = 0;
  for (int w = 0; w < W; ++w) {
    if (P.px[w]) { P.piv_word = w; P.piv_in_x = 1; P.piv_mask = P.px[w] & (~P.px[w] + 1); break; }
    if (P.pz[w]) { P.piv_word = w; P.piv_in_x = 0; P.piv_mask = P.pz[w] & (~P.pz[w] + 1); break; }
  }
  // 3-qubit groups (per 32-bit half word) that P touches
  for (int h = 0; h < 2 * W; ++h) {
    const uint32_t v = (uint32_t)((P.px[h >> 1] | P.pz[h >> 1]) >> (32 * (h & 1)));
    uint32_t bits = 0;
    for (int g = 0; g < kGroupsPerHalf; ++g) {
      const uint32_t m = (7u << (3 * g));
      if (v & m) bits |= m;
    }
    P.gbits[h] = bits;
  }
  return P;
}

int ilog2_ceil(int64_t v) {
  int m = 0;
  while ((1ll << m) < v) ++m;
  return m;
}

}  // namespace

namespace {

// Device memory of a store, one block: a 256-byte header of device scalars,
// the bucket table (off, cnt, lim) and the arena planes x[W][cap], z[W][cap],
// c[cap]; every array starts on a 256-byte boundary.
struct StoreLayout {
  int W = 0, mcap = 0;
  int64_t cap = 0;
  size_t off = 0, cnt = 0, lim = 0, x = 0, z = 0, c = 0, bytes = 0;
};

constexpr size_t kHeaderBytes = 256;

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

bool store_layout(int n_qubits, int64_t max_terms, uint32_t flags, StoreLayout& L) {
  if (n_qubits < 1 || n_qubits > 64 * kMaxWords) return false;
  if (max_terms < 1 || max_terms > (1ll << 38)) return false;
  if (flags & ~(uint32_t)IQCC_STORE_INPLACE) return false;
  L.W = (n_qubits + 63) / 64;
  L.mcap = ilog2_ceil(max_terms / 16 + 1) + 1;
  if (L.mcap > kMaxBucketBits) L.mcap = kMaxBucketBits;
  if (flags & IQCC_STORE_INPLACE) {
    // every bucket in a region of its own with room to grow (3 max_terms rows
    // in all), plus a pool of max_terms / 2 rows for buckets that outgrow
    // their region; rows are addressed with 32-bit offsets inside a step
    L.cap = 3 * max_terms + max_terms / 2 + 4096;
    if (L.cap >= (1ll << 31)) return false;
  } else {
    L.cap = 2 * max_terms + 1024;
  }
  const size_t B = (size_t)1 << L.mcap;
  size_t o = kHeaderBytes;
  L.off = o; o = align256(o + 8 * B);
  L.cnt = o; o = align256(o + 8 * B);
  L.lim = o; o = align256(o + 8 * B);
  L.x = o; o = align256(o + 8 * (size_t)L.W * L.cap);
  L.z = o; o = align256(o + 8 * (size_t)L.W * L.cap);
  L.c = o; o = align256(o + 8 * (size_t)L.cap);
  L.bytes = o;
  return true;
}

iqcc_store* store_from_memory(int n_qubits, int64_t max_terms, uint32_t flags, const StoreLayout& L,
                              void* mem, bool owned) {
  iqcc_store* st = new iqcc_store();
  st->nq = n_qubits;
  st->W = L.W;
  st->max_terms = max_terms;
  st->flags = flags;
  st->mem = mem;
  st->owned = owned;
  char* b = (char*)mem;
  st->d.total = (int64_t*)(b + 0);
  st->d.top = (int64_t*)(b + 8);
  st->d.m = (int*)(b + 16);
  st->d.err = (int*)(b + 20);
  st->d.stats = (int64_t*)(b + 24);
  st->d.aux = (int64_t*)(b + 40);
  st->d.off = (int64_t*)(b + L.off);
  st->d.cnt = (int64_t*)(b + L.cnt);
  st->d.lim = (int64_t*)(b + L.lim);
  st->d.x = (uint64_t*)(b + L.x);
  st->d.z = (uint64_t*)(b + L.z);
  st->d.c = (double*)(b + L.c);
  st->d.cap = L.cap;
  st->d.mcap = L.mcap;
  return st;
}

// An empty store: every scalar 0 and bucket 0 (the only bucket at m = 0) empty.
hipError_t store_clear(iqcc_store* st, hipStream_t s) {
  hipError_t e = hipMemsetAsync(st->mem, 0, kHeaderBytes, s);
  if (e == hipSuccess) e = hipMemsetAsync(st->d.off, 0, 8, s);
  if (e == hipSuccess) e = hipMemsetAsync(st->d.cnt, 0, 8, s);
  if (e == hipSuccess) e = hipMemsetAsync(st->d.lim, 0, 8, s);
  return e;
}

int store_open(iqcc_ctx* ctx, int n_qubits, int64_t max_terms, uint32_t flags, void* mem,
               int64_t bytes, iqcc_store** out, hipStream_t s) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!out) return fail(ctx, IQCC_ERR_INVALID_ARG, "store output pointer is null");
  *out = nullptr;
  if (n_qubits > 64 * kMaxWords) return fail(ctx, IQCC_ERR_UNSUPPORTED, "more than 256 qubits");
  StoreLayout L;
  if (!store_layout(n_qubits, max_terms, flags, L))
    return fail(ctx, IQCC_ERR_INVALID_ARG, "bad n_qubits, max_terms or flags");
  bool owned = false;
  if (!mem) {
    hipError_t e = hipMalloc(&mem, L.bytes);
    if (e != hipSuccess)
      return fail(ctx, IQCC_ERR_HIP, "store allocation (%lld rows, %zu bytes) failed: %s",
                  (long long)L.cap, L.bytes, hipGetErrorString(e));
    owned = true;
  } else {
    if (bytes < (int64_t)L.bytes)
      return fail(ctx, IQCC_ERR_CAPACITY, "store needs %zu bytes, got %lld", L.bytes, (long long)bytes);
    if (((uintptr_t)mem & 255) != 0) return fail(ctx, IQCC_ERR_INVALID_ARG, "store memory is not 256-byte aligned");
  }
  iqcc_store* st = store_from_memory(n_qubits, max_terms, flags, L, mem, owned);
  hipError_t e = store_clear(st, s);
  if (e == hipSuccess && owned) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    if (owned) hipFree(mem);
    delete st;
    return fail(ctx, IQCC_ERR_HIP, "store initialisation failed: %s", hipGetErrorString(e));
  }
  *out = st;
  return IQCC_OK;
}

// Bucket count and region rows of an in-place store: about
// inplace_bucket_terms terms per bucket at max_terms, and regions that share
// the arena minus a pool of max_terms / 2 rows.
void inplace_geometry(const iqcc_ctx* ctx, const iqcc_store* st, int& m, int64_t& R) {
  const double lg = std::log2((double)st->max_terms / (double)ctx->inplace_bucket_terms);
  m = lg <= 0.0 ? 0 : (int)std::lround(lg);
  if (m > st->d.mcap) m = st->d.mcap;
  const int64_t pool = st->max_terms / 2 + 1024;
  while (m > 0 && ((st->d.cap - pool) >> m) < 16) --m;   // regions of at least 16 rows
  const int64_t B = 1ll << m;
  R = ((st->d.cap - pool) / B) & ~(int64_t)15;
  if (ctx->inplace_region_rows && ctx->inplace_region_rows < R) R = (ctx->inplace_region_rows + 15) & ~(int64_t)15;
  if (R < 16) R = 16;
}

// ---- allocation-free QMF energy ----------------------------------------------
// Device scratch of iqcc_qmf_energy_noalloc: the 3-qubit group table of the
// QMF state (kMaxWords * 22 * 64 doubles) followed by the per-workgroup
// partial sums (at most kNoAllocPartials).  Every device the library runs on
// holds its own copy until the process ends; host code reaches it only
// through the per-device address from hipGetSymbolAddress.
constexpr int kNoAllocLut = 8192;   // energy table: 2 words x 16 nibbles x 256, or 4 x 22 x 64
static_assert(kNoAllocLut >= 2 * 16 * 256 && kNoAllocLut >= kMaxWords * kGroupsPerWord * kLutEntries,
              "the allocation-free energy table holds every table layout");
constexpr int kNoAllocPartials = 8192;
constexpr int kNoAllocDevices = 64;
static __device__ __align__(256) double scratch[kNoAllocLut + kNoAllocPartials];
double* g_scratch[kNoAllocDevices] = {};
std::mutex g_scratch_mu;

// Called once per device by iqcc_ctx_create with that device current.  A
// failure is not fatal for the context: only the allocation-free entry point
// then reports it.
void noalloc_setup(int device) {
  if (device < 0 || device >= kNoAllocDevices) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[device]) return;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) g_scratch[device] = (double*)p;
  else (void)hipGetLastError();
}

}  // namespace

extern "C" {

const char* iqcc_version(void) { return "iqcc-gfx950 0.1"; }

const char* iqcc_last_error(const iqcc_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int iqcc_ctx_create(iqcc_ctx** out, int device) {
  if (!out) return IQCC_ERR_INVALID_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return IQCC_ERR_HIP;
  iqcc_ctx* ctx = new iqcc_ctx();
  ctx->device = device;
  if (hipSetDevice(device) != hipSuccess) { delete ctx; return IQCC_ERR_HIP; }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) { delete ctx; return IQCC_ERR_HIP; }
  ctx->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
  {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeSharedMemPerBlockOptin, device) == hipSuccess && v > 0)
      ctx->lds_per_block = (size_t)v;
    else if (prop.sharedMemPerBlock > 0)
      ctx->lds_per_block = prop.sharedMemPerBlock;
    ctx->lds_per_cu = ctx->lds_per_block;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device) == hipSuccess &&
        (size_t)v > ctx->lds_per_cu)
      ctx->lds_per_cu = (size_t)v;
  }
  noalloc_setup(device);
  if (hipMalloc(&ctx->lut, sizeof(double) * 8192) != hipSuccess) {   // every energy table layout
    delete ctx;
    return IQCC_ERR_HIP;
  }
  *out = ctx;
  return IQCC_OK;
}

int iqcc_ctx_destroy(iqcc_ctx* ctx) {
  if (!ctx) return IQCC_OK;
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  if (ctx->lut) hipFree(ctx->lut);
  if (ctx->partial) hipFree(ctx->partial);
  if (ctx->scratch) hipFree(ctx->scratch);
  delete ctx;
  return IQCC_OK;
}

int iqcc_set_param(iqcc_ctx* ctx, const char* name, int64_t v) {
  if (!ctx || !name) return IQCC_ERR_INVALID_ARG;
  struct { const char* n; int64_t* p; int64_t lo, hi; } tab[] = {
      {"load_bucket_terms", &ctx->load_bucket_terms, 1, 1 << 14},
      {"split_bucket_terms", &ctx->split_bucket_terms, 1, 1 << 20},
      {"anti_cap", &ctx->anti_cap, 16, 8192},
      {"grid_per_cu", &ctx->grid_per_cu, 1, 16},
      {"batch_split_bucket_terms", &ctx->batch_split_bucket_terms, 1, 1 << 20},
      {"batch_anti_cap", &ctx->batch_anti_cap, 16, 8192},
      {"batch_unit_pairs", &ctx->batch_unit_pairs, 1, 1 << 16},
      {"energy_grid_per_cu", &ctx->energy_grid_per_cu, 1, 32},
      {"fuse_energy", &ctx->fuse_energy, 0, 1},
      {"dis_tile", &ctx->dis_tile, 1, 256},
      {"dis_bucket_ranges", &ctx->dis_bucket_ranges, 0, 4096},
      {"inplace_bucket_terms", &ctx->inplace_bucket_terms, 1, 1 << 14},
      {"inplace_item_terms", &ctx->inplace_item_terms, 0, 1 << 16},
      {"inplace_cap", &ctx->inplace_cap, 0, 512},
      {"inplace_region_rows", &ctx->inplace_region_rows, 0, 1 << 24},
  };
  for (auto& t : tab) {
    if (std::strcmp(t.n, name) == 0) {
      if (v < t.lo || v > t.hi) return fail(ctx, IQCC_ERR_INVALID_ARG, "%s out of range", name);
      *t.p = v;
      return IQCC_OK;
    }
  }
  return fail(ctx, IQCC_ERR_INVALID_ARG, "unknown parameter %s", name);
}

int iqcc_get_param(const iqcc_ctx* ctx, const char* name, int64_t* v) {
  if (!ctx || !name || !v) return IQCC_ERR_INVALID_ARG;
  const struct { const char* n; int64_t p; } tab[] = {
      {"load_bucket_terms", ctx->load_bucket_terms}, {"split_bucket_terms", ctx->split_bucket_terms},
      {"anti_cap", ctx->anti_cap}, {"grid_per_cu", ctx->grid_per_cu},
      {"batch_split_bucket_terms", ctx->batch_split_bucket_terms},
      {"batch_anti_cap", ctx->batch_anti_cap}, {"batch_unit_pairs", ctx->batch_unit_pairs},
      {"energy_grid_per_cu", ctx->energy_grid_per_cu},
      {"fuse_energy", ctx->fuse_energy}, {"dis_tile", ctx->dis_tile},
      {"dis_bucket_ranges", ctx->dis_bucket_ranges},
      {"inplace_bucket_terms", ctx->inplace_bucket_terms},
      {"inplace_item_terms", ctx->inplace_item_terms},
      {"inplace_cap", ctx->inplace_cap},
      {"inplace_region_rows", ctx->inplace_region_rows},
      {"n_cu", ctx->n_cu},
  };
  for (auto& t : tab)
    if (std::strcmp(t.n, name) == 0) { *v = t.p; return IQCC_OK; }
  return IQCC_ERR_INVALID_ARG;
}

// ---- stores -----------------------------------------------------------------

int iqcc_store_bytes(int n_qubits, int64_t max_terms, uint32_t flags, int64_t* bytes) {
  if (!bytes) return IQCC_ERR_INVALID_ARG;
  if (n_qubits > 64 * kMaxWords) return IQCC_ERR_UNSUPPORTED;
  StoreLayout L;
  if (!store_layout(n_qubits, max_terms, flags, L)) return IQCC_ERR_INVALID_ARG;
  *bytes = (int64_t)L.bytes;
  return IQCC_OK;
}

int iqcc_store_create(iqcc_ctx* ctx, int n_qubits, int64_t max_terms, iqcc_store** out) {
  return store_open(ctx, n_qubits, max_terms, 0u, nullptr, 0, out, nullptr);
}

int iqcc_store_create_ex(iqcc_ctx* ctx, int n_qubits, int64_t max_terms, uint32_t flags,
                         iqcc_store** out) {
  return store_open(ctx, n_qubits, max_terms, flags, nullptr, 0, out, nullptr);
}

int iqcc_store_wrap(iqcc_ctx* ctx, int n_qubits, int64_t max_terms, uint32_t flags, void* mem,
                    int64_t bytes, iqcc_store** out, void* stream) {
  if (ctx && !mem) return fail(ctx, IQCC_ERR_INVALID_ARG, "store memory is null");
  return store_open(ctx, n_qubits, max_terms, flags, mem, bytes, out, as_stream(stream));
}

int iqcc_store_destroy(iqcc_ctx* ctx, iqcc_store* st) {
  if (!st) return IQCC_OK;
  if (ctx) hipSetDevice(ctx->device);
  if (st->owned) {
    hipDeviceSynchronize();
    hipFree(st->mem);
  }
  delete st;
  return IQCC_OK;
}

int iqcc_store_shape(const iqcc_store* st, int* nq, int* W) {
  if (!st) return IQCC_ERR_INVALID_ARG;
  if (nq) *nq = st->nq;
  if (W) *W = st->W;
  return IQCC_OK;
}

int iqcc_store_load(iqcc_ctx* ctx, iqcc_store* st, const uint64_t* x, const uint64_t* z,
                    const double* c, int64_t n, int64_t ld, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!st) return fail(ctx, IQCC_ERR_INVALID_ARG, "store is null");
  if (n < 0 || (n > 0 && (!x || !z || !c)) || ld < n)
    return fail(ctx, IQCC_ERR_INVALID_ARG, "bad rows/pointers/leading dimension");
  if (n > st->d.cap) return fail(ctx, IQCC_ERR_CAPACITY, "store holds at most %lld rows", (long long)st->d.cap);
  int m = 0;
  while (m < st->d.mcap && (n >> m) > ctx->load_bucket_terms) ++m;
  const int64_t B = 1ll << m;
  hipStream_t s = as_stream(stream);
  if (getenv("IQCC_DEBUG_VALIDATE")) {
    rc = validate_rows(ctx, st->nq, st->W, x, z, n, ld, s);
    if (rc) return rc;
  }
  st->floor = 0.0;
  if (st->flags & IQCC_STORE_INPLACE) {
    int64_t R = 0;
    inplace_geometry(ctx, st, m, R);
    const int64_t Bi = 1ll << m;
    rc = ensure_scratch(ctx, 3 * Bi + Bi / 1024 + 16 + n);
    if (rc) return rc;
    launch_store_load_regions(st->W, st->d, x, z, c, n, ld, m, R, ctx->scratch, s);
    LAUNCH_CHECK(ctx);
    st->regions = true;
    st->region_m = m;
    return IQCC_OK;
  }
  rc = ensure_scratch(ctx, B + B / 1024 + 16 + n);
  if (rc) return rc;
  launch_store_load(st->W, st->d, x, z, c, n, ld, m, ctx->scratch, s);
  LAUNCH_CHECK(ctx);
  st->regions = false;
  return IQCC_OK;
}

int iqcc_store_copy(iqcc_ctx* ctx, const iqcc_store* src, iqcc_store* dst, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!src || !dst) return fail(ctx, IQCC_ERR_INVALID_ARG, "store is null");
  if (src == dst) return fail(ctx, IQCC_ERR_INVALID_ARG, "source and destination are the same store");
  if (!(dst->flags & IQCC_STORE_INPLACE))
    return fail(ctx, IQCC_ERR_INVALID_ARG, "destination is not an IQCC_STORE_INPLACE store");
  if (src->nq != dst->nq) return fail(ctx, IQCC_ERR_INVALID_ARG, "qubit counts differ");
  int m = 0;
  int64_t R = 0;
  inplace_geometry(ctx, dst, m, R);
  const int64_t B = 1ll << m;
  rc = ensure_scratch(ctx, B + B / 1024 + 16);
  if (rc) return rc;
  launch_store_copy_regions(dst->W, src->d, dst->d, m, R, ctx->scratch, as_stream(stream),
                            src->regions && src->region_m == m);
  LAUNCH_CHECK(ctx);
  dst->floor = src->floor;
  dst->regions = true;
  dst->region_m = m;
  return IQCC_OK;
}

int iqcc_store_count(iqcc_ctx* ctx, const iqcc_store* st, int64_t* n, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!st || !n) return fail(ctx, IQCC_ERR_INVALID_ARG, "null argument");
  char buf[64];
  hipStream_t s = as_stream(stream);
  HIP_TRY(ctx, hipMemcpyAsync(buf, st->mem, 64, hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  int64_t total;
  int err;
  std::memcpy(&total, buf, 8);
  std::memcpy(&err, buf + 20, 4);
  *n = total;
  if (err & 1) return fail(ctx, IQCC_ERR_CAPACITY, "dressing output exceeded the store arena");
  if (err & 2) return fail(ctx, IQCC_ERR_CAPACITY, "dressing output exceeded the bucket table");
  if (err & 4) return fail(ctx, IQCC_ERR_CAPACITY, "bucket pair beyond the hash-round limit");
  return IQCC_OK;
}

int iqcc_store_stats(iqcc_ctx* ctx, const iqcc_store* st, int64_t* n_anti, int64_t* n_new,
                     void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!st || !n_anti || !n_new) return fail(ctx, IQCC_ERR_INVALID_ARG, "null argument");
  char buf[64];
  hipStream_t s = as_stream(stream);
  HIP_TRY(ctx, hipMemcpyAsync(buf, st->mem, 64, hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  std::memcpy(n_anti, buf + 24, 8);
  std::memcpy(n_new, buf + 32, 8);
  return IQCC_OK;
}

int iqcc_store_sum_squares(iqcc_ctx* ctx, const iqcc_store* st, double* out, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!st || !out) return fail(ctx, IQCC_ERR_INVALID_ARG, "null argument");
  const int grid = (int)(ctx->n_cu * 4);
  rc = ensure_partial(ctx, grid);
  if (rc) return rc;
  hipStream_t s = as_stream(stream);
  launch_sum_squares(st->d, grid, ctx->partial, s);
  launch_finalize_sum(ctx->partial, grid, nullptr, out, s);
  LAUNCH_CHECK(ctx);
  return IQCC_OK;
}

int iqcc_store_lookup(iqcc_ctx* ctx, const iqcc_store* st, const uint64_t* qx, const uint64_t* qz,
                      int64_t n, int64_t ld, int8_t* found, double* val, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!st || n < 0 || ld < n || (n > 0 && (!qx || !qz || !found || !val)))
    return fail(ctx, IQCC_ERR_INVALID_ARG, "bad lookup arguments");
  launch_lookup(st->W, st->d, qx, qz, n, ld, found, val, as_stream(stream));
  LAUNCH_CHECK(ctx);
  return IQCC_OK;
}

int iqcc_store_export(iqcc_ctx* ctx, const iqcc_store* st, uint64_t* x, uint64_t* z, double* c,
                      int64_t cap, int64_t ld, int64_t* n, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!st || !n) return fail(ctx, IQCC_ERR_INVALID_ARG, "null argument");
  char buf[64];
  hipStream_t s = as_stream(stream);
  HIP_TRY(ctx, hipMemcpyAsync(buf, st->mem, 64, hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  int64_t total;
  int m, err;
  std::memcpy(&total, buf, 8);
  std::memcpy(&m, buf + 16, 4);
  std::memcpy(&err, buf + 20, 4);
  *n = total;
  if (err) return fail(ctx, IQCC_ERR_CAPACITY, "store is invalid (dressing ran out of capacity)");
  if (total > cap) return fail(ctx, IQCC_ERR_CAPACITY, "export needs %lld rows", (long long)total);
  if (total > 0 && (!x || !z || !c)) return fail(ctx, IQCC_ERR_INVALID_ARG, "null output");
  if (ld < cap) return fail(ctx, IQCC_ERR_INVALID_ARG, "leading dimension below cap");
  const int64_t B = 1ll << m;
  rc = ensure_scratch(ctx, B + B / 1024 + 16);
  if (rc) return rc;
  launch_store_export(st->W, st->d, m, x, z, c, ld, ctx->scratch, ctx->scratch + B, s);
  LAUNCH_CHECK(ctx);
  HIP_TRY(ctx, hipStreamSynchronize(s));
  return IQCC_OK;
}

// ---- dressing ---------------------------------------------------------------

static int dress_impl(iqcc_ctx* ctx, const iqcc_store* in, const uint64_t* px, const uint64_t* pz,
                      double tau, double eps, const double* theta, const double* phi,
                      const double* energy_in, double* energy, iqcc_store* out,
                      int32_t* tape_self, int32_t* tape_partner, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!in || !out || !px || !pz) return fail(ctx, IQCC_ERR_INVALID_ARG, "null argument");
  if (in == out) return fail(ctx, IQCC_ERR_INVALID_ARG, "output store must differ from input");
  if (in->nq != out->nq) return fail(ctx, IQCC_ERR_INVALID_ARG, "qubit counts differ");
  if (!std::isfinite(tau)) return fail(ctx, IQCC_ERR_INVALID_ARG, "tau is not finite");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(ctx, IQCC_ERR_INVALID_ARG, "eps must be finite and >= 0");
  const bool want_e = theta || phi || energy;
  if (want_e && !(theta && phi && energy))
    return fail(ctx, IQCC_ERR_INVALID_ARG, "theta, phi and energy must be given together");
  if (!padding_clear(in->nq, in->W, px, pz))
    return fail(ctx, IQCC_ERR_INVALID_ARG, "entangler has bits beyond n_qubits");
  if (out->d.cap < in->d.cap || out->d.mcap < in->d.mcap)
    return fail(ctx, IQCC_ERR_CAPACITY, "output store is smaller than the input store");
  if (tape_self && out->d.cap >= ((int64_t)1 << 30))
    return fail(ctx, IQCC_ERR_INVALID_ARG, "a taped step needs an output arena below 2^30 rows");
  const int W = in->W;
  Entangler P = make_entangler(W, px, pz);
  hipStream_t s = as_stream(stream);
  const bool fused = want_e && ctx->fuse_energy;
  const size_t lds = dress_lds_bytes(W, (int)ctx->anti_cap, fused, tape_self != nullptr);
  if (lds > ctx->lds_per_block)
    return fail(ctx, IQCC_ERR_INVALID_ARG, "anti_cap %d needs more LDS than a workgroup has",
                (int)ctx->anti_cap);
  const int grid = dress_grid(ctx, lds);
  rc = ensure_partial(ctx, grid);
  if (rc) return rc;
  DressConfig cfg{};
  cfg.C = std::cos(tau);
  cfg.S = std::sin(tau);
  cfg.eps = eps;
  cfg.split_thr = ctx->split_bucket_terms;
  cfg.anti_cap = (int)ctx->anti_cap;
  cfg.grid = grid;
  if (want_e) {
    launch_build_lut(W, in->nq, theta, phi, ctx->lut, s);
    LAUNCH_CHECK(ctx);
  }
  cfg.lut = fused ? ctx->lut : nullptr;
  // with the input's energy known, the fused pass accumulates only the change
  const bool delta = fused && energy_in;
  cfg.delta = delta ? 1 : 0;
  cfg.e_partial = ctx->partial;
  cfg.tape_self = tape_self;
  cfg.tape_partner = tape_partner;
  launch_zero_counters(out->d, s);
  launch_dress(W, in->d, out->d, P, cfg, s);
  LAUNCH_CHECK(ctx);
  out->floor = eps;
  out->regions = false;
  if (want_e) {
    if (!fused) launch_energy(W, out->d, grid, ctx->lut, ctx->partial, s);
    launch_finalize_sum(ctx->partial, grid, nullptr, energy, s, delta ? energy_in : nullptr);
    LAUNCH_CHECK(ctx);
  }
  return IQCC_OK;
}

int iqcc_dress(iqcc_ctx* ctx, const iqcc_store* in, const uint64_t* px, const uint64_t* pz,
               double tau, double eps, const double* theta, const double* phi, double* energy,
               iqcc_store* out, void* stream) {
  return dress_impl(ctx, in, px, pz, tau, eps, theta, phi, nullptr, energy, out, nullptr, nullptr,
                    stream);
}

int iqcc_dress_energy_update(iqcc_ctx* ctx, const iqcc_store* in, const uint64_t* px,
                             const uint64_t* pz, double tau, double eps, const double* theta,
                             const double* phi, const double* energy_in, double* energy_out,
                             iqcc_store* out, void* stream) {
  if (ctx && (!theta || !phi || !energy_in || !energy_out))
    return fail(ctx, IQCC_ERR_INVALID_ARG, "theta, phi, energy_in and energy_out are required");
  return dress_impl(ctx, in, px, pz, tau, eps, theta, phi, energy_in, energy_out, out, nullptr,
                    nullptr, stream);
}

int iqcc_dress_inplace(iqcc_ctx* ctx, iqcc_store* st, const uint64_t* px, const uint64_t* pz, double tau,
                       double eps, const double* theta, const double* phi, const double* energy_in,
                       double* energy_out, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!st || !px || !pz) return fail(ctx, IQCC_ERR_INVALID_ARG, "null argument");
  if (!(st->flags & IQCC_STORE_INPLACE) || !st->regions)
    return fail(ctx, IQCC_ERR_INVALID_ARG,
                "store is not laid out in bucket regions (load or copy it into an IQCC_STORE_INPLACE store)");
  if (!std::isfinite(tau)) return fail(ctx, IQCC_ERR_INVALID_ARG, "tau is not finite");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(ctx, IQCC_ERR_INVALID_ARG, "eps must be finite and >= 0");
  const bool want_e = theta || phi || energy_out;
  if (want_e && !(theta && phi && energy_out))
    return fail(ctx, IQCC_ERR_INVALID_ARG, "theta, phi and energy_out must be given together");
  if (energy_in && !want_e) return fail(ctx, IQCC_ERR_INVALID_ARG, "energy_in without theta, phi, energy_out");
  if (!padding_clear(st->nq, st->W, px, pz))
    return fail(ctx, IQCC_ERR_INVALID_ARG, "entangler has bits beyond n_qubits");
  const int W = st->W;
  Entangler P = make_entangler(W, px, pz);
  hipStream_t s = as_stream(stream);
  const bool fused = want_e && ctx->fuse_energy;
  const size_t budget = ctx->lds_per_block < ctx->lds_per_cu ? ctx->lds_per_block : ctx->lds_per_cu;
  int cap = inplace_cap(W, fused, budget);
  if (ctx->inplace_cap && ctx->inplace_cap < cap) cap = (int)ctx->inplace_cap;
  if (cap < 16 || inplace_lds_bytes(W, cap, fused) > budget)
    return fail(ctx, IQCC_ERR_UNSUPPORTED, "the in-place step does not fit the LDS of a workgroup");
  const int grid = ctx->n_cu;
  const int nparts = grid * inplace_waves_per_block();
  // energy partials, then five counts per wavefront
  rc = ensure_partial(ctx, 6 * (int64_t)nparts);
  if (rc) return rc;
  InplaceConfig cfg{};
  cfg.C = std::cos(tau);
  cfg.S = std::sin(tau);
  cfg.eps = eps;
  cfg.cap = cap;
  cfg.item_terms = ctx->inplace_item_terms ? (int)ctx->inplace_item_terms : (3 * cap) / 2;
  cfg.theta = fused ? theta : nullptr;
  cfg.phi = fused ? phi : nullptr;
  cfg.nq = st->nq;
  const bool delta = fused && energy_in;
  cfg.delta = delta ? 1 : 0;
  cfg.e_partial = ctx->partial;
  cfg.counts = reinterpret_cast<int64_t*>(ctx->partial + nparts);
  launch_dress_inplace(W, st->d, P, cfg, grid, delta ? energy_in : nullptr, fused ? energy_out : nullptr, s);
  LAUNCH_CHECK(ctx);
  st->floor = eps;
  if (want_e && !fused) {
    const int eg = (int)(ctx->n_cu * ctx->energy_grid_per_cu);
    rc = ensure_partial(ctx, eg);
    if (rc) return rc;
    launch_build_lut(W, st->nq, theta, phi, ctx->lut, s);
    launch_energy(W, st->d, eg, ctx->lut, ctx->partial, s);
    launch_finalize_sum(ctx->partial, eg, nullptr, energy_out, s);
    LAUNCH_CHECK(ctx);
  }
  return IQCC_OK;
}

int iqcc_store_inplace_stats(iqcc_ctx* ctx, const iqcc_store* st, int64_t* relocated, int64_t* freed,
                             int64_t* region_rows, int64_t* pool_used, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!st) return fail(ctx, IQCC_ERR_INVALID_ARG, "store is null");
  int64_t buf[13];
  hipStream_t s = as_stream(stream);
  HIP_TRY(ctx, hipMemcpyAsync(buf, st->mem, sizeof buf, hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  // header: total, top, m|err, stats[2], aux[8]
  if (relocated) *relocated = buf[5 + 3];
  if (freed) *freed = buf[5 + 4];
  if (region_rows) *region_rows = buf[5 + 1];
  if (pool_used) *pool_used = buf[1] - buf[5 + 2];
  return IQCC_OK;
}

int iqcc_store_rows(const iqcc_store* st, int64_t* rows) {
  if (!st || !rows) return IQCC_ERR_INVALID_ARG;
  *rows = st->d.cap;
  return IQCC_OK;
}

int iqcc_dress_taped(iqcc_ctx* ctx, const iqcc_store* in, const uint64_t* px, const uint64_t* pz,
                     double tau, double eps, iqcc_store* out, int32_t* tape_self,
                     int32_t* tape_partner, void* stream) {
  if (ctx && (!tape_self || !tape_partner)) return fail(ctx, IQCC_ERR_INVALID_ARG, "tape arrays are null");
  return dress_impl(ctx, in, px, pz, tau, eps, nullptr, nullptr, nullptr, nullptr, out, tape_self,
                    tape_partner, stream);
}

int iqcc_dress_backward(iqcc_ctx* ctx, const iqcc_store* in, const uint64_t* px,
                        const uint64_t* pz, double tau, const int32_t* tape_self,
                        const int32_t* tape_partner, const double* lambda_out,
                        double* lambda_in, double* dtau, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!in || !px || !pz || !tape_self || !tape_partner || !lambda_out || !lambda_in || !dtau)
    return fail(ctx, IQCC_ERR_INVALID_ARG, "null argument");
  if (!std::isfinite(tau)) return fail(ctx, IQCC_ERR_INVALID_ARG, "tau is not finite");
  if (!padding_clear(in->nq, in->W, px, pz))
    return fail(ctx, IQCC_ERR_INVALID_ARG, "entangler has bits beyond n_qubits");
  hipStream_t s = as_stream(stream);
  const int grid = (int)(ctx->n_cu * 4);
  rc = ensure_partial(ctx, 3 * (int64_t)grid);   // exact fixed-point parts
  if (rc) return rc;
  launch_dress_backward(in->W, in->d, std::cos(tau), std::sin(tau), tape_self, tape_partner,
                        lambda_out, lambda_in, ctx->partial, grid, s);
  launch_finalize_fixed(ctx->partial, grid, dtau, s);
  LAUNCH_CHECK(ctx);
  return IQCC_OK;
}

int iqcc_dress_count(iqcc_ctx* ctx, const iqcc_store* in, const uint64_t* px, const uint64_t* pz,
                     int64_t* n_anti, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!in || !px || !pz || !n_anti) return fail(ctx, IQCC_ERR_INVALID_ARG, "null argument");
  if (!padding_clear(in->nq, in->W, px, pz))
    return fail(ctx, IQCC_ERR_INVALID_ARG, "entangler has bits beyond n_qubits");
  hipStream_t s = as_stream(stream);
  rc = ensure_scratch(ctx, 1);
  if (rc) return rc;
  HIP_TRY(ctx, hipMemsetAsync(ctx->scratch, 0, 8, s));
  launch_count_anti(in->W, in->d, make_entangler(in->W, px, pz), (unsigned long long*)ctx->scratch,
                    (int)(ctx->n_cu * 4), s);
  LAUNCH_CHECK(ctx);
  int64_t v = 0;
  HIP_TRY(ctx, hipMemcpyAsync(&v, ctx->scratch, 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  *n_anti = v;
  return IQCC_OK;
}

int iqcc_pauli_products(iqcc_ctx* ctx, int nq, const uint64_t* x1, const uint64_t* z1,
                        const uint64_t* x2, const uint64_t* z2, int64_t n, int64_t ld, uint64_t* x3,
                        uint64_t* z3, int8_t* e, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (nq < 1 || nq > 64 * kMaxWords) return fail(ctx, IQCC_ERR_INVALID_ARG, "bad n_qubits");
  if (n < 0 || ld < n) return fail(ctx, IQCC_ERR_INVALID_ARG, "bad sizes");
  if (n > 0 && (!x1 || !z1 || !x2 || !z2 || !x3 || !z3 || !e))
    return fail(ctx, IQCC_ERR_INVALID_ARG, "null argument");
  launch_pauli_products((nq + 63) / 64, x1, z1, x2, z2, n, ld, x3, z3, e, as_stream(stream));
  LAUNCH_CHECK(ctx);
  return IQCC_OK;
}

int iqcc_chain_forward(iqcc_ctx* ctx, const iqcc_store* h0, int n_steps, const uint64_t* px,
                       const uint64_t* pz, const double* taus, double eps, iqcc_store* const* outs,
                       int32_t* const* tape_self, int32_t* const* tape_partner, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!h0 || n_steps < 0 || (n_steps > 0 && (!px || !pz || !taus || !outs || !tape_self || !tape_partner)))
    return fail(ctx, IQCC_ERR_INVALID_ARG, "bad chain arguments");
  for (int j = 0; j < n_steps; ++j) {
    if (!outs[j] || outs[j] == h0 || !tape_self[j] || !tape_partner[j])
      return fail(ctx, IQCC_ERR_INVALID_ARG, "chain step %d: null or aliased store/tape", j);
    for (int k = 0; k < j; ++k)
      if (outs[k] == outs[j]) return fail(ctx, IQCC_ERR_INVALID_ARG, "chain steps %d and %d share a store", k, j);
  }
  const int W = h0->W;
  const iqcc_store* src = h0;
  for (int j = 0; j < n_steps; ++j) {
    rc = iqcc_dress_taped(ctx, src, px + (size_t)j * W, pz + (size_t)j * W, taus[j], eps, outs[j],
                          tape_self[j], tape_partner[j], stream);
    if (rc) return rc;
    src = outs[j];
  }
  return IQCC_OK;
}

int iqcc_chain_backward(iqcc_ctx* ctx, const iqcc_store* h0, int n_steps, const uint64_t* px,
                        const uint64_t* pz, const double* taus, iqcc_store* const* outs,
                        int32_t* const* tape_self, int32_t* const* tape_partner,
                        const double* lambda_final, double* work0, double* work1, double* lambda_h0,
                        double* dtau, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!h0 || n_steps < 0 ||
      (n_steps > 0 && (!px || !pz || !taus || !outs || !tape_self || !tape_partner || !lambda_final ||
                       !work0 || !work1 || !dtau)))
    return fail(ctx, IQCC_ERR_INVALID_ARG, "bad chain arguments");
  const int W = h0->W;
  const double* lam_out = lambda_final;
  for (int j = n_steps - 1; j >= 0; --j) {
    if (!outs[j] || !tape_self[j] || !tape_partner[j])
      return fail(ctx, IQCC_ERR_INVALID_ARG, "chain step %d: null store/tape", j);
    const iqcc_store* src = j ? outs[j - 1] : h0;
    double* lam_in = (j == 0 && lambda_h0) ? lambda_h0 : ((n_steps - 1 - j) % 2 ? work1 : work0);
    rc = iqcc_dress_backward(ctx, src, px + (size_t)j * W, pz + (size_t)j * W, taus[j],
                             tape_self[j], tape_partner[j], lam_out, lam_in, dtau + j, stream);
    if (rc) return rc;
    lam_out = lam_in;
  }
  return IQCC_OK;
}

int iqcc_expectations(iqcc_ctx* ctx, const iqcc_store* h, const double* theta, const double* phi,
                      const double* scale, double* out, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!h || !theta || !phi || !out) return fail(ctx, IQCC_ERR_INVALID_ARG, "null argument");
  hipStream_t s = as_stream(stream);
  launch_build_lut(h->W, h->nq, theta, phi, ctx->lut, s);
  launch_expectations(h->W, h->d, ctx->lut, scale, out, (int)(ctx->n_cu * 4), s);
  LAUNCH_CHECK(ctx);
  return IQCC_OK;
}

static int batch_build(iqcc_ctx* ctx, int n_ham, const iqcc_store* const* ins,
                       iqcc_store* const* outs, const uint64_t* px, const uint64_t* pz,
                       const double* taus, double eps, iqcc_batch* b) {
  if (n_ham < 1 || n_ham > (1 << 20) || !ins || !outs || !px || !pz || !taus)
    return fail(ctx, IQCC_ERR_INVALID_ARG, "bad batch arguments");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(ctx, IQCC_ERR_INVALID_ARG, "eps must be finite and >= 0");
  const int W = ins[0] ? ins[0]->W : 0;
  if (!W) return fail(ctx, IQCC_ERR_INVALID_ARG, "null store in batch");
  BatchItem* h = new BatchItem[n_ham];
  for (int i = 0; i < n_ham; ++i) {
    const iqcc_store* a = ins[i];
    const iqcc_store* o = outs[i];
    if (!a || !o || a == o || a->nq != o->nq || a->W != W || !std::isfinite(taus[i]) ||
        o->d.cap < a->d.cap || o->d.mcap < a->d.mcap ||
        !padding_clear(a->nq, W, px + (size_t)i * W, pz + (size_t)i * W)) {
      delete[] h;
      return fail(ctx, IQCC_ERR_INVALID_ARG, "batch item %d is invalid", i);
    }
    h[i].in = a->d;
    h[i].out = o->d;
    const_cast<iqcc_store*>(o)->regions = false;
    h[i].P = make_entangler(W, px + (size_t)i * W, pz + (size_t)i * W);
    h[i].C = std::cos(taus[i]);
    h[i].S = std::sin(taus[i]);
  }
  for (int i = 0; i < n_ham; ++i)
    for (int j = 0; j < n_ham; ++j)
      if (i != j && (outs[i] == outs[j] || outs[i] == ins[j])) {
        delete[] h;
        return fail(ctx, IQCC_ERR_INVALID_ARG, "batch outputs alias (items %d, %d)", i, j);
      }
  b->n = n_ham;
  b->W = W;
  hipError_t e = hipMalloc(&b->d_items, sizeof(BatchItem) * n_ham);
  if (e == hipSuccess) e = hipMalloc(&b->d_plan, sizeof(BatchPlan) * (n_ham + 1));
  if (e == hipSuccess) e = hipMalloc(&b->d_queue, 64);
  if (e == hipSuccess) e = hipMemcpy(b->d_items, h, sizeof(BatchItem) * n_ham, hipMemcpyHostToDevice);
  delete[] h;
  if (e != hipSuccess) return fail(ctx, IQCC_ERR_HIP, "batch allocation: %s", hipGetErrorString(e));
  b->cfg = DressConfig{};
  b->cfg.eps = eps;
  b->cfg.split_thr = ctx->batch_split_bucket_terms;
  b->cfg.anti_cap = (int)ctx->batch_anti_cap;
  b->cfg.unit_pairs = (int)ctx->batch_unit_pairs;
  const size_t lds = dress_lds_bytes(W, b->cfg.anti_cap, false, false);
  if (lds > ctx->lds_per_block)
    return fail(ctx, IQCC_ERR_INVALID_ARG, "anti_cap needs more LDS than a workgroup has");
  b->cfg.grid = dress_grid(ctx, lds);
  set_dress_batch_attributes(W, b->cfg.anti_cap);
  return IQCC_OK;
}

static void batch_free(iqcc_batch* b) {
  if (!b) return;
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  if (b->cap_stream) hipStreamDestroy(b->cap_stream);
  if (b->d_items) hipFree(b->d_items);
  if (b->d_plan) hipFree(b->d_plan);
  if (b->d_queue) hipFree(b->d_queue);
  delete b;
}

int iqcc_dress_batched(iqcc_ctx* ctx, int n_ham, const iqcc_store* const* ins,
                       iqcc_store* const* outs, const uint64_t* px, const uint64_t* pz,
                       const double* taus, double eps, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  iqcc_batch* b = new iqcc_batch();
  rc = batch_build(ctx, n_ham, ins, outs, px, pz, taus, eps, b);
  if (rc) { batch_free(b); return rc; }
  hipStream_t s = as_stream(stream);
  launch_dress_batch(b->W, b->n, b->d_items, b->d_plan, b->cfg, b->d_queue, s);
  hipError_t e = hipGetLastError();
  hipStreamSynchronize(s);
  batch_free(b);
  if (e != hipSuccess) return fail(ctx, IQCC_ERR_HIP, "batched launch: %s", hipGetErrorString(e));
  return IQCC_OK;
}

int iqcc_batch_create(iqcc_ctx* ctx, int n_ham, const iqcc_store* const* ins,
                      iqcc_store* const* outs, const uint64_t* px, const uint64_t* pz,
                      const double* taus, double eps, iqcc_batch** out) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!out) return fail(ctx, IQCC_ERR_INVALID_ARG, "null output");
  *out = nullptr;
  iqcc_batch* b = new iqcc_batch();
  rc = batch_build(ctx, n_ham, ins, outs, px, pz, taus, eps, b);
  if (rc) { batch_free(b); return rc; }
  hipError_t e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    launch_dress_batch(b->W, b->n, b->d_items, b->d_plan, b->cfg, b->d_queue, b->cap_stream);
    e = hipStreamEndCapture(b->cap_stream, &b->graph);
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    batch_free(b);
    return fail(ctx, IQCC_ERR_HIP, "graph capture: %s", hipGetErrorString(e));
  }
  *out = b;
  return IQCC_OK;
}

int iqcc_batch_launch(iqcc_ctx* ctx, iqcc_batch* b, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!b || !b->exec) return fail(ctx, IQCC_ERR_INVALID_ARG, "null batch");
  HIP_TRY(ctx, hipGraphLaunch(b->exec, as_stream(stream)));
  return IQCC_OK;
}

int iqcc_batch_destroy(iqcc_ctx* ctx, iqcc_batch* b) {
  if (ctx) hipSetDevice(ctx->device);
  if (b) hipDeviceSynchronize();
  batch_free(b);
  return IQCC_OK;
}

int iqcc_dress_raw(iqcc_ctx* ctx, int nq, const uint64_t* x, const uint64_t* z, const double* c,
                   int64_t n, int64_t ld, const uint64_t* px, const uint64_t* pz, double tau,
                   uint64_t* ox, uint64_t* oz, double* oc, int8_t* flag, int64_t ld_out,
                   void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (nq < 1 || nq > 64 * kMaxWords) return fail(ctx, IQCC_ERR_INVALID_ARG, "bad n_qubits");
  if (n < 0 || ld < n || ld_out < 2 * n) return fail(ctx, IQCC_ERR_INVALID_ARG, "bad sizes");
  if (!px || !pz || (n > 0 && (!x || !z || !c || !ox || !oz || !oc || !flag)))
    return fail(ctx, IQCC_ERR_INVALID_ARG, "null argument");
  if (!std::isfinite(tau)) return fail(ctx, IQCC_ERR_INVALID_ARG, "tau is not finite");
  const int W = (nq + 63) / 64;
  if (!padding_clear(nq, W, px, pz)) return fail(ctx, IQCC_ERR_INVALID_ARG, "entangler has bits beyond n_qubits");
  Entangler P = make_entangler(W, px, pz);
  launch_dress_raw(W, x, z, c, n, ld, P, std::cos(tau), std::sin(tau), ox, oz, oc, flag, ld_out,
                   as_stream(stream));
  LAUNCH_CHECK(ctx);
  return IQCC_OK;
}

int iqcc_merge_truncate(iqcc_ctx* ctx, const uint64_t* x, const uint64_t* z, const double* c,
                        int64_t n, int64_t ld, double eps, iqcc_store* out, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!out) return fail(ctx, IQCC_ERR_INVALID_ARG, "output store is null");
  if (n < 0 || ld < n || (n > 0 && (!x || !z || !c)))
    return fail(ctx, IQCC_ERR_INVALID_ARG, "bad rows/pointers/leading dimension");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(ctx, IQCC_ERR_INVALID_ARG, "eps must be finite and >= 0");
  if (n > out->d.cap) return fail(ctx, IQCC_ERR_CAPACITY, "store holds at most %lld rows", (long long)out->d.cap);
  int m = 0;
  while (m < out->d.mcap && (n >> m) > 512) ++m;
  rc = ensure_scratch(ctx, merge_scratch_len(out->W, n, m));
  if (rc) return rc;
  launch_merge_buckets(out->W, out->d, x, z, c, n, ld, m, eps, ctx->scratch, ctx->n_scratch,
                       as_stream(stream));
  LAUNCH_CHECK(ctx);
  out->regions = false;
  return IQCC_OK;
}

// ---- energy -----------------------------------------------------------------

int iqcc_qmf_energy(iqcc_ctx* ctx, const iqcc_store* h, const double* theta, const double* phi,
                    double* energy, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!h || !theta || !phi || !energy) return fail(ctx, IQCC_ERR_INVALID_ARG, "null argument");
  hipStream_t s = as_stream(stream);
  const int grid = (int)(ctx->n_cu * ctx->energy_grid_per_cu);
  rc = ensure_partial(ctx, grid);
  if (rc) return rc;
  launch_energy_table(h->W, h->nq, h->d, grid, theta, phi, ctx->lut, ctx->partial, s);
  launch_finalize_sum(ctx->partial, grid, nullptr, energy, s);
  LAUNCH_CHECK(ctx);
  return IQCC_OK;
}

int iqcc_qmf_energy_noalloc(iqcc_ctx* ctx, const iqcc_store* h, const double* theta, const double* phi,
                            double* energy, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!h || !theta || !phi || !energy) return fail(ctx, IQCC_ERR_INVALID_ARG, "null argument");
  double* base = (ctx->device >= 0 && ctx->device < kNoAllocDevices) ? g_scratch[ctx->device] : nullptr;
  if (!base) return fail(ctx, IQCC_ERR_HIP, "the device scratch of the allocation-free entry point is unavailable");
  const int64_t grid = ctx->n_cu * ctx->energy_grid_per_cu;
  if (grid > kNoAllocPartials)
    return fail(ctx, IQCC_ERR_CAPACITY,
                "allocation-free energy holds %d workgroup partials, the grid needs %lld "
                "(lower energy_grid_per_cu)", kNoAllocPartials, (long long)grid);
  hipStream_t s = as_stream(stream);
  launch_energy_table(h->W, h->nq, h->d, (int)grid, theta, phi, base, base + kNoAllocLut, s);
  launch_finalize_sum(base + kNoAllocLut, (int)grid, nullptr, energy, s);
  LAUNCH_CHECK(ctx);
  return IQCC_OK;
}

int iqcc_qmf_energy_backward(iqcc_ctx* ctx, const iqcc_store* h, const double* theta,
                             const double* phi, const double* dE, double* dtheta, double* dphi,
                             double* lambda, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!h || !theta || !phi || !dtheta || !dphi) return fail(ctx, IQCC_ERR_INVALID_ARG, "null argument");
  hipStream_t s = as_stream(stream);
  const int grid = (int)(ctx->n_cu * energy_bwd_blocks_per_cu(h->W));
  rc = ensure_partial(ctx, (int64_t)grid * 3 * h->nq);
  if (rc) return rc;
  launch_build_lut(h->W, h->nq, theta, phi, ctx->lut, s);
  launch_energy_backward(h->W, h->nq, h->d, grid, theta, phi, ctx->lut, dE, lambda, ctx->partial, s);
  launch_backward_finalize(h->nq, grid, ctx->partial, theta, phi, dE, dtheta, dphi, s);
  LAUNCH_CHECK(ctx);
  return IQCC_OK;
}

// ---- DIS --------------------------------------------------------------------

int iqcc_dis_gradients(iqcc_ctx* ctx, const iqcc_store* h, const double* theta, const double* phi,
                       const uint64_t* cx, const uint64_t* cz, int64_t n_cand, int64_t ld_cand,
                       int mode, double* g, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!h || !theta || !phi || !g || (n_cand > 0 && (!cx || !cz)))
    return fail(ctx, IQCC_ERR_INVALID_ARG, "null argument");
  if (n_cand < 0 || ld_cand < n_cand) return fail(ctx, IQCC_ERR_INVALID_ARG, "bad candidate sizes");
  if (mode != IQCC_DIS_BATCHED && mode != IQCC_DIS_PLAIN) return fail(ctx, IQCC_ERR_INVALID_ARG, "bad mode");
  if (n_cand == 0) return IQCC_OK;
  hipStream_t s = as_stream(stream);
  launch_build_lut(h->W, h->nq, theta, phi, ctx->lut, s);
  if (mode == IQCC_DIS_BATCHED) {
    // candidate tiles x bucket ranges: about 8 workgroups per CU in total
    // unless "dis_bucket_ranges" fixes the number of ranges
    const int64_t tiles = (n_cand + ctx->dis_tile - 1) / ctx->dis_tile;
    int64_t gt = ctx->dis_bucket_ranges ? ctx->dis_bucket_ranges : (ctx->n_cu * 8 + tiles - 1) / tiles;
    if (gt < 1) gt = 1;
    if (gt > 4096) gt = 4096;
    const int64_t n_part = (gt * n_cand + 1) & ~int64_t(1);   // tables start 16-byte aligned
    rc = ensure_partial(ctx, n_part + dis_tables_doubles(h->W));
    if (rc) return rc;
    launch_dis(h->W, h->d, ctx->lut, cx, cz, n_cand, ld_cand, 0, (int)ctx->dis_tile, 0,
               ctx->partial, (int)gt, g, s, theta, phi, h->nq, ctx->partial + n_part);
  } else {
    const int grid = (int)(ctx->n_cu * dis_one_blocks_per_cu(h->W));
    rc = ensure_partial(ctx, grid + 1);   // per-workgroup sums and a finish counter
    if (rc) return rc;
    launch_dis(h->W, h->d, ctx->lut, cx, cz, n_cand, ld_cand, 1, 1, grid, ctx->partial, 0, g, s,
               theta, phi, h->nq, nullptr);
  }
  LAUNCH_CHECK(ctx);
  return IQCC_OK;
}


// ---- one iQCC iteration (Sec. II, iterative procedure; App. A) -------------

int iqcc_qmf_energy_anti(iqcc_ctx* ctx, const iqcc_store* h, const uint64_t* px, const uint64_t* pz,
                         const double* theta, const double* phi, double* energy_anti,
                         void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!h || !px || !pz || !theta || !phi || !energy_anti)
    return fail(ctx, IQCC_ERR_INVALID_ARG, "null argument");
  if (!padding_clear(h->nq, h->W, px, pz))
    return fail(ctx, IQCC_ERR_INVALID_ARG, "generator has bits beyond n_qubits");
  hipStream_t s = as_stream(stream);
  const int grid = (int)(ctx->n_cu * 4);
  rc = ensure_partial(ctx, grid);
  if (rc) return rc;
  PauliKey P{};
  for (int w = 0; w < h->W; ++w) {
    P.x[w] = px[w];
    P.z[w] = pz[w];
  }
  launch_build_lut(h->W, h->nq, theta, phi, ctx->lut, s);
  launch_energy_anti(h->W, h->d, P, grid, ctx->lut, ctx->partial, s);
  launch_finalize_sum(ctx->partial, grid, nullptr, energy_anti, s);
  LAUNCH_CHECK(ctx);
  return IQCC_OK;
}

namespace {

// a < b in canonical order: x words from the most significant down, then z
bool canon_less(int W, const uint64_t* ax, const uint64_t* az, const uint64_t* bx,
                const uint64_t* bz) {
  for (int w = W - 1; w >= 0; --w)
    if (ax[w] != bx[w]) return ax[w] < bx[w];
  for (int w = W - 1; w >= 0; --w)
    if (az[w] != bz[w]) return az[w] < bz[w];
  return false;
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) hipFree(p);
  }
};

}  // namespace

namespace {

// Distinct flip sets with 1 <= |F| <= w_max of h's terms, canonical order, as
// rows of W words in `out`.
int flip_sets_impl(iqcc_ctx* ctx, const iqcc_store* h, int w_max, std::vector<uint64_t>& out) {
  const int W = h->W;
  out.clear();
  int64_t live = 0;
  int rc = iqcc_store_count(ctx, h, &live, nullptr);
  if (rc) return rc;
  if (live == 0) return IQCC_OK;
  // rows (F, 0, 1.0) for every term with 1 <= |F| <= w_max, made unique by the merge
  const int64_t ld = live;
  DevBuf rows, cnt;
  HIP_TRY(ctx, hipMalloc(&rows.p, (size_t)ld * (16 * W + 8)));
  HIP_TRY(ctx, hipMalloc(&cnt.p, 64));
  HIP_TRY(ctx, hipMemset(cnt.p, 0, 64));
  uint64_t* rx = (uint64_t*)rows.p;
  uint64_t* rz = rx + (size_t)W * ld;
  double* rc1 = (double*)(rz + (size_t)W * ld);
  launch_flip_rows(W, h->d, w_max, rx, rz, rc1, ld, (unsigned long long*)cnt.p,
                   (int)(ctx->n_cu * 4), nullptr);
  LAUNCH_CHECK(ctx);
  unsigned long long nrows = 0;
  HIP_TRY(ctx, hipMemcpy(&nrows, cnt.p, 8, hipMemcpyDeviceToHost));
  if (nrows == 0) return IQCC_OK;
  iqcc_store* u = nullptr;
  rc = iqcc_store_create(ctx, h->nq, (int64_t)nrows, &u);
  if (rc) return rc;
  rc = iqcc_merge_truncate(ctx, rx, rz, rc1, (int64_t)nrows, ld, 0.0, u, nullptr);
  int64_t nu = 0;
  if (!rc) rc = iqcc_store_export(ctx, u, rx, rz, rc1, ld, ld, &nu, nullptr);
  std::vector<uint64_t> hx;
  if (!rc) {
    hx.resize((size_t)W * nu);
    for (int w = 0; w < W; ++w)
      if (hipMemcpy(hx.data() + (size_t)w * nu, rx + (size_t)w * ld, sizeof(uint64_t) * nu,
                    hipMemcpyDeviceToHost) != hipSuccess)
        rc = fail(ctx, IQCC_ERR_HIP, "flip-set copy failed");
  }
  iqcc_store_destroy(ctx, u);
  if (rc) return rc;
  std::vector<int64_t> order(nu);
  for (int64_t i = 0; i < nu; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    for (int w = W - 1; w >= 0; --w) {
      const uint64_t va = hx[(size_t)w * nu + a], vb = hx[(size_t)w * nu + b];
      if (va != vb) return va < vb;
    }
    return false;
  });
  out.resize((size_t)nu * W);
  for (int64_t i = 0; i < nu; ++i)
    for (int w = 0; w < W; ++w) out[i * W + w] = hx[(size_t)w * nu + order[i]];
  return IQCC_OK;
}

}  // namespace

int iqcc_flip_sets(iqcc_ctx* ctx, const iqcc_store* h, int w_max, uint64_t* fx, int64_t cap,
                   int64_t* n) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!h || !n || w_max < 1 || cap < 0) return fail(ctx, IQCC_ERR_INVALID_ARG, "bad flip-set arguments");
  std::vector<uint64_t> F;
  rc = flip_sets_impl(ctx, h, w_max, F);
  if (rc) return rc;
  const int64_t nu = (int64_t)(F.size() / h->W);
  *n = nu;
  if (nu > cap) return fail(ctx, IQCC_ERR_CAPACITY, "%lld flip sets, room for %lld", (long long)nu,
                            (long long)cap);
  if (nu > 0 && !fx) return fail(ctx, IQCC_ERR_INVALID_ARG, "null output");
  std::copy(F.begin(), F.end(), fx);
  return IQCC_OK;
}

int iqcc_qcc_iteration(iqcc_ctx* ctx, iqcc_store** h, iqcc_store** spare, const double* theta,
                       const double* phi, int w_max, int n_select, double eps, uint64_t* sel_x,
                       uint64_t* sel_z, double* sel_g, double* sel_tau, double* energy,
                       int64_t* n_candidates, int* n_applied) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!h || !spare || !*h || !*spare || *h == *spare || !theta || !phi || !sel_x || !sel_z ||
      !sel_g || !sel_tau || !energy || !n_candidates || !n_applied || n_select < 0 || w_max < 1)
    return fail(ctx, IQCC_ERR_INVALID_ARG, "bad iteration arguments");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(ctx, IQCC_ERR_INVALID_ARG, "eps must be finite and >= 0");
  const int W = (*h)->W;
  *n_applied = 0;
  *n_candidates = 0;
  DevBuf dscal;
  HIP_TRY(ctx, hipMalloc(&dscal.p, 64));
  double* d_e = (double*)dscal.p;   // [0] energy, [1] next energy, [2] b, [3] c
  rc = iqcc_qmf_energy(ctx, *h, theta, phi, d_e, nullptr);
  if (rc) return rc;
  double e_cur = 0.0;
  HIP_TRY(ctx, hipMemcpy(&e_cur, d_e, 8, hipMemcpyDeviceToHost));
  energy[0] = e_cur;
  // 1. flip sets, 2. DIS candidates: Y on one qubit of F, X on the rest of F
  std::vector<uint64_t> F;
  rc = flip_sets_impl(ctx, *h, w_max, F);
  if (rc) return rc;
  const int64_t nf = (int64_t)(F.size() / W);
  std::vector<uint64_t> cx, cz;
  for (int64_t f = 0; f < nf; ++f)
    for (int w = 0; w < W; ++w)
      for (uint64_t v = F[f * W + w]; v; v &= v - 1) {
        for (int u = 0; u < W; ++u) {
          cx.push_back(F[f * W + u]);
          cz.push_back(u == w ? (v & (~v + 1)) : 0ull);
        }
      }
  const int64_t nc = (int64_t)(cx.size() / W);
  *n_candidates = nc;
  if (nc == 0 || n_select == 0) return IQCC_OK;
  // 3. gradients of all candidates in one batched launch
  DevBuf dc;
  HIP_TRY(ctx, hipMalloc(&dc.p, (size_t)nc * (16 * W + 8)));
  uint64_t* dcx = (uint64_t*)dc.p;
  uint64_t* dcz = dcx + (size_t)W * nc;
  double* dg = (double*)(dcz + (size_t)W * nc);
  {
    std::vector<uint64_t> px((size_t)W * nc), pz((size_t)W * nc);
    for (int64_t i = 0; i < nc; ++i)
      for (int w = 0; w < W; ++w) {
        px[(size_t)w * nc + i] = cx[i * W + w];
        pz[(size_t)w * nc + i] = cz[i * W + w];
      }
    HIP_TRY(ctx, hipMemcpy(dcx, px.data(), sizeof(uint64_t) * W * nc, hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemcpy(dcz, pz.data(), sizeof(uint64_t) * W * nc, hipMemcpyHostToDevice));
  }
  rc = iqcc_dis_gradients(ctx, *h, theta, phi, dcx, dcz, nc, nc, IQCC_DIS_BATCHED, dg, nullptr);
  if (rc) return rc;
  std::vector<double> g(nc);
  HIP_TRY(ctx, hipMemcpy(g.data(), dg, sizeof(double) * nc, hipMemcpyDeviceToHost));
  // the n_select largest |g| (ties: canonical key ascending); zero gradients are never taken
  std::vector<int64_t> idx(nc);
  for (int64_t i = 0; i < nc; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
    const double ga = std::fabs(g[a]), gb = std::fabs(g[b]);
    if (ga != gb) return ga > gb;
    return canon_less(W, &cx[a * W], &cz[a * W], &cx[b * W], &cz[b * W]);
  });
  // 4. one closed-form step per selected generator, in rank order
  for (int k = 0; k < n_select && k < nc; ++k) {
    const int64_t i = idx[k];
    if (!(std::fabs(g[i]) > 0.0)) break;
    const uint64_t* px = &cx[i * W];
    const uint64_t* pz = &cz[i * W];
    rc = iqcc_qmf_energy_anti(ctx, *h, px, pz, theta, phi, d_e + 2, nullptr);
    if (rc) return rc;
    rc = iqcc_dis_gradients(ctx, *h, theta, phi, dcx + i, dcz + i, 1, nc, IQCC_DIS_PLAIN, d_e + 3,
                            nullptr);
    if (rc) return rc;
    double bc[2];
    HIP_TRY(ctx, hipMemcpy(bc, d_e + 2, 16, hipMemcpyDeviceToHost));
    // E(tau) = (E - b) + b cos(tau) + c sin(tau) is smallest at (cos, sin) = -(b, c) / |(b, c)|
    const double tau = (bc[0] == 0.0 && bc[1] == 0.0) ? 0.0 : std::atan2(-bc[1], -bc[0]);
    rc = iqcc_dress_energy_update(ctx, *h, px, pz, tau, eps, theta, phi, d_e, d_e + 1, *spare,
                                  nullptr);
    if (rc) return rc;
    std::swap(*h, *spare);
    double e_next = 0.0;
    HIP_TRY(ctx, hipMemcpy(&e_next, d_e + 1, 8, hipMemcpyDeviceToHost));
    HIP_TRY(ctx, hipMemcpy(d_e, d_e + 1, 8, hipMemcpyDeviceToDevice));
    for (int w = 0; w < W; ++w) {
      sel_x[k * W + w] = px[w];
      sel_z[k * W + w] = pz[w];
    }
    sel_g[k] = g[i];
    sel_tau[k] = tau;
    energy[k + 1] = e_next;
    *n_applied = k + 1;
  }
  int64_t nout = 0;
  return iqcc_store_count(ctx, *h, &nout, nullptr);
}


// ---- term-limit compression -------------------------------------------------

int iqcc_truncate_top(iqcc_ctx* ctx, const iqcc_store* in, int64_t max_terms, iqcc_store* out,
                      void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!in || !out || in == out || max_terms < 0) return fail(ctx, IQCC_ERR_INVALID_ARG, "bad arguments");
  if (in->nq != out->nq) return fail(ctx, IQCC_ERR_INVALID_ARG, "qubit counts differ");
  if (out->d.cap < in->d.cap || out->d.mcap < in->d.mcap)
    return fail(ctx, IQCC_ERR_CAPACITY, "output store is smaller than the input store");
  hipStream_t s = as_stream(stream);
  int64_t n = 0;
  rc = iqcc_store_count(ctx, in, &n, stream);
  if (rc) return rc;
  const int W = in->W;
  const int grid = (int)(ctx->n_cu * 4);
  DevBuf dss, dhist;
  HIP_TRY(ctx, hipMalloc(&dss.p, sizeof(SelState)));
  HIP_TRY(ctx, hipMalloc(&dhist.p, 2048 * sizeof(unsigned)));
  SelState* ss = (SelState*)dss.p;
  SelState h{};
  h.need = max_terms;
  HIP_TRY(ctx, hipMemcpyAsync(ss, &h, sizeof(h), hipMemcpyHostToDevice, s));
  HIP_TRY(ctx, hipMemsetAsync(dhist.p, 0, 2048 * sizeof(unsigned), s));
  launch_zero_counters(out->d, s);
  int keep_all = n <= max_terms ? 1 : max_terms == 0 ? -1 : 0;
  DevBuf keys, kcount;
  if (keep_all == 0) {
    launch_abs_select_first(W, in->d, ss, (unsigned*)dhist.p, grid, s);
    LAUNCH_CHECK(ctx);
    HIP_TRY(ctx, hipMemcpyAsync(&h, ss, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    // the terms that share the first digit: their |c| bits go to the reused
    // partial-sum buffer, followed by the append counter
    const int64_t ncand = h.at > 0 ? h.at : 1;
    rc = ensure_partial(ctx, ncand + 1);
    if (rc) return rc;
    uint64_t* cand = (uint64_t*)ctx->partial;
    unsigned long long* ccount = (unsigned long long*)(ctx->partial + ncand);
    HIP_TRY(ctx, hipMemsetAsync(ccount, 0, sizeof(unsigned long long), s));
    launch_abs_select_rest(W, in->d, ss, (unsigned*)dhist.p, grid, cand, ncand, ccount, s);
    LAUNCH_CHECK(ctx);
    HIP_TRY(ctx, hipMemcpyAsync(&h, ss, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (h.need < h.ties) {
      // not every term equal to the threshold fits: the smaller canonical keys go first
      HIP_TRY(ctx, hipMalloc(&keys.p, (size_t)h.ties * 2 * W * sizeof(uint64_t)));
      HIP_TRY(ctx, hipMalloc(&kcount.p, 64));
      HIP_TRY(ctx, hipMemsetAsync(kcount.p, 0, 64, s));
      launch_collect_ties(W, in->d, ss, (uint64_t*)keys.p, h.ties, (unsigned long long*)kcount.p,
                          grid, s);
      launch_key_select(W, (const uint64_t*)keys.p, h.ties, ss, (unsigned*)dhist.p, s);
      const int one = 1;
      HIP_TRY(ctx, hipMemcpyAsync(&ss->key_mode, &one, sizeof(int), hipMemcpyHostToDevice, s));
      LAUNCH_CHECK(ctx);
    }
  }
  launch_select_compact(W, in->d, out->d, ss, keep_all, grid, s);
  out->regions = false;
  LAUNCH_CHECK(ctx);
  HIP_TRY(ctx, hipStreamSynchronize(s));
  return IQCC_OK;
}


// ---- sortless dressing (App. D), the comparison path -------------------------

int iqcc_sortless_dress(iqcc_ctx* ctx, int n_qubits, const uint64_t* x, const uint64_t* z,
                        const double* c, int64_t n, int64_t ld, const uint64_t* px,
                        const uint64_t* pz, double tau, double eps, uint64_t* ox, uint64_t* oz,
                        double* oc, int64_t cap, int64_t ld_out, int64_t* n_out, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (n_qubits < 1 || n_qubits > 64 * kMaxWords || n < 0 || ld < n || cap < 0 || ld_out < cap ||
      !px || !pz || !n_out || (n > 0 && (!x || !z || !c)) || (cap > 0 && (!ox || !oz || !oc)))
    return fail(ctx, IQCC_ERR_INVALID_ARG, "bad sortless-dressing arguments");
  if (n >= (int64_t)1 << 32) return fail(ctx, IQCC_ERR_INVALID_ARG, "at most 2^32 - 1 terms");
  if (!std::isfinite(tau)) return fail(ctx, IQCC_ERR_INVALID_ARG, "tau is not finite");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(ctx, IQCC_ERR_INVALID_ARG, "eps must be finite and >= 0");
  const int W = (n_qubits + 63) / 64;
  if (!padding_clear(n_qubits, W, px, pz))
    return fail(ctx, IQCC_ERR_INVALID_ARG, "entangler has bits beyond n_qubits");
  PauliKey P{};
  int nbits = 0;
  for (int w = 0; w < W; ++w) {
    P.x[w] = px[w];
    P.z[w] = pz[w];
    nbits += __builtin_popcountll(px[w]) + __builtin_popcountll(pz[w]);
  }
  if (nbits > 20) return fail(ctx, IQCC_ERR_INVALID_ARG, "entangler flips %d key bits (at most 20)", nbits);
  *n_out = 0;
  if (n == 0) return IQCC_OK;
  const hipError_t e = sortless_dress_run(W, x, z, c, n, ld, P, nbits, std::cos(tau), std::sin(tau),
                                          eps, ox, oz, oc, cap, ld_out, n_out, as_stream(stream));
  if (e == hipErrorInvalidValue && *n_out > cap)
    return fail(ctx, IQCC_ERR_CAPACITY, "result has %lld terms, room for %lld", (long long)*n_out,
                (long long)cap);
  if (e != hipSuccess) return fail(ctx, IQCC_ERR_HIP, "sortless dressing: %s", hipGetErrorString(e));
  return IQCC_OK;
}


// ---- several generators at once: exact energy polynomial (Eqs. 5, 6) ---------

namespace {

// f_b(tau) for the basis (1, cos, sin) at the grid angles 0, pi/2, pi, computed
// exactly as the dressing computes its cos and sin.
void grid_basis(double M[3][3]) {
  const double t[3] = {0.0, 0.5 * M_PI, M_PI};
  for (int r = 0; r < 3; ++r) {
    M[r][0] = 1.0;
    M[r][1] = std::cos(t[r]);
    M[r][2] = std::sin(t[r]);
  }
}

bool invert3(const double A[3][3], double B[3][3]) {
  const double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                     A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                     A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
  if (det == 0.0) return false;
  B[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / det;
  B[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / det;
  B[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det;
  B[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / det;
  B[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / det;
  B[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / det;
  B[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / det;
  B[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / det;
  B[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / det;
  return true;
}

}  // namespace

int iqcc_energy_trig_poly(iqcc_ctx* ctx, const iqcc_store* h, int n, const uint64_t* px,
                          const uint64_t* pz, const double* theta, const double* phi,
                          iqcc_store* const* work, double* coef) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!h || n < 1 || n > 8 || !px || !pz || !theta || !phi || !work || !coef)
    return fail(ctx, IQCC_ERR_INVALID_ARG, "bad trigonometric-polynomial arguments");
  const int W = h->W;
  for (int k = 0; k < n; ++k) {
    if (!work[k] || work[k] == h) return fail(ctx, IQCC_ERR_INVALID_ARG, "work store %d is invalid", k);
    for (int j = 0; j < k; ++j)
      if (work[j] == work[k]) return fail(ctx, IQCC_ERR_INVALID_ARG, "work stores alias");
  }
  const int64_t npts = (int64_t)std::pow(3.0, n);
  std::vector<double> grid(npts);
  DevBuf de;
  HIP_TRY(ctx, hipMalloc(&de.p, 8));
  const double tgrid[3] = {0.0, 0.5 * M_PI, M_PI};
  // depth-first over the grid: level k dresses work[k-1] (or h) into work[k]
  std::vector<int> digit(n, 0);
  int level = 0;
  int64_t done = 0;
  while (done < npts) {
    for (; level < n; ++level) {
      const iqcc_store* src = level == 0 ? h : work[level - 1];
      rc = iqcc_dress(ctx, src, px + (size_t)level * W, pz + (size_t)level * W, tgrid[digit[level]], 0.0,
                      nullptr, nullptr, nullptr, work[level], nullptr);
      if (rc) return rc;
    }
    rc = iqcc_qmf_energy(ctx, work[n - 1], theta, phi, (double*)de.p, nullptr);
    if (rc) return rc;
    int64_t idx = 0;
    for (int k = n - 1; k >= 0; --k) idx = idx * 3 + digit[k];
    HIP_TRY(ctx, hipMemcpy(&grid[idx], de.p, 8, hipMemcpyDeviceToHost));
    ++done;
    // next grid point: increment the last digit, carrying upwards
    int k = n - 1;
    while (k >= 0 && digit[k] == 2) digit[k--] = 0;
    if (k < 0) break;
    ++digit[k];
    level = k;
  }
  // E(grid t) = sum_s coef[s] prod_k M[t_k][s_k]: apply M^-1 along every axis
  double M[3][3], Mi[3][3];
  grid_basis(M);
  if (!invert3(M, Mi)) return fail(ctx, IQCC_ERR_INVALID_ARG, "singular grid");
  std::vector<double> a = grid, b(npts);
  int64_t stride = 1;
  for (int k = 0; k < n; ++k, stride *= 3) {
    for (int64_t i = 0; i < npts; ++i) {
      const int64_t d = (i / stride) % 3;
      const int64_t base = i - d * stride;
      b[i] = Mi[d][0] * a[base] + Mi[d][1] * a[base + stride] + Mi[d][2] * a[base + 2 * stride];
    }
    std::swap(a, b);
  }
  std::copy(a.begin(), a.end(), coef);
  return IQCC_OK;
}

double iqcc_trig_poly_eval(int n, const double* coef, const double* tau) {
  if (n < 1 || n > 8 || !coef || !tau) return std::nan("");
  const int64_t npts = (int64_t)std::pow(3.0, n);
  double e = 0.0;
  for (int64_t s = 0; s < npts; ++s) {
    double p = coef[s];
    int64_t v = s;
    for (int k = 0; k < n; ++k, v /= 3) {
      const int d = (int)(v % 3);
      p *= d == 0 ? 1.0 : d == 1 ? std::cos(tau[k]) : std::sin(tau[k]);
    }
    e += p;
  }
  return e;
}

int iqcc_trig_poly_minimize(int n, const double* coef, double* tau, int sweeps, double* energy) {
  if (n < 1 || n > 8 || !coef || !tau || !energy || sweeps < 0) return IQCC_ERR_INVALID_ARG;
  const int64_t npts = (int64_t)std::pow(3.0, n);
  double e = iqcc_trig_poly_eval(n, coef, tau);
  for (int sw = 0; sw < sweeps; ++sw) {
    const double e0 = e;
    for (int k = 0; k < n; ++k) {
      // with the other amplitudes fixed, E = a + b cos(tau_k) + c sin(tau_k)
      double abc[3] = {0.0, 0.0, 0.0};
      int64_t pk = 1;
      for (int j = 0; j < k; ++j) pk *= 3;
      for (int64_t s = 0; s < npts; ++s) {
        double p = coef[s];
        int64_t v = s;
        for (int j = 0; j < n; ++j, v /= 3) {
          if (j == k) continue;
          const int d = (int)(v % 3);
          p *= d == 0 ? 1.0 : d == 1 ? std::cos(tau[j]) : std::sin(tau[j]);
        }
        abc[(s / pk) % 3] += p;
      }
      if (abc[1] != 0.0 || abc[2] != 0.0) tau[k] = std::atan2(-abc[2], -abc[1]);
    }
    e = iqcc_trig_poly_eval(n, coef, tau);
    if (!(e < e0)) break;
  }
  *energy = e;
  return IQCC_OK;
}

}  // extern "C"
