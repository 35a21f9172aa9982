// CPU stand-in of the HIP runtime, for host-side tests of libtrals.
//
// The library's objects (built by hipcc as usual) are linked against this file
// instead of libamdhip64, so that its host code -- context set-up, the sweep
// driver, graph capture, the serving executor -- runs on a machine without a
// GPU.  Kernels are not executed: "device" memory is zero-filled host memory,
// so status words read back as clear and the host logic takes its normal path.
// Every call is checked instead:
//   * launches: grid and block shape, dynamic LDS against the 160 KB limit and
//     against the function's raised limit above 64 KB, every pointer argument
//     inside a live allocation, and for the kernels listed in check_extents()
//     the byte range each operand covers inside its allocation;
//   * copies and fills: both ranges inside live allocations (device side);
//   * graph capture: no fill, allocation, free or synchronisation of a
//     capturing stream while a capture is open; captured launches re-checked
//     when the graph is replayed (their buffers must still be live);
//   * threads: between fakehip_window_begin() and fakehip_window_end() the
//     distinct host threads that call into the runtime are counted.
// Problems are collected as text (fakehip_violation) rather than aborting, so
// a test can report them all.
#include <cxxabi.h>
#include <sys/mman.h>

#include <algorithm>
#include <array>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <chrono>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "../../paper_2210_11362_amd/csrc/common.h"
#include "../../paper_2210_11362_amd/csrc/tiny.h"

struct Capture;

struct ihipStream_t {
  unsigned flags = 0;
  Capture* cap = nullptr;     // capture this stream records into
};

struct ihipEvent_t {
  Capture* cap = nullptr;     // recorded inside this capture
  long long ready_at = 0;     // steady-clock microseconds at which the recorded work "completes"
};

namespace {

constexpr size_t LDS_MAX = 160 * 1024;
constexpr size_t LDS_DEFAULT = 64 * 1024;

struct Range { uintptr_t p; size_t bytes; std::string what; };

struct Op {                   // one captured launch: its name and the ranges it covers
  std::string name;
  std::vector<Range> ranges;
};

struct Alloc { size_t size; bool mapped; bool host; bool var = false; };

std::recursive_mutex& mu() {   // built on first use, like names()
  static auto* m = new std::recursive_mutex();
  return *m;
}
// start -> allocation; built on first use (device variables are registered by
// the library's constructors, possibly before this file's globals exist)
std::map<uintptr_t, Alloc>& allocs() {
  static auto* m = new std::map<uintptr_t, Alloc>();
  return *m;
}
// host stub -> demangled kernel; built on first use, since the library's
// registration constructors may run before this file's globals exist
std::unordered_map<const void*, std::string>& names() {
  static auto* m = new std::unordered_map<const void*, std::string>();
  return *m;
}
std::unordered_map<const void*, int> g_lds_limit;     // raised dynamic-LDS limit
std::vector<std::string> g_viol;
std::map<std::string, long> g_launches;
// allocations, frees, synchronisations (first use may come from a constructor)
std::map<std::string, long>& calls() {
  static auto* m = new std::map<std::string, long>();
  return *m;
}
std::vector<std::array<long long, 4>> g_gemm_log;     // M, N, realign, pair member
int g_open_captures = 0;
long long g_delay_us = 0;                             // simulated device time of recorded work

long long now_us() {
  return std::chrono::duration_cast<std::chrono::microseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}
bool g_window = false;
std::set<std::thread::id> g_window_threads;
thread_local hipError_t t_last = hipSuccess;
struct CallCfg { dim3 g, b; size_t shm; hipStream_t s; };
thread_local std::vector<CallCfg> t_cfg;
thread_local unsigned t_grid_x = 0;   // grid of the launch being checked

}  // namespace

struct Capture {
  std::vector<Op> ops;
  std::vector<hipStream_t> joined;
};
struct ihipGraph { std::vector<Op> ops; };
struct hipGraphExec { std::vector<Op> ops; };

namespace {

void viol(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_viol.emplace_back(buf);
}

void touch() {
  if (g_window) g_window_threads.insert(std::this_thread::get_id());
}

hipError_t ret(hipError_t e) {
  t_last = e == hipSuccess ? t_last : e;
  return e;
}

const Alloc* find(uintptr_t p, uintptr_t* start) {
  auto it = allocs().upper_bound(p);
  if (it == allocs().begin()) return nullptr;
  --it;
  if (p >= it->first + std::max<size_t>(it->second.size, 1)) return nullptr;
  *start = it->first;
  return &it->second;
}

// [p, p + bytes) must lie inside one live allocation
bool in_bounds(uintptr_t p, size_t bytes) {
  uintptr_t st = 0;
  const Alloc* a = find(p, &st);
  return a && p + bytes <= st + a->size;
}

void check_range(const std::string& who, const Range& r) {
  if (!r.p) {
    if (r.bytes) viol("%s: %s is null but covers %zu bytes", who.c_str(), r.what.c_str(), r.bytes);
    return;
  }
  uintptr_t st = 0;
  const Alloc* a = find(r.p, &st);
  if (!a) {
    viol("%s: %s at %#lx is not inside a live allocation", who.c_str(), r.what.c_str(), (unsigned long)r.p);
    return;
  }
  if (r.p + r.bytes > st + a->size)
    viol("%s: %s covers %zu bytes from offset %zu of a %zu-byte allocation (%zu bytes past its end)", who.c_str(),
         r.what.c_str(), r.bytes, (size_t)(r.p - st), a->size, (size_t)(r.p + r.bytes - st - a->size));
}

std::string demangle(const char* m0) {
  // the host demangler does not know clang's mangling of __bf16 (DF16b):
  // spell it as a vendor-extended type, which demangles to its name
  std::string mm(m0);
  for (size_t q; (q = mm.find("DF16b")) != std::string::npos;) mm.replace(q, 5, "u6__bf16");
  const char* m = mm.c_str();
  int st = 0;
  char* d = abi::__cxa_demangle(m, nullptr, nullptr, &st);
  std::string s = (st == 0 && d) ? d : m;
  free(d);
  const std::string anon = "(anonymous namespace)::";
  for (size_t q; (q = s.find(anon)) != std::string::npos;) s.erase(q, anon.size());
  return s;
}

// "ns::name<...>(T1, T2)" -> "name"
std::string base_name(const std::string& full) {   // template kernels demangle with a "void " prefix
  size_t end = full.find_first_of("<(");
  std::string s = full.substr(0, end);
  const size_t sp = s.rfind(' ');
  if (sp != std::string::npos) s = s.substr(sp + 1);
  const size_t c = s.rfind("::");
  return c == std::string::npos ? s : s.substr(c + 2);
}

// parameter types of "name<...>(T1, T2<a, b>, T3)"
std::vector<std::string> param_types(const std::string& full) {
  std::vector<std::string> out;
  size_t open = std::string::npos;
  int depth = 0;
  for (size_t q = 0; q < full.size(); ++q) {   // the '(' of the parameter list at depth 0
    const char ch = full[q];
    if (ch == '<') depth++;
    else if (ch == '>') depth--;
    else if (ch == '(' && depth == 0) {
      open = q;
      break;
    }
  }
  if (open == std::string::npos) return out;
  const size_t close = full.rfind(')');
  std::string cur;
  depth = 0;
  for (size_t q = open + 1; q < close; ++q) {
    const char ch = full[q];
    if (ch == '<' || ch == '(') depth++;
    if (ch == '>' || ch == ')') depth--;
    if (ch == ',' && depth == 0) {
      out.push_back(cur);
      cur.clear();
      continue;
    }
    if (!(cur.empty() && ch == ' ')) cur += ch;
  }
  if (!cur.empty()) out.push_back(cur);
  return out;
}

template <class T>
T arg(void** args, int i) {
  T v;
  std::memcpy(&v, args[i], sizeof(T));
  return v;
}

int template_int(const std::string& full, int which) {   // which-th integer template argument
  const size_t lt = full.find('<');
  if (lt == std::string::npos) return -1;
  int k = 0;
  size_t q = lt + 1;
  while (q < full.size() && full[q] != '>') {
    size_t e = full.find_first_of(",>", q);
    std::string t = full.substr(q, e - q);
    while (!t.empty() && t[0] == ' ') t.erase(0, 1);
    if (k == which) return (t.empty() || !(isdigit((unsigned char)t[0]))) ? -1 : atoi(t.c_str());
    ++k;
    q = e + (full[e] == ',' ? 1 : 0);
    if (full[e] == '>') break;
  }
  return -1;
}

size_t view_bytes(const MatView& v, int64_t rows, int64_t cols) {
  if (v.kind == 1) return (size_t)v.Rl * v.Rr * v.Rl * v.Rr * 8;
  if (v.kind == 2) return (size_t)(v.ld * (rows - 1) + cols) * 8;
  return (size_t)(v.ld * (cols - 1) + rows) * 8;
}

void gemm_ranges(const Gemm64Desc& g, const char* tag, std::vector<Range>* r, bool pair_member) {
  const std::string t(tag);
  r->push_back({(uintptr_t)g.A.p, view_bytes(g.A, g.M, g.K), t + "A"});
  r->push_back({(uintptr_t)g.B.p, view_bytes(g.B, g.K, g.N), t + "B"});
  if (g.beta != 0.0) r->push_back({(uintptr_t)g.Cin, (size_t)(g.ldcin * (g.N - 1) + g.M) * 8, t + "Cin"});
  const size_t cb = g.Ra > 0 ? (size_t)g.Ra * g.Rb * g.Ra * g.Rb * 8 : (size_t)(g.ldc * (g.N - 1) + g.M) * 8;
  r->push_back({(uintptr_t)g.C, cb, t + "C"});
  g_gemm_log.push_back({g.M, g.N, g.Ra > 0 ? 1 : 0, pair_member ? 1 : 0});
}

size_t es_of_prec(int p) { return p == 0 ? 8 : p == 1 ? 4 : p == 2 ? 2 : 1; }

// Byte ranges of the operands of the kernels whose extents are modelled here.
void check_extents(const std::string& full, const std::string& nm, void** a, std::vector<Range>* r) {
  auto D = [&](int i) { return (uintptr_t)arg<const void*>(a, i); };
  auto L = [&](int i) { return arg<int64_t>(a, i); };
  auto I = [&](int i) { return (int64_t)arg<int>(a, i); };
  if (nm == "gemm64_kernel") {
    gemm_ranges(arg<Gemm64Desc>(a, 0), "", r, false);
  } else if (nm == "gemm64_pair_kernel") {
    gemm_ranges(arg<Gemm64Desc>(a, 0), "first ", r, true);
    gemm_ranges(arg<Gemm64Desc>(a, 1), "second ", r, true);
  } else if (nm == "realign_S_kernel") {
    const MatView W = arg<MatView>(a, 0);
    const int64_t Ra = I(1), Rb = I(2);
    r->push_back({(uintptr_t)W.p, view_bytes(W, Rb * Rb, Ra * Ra), "W"});
    r->push_back({D(3), (size_t)(Ra * Rb * Ra * Rb * 8), "S"});
  } else if (nm == "chain_step_kernel") {   // (T, J, Rl, Rm, core, I, Rr, out)
    const int64_t J = L(1), Rl = I(2), Rm = I(3), In = L(5), Rr = I(6);
    r->push_back({D(0), (size_t)(J * Rl * Rm * 8), "T"});
    r->push_back({D(4), (size_t)(Rm * In * Rr * 8), "core"});
    r->push_back({D(7), (size_t)(J * In * Rl * Rr * 8), "out"});
  } else if (nm == "core_to_table_kernel" || nm == "core_unfold_kernel") {   // (core, Rl, I, Rr, out)
    const size_t b = (size_t)(I(1) * L(2) * I(3) * 8);
    r->push_back({D(0), b, "core"});
    r->push_back({D(4), b, "out"});
  } else if (nm == "identity_table_kernel") {
    r->push_back({D(1), (size_t)(I(0) * I(0) * 8), "out"});
  } else if (nm == "gram_kernel") {   // (core, Rl, I, Rr, E)
    const int64_t n = I(1) * I(3);
    r->push_back({D(0), (size_t)(n * L(2) * 8), "core"});
    r->push_back({D(4), (size_t)(n * n * 8), "E"});
  } else if (nm == "commit_gram_kernel") {   // (G, I, Ra, Rb, core, E, status)
    const int64_t n = I(2) * I(3);
    r->push_back({D(0), (size_t)(L(1) * n * 8), "G"});
    r->push_back({D(4), (size_t)(L(1) * n * 8), "core"});
    r->push_back({D(5), (size_t)(n * n * 8), "E"});
    r->push_back({D(6), 4, "status"});
  } else if (nm == "commit_core_kernel") {   // (G, I, Ra, Rb, core, status)
    const int64_t n = I(2) * I(3);
    r->push_back({D(0), (size_t)(L(1) * n * 8), "G"});
    r->push_back({D(4), (size_t)(L(1) * n * 8), "core"});
  } else if (nm == "ne_apply_kernel") {   // (M, I, n, S, Sinv, refine, G, status)
    const int64_t n = I(2);
    r->push_back({D(0), (size_t)(L(1) * n * 8), "M"});
    r->push_back({D(3), (size_t)(n * n * 8), "S"});
    r->push_back({D(4), (size_t)(n * n * 8), "Sinv"});
    r->push_back({D(6), (size_t)(L(1) * n * 8), "G"});
    r->push_back({D(7), 4, "status"});
  } else if (nm == "widen_f32_kernel") {   // (x, n, out)
    r->push_back({D(0), (size_t)(L(1) * 4), "x"});
    r->push_back({D(2), (size_t)(L(1) * 8), "out"});
  } else if (nm == "transpose_kernel") {   // (A, rows, cols, At)
    r->push_back({D(0), (size_t)(L(1) * L(2) * 8), "A"});
    r->push_back({D(3), (size_t)(L(1) * L(2) * 8), "At"});
  } else if (nm == "table_absmax_kernel") {   // (T, n, out)
    r->push_back({D(0), (size_t)(L(1) * 8), "T"});
    r->push_back({D(2), 8, "out"});
  } else if (nm == "zero_double_kernel") {   // (out)
    r->push_back({D(0), 8, "out"});
  } else if (nm == "v2_direct_kernel") {   // (Tp, Jp, core, I, Rm, Ra, Rb, L, rows, V2)
    const int64_t Jp = L(1), In = L(3), Rm = I(4), Ra = I(5), Rb = I(6), rows = I(8);
    r->push_back({D(0), (size_t)(Jp * Rb * Rm * 8), "Tp"});
    r->push_back({D(2), (size_t)(Rm * In * Ra * 8), "core"});
    r->push_back({D(9), (size_t)(Jp * In * Ra * Rb * 8), "V2"});
    if (rows < 1 || 256 % rows != 0) viol("v2_direct_kernel: rows %lld does not divide the block", (long long)rows);
  } else if (nm == "slice_transpose_kernel") {   // (in, L, I, T, out)
    const size_t b = (size_t)(L(1) * L(2) * L(3) * 8);
    r->push_back({D(0), b, "in"});
    r->push_back({D(4), b, "out"});
  } else if (nm == "spd_block_inv_kernel") {   // (S, n, Sinv, status)
    const int64_t n = I(1);
    r->push_back({D(0), (size_t)(n * n * 8), "S"});
    r->push_back({D(2), (size_t)(n * n * 8), "Sinv"});
  } else if (nm == "bond_to_M_kernel") {   // (Y, In, Ru, Rc, M)
    const size_t b = (size_t)(L(1) * I(2) * I(3) * 8);
    r->push_back({D(0), b, "Y"});
    r->push_back({D(4), b, "M"});
  } else if (nm == "table_to_bt_fp8_kernel") {   // (T, K, C, Crows, ldb, tmax, Bt)
    r->push_back({D(0), (size_t)(L(1) * I(2) * 8), "T"});
    r->push_back({D(5), 8, "tmax"});
    r->push_back({D(6), (size_t)(2 * I(3) * L(4)), "Bt"});
  } else if (nm == "xg_reduce_kernel") {   // <prec>(XgArgs, int, double, Y, status)
    const XgArgs g = arg<XgArgs>(a, 0);
    if (g.tmax) r->push_back({(uintptr_t)g.tmax, 8, "tmax"});
    const size_t es = template_int(full, 0) == 0 ? 8 : 4;
    r->push_back({(uintptr_t)g.partial, (size_t)g.nsplit * g.n_mt * g.n_nt * g.MT * g.NT * es, "partial"});
    r->push_back({D(3), (size_t)(g.M * g.C * 8), "Y"});
  } else if (nm == "xgemm_kernel") {   // <prec, T, ...>(XgArgs)
    const XgArgs g = arg<XgArgs>(a, 0);
    const int p = template_int(full, 0);
    const size_t xes = p == 0 ? (full.find("float") != std::string::npos ? 4 : 8) : p == 1 ? 4 : es_of_prec(p);
    const size_t bes = p == 0 ? 8 : p == 1 ? 4 : es_of_prec(p);
    r->push_back({(uintptr_t)g.X, (size_t)(g.M * g.K) * xes, "X"});
    r->push_back({(uintptr_t)g.Bt, (size_t)g.n_nt * g.NT * g.ldb * bes * (p == 3 ? 2 : 1), "Bt"});   // FP8: hi, lo
    if (p == 3) r->push_back({(uintptr_t)g.tmax, 8, "tmax"});
    r->push_back({(uintptr_t)g.partial, (size_t)g.nsplit * g.n_mt * g.n_nt * g.MT * g.NT * (p == 0 ? 8 : 4),
                  "partial"});
  } else if (nm == "xs_reduce_kernel") {   // <prec>(XsArgs, double, M, status)
    const XsArgs x = arg<XsArgs>(a, 0);
    if (x.tmax) r->push_back({(uintptr_t)x.tmax, 16, "tmax"});
    const size_t es = template_int(full, 0) == 0 ? 8 : 4;
    r->push_back({(uintptr_t)x.partial, (size_t)x.nsplit * x.n_mt * x.n_nt * x.MT * x.NT * es, "partial"});
    r->push_back({D(2), (size_t)(x.I * x.Ra * x.Rb * 8), "M"});
  } else if (nm == "xstream_kernel") {
    const XsArgs x = arg<XsArgs>(a, 0);
    const int p = template_int(full, 0);
    if (p == 3) r->push_back({(uintptr_t)x.tmax, 16, "tmax"});
    r->push_back({(uintptr_t)x.partial, (size_t)x.nsplit * x.n_mt * x.n_nt * x.MT * x.NT * (p == 0 ? 8 : 4),
                  "partial"});
  } else if (nm == "to_bf16_kernel" || nm == "to_fp8_kernel" || nm == "sumsq_kernel" || nm == "absmax_kernel") {
    const size_t es = full.find("<double>") != std::string::npos ? 8 : 4;
    r->push_back({D(0), (size_t)L(1) * es, "X"});
    if (nm == "to_bf16_kernel") r->push_back({D(2), (size_t)L(1) * 2, "out"});
    if (nm == "to_fp8_kernel") r->push_back({D(4), (size_t)L(1), "out"});
  } else if (nm == "to_lowp_t_kernel") {   // <T, fp8>(X, M, K, absmax, out)
    const size_t es = full.find("<double") != std::string::npos ? 8 : 4;
    const size_t n = (size_t)(L(1) * L(2));
    r->push_back({D(0), n * es, "X"});
    r->push_back({D(4), n * (full.find("true>") != std::string::npos ? 1 : 2), "out"});
  } else if (nm == "xslab_kernel" || nm == "xslab_reduce_kernel" || nm == "xslab_table_kernel") {
    const XslabArgs x = arg<XslabArgs>(a, 0);
    const bool f64 = full.find("<0") != std::string::npos || full.find("<double") != std::string::npos;
    const size_t es = f64 ? 8 : (full.find("float") != std::string::npos ? 4 : 2);
    const size_t pes = full.find("<0") != std::string::npos ? 8 : 4;   // partials of the FP64 path
    const size_t parts = (size_t)x.nsplit * x.n_mt * x.n_g * 128 * x.OWg;
    if (nm == "xslab_kernel") {
      // X: the last element of the largest slab range the kernel walks
      const size_t xes = full.find(", double") != std::string::npos ? 8 : full.find(", float") != std::string::npos ? 4 : 2;
      const int64_t last = (x.In - 1) * x.sn + (x.Ik - 1) * x.sk + (x.Il - 1) * x.sl;
      r->push_back({(uintptr_t)x.X, (size_t)(last + 1) * xes, "X"});
      r->push_back({(uintptr_t)x.Bt, (size_t)x.n_g * x.TWg * x.ldb * (f64 ? 8 : es == 2 ? 4 : es), "table"});
      r->push_back({(uintptr_t)x.partial, parts * (full.find("<0") != std::string::npos ? 8 : 4), "partial"});
      r->push_back({(uintptr_t)x.Gl, (size_t)x.Rm * x.Il * x.Ro * 8, "absorbed core"});
    } else if (nm == "xslab_reduce_kernel") {
      r->push_back({(uintptr_t)x.partial, parts * pes, "partial"});
      r->push_back({D(2), (size_t)(x.In * x.Rn * (x.caseB ? x.Ro : x.Rg) * 8), "M"});
    } else {
      r->push_back({D(2), (size_t)x.n_g * x.TWg * x.ldb * (es == 2 ? 4 : es), "table"});   // BF16: hi and lo
      r->push_back({D(1), (size_t)x.Rm * x.Ik * x.Rg * 8, "core"});
    }
  } else if (nm == "copy_block_kernel") {   // (src, lds, rows, cols, dst, ldd, trans, add)
    const int64_t rows = I(2), cols = I(3), lds_ = L(1), ldd = L(5);
    if (D(0)) r->push_back({D(0), (size_t)((arg<int>(a, 6) ? lds_ * (rows - 1) + cols : lds_ * (cols - 1) + rows) * 8),
                            "src"});
    r->push_back({D(4), (size_t)((ldd * (cols - 1) + rows) * 8), "dst"});
  } else if (nm == "chol_lds_kernel") {     // (S, n, L, LT, status, rdiag)
    const size_t b = (size_t)(I(1) * I(1) * 8);
    r->push_back({D(0), b, "S"});
    r->push_back({D(2), b, "L"});
    r->push_back({D(3), b, "LT"});
    r->push_back({D(5), (size_t)((I(1) + 7) / 8 * 8 * 8), "rdiag"});   // padded to 8-column blocks
  } else if (nm == "trsm_rhs_kernel") {     // (L, rdiag, n, Rhs, I, G, accumulate, status, mode)
    const int64_t n = I(2), rows = L(4);
    r->push_back({D(0), (size_t)(n * n * 8), "L"});
    if (D(3)) r->push_back({D(3), (size_t)(rows * n * 8), "Rhs"});
    r->push_back({D(5), (size_t)(rows * n * 8), "G"});
  } else if (nm == "philox_normal_kernel") {
    r->push_back({D(0), (size_t)L(1) * 8, "out"});
  } else if (nm == "tiny_als_kernel") {
    // one descriptor per workgroup (the grid size is checked with the launch
    // shape); each job's operands, and its status word, which the kernel
    // always writes at the end (modelled here as a clear status)
    const TinyJob* jobs = arg<const TinyJob*>(a, 0);
    r->push_back({(uintptr_t)jobs, sizeof(TinyJob), "job descriptors"});
    if (in_bounds((uintptr_t)jobs, sizeof(TinyJob)))
      for (unsigned q = 0; q < t_grid_x && in_bounds((uintptr_t)(jobs + q), sizeof(TinyJob)); ++q) {
        const TinyJob& j = jobs[q];
        int64_t numel = 1;
        for (int k = 0; k < j.N && k < 4; ++k) numel *= j.dims[k];
        r->push_back({(uintptr_t)j.X, (size_t)numel * (j.xdt == 0 ? 8 : 4), "job X"});
        for (int k = 0; k < j.N && k < 4; ++k)
          r->push_back({(uintptr_t)j.cores[k], (size_t)(j.R[k] * j.dims[k] * j.R[k + 1] * 8), "job core"});
        r->push_back({(uintptr_t)j.status, 4, "job status"});
        r->push_back({(uintptr_t)j.scal, 16, "job norms"});
        if (in_bounds((uintptr_t)j.status, 4)) *j.status = 0;
      }
  }
}

void launch_checks(const void* f, dim3 g, dim3 b, void** args, size_t shm, Op* op) {
  auto it = names().find(f);
  const std::string full = it == names().end() ? std::string("<unregistered kernel>") : it->second;
  const std::string nm = base_name(full);
  op->name = nm;
  g_launches[nm]++;
  t_grid_x = g.x;
  if (!g.x || !g.y || !g.z) viol("%s: empty grid (%u, %u, %u)", nm.c_str(), g.x, g.y, g.z);
  const unsigned long nt = (unsigned long)b.x * b.y * b.z;
  if (nt == 0 || nt > 1024) viol("%s: block of %lu threads", nm.c_str(), nt);
  if (shm > LDS_MAX) viol("%s: %zu bytes of dynamic LDS", nm.c_str(), shm);
  if (shm > LDS_DEFAULT) {
    auto lim = g_lds_limit.find(f);
    if (lim == g_lds_limit.end() || (size_t)lim->second < shm)
      viol("%s: %zu bytes of dynamic LDS without a raised limit", nm.c_str(), shm);
  }
  const std::vector<std::string> ts = param_types(full);
  for (size_t q = 0; q < ts.size(); ++q)
    if (!ts[q].empty() && ts[q].back() == '*') {
      const uintptr_t p = (uintptr_t)arg<const void*>(args, (int)q);
      if (p) op->ranges.push_back({p, 1, "argument " + std::to_string(q) + " (" + ts[q] + ")"});
    }
  check_extents(full, nm, args, &op->ranges);
  for (const Range& r : op->ranges) check_range(nm, r);
}

Capture* capture_of(hipStream_t s) { return s ? s->cap : nullptr; }

}  // namespace

// ---------------------------------------------------------------------------
// the runtime entry points the library uses
// ---------------------------------------------------------------------------
extern "C" {

void** __hipRegisterFatBinary(const void*) {
  static void* mod = nullptr;
  return &mod;
}
void __hipUnregisterFatBinary(void**) {}
void __hipRegisterFunction(void**, const void* hostFunction, char*, const char* deviceName, unsigned int, uint3*,
                           uint3*, dim3*, dim3*, int*) {
  std::lock_guard<std::recursive_mutex> lk(mu());
  names()[hostFunction] = demangle(deviceName);
}
// device variables: host shadow -> stand-in device allocation of the same size
static std::unordered_map<const void*, void*>& vars() {
  static auto* m = new std::unordered_map<const void*, void*>();
  return *m;
}
static hipError_t do_alloc(void** p, size_t bytes, bool host);
void __hipRegisterVar(void**, void* var, char*, char*, int, size_t size, int, int) {
  std::lock_guard<std::recursive_mutex> lk(mu());
  void* p = nullptr;
  if (do_alloc(&p, size, false) == hipSuccess) {
    vars()[var] = p;
    allocs()[(uintptr_t)p].var = true;
  }
}
hipError_t hipGetSymbolAddress(void** devPtr, const void* symbol) {
  std::lock_guard<std::recursive_mutex> lk(mu());
  touch();
  auto it = vars().find(symbol);
  if (!devPtr || it == vars().end()) return ret(hipErrorInvalidSymbol);
  *devPtr = it->second;
  return hipSuccess;
}
hipError_t __hipPushCallConfiguration(dim3 g, dim3 b, size_t shm, hipStream_t s) {
  t_cfg.push_back({g, b, shm, s});
  return hipSuccess;
}
hipError_t __hipPopCallConfiguration(dim3* g, dim3* b, size_t* shm, hipStream_t* s) {
  if (t_cfg.empty()) return hipErrorInvalidConfiguration;
  const CallCfg c = t_cfg.back();
  t_cfg.pop_back();
  *g = c.g; *b = c.b; *shm = c.shm; *s = c.s;
  return hipSuccess;
}

hipError_t hipLaunchKernel(const void* f, dim3 g, dim3 b, void** args, size_t shm, hipStream_t s) {
  std::lock_guard<std::recursive_mutex> lk(mu());
  touch();
  Op op;
  launch_checks(f, g, b, args, shm, &op);
  if (!g.x || !g.y || !g.z) return ret(hipErrorInvalidConfiguration);
  if (Capture* c = capture_of(s)) c->ops.push_back(std::move(op));
  return hipSuccess;
}

hipError_t hipFuncSetAttribute(const void* f, hipFuncAttribute attr, int value) {
  std::lock_guard<std::recursive_mutex> lk(mu());
  touch();
  if (attr == hipFuncAttributeMaxDynamicSharedMemorySize) {
    if (value < 0 || (size_t)value > LDS_MAX) return ret(hipErrorInvalidValue);
    g_lds_limit[f] = value;
  }
  return hipSuccess;
}

static hipError_t do_alloc(void** p, size_t bytes, bool host) {
  std::lock_guard<std::recursive_mutex> lk(mu());
  touch();
  if (!p) return ret(hipErrorInvalidValue);
  if (g_open_captures && !host) viol("hipMalloc of %zu bytes while a stream capture is open", bytes);
  calls()[host ? "host alloc" : "alloc"]++;
  const size_t sz = std::max<size_t>(bytes, 1);
  const size_t mapped = (sz + 4095) / 4096 * 4096;
  void* m = mmap(nullptr, mapped, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
  if (m == MAP_FAILED) { *p = nullptr; return ret(hipErrorOutOfMemory); }
  allocs()[(uintptr_t)m] = {bytes, true, host};
  *p = m;
  return hipSuccess;
}

static hipError_t do_free(void* p) {
  std::lock_guard<std::recursive_mutex> lk(mu());
  touch();
  if (!p) return hipSuccess;
  if (g_open_captures) viol("free while a stream capture is open");
  calls()["free"]++;
  auto it = allocs().find((uintptr_t)p);
  if (it == allocs().end()) {
    viol("free of %p, which is not the start of a live allocation", p);
    return ret(hipErrorInvalidValue);
  }
  munmap(p, (std::max<size_t>(it->second.size, 1) + 4095) / 4096 * 4096);
  allocs().erase(it);
  return hipSuccess;
}

hipError_t hipMalloc(void** p, size_t bytes) { return do_alloc(p, bytes, false); }
hipError_t hipFree(void* p) { return do_free(p); }
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned int) { return do_alloc(p, bytes, true); }
hipError_t hipHostFree(void* p) { return do_free(p); }

hipError_t hipMemGetInfo(size_t* fr, size_t* tot) {
  touch();
  *fr = (size_t)16 << 30;
  *tot = (size_t)288 << 30;
  return hipSuccess;
}

static hipError_t copy(void* dst, const void* src, size_t n, hipMemcpyKind kind, hipStream_t s, bool async) {
  std::lock_guard<std::recursive_mutex> lk(mu());
  touch();
  const bool dd = kind == hipMemcpyDeviceToDevice || kind == hipMemcpyHostToDevice || kind == hipMemcpyDefault;
  const bool sd = kind == hipMemcpyDeviceToDevice || kind == hipMemcpyDeviceToHost || kind == hipMemcpyDefault;
  if (dd && !in_bounds((uintptr_t)dst, n)) viol("copy of %zu bytes: destination %p out of bounds", n, dst);
  if (sd && !in_bounds((uintptr_t)src, n)) viol("copy of %zu bytes: source %p out of bounds", n, src);
  Capture* c = async ? capture_of(s) : nullptr;
  if (!async && g_open_captures) viol("synchronous copy while a stream capture is open");
  if (c) {
    if (kind != hipMemcpyDeviceToDevice) viol("host copy recorded into a graph");
    Op op;
    op.name = "memcpy";
    op.ranges = {{(uintptr_t)dst, n, "dst"}, {(uintptr_t)src, n, "src"}};
    c->ops.push_back(op);
    return hipSuccess;
  }
  if (n) std::memmove(dst, src, n);
  return hipSuccess;
}

hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind k) { return copy(d, s, n, k, nullptr, false); }
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t st) {
  return copy(d, s, n, k, st, true);
}

hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t s) {
  std::lock_guard<std::recursive_mutex> lk(mu());
  touch();
  if (!in_bounds((uintptr_t)d, n)) viol("fill of %zu bytes at %p out of bounds", n, d);
  if (capture_of(s)) viol("fill recorded into a graph");
  else if (n) std::memset(d, v, n);
  return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int flags) {
  std::lock_guard<std::recursive_mutex> lk(mu());
  touch();
  *s = new ihipStream_t;
  (*s)->flags = flags;
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  std::lock_guard<std::recursive_mutex> lk(mu());
  touch();
  if (s && s->cap) viol("destroy of a capturing stream");
  delete s;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  std::lock_guard<std::recursive_mutex> lk(mu());
  touch();
  if (capture_of(s)) viol("synchronisation of a capturing stream");
  calls()["sync"]++;
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int) {
  std::lock_guard<std::recursive_mutex> lk(mu());
  touch();
  if (e && e->cap && s && !s->cap) {   // the waiting stream joins the capture
    s->cap = e->cap;
    e->cap->joined.push_back(s);
  }
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  std::lock_guard<std::recursive_mutex> lk(mu());
  touch();
  if (!s) return ret(hipErrorStreamCaptureUnsupported);
  if (s->cap) return ret(hipErrorIllegalState);
  s->cap = new Capture;
  g_open_captures++;
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  std::lock_guard<std::recursive_mutex> lk(mu());
  touch();
  if (!s || !s->cap) return ret(hipErrorIllegalState);
  Capture* c = s->cap;
  for (hipStream_t j : c->joined) j->cap = nullptr;
  s->cap = nullptr;
  g_open_captures--;
  *g = new ihipGraph{std::move(c->ops)};
  delete c;
  return hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t* ex, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  std::lock_guard<std::recursive_mutex> lk(mu());
  touch();
  *ex = new hipGraphExec{g->ops};
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  touch();
  delete g;
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t ex) {
  touch();
  delete ex;
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t ex, hipStream_t s) {
  std::lock_guard<std::recursive_mutex> lk(mu());
  touch();
  if (capture_of(s)) viol("graph launched into a capture");
  for (const Op& op : ex->ops) {
    g_launches[op.name]++;
    for (const Range& r : op.ranges) check_range("replayed " + op.name, r);
  }
  return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t* e) {
  touch();
  *e = new ihipEvent_t;
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned int) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
  touch();
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  std::lock_guard<std::recursive_mutex> lk(mu());
  touch();
  e->cap = capture_of(s);
  e->ready_at = now_us() + g_delay_us;
  return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
  touch();
  return (e && now_us() < e->ready_at) ? hipErrorNotReady : hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t) {
  touch();
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  touch();
  *ms = 0.001f;
  return hipSuccess;
}

hipError_t hipGetDevice(int* d) {
  touch();
  *d = 0;
  return hipSuccess;
}
hipError_t hipSetDevice(int) {
  touch();
  return hipSuccess;
}
hipError_t hipGetLastError(void) {
  const hipError_t e = t_last;
  t_last = hipSuccess;
  return e;
}
const char* hipGetErrorString(hipError_t e) {
  static thread_local char buf[64];
  snprintf(buf, sizeof buf, "stand-in HIP error %d", (int)e);
  return buf;
}

// ---------------------------------------------------------------------------
// inspection, for the tests
// ---------------------------------------------------------------------------
int fakehip_violation_count(void) {
  std::lock_guard<std::recursive_mutex> lk(mu());
  return (int)g_viol.size();
}
const char* fakehip_violation(int k) {
  std::lock_guard<std::recursive_mutex> lk(mu());
  return (k >= 0 && k < (int)g_viol.size()) ? g_viol[k].c_str() : "";
}
void fakehip_reset(void) {
  std::lock_guard<std::recursive_mutex> lk(mu());
  g_viol.clear();
  g_launches.clear();
  g_gemm_log.clear();
  calls().clear();
}
// allocations ("alloc", "host alloc"), frees ("free") and stream
// synchronisations ("sync") since the last reset
long fakehip_calls(const char* what) {
  std::lock_guard<std::recursive_mutex> lk(mu());
  auto it = calls().find(what ? what : "");
  return it == calls().end() ? 0 : it->second;
}
long fakehip_launches(const char* kernel) {
  std::lock_guard<std::recursive_mutex> lk(mu());
  if (!kernel) {
    long n = 0;
    for (auto& kv : g_launches) n += kv.second;
    return n;
  }
  auto it = g_launches.find(kernel);
  return it == g_launches.end() ? 0 : it->second;
}
// FP64 GEMM launches since the last reset: rows, columns, whether the output
// is stored realigned as a coefficient matrix, whether it was one of a pair
int fakehip_gemm_log(long long* out, int cap) {
  std::lock_guard<std::recursive_mutex> lk(mu());
  const int n = (int)g_gemm_log.size();
  for (int k = 0; k < n && k < cap; ++k)
    for (int q = 0; q < 4; ++q) out[4 * k + q] = g_gemm_log[k][q];
  return n;
}
int fakehip_live_allocations(void) {   // allocated by calls, not the library's device variables
  std::lock_guard<std::recursive_mutex> lk(mu());
  int n = 0;
  for (auto& kv : allocs()) n += kv.second.var ? 0 : 1;
  return n;
}
// completion of recorded work is reported this many microseconds after it
// was recorded, so that callers polling events see work in flight
void fakehip_set_delay_us(long long us) {
  std::lock_guard<std::recursive_mutex> lk(mu());
  g_delay_us = us;
}
void fakehip_window_begin(void) {
  std::lock_guard<std::recursive_mutex> lk(mu());
  g_window = true;
  g_window_threads.clear();
}
int fakehip_window_end(void) {
  std::lock_guard<std::recursive_mutex> lk(mu());
  g_window = false;
  return (int)g_window_threads.size();
}
void* fakehip_device_alloc(size_t bytes) {
  void* p = nullptr;
  return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
}
void fakehip_device_free(void* p) { (void)hipFree(p); }

}  // extern "C"

// ---------------------------------------------------------------------------
// rocBLAS calls of the library (QR-based variants, R_n R_{n+1} > 128): the
// operand extents are checked like a kernel's, the call is counted as a launch
// under its own name, and none may be issued on a stream under capture
// ---------------------------------------------------------------------------
#include <rocblas/rocblas.h>

namespace {
struct FakeBlas { hipStream_t s = nullptr; };

size_t mat_bytes(int64_t rows, int64_t cols, int64_t ld) {
  if (rows <= 0 || cols <= 0) return 0;
  if (ld < rows) viol("rocBLAS: leading dimension %lld below %lld rows", (long long)ld, (long long)rows);
  return (size_t)(ld * (cols - 1) + rows) * sizeof(double);
}

void blas_call(rocblas_handle h, const char* nm, std::initializer_list<Range> rs) {
  touch();
  g_launches[nm]++;
  FakeBlas* b = reinterpret_cast<FakeBlas*>(h);
  if (capture_of(b->s)) viol("%s on a stream under capture", nm);
  for (const Range& r : rs) check_range(nm, r);
}
}  // namespace

extern "C" {
rocblas_status rocblas_create_handle(rocblas_handle* h) {
  *h = reinterpret_cast<rocblas_handle>(new FakeBlas());
  return rocblas_status_success;
}
rocblas_status rocblas_destroy_handle(rocblas_handle h) {
  delete reinterpret_cast<FakeBlas*>(h);
  return rocblas_status_success;
}
rocblas_status rocblas_set_stream(rocblas_handle h, hipStream_t s) {
  reinterpret_cast<FakeBlas*>(h)->s = s;
  return rocblas_status_success;
}
const char* rocblas_status_to_string(rocblas_status) { return "stand-in"; }

rocblas_status rocblas_dsyrk(rocblas_handle h, rocblas_fill, rocblas_operation t, rocblas_int n, rocblas_int k,
                             const double*, const double* A, rocblas_int lda, const double*, double* C,
                             rocblas_int ldc) {
  const bool tr = t != rocblas_operation_none;
  blas_call(h, "rocblas_dsyrk", {{(uintptr_t)A, tr ? mat_bytes(k, n, lda) : mat_bytes(n, k, lda), "A"},
                                 {(uintptr_t)C, mat_bytes(n, n, ldc), "C"}});
  return rocblas_status_success;
}
rocblas_status rocblas_dtrsm(rocblas_handle h, rocblas_side side, rocblas_fill, rocblas_operation, rocblas_diagonal,
                             rocblas_int m, rocblas_int n, const double*, const double* A, rocblas_int lda, double* B,
                             rocblas_int ldb) {
  const int64_t k = side == rocblas_side_right ? n : m;
  blas_call(h, "rocblas_dtrsm", {{(uintptr_t)A, mat_bytes(k, k, lda), "A"}, {(uintptr_t)B, mat_bytes(m, n, ldb), "B"}});
  return rocblas_status_success;
}
rocblas_status rocblas_dgemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, rocblas_int m,
                             rocblas_int n, rocblas_int k, const double*, const double* A, rocblas_int lda,
                             const double* B, rocblas_int ldb, const double*, double* C, rocblas_int ldc) {
  const bool a_t = ta != rocblas_operation_none, b_t = tb != rocblas_operation_none;
  blas_call(h, "rocblas_dgemm", {{(uintptr_t)A, a_t ? mat_bytes(k, m, lda) : mat_bytes(m, k, lda), "A"},
                                 {(uintptr_t)B, b_t ? mat_bytes(n, k, ldb) : mat_bytes(k, n, ldb), "B"},
                                 {(uintptr_t)C, mat_bytes(m, n, ldc), "C"}});
  return rocblas_status_success;
}
rocblas_status rocblas_dgemm_strided_batched(rocblas_handle h, rocblas_operation ta, rocblas_operation tb,
                                             rocblas_int m, rocblas_int n, rocblas_int k, const double*,
                                             const double* A, rocblas_int lda, rocblas_stride sa, const double* B,
                                             rocblas_int ldb, rocblas_stride sb, const double*, double* C,
                                             rocblas_int ldc, rocblas_stride sc, rocblas_int batch) {
  const bool a_t = ta != rocblas_operation_none, b_t = tb != rocblas_operation_none;
  const size_t last = batch > 0 ? (size_t)(batch - 1) : 0;
  blas_call(h, "rocblas_dgemm_strided_batched",
            {{(uintptr_t)A, last * sa * 8 + (a_t ? mat_bytes(k, m, lda) : mat_bytes(m, k, lda)), "A"},
             {(uintptr_t)B, last * sb * 8 + (b_t ? mat_bytes(n, k, ldb) : mat_bytes(k, n, ldb)), "B"},
             {(uintptr_t)C, last * sc * 8 + mat_bytes(m, n, ldc), "C"}});
  return rocblas_status_success;
}
}  // extern "C"
