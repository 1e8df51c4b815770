// Problem-specialised walk and branching kernels: source generation, runtime
// compilation (hiprtc) and a two-level cache of the compiled code objects.
#include "pdd_spec.hpp"

#include <hip/hiprtc.h>
#include <sys/stat.h>
#include <unistd.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>

namespace pdd {

// Text of the device headers, embedded at build time (rtc_sources.cpp).
extern const int kRtcHeaderCount;
extern const char* const kRtcHeaderNames[];
extern const char* const kRtcHeaderBodies[];

namespace {

bool literal(double v, std::string* out) {
  if (!std::isfinite(v)) return false;
  char b[64];
  std::snprintf(b, sizeof b, "%a", v);
  *out = std::string("(R)") + b;
  return true;
}

const char* kFunNames[6] = {"b0", "b1", "b2", "c", "f", "g"};

const DevFun& fun_at(const LinearParams& P, int w) {
  if (w < 3) return P.b[w];
  if (w == 3) return P.c;
  if (w == 4) return P.f;
  return P.g;
}

uint64_t fnv1a(const std::string& s) {
  uint64_t h = 1469598103934665603ull;
  for (unsigned char ch : s) {
    h ^= ch;
    h *= 1099511628211ull;
  }
  return h;
}

std::string cache_dir() {
  const char* e = std::getenv("PDD_JIT_CACHE");
  if (e && *e) return e;
  const char* home = std::getenv("HOME");
  if (!home || !*home) return "";
  return std::string(home) + "/.cache/pdd_jit";
}

// One cache entry is one file, written to a temporary name and renamed into
// place, so a reader sees either a whole entry or none:
//   "PDDJIT3\n", four little-endian uint64 (the lengths of the key, the
//   symbol and the code object, then a 64-bit FNV-1a checksum of those three
//   byte strings in that order), then the three byte strings.
// An entry whose checksum does not match (damaged in place) is treated as
// missing: the kernel is compiled again and the entry replaced.  The checksum
// guards against damage, not against someone who can write the cache
// directory.
constexpr char kEntryMagic[8] = {'P', 'D', 'D', 'J', 'I', 'T', '3', '\n'};

uint64_t entry_checksum(const char* p, size_t n) {
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= (unsigned char)p[i];
    h *= 1099511628211ull;
  }
  return h;
}

bool read_entry(const std::string& p, const std::string& key, std::string* sym, std::string* code) {
  std::ifstream f(p, std::ios::binary);
  if (!f) return false;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string d = ss.str();
  const size_t head = sizeof kEntryMagic + 4 * sizeof(uint64_t);
  if (d.size() < head || d.compare(0, sizeof kEntryMagic, kEntryMagic, sizeof kEntryMagic) != 0) return false;
  uint64_t n[4];
  std::memcpy(n, d.data() + sizeof kEntryMagic, sizeof n);
  if (n[0] > d.size() || n[1] > d.size() || n[2] > d.size() || head + n[0] + n[1] + n[2] != d.size()) return false;
  if (n[1] == 0 || n[2] == 0 || d.compare(head, n[0], key) != 0) return false;
  if (entry_checksum(d.data() + head, n[0] + n[1] + n[2]) != n[3]) return false;
  sym->assign(d, head + n[0], n[1]);
  code->assign(d, head + n[0] + n[1], n[2]);
  return true;
}

void write_entry(const std::string& p, const std::string& key, const std::string& sym, const std::string& code) {
  const std::string tmp = p + ".tmp" + std::to_string((long)getpid());
  {
    std::ofstream f(tmp, std::ios::binary);
    if (!f) return;
    const std::string body = key + sym + code;
    const uint64_t n[4] = {key.size(), sym.size(), code.size(), entry_checksum(body.data(), body.size())};
    f.write(kEntryMagic, sizeof kEntryMagic);
    f.write(reinterpret_cast<const char*>(n), sizeof n);
    f << body;
    if (!f) {
      f.close();
      std::remove(tmp.c_str());
      return;
    }
  }
  if (std::rename(tmp.c_str(), p.c_str()) != 0) std::remove(tmp.c_str());
}

void make_dirs(const std::string& d) {
  for (size_t i = 1; i <= d.size(); ++i)
    if (i == d.size() || d[i] == '/') mkdir(d.substr(0, i).c_str(), 0755);
}

std::mutex g_spec_mu;
std::map<std::string, hipFunction_t> g_spec;   // (device, key) -> loaded kernel

}  // namespace

bool spec_compile(const std::string& src, const std::string& name, const std::string& arch, std::string* code,
                  std::string* lowered, std::string* err) {
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "pdd_spec.hip", kRtcHeaderCount, kRtcHeaderBodies, kRtcHeaderNames) !=
      HIPRTC_SUCCESS) {
    *err = "hiprtcCreateProgram failed";
    return false;
  }
  hiprtcAddNameExpression(prog, name.c_str());
  const std::string a = "--offload-arch=" + arch;
  // the same code-generation flags as the precompiled kernels (no packed FP32)
  const char* opts[] = {a.c_str(), "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
  const hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
  if (r != HIPRTC_SUCCESS) {
    size_t n = 0;
    hiprtcGetProgramLogSize(prog, &n);
    std::string log(n, '\0');
    if (n) hiprtcGetProgramLog(prog, &log[0]);
    *err = std::string("runtime compilation failed: ") + hiprtcGetErrorString(r) + "\n" + log.substr(0, 4000);
    hiprtcDestroyProgram(&prog);
    return false;
  }
  const char* low = nullptr;
  if (hiprtcGetLoweredName(prog, name.c_str(), &low) != HIPRTC_SUCCESS || low == nullptr) {
    *err = "hiprtcGetLoweredName failed";
    hiprtcDestroyProgram(&prog);
    return false;
  }
  *lowered = low;
  size_t n = 0;
  hiprtcGetCodeSize(prog, &n);
  code->assign(n, '\0');
  if (n == 0 || hiprtcGetCode(prog, &(*code)[0]) != HIPRTC_SUCCESS) {
    *err = "hiprtcGetCode failed";
    hiprtcDestroyProgram(&prog);
    return false;
  }
  hiprtcDestroyProgram(&prog);
  return true;
}

std::string spec_terms_source(const LinearParams& P, const std::vector<DevFactor>& fac) {
  std::ostringstream term, sum, load;
  bool first = true;
  int nst = 0;   // state slots: the term coefficients of b, c and f
  for (int w = 0; w < 6; ++w) {
    const DevFun& F = fun_at(P, w);
    if (F.n_terms <= 0) continue;
    const char* el = first ? "" : "else ";
    first = false;
    term << "    " << el << "if constexpr (W == " << w << ") {  // " << kFunNames[w] << "\n";
    sum << "    " << el << "if constexpr (W == " << w << ") {\n";
    for (int t = 0; t < F.n_terms; ++t) {
      term << "      " << (t ? "else " : "") << "if (t == " << t << ") {";
      for (int j = 0; j < F.n_factors; ++j) {
        const DevFactor& d = fac[(size_t)(F.fac_off + t * F.n_factors + j)];
        std::string a, b;
        if (!literal(d.ad, &a) || !literal(d.bd, &b)) return "";
        term << "\n        v *= pdd::factor_fixed<R, DIM, " << d.fn << ", " << d.power << ">(x, " << d.dim << ", " << a
             << ", " << b << ");";
      }
      term << "\n      }\n";
      if (w == 5) {
        // g is evaluated once per exit: its coefficients stay in the table
        sum << "      s += c[" << (F.coef_off + t) << "] * term<R, DIM, W>(P, " << t << ", x);\n";
      } else {
        load << "    st.c[" << nst << "] = c[" << (F.coef_off + t) << "];\n"
             << "    asm volatile(\"\" : \"+v\"(st.c[" << nst << "]));\n";
        sum << "      s += st.c[" << nst << "] * term<R, DIM, W>(P, " << t << ", x);\n";
        ++nst;
      }
    }
    term << "    }\n";
    sum << "    }\n";
  }
  std::ostringstream o;
  o << "namespace pdd_spec {\n"
       "struct SpecTerms {\n"
       "  template <typename R>\n"
       "  struct State {\n"
       "    R c["
    << (nst > 0 ? nst : 1)
    << "];\n"
       "  };\n"
       "  template <typename R>\n"
       "  __device__ static __forceinline__ State<R> load(const pdd::LinearParams& P) {\n"
       "    State<R> st;\n"
       "    const R PDD_CONST_AS* c = pdd::coef_table<R>(P);\n"
       "    (void)c;\n"
    << load.str()
    << "    return st;\n"
       "  }\n"
       "  template <typename R, int DIM, int W>\n"
       "  __device__ static __forceinline__ R term(const pdd::LinearParams& P, int t, const R* x) {\n"
       "    (void)P;\n"
       "    R v = (R)1;\n"
    << term.str()
    << "    return v;\n"
       "  }\n"
       "  template <typename R, int DIM, int W>\n"
       "  __device__ static __forceinline__ R sum(const pdd::LinearParams& P, const State<R>& st, const R* x) {\n"
       "    const R PDD_CONST_AS* c = pdd::coef_table<R>(P);\n"
       "    (void)c;\n"
       "    (void)st;\n"
       "    R s = (R)0;\n"
    << sum.str()
    << "    return s;\n"
       "  }\n"
       "};\n"
       "}  // namespace pdd_spec\n";
  return o.str();
}

namespace {

// Sum of the generic terms of F at the coordinates `x` (DIMS of them), then
// its dense polynomial part at `xp` (degree and offset written in, so the
// loops unroll), into `v`: the operations of terms_sum and poly_nested in
// their order.
bool emit_fun(std::ostringstream& o, const DevFun& F, const std::vector<DevFactor>& fac, const char* dims,
              const char* x, const char* xp) {
  o << "    R v = (R)0;\n";
  if (F.n_terms > 0) {
    o << "    {\n      R s = (R)0;\n";
    for (int t = 0; t < F.n_terms; ++t) {
      o << "      {\n        R p = (R)1;\n";
      for (int j = 0; j < F.n_factors; ++j) {
        const DevFactor& d = fac[(size_t)(F.fac_off + t * F.n_factors + j)];
        std::string a, b;
        if (!literal(d.ad, &a) || !literal(d.bd, &b)) return false;
        o << "        p *= pdd::factor_fixed<R, " << dims << ", " << d.fn << ", " << d.power << ">(" << x << ", "
          << d.dim << ", " << a << ", " << b << ");\n";
      }
      o << "        s += pdd::coef_const<R>(P.cd, P.cf, " << (F.coef_off + t) << ") * p;\n      }\n";
    }
    o << "      v = s;\n    }\n";
  }
  if (F.poly_deg >= 0)
    o << "    v += pdd::poly_nested<R, DIM>(P.cd, P.cf, " << F.poly_deg << ", " << F.poly_off << ", " << xp << ");\n";
  o << "    return v;\n";
  return true;
}

}  // namespace

std::string spec_psi_source(const DevFun& psi, const DevFun* g, const std::vector<DevFactor>& fac) {
  std::ostringstream o;
  o << "namespace pdd_spec {\n"
       "struct SpecPsi {\n"
       "  template <typename R, int DIM>\n"
       "  __device__ static __forceinline__ R psi(const pdd::BranchParams& P, const R* x) {\n"
       "    (void)P;\n";
  if (!emit_fun(o, psi, fac, "DIM", "x", "x")) return "";
  o << "  }\n";
  if (g != nullptr) {
    o << "  template <typename R, int DIM>\n"
         "  __device__ static __forceinline__ R g(const pdd::BranchParams& P, const pdd::BranchBoundary& B,\n"
         "                                        const R* xp, R ts) {\n"
         "    (void)P;\n"
         "    (void)B;\n"
         "    R xs[DIM + 1];\n"
         "#pragma unroll\n"
         "    for (int k = 0; k < DIM; ++k) xs[k] = xp[k];\n"
         "    xs[DIM] = ts;\n"
         "    (void)xs;\n";
    if (!emit_fun(o, *g, fac, "DIM + 1", "xs", "xp")) return "";
    o << "  }\n";
  }
  o << "};\n"
       "}  // namespace pdd_spec\n";
  return o.str();
}

namespace {

// Loads the instantiation `name` of `src` for the current device: from the
// in-memory table, else from the disk cache, else compiled now.
bool load_spec(const std::string& name, const std::string& src, hipFunction_t* fn, std::string* err) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    *err = "hipGetDevice failed";
    return false;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    *err = "hipGetDeviceProperties failed";
    return false;
  }
  const std::string arch = prop.gcnArchName;
  // the key covers the generated source, the instantiation, the target and
  // the embedded device headers
  std::string key = arch + "\n" + name + "\n" + src;
  for (int i = 0; i < kRtcHeaderCount; ++i) key += std::string("\n") + kRtcHeaderBodies[i];
  std::lock_guard<std::mutex> lk(g_spec_mu);
  const std::string mkey = std::to_string(dev) + "\n" + key;
  auto it = g_spec.find(mkey);
  if (it != g_spec.end()) {
    *fn = it->second;
    return true;
  }
  // disk cache: <hash>.pddjit holds the full key (compared on read), the
  // lowered kernel name and the code object
  const std::string dir = cache_dir();
  char hx[32];
  std::snprintf(hx, sizeof hx, "%016llx", (unsigned long long)fnv1a(key));
  const std::string path = dir.empty() ? "" : dir + "/" + hx + ".pddjit";
  std::string code, lowered;
  const bool have = !path.empty() && read_entry(path, key, &lowered, &code);
  if (!have) {
    if (!spec_compile(src, name, arch, &code, &lowered, err)) return false;
    if (!path.empty()) {
      make_dirs(dir);
      write_entry(path, key, lowered, code);
    }
  }
  hipModule_t mod;
  hipError_t e = hipModuleLoadData(&mod, code.data());
  if (e != hipSuccess && have) {
    // an entry that does not load (written by another runtime version, or
    // damaged in place): compile afresh and replace it
    (void)hipGetLastError();
    if (!spec_compile(src, name, arch, &code, &lowered, err)) return false;
    e = hipModuleLoadData(&mod, code.data());
    if (e == hipSuccess) write_entry(path, key, lowered, code);
  }
  if (e != hipSuccess) {
    *err = std::string("hipModuleLoadData: ") + hipGetErrorString(e);
    return false;
  }
  hipFunction_t f;
  e = hipModuleGetFunction(&f, mod, lowered.c_str());
  if (e != hipSuccess) {
    *err = std::string("hipModuleGetFunction: ") + hipGetErrorString(e);
    return false;
  }
  g_spec[mkey] = f;
  *fn = f;
  return true;
}

}  // namespace

std::string spec_walk_name(bool fp32, int dim, int dfc, int layout, bool adjoint) {
  std::ostringstream nm;
  nm << "pdd::k_walk<" << (fp32 ? "float" : "double") << ", " << dim << ", " << dfc << ", " << layout << ", true, "
     << (adjoint ? "true" : "false") << ", false, pdd_spec::SpecTerms>";
  return nm.str();
}

std::string spec_walk_source(const std::string& terms_src) { return "#include \"walk_kernels.hpp\"\n" + terms_src; }

bool spec_walk_kernel(const std::string& terms_src, bool fp32, int dim, int dfc, int layout, bool adjoint,
                      hipFunction_t* fn, std::string* err) {
  return load_spec(spec_walk_name(fp32, dim, dfc, layout, adjoint), spec_walk_source(terms_src), fn, err);
}

std::string spec_branch_name(bool fp32, int dim, int layout, bool boundary) {
  std::ostringstream nm;
  nm << "pdd::" << (boundary ? "k_branch_bvp<" : "k_branch<") << (fp32 ? "float" : "double") << ", " << dim << ", "
     << layout << ", pdd_spec::SpecPsi>";
  return nm.str();
}

std::string spec_branch_source(const std::string& psi_src) { return "#include \"branch_kernels.hpp\"\n" + psi_src; }

bool spec_branch_kernel(const std::string& psi_src, bool fp32, int dim, int layout, bool boundary,
                        hipFunction_t* fn, std::string* err) {
  return load_spec(spec_branch_name(fp32, dim, layout, boundary), spec_branch_source(psi_src), fn, err);
}

}  // namespace pdd
