// Runtime-compiled user kernels (Sec. 3.5 "Runtime Kernel Compilation").
//
// A user supplies the source of a HIP __device__ function that takes the
// virtual block index as its first argument and its arrays as view types
// (lt::Vector / lt::Matrix / lt::Tensor for 1-, 2- and 3-D arrays), plus the
// parameter list and an annotation.  The runtime generates a __global__
// wrapper around it and compiles the pair with hipRTC for gfx950.
//
// What the wrapper does, per workgroup:
//   - finds its task (superblock) in a table passed by value (up to RTC_MAXG
//     tasks share one dispatch, as in the grouped executor) and turns its
//     position in the task's block box into the virtual block index
//     (the task's first block + the local block; Sec. 3.5 adds an offset to
//     the physical block index in the same way);
//   - builds each array view from a base address that the host has already
//     moved by the region's origin, so the user's code indexes with global
//     array indices and no offset is subtracted per element access;
//   - calls the user's function.
// What is baked into the code as constants (one compiled version per
// combination, cached for the process): the block shape (also the
// __launch_bounds__), every view's element strides, and the values of
// scalar parameters the user marks constant.  Strides depend on where a
// region lives (a chunk, a run of chunks, an assembled temporary); tasks
// whose views have different strides go to different versions.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <cctype>
#include <cinttypes>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.h"
#include "lt_internal.h"

namespace lt {

namespace {

constexpr int RTC_MAXG = 16;  // tasks per dispatch (the argument block stays under 2 KiB)

// Header the user's source is compiled against: the view types.  A view
// holds the byte address of element (0, 0, 0) (which may lie outside the
// memory that backs the region) and element strides; an access is one
// integer multiply-add per axis on top of that address.
const char *kPrelude = R"LT(#pragma once
namespace lt {
template <typename T>
struct Vector {
    long long base, s0;
    __device__ __forceinline__ Vector(long long b, long long a0) : base(b), s0(a0) {}
    __device__ __forceinline__ T &operator[](long long i) const {
        return *reinterpret_cast<T *>(base + (long long)sizeof(T) * (i * s0));
    }
    __device__ __forceinline__ T &operator()(long long i) const { return (*this)[i]; }
};
template <typename T>
struct Row {
    long long base, s1;
    __device__ __forceinline__ T &operator[](long long j) const {
        return *reinterpret_cast<T *>(base + (long long)sizeof(T) * (j * s1));
    }
};
template <typename T>
struct Matrix {
    long long base, s0, s1;
    __device__ __forceinline__ Matrix(long long b, long long a0, long long a1) : base(b), s0(a0), s1(a1) {}
    __device__ __forceinline__ T &operator()(long long i, long long j) const {
        return *reinterpret_cast<T *>(base + (long long)sizeof(T) * (i * s0 + j * s1));
    }
    __device__ __forceinline__ Row<T> operator[](long long i) const {
        return Row<T>{base + (long long)sizeof(T) * (i * s0), s1};
    }
};
template <typename T>
struct Plane {
    long long base, s1, s2;
    __device__ __forceinline__ Row<T> operator[](long long j) const {
        return Row<T>{base + (long long)sizeof(T) * (j * s1), s2};
    }
};
template <typename T>
struct Tensor {
    long long base, s0, s1, s2;
    __device__ __forceinline__ Tensor(long long b, long long a0, long long a1, long long a2)
        : base(b), s0(a0), s1(a1), s2(a2) {}
    __device__ __forceinline__ T &operator()(long long i, long long j, long long k) const {
        return *reinterpret_cast<T *>(base + (long long)sizeof(T) * (i * s0 + j * s1 + k * s2));
    }
    __device__ __forceinline__ Plane<T> operator[](long long i) const {
        return Plane<T>{base + (long long)sizeof(T) * (i * s0), s1, s2};
    }
};
}  // namespace lt
)LT";

const char *ctype_of(lt_dtype d) {
    switch (d) {
        case LT_F32: return "float";
        case LT_I32: return "int";
        case LT_F64: return "double";
        case LT_I64: return "long long";
        case LT_U8: return "unsigned char";
    }
    return nullptr;
}

// One compiled version: the block shape, each array parameter's strides
// and the constant scalars' values.
struct Spec {
    int64_t block[3] = {1, 1, 1};  // x, y, z
    int64_t strides[MAXPARAM][3] = {};
    int64_t ival[MAXPARAM] = {};
    double fval[MAXPARAM] = {};

    std::string key(const RtcKernel &K) const {
        std::string k = K.source_key;
        char buf[96];
        snprintf(buf, sizeof buf, "|b%lld,%lld,%lld", (long long)block[0], (long long)block[1],
                 (long long)block[2]);
        k += buf;
        for (int p = 0; p < K.def.nparam; ++p) {
            const ParamDef &pd = K.def.params[p];
            if (pd.kind == P_ARRAY) {
                snprintf(buf, sizeof buf, "|s%lld,%lld,%lld", (long long)strides[p][0], (long long)strides[p][1],
                         (long long)strides[p][2]);
                k += buf;
            } else if (K.is_const[p]) {
                if (pd.kind == P_INT) snprintf(buf, sizeof buf, "|i%lld", (long long)ival[p]);
                else {
                    long long bits;
                    memcpy(&bits, &fval[p], sizeof bits);
                    snprintf(buf, sizeof buf, "|f%llx", (unsigned long long)bits);
                }
                k += buf;
            }
        }
        return k;
    }
};

uint64_t fnv1a(const std::string &s) {
    uint64_t h = 1469598103934665603ull;
    for (unsigned char c : s) {
        h ^= c;
        h *= 1099511628211ull;
    }
    return h;
}

// The generated translation unit: prelude, the user's source, the wrapper.
std::string wrapper_source(const RtcKernel &K, const Spec &sp, const std::string &sym) {
    const KernelDef &d = K.def;
    const int np = d.nparam;
    int narr = 0;
    for (int p = 0; p < np; ++p) narr += d.params[p].kind == P_ARRAY;
    std::string s = "#include \"lt_rtc.h\"\n#line 1 \"" + K.function + ".hip\"\n" + K.source + "\n";
    char buf[4096];
    snprintf(buf, sizeof buf,
             "namespace %s_ns {\n"
             "struct Task { long long b[3]; long long nb[3]; long long base[%d]; };\n"
             "struct Args { long long ntask; long long begin[%d]; Task t[%d]; long long iarg[%d]; "
             "double farg[%d]; };\n"
             "}\n",
             sym.c_str(), narr > 0 ? narr : 1, RTC_MAXG + 1, RTC_MAXG, np > 0 ? np : 1, np > 0 ? np : 1);
    s += buf;
    const long long nthreads = (long long)(sp.block[0] * sp.block[1] * sp.block[2]);
    snprintf(buf, sizeof buf,
             "extern \"C\" __global__ __launch_bounds__(%lld) void %s(%s_ns::Args a) {\n"
             "    const long long bid = blockIdx.x;\n"
             "    int k = 0;\n"
             "    while (k + 1 < a.ntask && bid >= a.begin[k + 1]) ++k;\n"
             "    const %s_ns::Task &t = a.t[k];\n"
             "    long long l = bid - a.begin[k];\n"
             "    const long long lx = l %% t.nb[0];\n"
             "    l /= t.nb[0];\n"
             "    const long long ly = l %% t.nb[1];\n"
             "    const long long lz = l / t.nb[1];\n"
             "    const dim3 vb((unsigned)(t.b[0] + lx), (unsigned)(t.b[1] + ly), (unsigned)(t.b[2] + lz));\n",
             nthreads, sym.c_str(), sym.c_str(), sym.c_str());
    s += buf;
    std::string call = "    " + K.function + "(vb";
    int a = 0;
    for (int p = 0; p < np; ++p) {
        const ParamDef &pd = d.params[p];
        char arg[64];
        if (pd.kind == P_ARRAY) {
            const char *ty = ctype_of(pd.dtype);
            const int64_t *st = sp.strides[p];
            if (pd.ndim == 1)
                snprintf(buf, sizeof buf, "    const lt::Vector<%s> v%d(t.base[%d], %lldLL);\n", ty, p, a,
                         (long long)st[0]);
            else if (pd.ndim == 2)
                snprintf(buf, sizeof buf, "    const lt::Matrix<%s> v%d(t.base[%d], %lldLL, %lldLL);\n", ty, p, a,
                         (long long)st[0], (long long)st[1]);
            else
                snprintf(buf, sizeof buf, "    const lt::Tensor<%s> v%d(t.base[%d], %lldLL, %lldLL, %lldLL);\n", ty,
                         p, a, (long long)st[0], (long long)st[1], (long long)st[2]);
            s += buf;
            snprintf(arg, sizeof arg, ", v%d", p);
            ++a;
        } else if (pd.kind == P_INT) {
            if (K.is_const[p]) snprintf(arg, sizeof arg, ", (long long)%lldLL", (long long)sp.ival[p]);
            else snprintf(arg, sizeof arg, ", a.iarg[%d]", p);
        } else {
            if (K.is_const[p]) {
                // the exact bits, whatever the value (NaN and infinities included)
                long long bits;
                memcpy(&bits, &sp.fval[p], sizeof bits);
                snprintf(arg, sizeof arg, ", __longlong_as_double(%lldLL)", bits);
            }
            else snprintf(arg, sizeof arg, ", a.farg[%d]", p);
        }
        call += arg;
    }
    s += call + ");\n}\n";
    return s;
}

const char *kOptions[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};

// hipRTC compile; on failure *log holds the compiler's messages.
bool rtc_compile(const std::string &src, const std::string &name, std::vector<char> *code, std::string *log) {
    // LT_RTC_DUMP=1: every generated translation unit goes to stderr
    static const bool dump = getenv("LT_RTC_DUMP") && atoi(getenv("LT_RTC_DUMP")) != 0;
    if (dump) fprintf(stderr, "---- %s (generated)\n%s---- end\n", name.c_str(), src.c_str());
    hiprtcProgram prog;
    const char *hname = "lt_rtc.h";
    hiprtcResult r = hiprtcCreateProgram(&prog, src.c_str(), (name + ".hip").c_str(), 1, &kPrelude, &hname);
    if (r != HIPRTC_SUCCESS) {
        *log = std::string("hiprtcCreateProgram: ") + hiprtcGetErrorString(r);
        return false;
    }
    r = hiprtcCompileProgram(prog, (int)(sizeof kOptions / sizeof kOptions[0]), kOptions);
    size_t ls = 0;
    hiprtcGetProgramLogSize(prog, &ls);
    std::string lg(ls, '\0');
    if (ls) hiprtcGetProgramLog(prog, &lg[0]);
    while (!lg.empty() && (lg.back() == '\0' || lg.back() == '\n')) lg.pop_back();
    if (r != HIPRTC_SUCCESS) {
        *log = std::string(hiprtcGetErrorString(r)) + (lg.empty() ? "" : ":\n" + lg);
        hiprtcDestroyProgram(&prog);
        return false;
    }
    size_t cs = 0;
    hiprtcGetCodeSize(prog, &cs);
    code->resize(cs);
    if (cs) hiprtcGetCode(prog, code->data());
    hiprtcDestroyProgram(&prog);
    return cs > 0;
}

// Process-wide caches: code objects by specialisation key, loaded functions
// by (key, device).  Modules stay loaded until the process ends.
struct Cache {
    std::mutex mu;
    std::map<std::string, std::vector<char>> code;
    std::map<std::pair<std::string, int>, hipFunction_t> fn;
    uint64_t compiles = 0, loads = 0;
    double compile_s = 0;
};
Cache &cache() {
    static Cache c;
    return c;
}

double mono_s() {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

bool get_function(RtcKernel &K, const Spec &sp, hipFunction_t *out) {
    const std::string key = sp.key(K);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        K.last_error = "hipGetDevice failed";
        return false;
    }
    Cache &C = cache();
    std::lock_guard<std::mutex> lock(C.mu);
    auto fit = C.fn.find({key, dev});
    if (fit != C.fn.end()) {
        *out = fit->second;
        return true;
    }
    char sym[64];
    snprintf(sym, sizeof sym, "lt_rtc_%016" PRIx64, fnv1a(key));
    auto cit = C.code.find(key);
    if (cit == C.code.end()) {
        std::vector<char> code;
        std::string log;
        double t0 = mono_s();
        if (!rtc_compile(wrapper_source(K, sp, sym), K.function, &code, &log)) {
            K.last_error = "runtime compilation of " + K.function + " failed: " + log;
            return false;
        }
        C.compile_s += mono_s() - t0;
        C.compiles++;
        cit = C.code.emplace(key, std::move(code)).first;
    }
    hipModule_t mod;
    hipError_t r = hipModuleLoadData(&mod, cit->second.data());
    if (r != hipSuccess) {
        K.last_error = std::string("hipModuleLoadData: ") + hipGetErrorString(r);
        return false;
    }
    hipFunction_t f;
    r = hipModuleGetFunction(&f, mod, sym);
    if (r != hipSuccess) {
        K.last_error = std::string("hipModuleGetFunction: ") + hipGetErrorString(r);
        return false;
    }
    C.loads++;
    C.fn[{key, dev}] = f;
    *out = f;
    return true;
}

}  // namespace

// Host launcher of every user kernel: tasks with equal view strides share a
// dispatch (up to RTC_MAXG), one compiled version per stride combination.
hipError_t launch_rtc(const KLaunch &L) {
    RtcKernel &K = *static_cast<RtcKernel *>(const_cast<void *>(L.user));
    const KernelDef &d = K.def;
    const int nd = L.ndim;
    Spec sp;
    // logical axis a (0 = slowest) runs along hardware axis nd-1-a (x fastest)
    for (int a = 0; a < nd; ++a) sp.block[nd - 1 - a] = L.block[a];
    for (int p = 0; p < d.nparam; ++p) {
        sp.ival[p] = L.iarg[p];
        sp.fval[p] = L.farg[p];
    }
    const int np = d.nparam;
    int narr = 0;
    for (int p = 0; p < np; ++p) narr += d.params[p].kind == P_ARRAY;
    const int nb = narr > 0 ? narr : 1, npa = np > 0 ? np : 1;
    // argument block, laid out as the generated Args struct (all 8-byte words)
    const size_t task_words = 6 + (size_t)nb;
    std::vector<int64_t> buf(1 + (RTC_MAXG + 1) + RTC_MAXG * task_words + 2 * (size_t)npa, 0);
    int i = 0;
    while (i < L.ntask) {
        // strides of this task's views
        for (int p = 0; p < np; ++p)
            if (d.params[p].kind == P_ARRAY)
                for (int a = 0; a < 3; ++a) sp.strides[p][a] = a < d.params[p].ndim ? L.tasks[i].v[p].s[a] : 0;
        // the run of following tasks with the same strides
        int j = i + 1;
        for (; j < L.ntask && j - i < RTC_MAXG; ++j) {
            bool same = true;
            for (int p = 0; p < np && same; ++p)
                if (d.params[p].kind == P_ARRAY)
                    for (int a = 0; a < d.params[p].ndim; ++a) same = same && L.tasks[j].v[p].s[a] == sp.strides[p][a];
            if (!same) break;
        }
        hipFunction_t fn;
        if (!get_function(K, sp, &fn)) return hipErrorInvalidImage;
        std::fill(buf.begin(), buf.end(), 0);
        int64_t *ntask = &buf[0];
        int64_t *begin = &buf[1];
        int64_t *tasks = &buf[1 + RTC_MAXG + 1];
        int64_t *iarg = tasks + RTC_MAXG * task_words;
        double *farg = reinterpret_cast<double *>(iarg + npa);
        int64_t total = 0;
        *ntask = j - i;
        for (int t = i; t < j; ++t) {
            int64_t *T = tasks + (size_t)(t - i) * task_words;
            int64_t cnt = 1;
            for (int a = 0; a < 3; ++a) {
                T[a] = 0;
                T[3 + a] = 1;
            }
            for (int a = 0; a < nd; ++a) {
                const int hw = nd - 1 - a;
                const int64_t lo = L.tasks[t].lo[a], hi = L.tasks[t].hi[a];
                T[hw] = lo / L.block[a];
                T[3 + hw] = (hi - lo) / L.block[a];
                cnt *= T[3 + hw];
            }
            int q = 0;
            for (int p = 0; p < np; ++p)
                if (d.params[p].kind == P_ARRAY) T[6 + q++] = L.tasks[t].v[p].base;
            begin[t - i] = total;
            total += cnt;
        }
        begin[j - i] = total;
        for (int t = j - i + 1; t <= RTC_MAXG; ++t) begin[t] = total;
        for (int p = 0; p < np; ++p) {
            iarg[p] = L.iarg[p];
            farg[p] = L.farg[p];
        }
        if (total > 0) {
            if (total > 0x7fffffffLL) {
                K.last_error = "a dispatch of " + K.function + " needs more than 2^31 - 1 workgroups";
                return hipErrorInvalidConfiguration;
            }
            size_t bytes = buf.size() * sizeof(int64_t);
            void *config[] = {HIP_LAUNCH_PARAM_BUFFER_POINTER, buf.data(), HIP_LAUNCH_PARAM_BUFFER_SIZE, &bytes,
                              HIP_LAUNCH_PARAM_END};
            hipError_t r = hipModuleLaunchKernel(fn, (unsigned)total, 1, 1, (unsigned)sp.block[0],
                                                 (unsigned)sp.block[1], (unsigned)sp.block[2], 0, L.stream,
                                                 nullptr, config);
            if (r != hipSuccess) {
                K.last_error = std::string("hipModuleLaunchKernel: ") + hipGetErrorString(r);
                return r;
            }
        }
        i = j;
    }
    return hipSuccess;
}

static bool ident(const char *s) {
    if (!s || !*s || !(isalpha((unsigned char)*s) || *s == '_')) return false;
    for (const char *c = s; *c; ++c)
        if (!(isalnum((unsigned char)*c) || *c == '_')) return false;
    return true;
}

// Validates the parameter list, parses the annotation against it and
// compiles one version (block 64 along x, unit strides) so that errors in
// the source surface here, with the compiler's log.
lt_status rtc_define(Ctx *ctx, const char *source, const char *function, const lt_param *params, int32_t nparams,
                     const char *annotation, lt_kernel **out) {
    if (!out) return LT_ERR_INVALID;
    *out = nullptr;
    if (!source || !function || !annotation) return set_err(ctx, LT_ERR_INVALID, "source, function and annotation are required");
    if (!ident(function)) return set_err(ctx, LT_ERR_INVALID, "'%s' is not a function name", function);
    if (nparams < 0 || nparams > MAXPARAM || nparams > KMAXP || (nparams > 0 && !params))
        return set_err(ctx, LT_ERR_INVALID, "a user kernel takes 0..%d parameters", MAXPARAM);
    auto K = std::make_unique<RtcKernel>();
    K->source = source;
    K->function = function;
    K->names.resize((size_t)nparams);
    int narr = 0;
    for (int p = 0; p < nparams; ++p) {
        const lt_param &q = params[p];
        if (!ident(q.name)) return set_err(ctx, LT_ERR_INVALID, "parameter %d has no valid name", p);
        for (int r = 0; r < p; ++r)
            if (!strcmp(q.name, params[r].name)) return set_err(ctx, LT_ERR_INVALID, "parameter '%s' given twice", q.name);
        K->names[p] = q.name;
        ParamDef &pd = K->def.params[p];
        pd.name = nullptr;  // set below, once names no longer moves
        pd.dtype = LT_F32;
        pd.ndim = 0;
        if (q.kind == LT_ARG_ARRAY) {
            if (!ctype_of((lt_dtype)q.dtype))
                return set_err(ctx, LT_ERR_INVALID, "parameter '%s': unknown dtype %d", q.name, q.dtype);
            if (q.ndim < 1 || q.ndim > 3)
                return set_err(ctx, LT_ERR_INVALID, "parameter '%s': arrays have 1..3 dimensions", q.name);
            if (q.flags & LT_PARAM_CONST)
                return set_err(ctx, LT_ERR_INVALID, "parameter '%s': only scalars can be constant", q.name);
            pd.kind = P_ARRAY;
            pd.dtype = (lt_dtype)q.dtype;
            pd.ndim = q.ndim;
            ++narr;
        } else if (q.kind == LT_ARG_INT) {
            pd.kind = P_INT;
        } else if (q.kind == LT_ARG_FLOAT) {
            pd.kind = P_FLOAT;
        } else {
            return set_err(ctx, LT_ERR_INVALID, "parameter '%s': unknown kind %d", q.name, q.kind);
        }
        K->is_const[p] = (q.flags & LT_PARAM_CONST) != 0;
    }
    for (int p = 0; p < nparams; ++p) K->def.params[p].name = K->names[p].c_str();
    K->def.name = K->function.c_str();
    K->def.annotation = nullptr;
    K->def.nparam = nparams;
    K->def.fn = launch_rtc;
    K->def.max_group = RTC_MAXG;
    K->def.dkind = -1;
    K->def.slots = nullptr;
    K->def.user = K.get();
    char head[160];
    snprintf(head, sizeof head, "%016" PRIx64 ":%s:", fnv1a(K->source), function);
    K->source_key = head;
    for (int p = 0; p < nparams; ++p) {
        char b[64];
        snprintf(b, sizeof b, "%d.%d.%d.%d,", params[p].kind, params[p].dtype, params[p].ndim, K->is_const[p] ? 1 : 0);
        K->source_key += b;
    }
    // annotation: the grid rank is the number of names it binds
    auto k = std::make_unique<lt_kernel>();
    k->def = &K->def;
    K->def.grid_ndim = 1;
    lt_status st = compile_annotation(ctx, &K->def, annotation, &k->annot);
    if (st) return st;
    int nd = -1;
    for (int kd = 0; kd < 3; ++kd)
        if (k->annot->nbound[kd] > 0) nd = nd < 0 ? k->annot->nbound[kd] : nd;
    if (nd < 1 || nd > 3) return set_err(ctx, LT_ERR_PARSE, "the annotation must bind 1..3 index names");
    K->def.grid_ndim = nd;
    // check build: the source compiles against the view types and the call
    Spec sp;
    sp.block[0] = 64;
    for (int p = 0; p < nparams; ++p)
        for (int a = 0; a < 3; ++a) sp.strides[p][a] = 1;
    std::vector<char> code;
    std::string log;
    char sym[64];
    snprintf(sym, sizeof sym, "lt_rtc_check_%016" PRIx64, fnv1a(sp.key(*K)));
    double t0 = mono_s();
    if (!rtc_compile(wrapper_source(*K, sp, sym), K->function, &code, &log))
        return set_err(ctx, LT_ERR_COMPILE, "%s: %s", function, log.c_str());
    {
        Cache &C = cache();
        std::lock_guard<std::mutex> lock(C.mu);
        C.compile_s += mono_s() - t0;
        C.compiles++;
    }
    *out = k.get();
    ctx->kernels.push_back(std::move(k));
    ctx->rtc_kernels.push_back(std::move(K));
    return LT_OK;
}

const char *rtc_last_error(const KernelDef *def) {
    if (!def || !def->user) return nullptr;
    const RtcKernel *K = static_cast<const RtcKernel *>(def->user);
    return K->last_error.empty() ? nullptr : K->last_error.c_str();
}

void rtc_counters(uint64_t *compiles, uint64_t *loads, double *compile_s) {
    Cache &C = cache();
    std::lock_guard<std::mutex> lock(C.mu);
    *compiles = C.compiles;
    *loads = C.loads;
    *compile_s = C.compile_s;
}

}  // namespace lt
