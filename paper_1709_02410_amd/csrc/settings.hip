// Run-time settings of librpywall.so read from the environment, and the
// persisted launch-shape cache.
//
//   RPYW_LOG=1                 one line per entry-point call on stderr (name,
//                              sizes, precision, chosen launch shape, status)
//   RPYW_TILE=64|256           source tile of the plain pair kernel, for every
//                              product (overrides tuned and built-in shapes)
//   RPYW_RHS_WIDTH=1|2|4|8|16  right-hand sides per pass (FP64: 16 only on the matrix cores);
//                              widths above 4 use the plain kernel, or in
//                              FP32C the matrix-core kernel where the shape
//                              selects it
//   RPYW_SYM_SPLIT=ns,nseg     how the symmetric kernel with groups of 64
//                              splits the passes of an item: over ns waves
//                              of a workgroup (1 or 4) and nseg workgroups
//                              (1, 2 or 4); by default chosen from the
//                              number of items
//   RPYW_AUTOTUNE_CACHE=path   JSON file of tuned launch shapes, keyed by
//                              (GPU architecture, precision, size class of N
//                              = floor(log2 N), RHS class k); read at the
//                              first shape lookup, rewritten after every
//                              rpy_wall_autotune call (entries of other
//                              architectures are kept)
//
// Values that are not recognised are ignored (and reported when RPYW_LOG is
// set).  The file format is one JSON object:
//   {"version": 1, "entries": [{"arch": "gfx950", "precision": 1,
//     "size_class": 16, "k": 1, "tpl": 1, "tile": 256, "kblk": 1, "sym": 1,
//     "ipw": 2, "mat": 0}, ...]}   ("mat" may be missing: 0)
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "rpyw_internal.h"

namespace rpyw {

namespace {

int env_int(const char* name, int dflt) {
    const char* v = std::getenv(name);
    if (!v || !*v) return dflt;
    char* end = nullptr;
    const long x = std::strtol(v, &end, 10);
    if (end == v || *end) return dflt;
    return (int)x;
}

struct Env {
    bool log;
    int tile;       // 0: no override
    int rhs_width;  // 0: no override
    int sym_ns = 0, sym_nseg = 0;  // 0: no override
    std::string cache;
    Env() {
        log = env_int("RPYW_LOG", 0) != 0;
        const int t = env_int("RPYW_TILE", 0);
        tile = (t == 64 || t == 256) ? t : 0;
        const int w = env_int("RPYW_RHS_WIDTH", 0);
        rhs_width = (w == 1 || w == 2 || w == 4 || w == 8 || w == 16) ? w : 0;
        if (const char* sp = std::getenv("RPYW_SYM_SPLIT")) {
            int a = 0, b = 0;
            char tail = 0;
            if (std::sscanf(sp, "%d,%d%c", &a, &b, &tail) == 2 && (a == 1 || a == 4) &&
                (b == 1 || b == 2 || b == 4)) {
                sym_ns = a;
                sym_nseg = b;
            } else if (log) {
                std::fprintf(stderr, "[rpywall] ignoring RPYW_SYM_SPLIT (ns,nseg with ns 1 or 4, nseg 1, 2 or 4)\n");
            }
        }
        const char* c = std::getenv("RPYW_AUTOTUNE_CACHE");
        cache = c ? c : "";
        if (log) {
            if (std::getenv("RPYW_TILE") && !tile) std::fprintf(stderr, "[rpywall] ignoring RPYW_TILE (64 or 256)\n");
            if (std::getenv("RPYW_RHS_WIDTH") && !rhs_width)
                std::fprintf(stderr, "[rpywall] ignoring RPYW_RHS_WIDTH (1, 2, 4, 8 or 16)\n");
        }
    }
};

const Env& env() {
    static const Env e;
    return e;
}

// Value of an integer field "key": <int> inside one JSON object text.
bool field_int(const std::string& obj, const char* key, int* out) {
    const std::string k = std::string("\"") + key + "\"";
    const size_t p = obj.find(k);
    if (p == std::string::npos) return false;
    size_t q = obj.find(':', p + k.size());
    if (q == std::string::npos) return false;
    const char* s = obj.c_str() + q + 1;
    char* end = nullptr;
    const long v = std::strtol(s, &end, 10);
    if (end == s) return false;
    *out = (int)v;
    return true;
}

bool field_str(const std::string& obj, const char* key, std::string* out) {
    const std::string k = std::string("\"") + key + "\"";
    const size_t p = obj.find(k);
    if (p == std::string::npos) return false;
    const size_t q = obj.find('"', obj.find(':', p + k.size()) + 1);
    if (q == std::string::npos) return false;
    const size_t r = obj.find('"', q + 1);
    if (r == std::string::npos) return false;
    *out = obj.substr(q + 1, r - q - 1);
    return true;
}

}  // namespace

bool log_enabled() { return env().log; }

void log_line(const char* fmt, ...) {
    if (!env().log) return;
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    std::fprintf(stderr, "[rpywall] %s\n", buf);
}

Shape apply_env_overrides(Shape s) {
    const Env& e = env();
    if (e.tile) s.tile = e.tile;
    if (e.rhs_width) s.kblk = e.rhs_width;
    return s;
}

bool sym_split_override(int* ns, int* nseg) {
    if (!env().sym_ns) return false;
    *ns = env().sym_ns;
    *nseg = env().sym_nseg;
    return true;
}

const char* autotune_cache_path() { return env().cache.empty() ? nullptr : env().cache.c_str(); }

std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string a = p.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

int read_shape_cache(const char* path, std::vector<CachedShape>& out) {
    out.clear();
    FILE* f = std::fopen(path, "rb");
    if (!f) return -1;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
    std::fclose(f);
    const size_t ent = text.find("\"entries\"");
    if (ent == std::string::npos) return -1;
    size_t p = text.find('[', ent);
    while (p != std::string::npos) {
        const size_t a = text.find('{', p);
        if (a == std::string::npos) break;
        const size_t b = text.find('}', a);
        if (b == std::string::npos) break;
        const std::string obj = text.substr(a, b - a + 1);
        CachedShape c;
        if (field_str(obj, "arch", &c.arch) && field_int(obj, "precision", &c.prec) &&
            field_int(obj, "size_class", &c.size_class) && field_int(obj, "k", &c.kclass) &&
            field_int(obj, "tpl", &c.s.tpl) && field_int(obj, "tile", &c.s.tile) &&
            field_int(obj, "kblk", &c.s.kblk) && field_int(obj, "sym", &c.s.sym) && field_int(obj, "ipw", &c.s.ipw)) {
            if (!field_int(obj, "mat", &c.s.mat)) c.s.mat = 0;  // entries written before the field existed
            out.push_back(c);
        }
        p = b + 1;
    }
    return 0;
}

int write_shape_cache(const char* path, const std::vector<CachedShape>& entries) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return -1;
    std::fprintf(f, "{\"version\": 1, \"entries\": [");
    for (size_t i = 0; i < entries.size(); ++i) {
        const CachedShape& c = entries[i];
        std::fprintf(f,
                     "%s\n  {\"arch\": \"%s\", \"precision\": %d, \"size_class\": %d, \"k\": %d, \"tpl\": %d, "
                     "\"tile\": %d, \"kblk\": %d, \"sym\": %d, \"ipw\": %d, \"mat\": %d}",
                     i ? "," : "", c.arch.c_str(), c.prec, c.size_class, c.kclass, c.s.tpl, c.s.tile, c.s.kblk,
                     c.s.sym, c.s.ipw, c.s.mat);
    }
    std::fprintf(f, "\n]}\n");
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return -1;
    }
    return 0;
}

}  // namespace rpyw
