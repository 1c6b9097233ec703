// Tile shapes of the Cholesky factorisation, per matrix order and factor
// class, from the cache the autotuner writes (paper_2203_11733_amd/autotune.py
// times every candidate on the GPU and keeps the fastest per order bucket).
// The shapes change the schedule only, never the arithmetic of an entry:
//   outer_width   columns per outer panel (256 or 512; the matrix order is a
//                 multiple of 512, so both divide it)
//   super_panels  outer panels per trailing update of the 16-bit factors
//                 (1, 2 or 4, K = super_panels * outer_width <= 2048; 1: the
//                 trailing matrix is updated after every panel)
// Cache format (JSON, written by the autotuner): {"entries": [{"factor":
// "16bit" | "f32" | "f64", "npad_min": a, "npad_max": b, "outer_width": w,
// "super_panels": p, ...}, ...], ...}; an entry applies to padded orders
// a <= npad < b.  Without a cache (or outside every entry) the built-in
// defaults below apply.
#include <dlfcn.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "gbem_internal.h"

namespace gbem {

namespace {
struct Entry {
    int cls;   // 0: 16-bit trailing updates, 1: FP32, 2: FP64
    int64_t lo, hi;
    CholShape shape;
};
std::mutex g_mu;
std::vector<Entry> g_table;
CholShape g_override{0, 0};
bool g_autoloaded = false;
std::string g_source = "built-in defaults";

int class_of(int dtype) { return dtype == GBEM_F64 ? 2 : (dtype == GBEM_F32 ? 1 : 0); }

// Built-in shapes (measured on the MI355X in mixed and FP64 mode):
// 512-wide panels from order 16,384 (the look-ahead chain dominates below);
// 4 panels per 16-bit super-panel from order 32,768.
CholShape defaults(int cls, int64_t npad)
{
    CholShape s;
    s.outer_width = npad >= 16384 ? 512 : 256;
    s.super_panels = cls == 0 ? (npad >= 32768 ? 4 : 2) : 1;
    return s;
}

// value after "key": in [p, end): integer or quoted string
bool find_key(const char *p, const char *end, const char *key, const char **val)
{
    const size_t kl = strlen(key);
    for (const char *q = p; q + kl + 2 < end; ++q) {
        if (q[0] == '"' && strncmp(q + 1, key, kl) == 0 && q[kl + 1] == '"') {
            const char *r = q + kl + 2;
            while (r < end && (*r == ' ' || *r == ':' || *r == '\t' || *r == '\n')) ++r;
            *val = r;
            return r < end;
        }
    }
    return false;
}

bool parse(const std::string &text, std::vector<Entry> &out, std::string &why)
{
    const char *s = text.c_str(), *end = s + text.size();
    const char *e = strstr(s, "\"entries\"");
    if (!e) {
        why = "no \"entries\" array";
        return false;
    }
    const char *p = strchr(e, '[');
    if (!p) {
        why = "\"entries\" is not an array";
        return false;
    }
    ++p;
    for (;;) {
        while (p < end && *p != '{' && *p != ']') ++p;
        if (p >= end || *p == ']') break;
        // the object: up to its matching brace (entries hold flat objects and
        // one nested object of timings)
        int depth = 0;
        const char *q = p;
        for (; q < end; ++q) {
            if (*q == '{') ++depth;
            if (*q == '}' && --depth == 0) break;
        }
        if (q >= end) {
            why = "unterminated entry";
            return false;
        }
        const char *v;
        Entry en{};
        if (!find_key(p, q, "factor", &v) || *v != '"') {
            why = "entry without \"factor\"";
            return false;
        }
        if (strncmp(v, "\"16bit\"", 7) == 0) en.cls = 0;
        else if (strncmp(v, "\"f32\"", 5) == 0) en.cls = 1;
        else if (strncmp(v, "\"f64\"", 5) == 0) en.cls = 2;
        else {
            why = "unknown \"factor\"";
            return false;
        }
        long long a, b, w, sp = 1;
        if (!find_key(p, q, "npad_min", &v) || sscanf(v, "%lld", &a) != 1 || !find_key(p, q, "npad_max", &v) ||
            sscanf(v, "%lld", &b) != 1 || !find_key(p, q, "outer_width", &v) || sscanf(v, "%lld", &w) != 1) {
            why = "entry without npad_min / npad_max / outer_width";
            return false;
        }
        if (find_key(p, q, "super_panels", &v) && sscanf(v, "%lld", &sp) != 1) sp = 1;
        if ((w != 256 && w != 512) || a < 0 || b <= a || (en.cls == 0 && sp != 1 && sp != 2 && sp != 4)) {
            why = "entry outside the supported shapes (outer_width 256 | 512, super_panels 1 | 2 | 4)";
            return false;
        }
        en.lo = a;
        en.hi = b;
        en.shape.outer_width = (int)w;
        en.shape.super_panels = en.cls == 0 ? (int)sp : 1;
        out.push_back(en);
        p = q + 1;
    }
    return true;
}

std::string default_path()
{
    Dl_info info;
    if (dladdr((const void *)&default_path, &info) && info.dli_fname) {
        std::string so = info.dli_fname;
        const size_t slash = so.rfind('/');
        return (slash == std::string::npos ? std::string(".") : so.substr(0, slash)) + "/tune_gfx950.json";
    }
    return "tune_gfx950.json";
}

gbem_status load_locked(const std::string &path, bool quiet_missing)
{
    FILE *f = fopen(path.c_str(), "rb");
    if (!f) {
        if (quiet_missing) return GBEM_OK;
        set_error("gbem_load_tuning: cannot open " + path);
        return GBEM_EINVAL;
    }
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
    fclose(f);
    std::vector<Entry> t;
    std::string why;
    if (!parse(text, t, why)) {
        set_error("gbem_load_tuning: " + path + ": " + why);
        return GBEM_EINVAL;
    }
    g_table.swap(t);
    g_source = path;
    return GBEM_OK;
}
}  // namespace

void tuning_autoload()
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_autoloaded) return;
    g_autoloaded = true;
    const char *env = getenv("GBEM_TUNE_FILE");
    (void)load_locked(env ? std::string(env) : default_path(), true);
}

CholShape chol_shape(int dtype, int64_t npad)
{
    const int cls = class_of(dtype);
    std::lock_guard<std::mutex> lk(g_mu);
    CholShape s = defaults(cls, npad);
    for (const Entry &e : g_table)
        if (e.cls == cls && npad >= e.lo && npad < e.hi) {
            s = e.shape;
            break;
        }
    if (g_override.outer_width) s.outer_width = g_override.outer_width;
    if (cls == 0 && g_override.super_panels) s.super_panels = g_override.super_panels;
    return s;
}

}  // namespace gbem

using namespace gbem;

extern "C" gbem_status gbem_load_tuning(const char *path)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_autoloaded = true;
    if (!path) {
        g_table.clear();
        g_source = "built-in defaults";
        return GBEM_OK;
    }
    return load_locked(path, false);
}

extern "C" gbem_status gbem_set_tuning_override(const gbem_tuning *t)
{
    if (t && ((t->outer_width != 0 && t->outer_width != 256 && t->outer_width != 512) ||
              (t->super_panels != 0 && t->super_panels != 1 && t->super_panels != 2 && t->super_panels != 4))) {
        set_error("gbem_set_tuning_override: outer_width must be 0, 256 or 512 and super_panels 0, 1, 2 or 4");
        return GBEM_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_override.outer_width = t ? t->outer_width : 0;
    g_override.super_panels = t ? t->super_panels : 0;
    return GBEM_OK;
}

extern "C" const char *gbem_tuning_source(void)
{
    static thread_local std::string s;
    std::lock_guard<std::mutex> lk(g_mu);
    s = g_source;
    return s.c_str();
}
