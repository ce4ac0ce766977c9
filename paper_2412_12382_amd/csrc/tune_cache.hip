// Autotune cache: the context's tuned launch parameters persisted in a JSON
// text file, one entry per (device architecture, graph size bucket, tuning
// version).  Host code only.
//
// File format (written by mcd_tune_cache_store, read by mcd_tune_cache_load):
//   {"format": "mcd-tune-cache", "version": 1, "entries": [
//     {"arch": "gfx950:sramecc+:xnack-", "tune_version": 2, "log2_n": 26,
//      "log2_m": 29, "ms": 300.5, "params": {"tc_chunk": 512, ...}}, ...]}
// The size bucket is (floor(log2 n), floor(log2 m)); tune_version changes
// whenever the kernels a parameter steers change, so that entries tuned for
// older kernels are not used.
#include <hip/hip_runtime.h>

#include <cctype>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "common.hpp"

// The library is built with hidden visibility; the C ABI is exported.
#pragma GCC visibility push(default)
#include "mcd.h"
#pragma GCC visibility pop

namespace {

constexpr int kTuneVersion = 2;
const char* const kParams[] = {"tc_chunk",        "tc_lds_max",          "tc_packed_range",
                               "tc_window_max",   "tc_window_occupancy", "sweep_shape"};
constexpr int kNumParams = 6;

// --------------------------------------------------------------- a JSON subset
// Values: objects, arrays, strings (escapes \" \\ \/ only), numbers, true,
// false, null.  Enough for the cache's own files; anything else is an error.
struct Json {
    enum Kind { NUL, BOOL, NUM, STR, ARR, OBJ } kind = NUL;
    double num = 0;
    bool b = false;
    std::string str;
    std::vector<Json> arr;
    std::vector<std::pair<std::string, Json>> obj;
    const Json* get(const char* key) const {
        for (const auto& kv : obj)
            if (kv.first == key) return &kv.second;
        return nullptr;
    }
};

struct Parser {
    const char* p;
    const char* end;
    int depth = 0;
    void ws() {
        while (p < end && std::isspace((unsigned char)*p)) ++p;
    }
    bool lit(const char* s) {
        const size_t n = std::strlen(s);
        if ((size_t)(end - p) < n || std::strncmp(p, s, n) != 0) return false;
        p += n;
        return true;
    }
    bool string(std::string& out) {
        if (p >= end || *p != '"') return false;
        ++p;
        while (p < end && *p != '"') {
            if (*p == '\\') {
                if (++p >= end || (*p != '"' && *p != '\\' && *p != '/')) return false;
            } else if ((unsigned char)*p < 0x20) {
                return false;
            }
            out.push_back(*p++);
        }
        if (p >= end) return false;
        ++p;
        return true;
    }
    bool value(Json& v) {
        if (++depth > 16) return false;
        ws();
        if (p >= end) return false;
        bool ok = true;
        if (*p == '{') {
            v.kind = Json::OBJ;
            ++p;
            ws();
            if (p < end && *p == '}') {
                ++p;
            } else {
                for (;;) {
                    ws();
                    std::string k;
                    Json x;
                    if (!string(k)) return false;
                    ws();
                    if (p >= end || *p != ':') return false;
                    ++p;
                    if (!value(x)) return false;
                    v.obj.emplace_back(std::move(k), std::move(x));
                    ws();
                    if (p < end && *p == ',') { ++p; continue; }
                    if (p < end && *p == '}') { ++p; break; }
                    return false;
                }
            }
        } else if (*p == '[') {
            v.kind = Json::ARR;
            ++p;
            ws();
            if (p < end && *p == ']') {
                ++p;
            } else {
                for (;;) {
                    Json x;
                    if (!value(x)) return false;
                    v.arr.push_back(std::move(x));
                    ws();
                    if (p < end && *p == ',') { ++p; continue; }
                    if (p < end && *p == ']') { ++p; break; }
                    return false;
                }
            }
        } else if (*p == '"') {
            v.kind = Json::STR;
            ok = string(v.str);
        } else if (lit("true")) {
            v.kind = Json::BOOL;
            v.b = true;
        } else if (lit("false")) {
            v.kind = Json::BOOL;
        } else if (lit("null")) {
            v.kind = Json::NUL;
        } else {
            // a number: strtod on a bounded copy (the buffer is not terminated)
            const char* q = p;
            while (q < end && (std::isdigit((unsigned char)*q) || *q == '-' || *q == '+' || *q == '.' ||
                               *q == 'e' || *q == 'E'))
                ++q;
            if (q == p || q - p > 40) return false;
            char buf[48];
            std::memcpy(buf, p, (size_t)(q - p));
            buf[q - p] = 0;
            char* e = nullptr;
            v.kind = Json::NUM;
            v.num = std::strtod(buf, &e);
            ok = e == buf + (q - p) && std::isfinite(v.num);
            p = q;
        }
        --depth;
        return ok;
    }
};

// Reads the file; a missing file is an empty cache (*exists = false).
mcd_status read_cache(const char* path, Json& root, bool* exists) {
    *exists = false;
    FILE* f = std::fopen(path, "rb");
    if (!f) return errno == ENOENT ? MCD_OK : MCD_ERR_CHECKPOINT;
    std::string text;
    char buf[65536];
    size_t k;
    while ((k = std::fread(buf, 1, sizeof buf, f)) > 0) {
        text.append(buf, k);
        if (text.size() > (64u << 20)) break;
    }
    const bool bad = std::ferror(f) != 0 || text.size() > (64u << 20);
    std::fclose(f);
    if (bad) return MCD_ERR_CHECKPOINT;
    *exists = true;
    Parser ps{text.data(), text.data() + text.size()};
    if (!ps.value(root)) return MCD_ERR_CHECKPOINT;
    ps.ws();
    if (ps.p != ps.end || root.kind != Json::OBJ) return MCD_ERR_CHECKPOINT;
    const Json* fmt = root.get("format");
    const Json* ver = root.get("version");
    const Json* ent = root.get("entries");
    if (!fmt || fmt->kind != Json::STR || fmt->str != "mcd-tune-cache" || !ver || ver->kind != Json::NUM ||
        ver->num != 1 || !ent || ent->kind != Json::ARR)
        return MCD_ERR_CHECKPOINT;
    return MCD_OK;
}

struct Key {
    std::string arch;
    int log2_n, log2_m;
};

int floor_log2(int64_t x) {
    int r = 0;
    while (x > 1) {
        x >>= 1;
        ++r;
    }
    return r;
}

mcd_status key_of(const mcd_graph* g, Key& k) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, g->ctx->device) != hipSuccess) return MCD_ERR_DEVICE;
    k.arch = prop.gcnArchName;
    k.log2_n = floor_log2(g->n);
    k.log2_m = floor_log2(g->m);
    return MCD_OK;
}

bool same_key(const Json& e, const Key& k) {
    const Json* a = e.get("arch");
    const Json* v = e.get("tune_version");
    const Json* ln = e.get("log2_n");
    const Json* lm = e.get("log2_m");
    return a && a->kind == Json::STR && a->str == k.arch && v && v->kind == Json::NUM && v->num == kTuneVersion &&
           ln && ln->kind == Json::NUM && ln->num == k.log2_n && lm && lm->kind == Json::NUM && lm->num == k.log2_m;
}

void escape_into(std::string& out, const std::string& s) {
    for (char c : s) {
        if (c == '"' || c == '\\') out.push_back('\\');
        out.push_back(c);
    }
}

}  // namespace

#pragma GCC visibility push(default)
extern "C" {

mcd_status mcd_tune_cache_load(mcd_ctx* ctx, const mcd_graph* g, const char* path, int32_t* hit) {
    if (!ctx || !g || !path || !hit || g->ctx != ctx) return MCD_ERR_INVALID_ARG;
    *hit = 0;
    Key k;
    mcd_status st = key_of(g, k);
    if (st != MCD_OK) return st;
    Json root;
    bool exists = false;
    if ((st = read_cache(path, root, &exists)) != MCD_OK || !exists) return st;
    for (const Json& e : root.get("entries")->arr) {
        if (e.kind != Json::OBJ || !same_key(e, k)) continue;
        const Json* prm = e.get("params");
        if (!prm || prm->kind != Json::OBJ) return MCD_ERR_CHECKPOINT;
        int64_t val[kNumParams];
        for (int i = 0; i < kNumParams; ++i) {
            const Json* x = prm->get(kParams[i]);
            if (!x || x->kind != Json::NUM || x->num != std::floor(x->num) || std::fabs(x->num) > 9.0e15)
                return MCD_ERR_CHECKPOINT;
            val[i] = (int64_t)x->num;
        }
        // every value through the context's own checks; the context is
        // changed only when all of them pass
        mcd_ctx probe = *ctx;
        for (int i = 0; i < kNumParams; ++i)
            if (mcd_ctx_set_param(&probe, kParams[i], val[i]) != MCD_OK) return MCD_ERR_CHECKPOINT;
        for (int i = 0; i < kNumParams; ++i) (void)mcd_ctx_set_param(ctx, kParams[i], val[i]);
        *hit = 1;
        return MCD_OK;
    }
    return MCD_OK;
}

mcd_status mcd_tune_cache_store(const mcd_ctx* ctx, const mcd_graph* g, const char* path, float ms) {
    if (!ctx || !g || !path || g->ctx != ctx || !std::isfinite(ms)) return MCD_ERR_INVALID_ARG;
    Key k;
    mcd_status st = key_of(g, k);
    if (st != MCD_OK) return st;
    Json root;
    bool exists = false;
    if ((st = read_cache(path, root, &exists)) != MCD_OK) return st;
    std::string out = "{\"format\": \"mcd-tune-cache\", \"version\": 1, \"entries\": [\n";
    bool first = true;
    char line[512];
    // earlier entries of other keys, re-written as read
    if (exists) {
        for (const Json& e : root.get("entries")->arr) {
            if (e.kind != Json::OBJ || same_key(e, k)) continue;
            const Json* a = e.get("arch");
            const Json* v = e.get("tune_version");
            const Json* ln = e.get("log2_n");
            const Json* lm = e.get("log2_m");
            const Json* t = e.get("ms");
            const Json* prm = e.get("params");
            if (!a || a->kind != Json::STR || !v || v->kind != Json::NUM || !ln || ln->kind != Json::NUM || !lm ||
                lm->kind != Json::NUM || !t || t->kind != Json::NUM || !prm || prm->kind != Json::OBJ)
                return MCD_ERR_CHECKPOINT;
            std::string s = first ? "  " : ",\n  ";
            s += "{\"arch\": \"";
            escape_into(s, a->str);
            std::snprintf(line, sizeof line, "\", \"tune_version\": %.0f, \"log2_n\": %.0f, \"log2_m\": %.0f, \"ms\": %.6g, \"params\": {",
                          v->num, ln->num, lm->num, t->num);
            s += line;
            bool pf = true;
            for (const auto& kv : prm->obj) {
                if (kv.second.kind != Json::NUM) return MCD_ERR_CHECKPOINT;
                s += pf ? "\"" : ", \"";
                escape_into(s, kv.first);
                std::snprintf(line, sizeof line, "\": %.0f", kv.second.num);
                s += line;
                pf = false;
            }
            s += "}}";
            out += s;
            first = false;
        }
    }
    // this graph's entry: the context's current parameters
    std::string s = first ? "  " : ",\n  ";
    s += "{\"arch\": \"";
    escape_into(s, k.arch);
    std::snprintf(line, sizeof line, "\", \"tune_version\": %d, \"log2_n\": %d, \"log2_m\": %d, \"ms\": %.6g, \"params\": {",
                  kTuneVersion, k.log2_n, k.log2_m, (double)ms);
    s += line;
    for (int i = 0; i < kNumParams; ++i) {
        int64_t v = 0;
        (void)mcd_ctx_get_param(ctx, kParams[i], &v);
        std::snprintf(line, sizeof line, "%s\"%s\": %lld", i ? ", " : "", kParams[i], (long long)v);
        s += line;
    }
    s += "}}";
    out += s;
    out += "\n]}\n";
    // written beside the target, then renamed over it
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return MCD_ERR_CHECKPOINT;
    const bool ok = std::fwrite(out.data(), 1, out.size(), f) == out.size();
    if (std::fclose(f) != 0 || !ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return MCD_ERR_CHECKPOINT;
    }
    return MCD_OK;
}

mcd_status mcd_tune_cache_check_file(const char* path) {
    if (!path) return MCD_ERR_INVALID_ARG;
    Json root;
    bool exists = false;
    const mcd_status st = read_cache(path, root, &exists);
    if (st != MCD_OK || !exists) return st;
    for (const Json& e : root.get("entries")->arr) {
        const Json* a = e.kind == Json::OBJ ? e.get("arch") : nullptr;
        const Json* prm = e.kind == Json::OBJ ? e.get("params") : nullptr;
        if (!a || a->kind != Json::STR || !prm || prm->kind != Json::OBJ) return MCD_ERR_CHECKPOINT;
        for (const char* name : {"tune_version", "log2_n", "log2_m", "ms"}) {
            const Json* x = e.get(name);
            if (!x || x->kind != Json::NUM) return MCD_ERR_CHECKPOINT;
        }
        for (const auto& kv : prm->obj)
            if (kv.second.kind != Json::NUM) return MCD_ERR_CHECKPOINT;
    }
    return MCD_OK;
}

}  // extern "C"
#pragma GCC visibility pop
