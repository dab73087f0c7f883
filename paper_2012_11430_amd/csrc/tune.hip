// Tuning entries from the autotuner's JSON cache, and queries of the registered
// entries (host code only).
//
// The cache (written by paper_2012_11430_amd/autotune.py) has the form
//   {"devices": {"<arch>:<compute units>": {"d,n,m,prec,mode": target, ...}, ...},
//    "version": 1}
// with prec one of fp64 / fp32 / bf16x3 and mode single / batch. The loader
// reads the object of this handle's device and registers every entry through
// prony_tune_set, so the same validation applies.
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>
#include <string>

#include "common.h"

namespace prony {
namespace {

struct Cursor {
    const std::string& s;
    size_t i = 0;
    void ws() {
        while (i < s.size() && (s[i] == ' ' || s[i] == '\n' || s[i] == '\r' || s[i] == '\t')) ++i;
    }
    bool eat(char c) {
        ws();
        if (i < s.size() && s[i] == c) {
            ++i;
            return true;
        }
        return false;
    }
    bool string(std::string& out) {   // no escapes occur in the cache's keys
        ws();
        if (i >= s.size() || s[i] != '"') return false;
        const size_t end = s.find('"', i + 1);
        if (end == std::string::npos) return false;
        out = s.substr(i + 1, end - i - 1);
        i = end + 1;
        return true;
    }
    bool integer(long& out) {
        ws();
        const char* p = s.c_str() + i;
        char* e = nullptr;
        out = std::strtol(p, &e, 10);
        if (e == p) return false;
        i += (size_t)(e - p);
        return true;
    }
};

// "d,n,m,prec,mode" -> fields; false if malformed
bool parse_key(const std::string& key, int& d, int& n, int& m, prony_prec_t& prec, unsigned& flags) {
    char p[16] = {}, mode[16] = {};
    if (std::sscanf(key.c_str(), "%d,%d,%d,%15[^,],%15s", &d, &n, &m, p, mode) != 5) return false;
    const std::string ps(p), ms(mode);
    if (ps == "fp64")
        prec = PRONY_FP64;
    else if (ps == "fp32")
        prec = PRONY_FP32;
    else if (ps == "bf16x3")
        prec = PRONY_BF16X3;
    else
        return false;
    if (ms == "single")
        flags = 0;
    else if (ms == "batch")
        flags = PRONY_TUNE_BATCHED;
    else
        return false;
    return true;
}

}  // namespace
}  // namespace prony

using namespace prony;

extern "C" prony_status_t prony_autotune(prony_handle_t h, const char* cache_json_path) {
    if (!h) return PRONY_EINVAL;
    if (!cache_json_path) return fail(h, PRONY_EINVAL, "prony_autotune: null path");
    std::ifstream in(cache_json_path);
    if (!in) return fail(h, PRONY_EINVAL, std::string("prony_autotune: cannot read ") + cache_json_path);
    std::stringstream buf;
    buf << in.rdbuf();
    const std::string text = buf.str();
    if (h->device < 0) return fail(h, PRONY_ENODEV, "validation-only handle has no device");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, h->device) != hipSuccess)
        return fail(h, PRONY_EHIP, "prony_autotune: hipGetDeviceProperties failed");
    const std::string dev_key = std::string(prop.gcnArchName) + ":" + std::to_string(prop.multiProcessorCount);
    // locate "devices": { ... "<dev_key>": { entries } ... }
    const size_t at = text.find("\"" + dev_key + "\"");
    if (at == std::string::npos) return PRONY_OK;   // nothing cached for this device
    Cursor c{text, at};
    std::string key;
    if (!c.string(key) || !c.eat(':') || !c.eat('{'))
        return fail(h, PRONY_EINVAL, "prony_autotune: malformed cache entry of this device");
    if (c.eat('}')) return PRONY_OK;
    for (;;) {
        long target = 0;
        if (!c.string(key) || !c.eat(':') || !c.integer(target))
            return fail(h, PRONY_EINVAL, "prony_autotune: malformed cache entry of this device");
        int d, n, m;
        prony_prec_t prec;
        unsigned flags;
        if (!parse_key(key, d, n, m, prec, flags) || target < 0 || target > (1 << 20))
            return fail(h, PRONY_EINVAL, "prony_autotune: bad cache key " + key);
        const prony_status_t st = prony_tune_set(h, d, n, m, prec, flags, (int)target);
        if (st != PRONY_OK) return st;
        if (c.eat('}')) return PRONY_OK;
        if (!c.eat(',')) return fail(h, PRONY_EINVAL, "prony_autotune: malformed cache entry of this device");
    }
}

extern "C" prony_status_t prony_tune_get(prony_handle_t h, int d, int n, int m, prony_prec_t prec, unsigned flags,
                                         int* target_wgs) {
    if (!h || !target_wgs) return PRONY_EINVAL;
    if (flags & ~PRONY_TUNE_BATCHED) return fail(h, PRONY_EINVAL, "prony_tune_get: unknown flag");
    const auto it = h->split_targets.find(std::make_tuple(d, n, m, (int)prec, (flags & PRONY_TUNE_BATCHED) ? 1 : 0));
    *target_wgs = it == h->split_targets.end() ? 0 : it->second;
    return PRONY_OK;
}
