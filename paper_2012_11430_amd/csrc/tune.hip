// Tuning entries from the autotuner's JSON cache, and queries of the registered
// entries (host code only).
//
// The cache (written by paper_2012_11430_amd/autotune.py) has the form
//   {"version": 2,
//    "devices": {"<arch>:<compute units>": {"<key>": <value>, ...}, ...}}
// with <key> "d,n,m,prec,mode" (an exact shape) or "bucket:d,n,m,prec,mode" (the
// bucket of that shape), prec one of fp64 / fp32 / bf16x3, mode single / batch,
// and <value> an integer (the split target) or an object
// {"target": <int>, "fragments": <int>} (either member may be missing: 0).
// Version 1 caches (integer values only) are read the same way.
//
// The loader parses the whole document with a small recursive-descent JSON
// parser (strings with escapes, numbers, literals, nested arrays and objects up to
// a fixed depth), takes the object of the requested device key from "devices" and
// registers every entry through prony_tune_set_tile, so the same validation applies.
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <memory>
#include <sstream>
#include <string>
#include <utility>
#include <vector>

#include "common.h"

namespace prony {
namespace {

struct Json {
    enum Kind { Null, Bool, Number, String, Array, Object } kind = Null;
    bool b = false;
    double num = 0.0;
    bool integral = false;   // the number was written without fraction or exponent
    long long ival = 0;
    std::string str;
    std::vector<Json> items;                            // Array
    std::vector<std::pair<std::string, Json>> members;  // Object, in document order
};

class Parser {
  public:
    explicit Parser(const std::string& text) : s_(text) {}

    bool parse(Json& out, std::string& err) {
        if (!value(out, 0)) {
            err = err_ + " at byte " + std::to_string(i_);
            return false;
        }
        ws();
        if (i_ != s_.size()) {
            err = "trailing characters at byte " + std::to_string(i_);
            return false;
        }
        return true;
    }

  private:
    static constexpr int kMaxDepth = 32;
    const std::string& s_;
    size_t i_ = 0;
    std::string err_;

    bool fail(const char* what) {
        err_ = what;
        return false;
    }
    void ws() {
        while (i_ < s_.size() && (s_[i_] == ' ' || s_[i_] == '\n' || s_[i_] == '\r' || s_[i_] == '\t')) ++i_;
    }
    bool literal(const char* word) {
        size_t k = 0;
        while (word[k]) {
            if (i_ + k >= s_.size() || s_[i_ + k] != word[k]) return fail("bad literal");
            ++k;
        }
        i_ += k;
        return true;
    }
    static void put_utf8(std::string& out, unsigned cp) {
        if (cp < 0x80) {
            out += (char)cp;
        } else if (cp < 0x800) {
            out += (char)(0xC0 | (cp >> 6));
            out += (char)(0x80 | (cp & 0x3F));
        } else if (cp < 0x10000) {
            out += (char)(0xE0 | (cp >> 12));
            out += (char)(0x80 | ((cp >> 6) & 0x3F));
            out += (char)(0x80 | (cp & 0x3F));
        } else {
            out += (char)(0xF0 | (cp >> 18));
            out += (char)(0x80 | ((cp >> 12) & 0x3F));
            out += (char)(0x80 | ((cp >> 6) & 0x3F));
            out += (char)(0x80 | (cp & 0x3F));
        }
    }
    bool hex4(unsigned& v) {
        if (i_ + 4 > s_.size()) return fail("short \\u escape");
        v = 0;
        for (int k = 0; k < 4; ++k) {
            const char c = s_[i_++];
            v <<= 4;
            if (c >= '0' && c <= '9')
                v |= (unsigned)(c - '0');
            else if (c >= 'a' && c <= 'f')
                v |= (unsigned)(c - 'a' + 10);
            else if (c >= 'A' && c <= 'F')
                v |= (unsigned)(c - 'A' + 10);
            else
                return fail("bad \\u escape");
        }
        return true;
    }
    bool string(std::string& out) {
        if (i_ >= s_.size() || s_[i_] != '"') return fail("expected a string");
        ++i_;
        out.clear();
        while (i_ < s_.size()) {
            const unsigned char c = (unsigned char)s_[i_++];
            if (c == '"') return true;
            if (c < 0x20) return fail("control character in a string");
            if (c != '\\') {
                out += (char)c;
                continue;
            }
            if (i_ >= s_.size()) break;
            const char e = s_[i_++];
            switch (e) {
                case '"': out += '"'; break;
                case '\\': out += '\\'; break;
                case '/': out += '/'; break;
                case 'b': out += '\b'; break;
                case 'f': out += '\f'; break;
                case 'n': out += '\n'; break;
                case 'r': out += '\r'; break;
                case 't': out += '\t'; break;
                case 'u': {
                    unsigned cp = 0;
                    if (!hex4(cp)) return false;
                    if (cp >= 0xD800 && cp < 0xDC00) {   // a surrogate pair
                        unsigned lo = 0;
                        if (i_ + 2 > s_.size() || s_[i_] != '\\' || s_[i_ + 1] != 'u') return fail("lone surrogate");
                        i_ += 2;
                        if (!hex4(lo)) return false;
                        if (lo < 0xDC00 || lo >= 0xE000) return fail("bad surrogate pair");
                        cp = 0x10000 + ((cp - 0xD800) << 10) + (lo - 0xDC00);
                    } else if (cp >= 0xDC00 && cp < 0xE000) {
                        return fail("lone surrogate");
                    }
                    put_utf8(out, cp);
                    break;
                }
                default:
                    return fail("bad escape");
            }
        }
        return fail("unterminated string");
    }
    bool number(Json& out) {
        const size_t start = i_;
        if (i_ < s_.size() && s_[i_] == '-') ++i_;
        if (i_ >= s_.size() || s_[i_] < '0' || s_[i_] > '9') return fail("bad number");
        if (s_[i_] == '0') {
            ++i_;
        } else {
            while (i_ < s_.size() && s_[i_] >= '0' && s_[i_] <= '9') ++i_;
        }
        bool integral = true;
        if (i_ < s_.size() && s_[i_] == '.') {
            integral = false;
            ++i_;
            if (i_ >= s_.size() || s_[i_] < '0' || s_[i_] > '9') return fail("bad number");
            while (i_ < s_.size() && s_[i_] >= '0' && s_[i_] <= '9') ++i_;
        }
        if (i_ < s_.size() && (s_[i_] == 'e' || s_[i_] == 'E')) {
            integral = false;
            ++i_;
            if (i_ < s_.size() && (s_[i_] == '+' || s_[i_] == '-')) ++i_;
            if (i_ >= s_.size() || s_[i_] < '0' || s_[i_] > '9') return fail("bad number");
            while (i_ < s_.size() && s_[i_] >= '0' && s_[i_] <= '9') ++i_;
        }
        const std::string text = s_.substr(start, i_ - start);
        out.kind = Json::Number;
        out.num = std::strtod(text.c_str(), nullptr);
        out.integral = integral && text.size() <= 18;   // fits a long long
        out.ival = out.integral ? std::strtoll(text.c_str(), nullptr, 10) : 0;
        return true;
    }
    bool value(Json& out, int depth) {
        if (depth > kMaxDepth) return fail("nesting too deep");
        ws();
        if (i_ >= s_.size()) return fail("unexpected end");
        const char c = s_[i_];
        if (c == '{') {
            ++i_;
            out.kind = Json::Object;
            ws();
            if (i_ < s_.size() && s_[i_] == '}') {
                ++i_;
                return true;
            }
            for (;;) {
                ws();
                std::string key;
                if (!string(key)) return false;
                ws();
                if (i_ >= s_.size() || s_[i_] != ':') return fail("expected ':'");
                ++i_;
                Json v;
                if (!value(v, depth + 1)) return false;
                out.members.emplace_back(std::move(key), std::move(v));
                ws();
                if (i_ < s_.size() && s_[i_] == ',') {
                    ++i_;
                    continue;
                }
                if (i_ < s_.size() && s_[i_] == '}') {
                    ++i_;
                    return true;
                }
                return fail("expected ',' or '}'");
            }
        }
        if (c == '[') {
            ++i_;
            out.kind = Json::Array;
            ws();
            if (i_ < s_.size() && s_[i_] == ']') {
                ++i_;
                return true;
            }
            for (;;) {
                Json v;
                if (!value(v, depth + 1)) return false;
                out.items.push_back(std::move(v));
                ws();
                if (i_ < s_.size() && s_[i_] == ',') {
                    ++i_;
                    continue;
                }
                if (i_ < s_.size() && s_[i_] == ']') {
                    ++i_;
                    return true;
                }
                return fail("expected ',' or ']'");
            }
        }
        if (c == '"') {
            out.kind = Json::String;
            return string(out.str);
        }
        if (c == 't') {
            out.kind = Json::Bool;
            out.b = true;
            return literal("true");
        }
        if (c == 'f') {
            out.kind = Json::Bool;
            return literal("false");
        }
        if (c == 'n') return literal("null");
        return number(out);
    }
};

const Json* member(const Json& obj, const std::string& key) {
    if (obj.kind != Json::Object) return nullptr;
    const Json* found = nullptr;   // the last of duplicate keys wins, as in most readers
    for (const auto& kv : obj.members)
        if (kv.first == key) found = &kv.second;
    return found;
}

// "d,n,m,prec,mode" (optionally prefixed "bucket:") -> fields; false if malformed
bool parse_key(const std::string& key, int& d, int& n, int& m, prony_prec_t& prec, unsigned& flags) {
    std::string k = key;
    flags = 0;
    static const std::string kBucket = "bucket:";
    if (k.compare(0, kBucket.size(), kBucket) == 0) {
        k = k.substr(kBucket.size());
        flags |= PRONY_TUNE_BUCKET;
    }
    char p[16] = {}, mode[16] = {};
    int used = 0;
    if (std::sscanf(k.c_str(), "%d,%d,%d,%15[^,],%15s%n", &d, &n, &m, p, mode, &used) != 5 || (size_t)used != k.size())
        return false;
    const std::string ps(p), ms(mode);
    if (ps == "fp64")
        prec = PRONY_FP64;
    else if (ps == "fp32")
        prec = PRONY_FP32;
    else if (ps == "bf16x3")
        prec = PRONY_BF16X3;
    else
        return false;
    if (ms == "batch")
        flags |= PRONY_TUNE_BATCHED;
    else if (ms != "single")
        return false;
    return true;
}

bool small_int(const Json* v, int& out) {
    if (!v) {
        out = 0;
        return true;
    }
    if (v->kind != Json::Number || !v->integral || v->ival < 0 || v->ival > (1 << 20)) return false;
    out = (int)v->ival;
    return true;
}

prony_status_t load_cache(prony_handle_t h, const char* path, const std::string& dev_key) {
    std::ifstream in(path);
    if (!in) return fail(h, PRONY_EINVAL, std::string("prony_autotune: cannot read ") + path);
    std::stringstream buf;
    buf << in.rdbuf();
    const std::string text = buf.str();
    Json doc;
    std::string err;
    if (!Parser(text).parse(doc, err)) return fail(h, PRONY_EINVAL, "prony_autotune: malformed JSON: " + err);
    if (doc.kind != Json::Object) return fail(h, PRONY_EINVAL, "prony_autotune: the cache is not a JSON object");
    const Json* version = member(doc, "version");
    if (version && !(version->kind == Json::Number && version->integral && (version->ival == 1 || version->ival == 2)))
        return fail(h, PRONY_EINVAL, "prony_autotune: unsupported cache version");
    const Json* devices = member(doc, "devices");
    if (!devices) return PRONY_OK;   // an empty cache
    if (devices->kind != Json::Object) return fail(h, PRONY_EINVAL, "prony_autotune: \"devices\" is not an object");
    const Json* entries = member(*devices, dev_key);
    if (!entries) return PRONY_OK;   // nothing cached for this device
    if (entries->kind != Json::Object)
        return fail(h, PRONY_EINVAL, "prony_autotune: the entries of this device are not an object");
    for (const auto& kv : entries->members) {
        int d, n, m;
        prony_prec_t prec;
        unsigned flags;
        if (!parse_key(kv.first, d, n, m, prec, flags)) return fail(h, PRONY_EINVAL, "prony_autotune: bad cache key " + kv.first);
        int target = 0, fragments = 0;
        bool ok;
        if (kv.second.kind == Json::Object)
            ok = small_int(member(kv.second, "target"), target) && small_int(member(kv.second, "fragments"), fragments);
        else
            ok = small_int(&kv.second, target);
        if (!ok) return fail(h, PRONY_EINVAL, "prony_autotune: bad cache value of " + kv.first);
        const prony_status_t st = prony_tune_set_tile(h, d, n, m, prec, flags, fragments, target);
        if (st != PRONY_OK) return st;
    }
    return PRONY_OK;
}

}  // namespace
}  // namespace prony

using namespace prony;

extern "C" prony_status_t prony_autotune_device(prony_handle_t h, const char* cache_json_path, const char* device_key) {
    if (!h) return PRONY_EINVAL;
    if (!cache_json_path || !device_key) return fail(h, PRONY_EINVAL, "prony_autotune: null argument");
    return load_cache(h, cache_json_path, device_key);
}

extern "C" prony_status_t prony_autotune(prony_handle_t h, const char* cache_json_path) {
    if (!h) return PRONY_EINVAL;
    if (!cache_json_path) return fail(h, PRONY_EINVAL, "prony_autotune: null path");
    if (!std::ifstream(cache_json_path))
        return fail(h, PRONY_EINVAL, std::string("prony_autotune: cannot read ") + cache_json_path);
    if (h->device < 0) return fail(h, PRONY_ENODEV, "validation-only handle has no device");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, h->device) != hipSuccess)
        return fail(h, PRONY_EHIP, "prony_autotune: hipGetDeviceProperties failed");
    return load_cache(h, cache_json_path, std::string(prop.gcnArchName) + ":" + std::to_string(prop.multiProcessorCount));
}

extern "C" prony_status_t prony_tune_get_tile(prony_handle_t h, int d, int n, int m, prony_prec_t prec, unsigned flags,
                                              int* fragments, int* target_wgs) {
    if (!h || !fragments || !target_wgs) return PRONY_EINVAL;
    if (flags & ~(PRONY_TUNE_BATCHED | PRONY_TUNE_BUCKET)) return fail(h, PRONY_EINVAL, "prony_tune_get: unknown flag");
    if (d < 1 || d > 3 || n < 1 || m < 1 || ipow(2 * (int64_t)n + 2, d) > (int64_t(1) << 30))
        return fail(h, PRONY_EINVAL, "prony_tune_get: bad shape");
    const auto it = h->tune.find(tune_key(d, n, m, (int)prec, (flags & PRONY_TUNE_BATCHED) != 0,
                                          (flags & PRONY_TUNE_BUCKET) != 0));
    *fragments = it == h->tune.end() ? 0 : it->second.fragments;
    *target_wgs = it == h->tune.end() ? 0 : it->second.target;
    return PRONY_OK;
}

extern "C" prony_status_t prony_tune_get(prony_handle_t h, int d, int n, int m, prony_prec_t prec, unsigned flags,
                                         int* target_wgs) {
    if (!h || !target_wgs) return PRONY_EINVAL;
    int fragments = 0;
    return prony_tune_get_tile(h, d, n, m, prec, flags, &fragments, target_wgs);
}
