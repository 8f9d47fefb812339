// Tuning table: the autotuner's choice of table shape (line width, probe
// sequence, lanes per state) per table kind, state width and capacity, read
// from its JSON file and consulted when the library creates tables.
//
// The reader accepts standard JSON (objects, arrays, strings with escapes,
// numbers, true/false/null) and keeps only the fields it knows.
#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace {

struct JVal {
    enum Kind { Null, Bool, Num, Str, Arr, Obj } kind = Null;
    bool b = false;
    double num = 0;
    std::string str;
    std::vector<JVal> arr;
    std::vector<std::pair<std::string, JVal>> obj;

    const JVal *get(const char *key) const {
        if (kind != Obj)
            return nullptr;
        for (const auto &kv : obj)
            if (kv.first == key)
                return &kv.second;
        return nullptr;
    }
};

class JParser {
public:
    explicit JParser(const std::string &text) : s_(text) {}

    bool parse(JVal &out) {
        if (!value(out, 0))
            return false;
        ws();
        return i_ == s_.size();
    }

private:
    static constexpr int kMaxDepth = 64;
    const std::string &s_;
    size_t i_ = 0;

    void ws() {
        while (i_ < s_.size() && (s_[i_] == ' ' || s_[i_] == '\t' || s_[i_] == '\n' || s_[i_] == '\r'))
            ++i_;
    }
    bool lit(const char *w) {
        const size_t n = std::strlen(w);
        if (s_.compare(i_, n, w) != 0)
            return false;
        i_ += n;
        return true;
    }
    static bool hex4(const std::string &s, size_t at, uint32_t &cp) {
        if (at + 4 > s.size())
            return false;
        cp = 0;
        for (size_t k = 0; k < 4; ++k) {
            const char c = s[at + k];
            cp <<= 4;
            if (c >= '0' && c <= '9')
                cp |= (uint32_t)(c - '0');
            else if (c >= 'a' && c <= 'f')
                cp |= (uint32_t)(c - 'a' + 10);
            else if (c >= 'A' && c <= 'F')
                cp |= (uint32_t)(c - 'A' + 10);
            else
                return false;
        }
        return true;
    }
    static void utf8(std::string &o, uint32_t cp) {
        if (cp < 0x80) {
            o += (char)cp;
        } else if (cp < 0x800) {
            o += (char)(0xC0 | (cp >> 6));
            o += (char)(0x80 | (cp & 0x3F));
        } else if (cp < 0x10000) {
            o += (char)(0xE0 | (cp >> 12));
            o += (char)(0x80 | ((cp >> 6) & 0x3F));
            o += (char)(0x80 | (cp & 0x3F));
        } else {
            o += (char)(0xF0 | (cp >> 18));
            o += (char)(0x80 | ((cp >> 12) & 0x3F));
            o += (char)(0x80 | ((cp >> 6) & 0x3F));
            o += (char)(0x80 | (cp & 0x3F));
        }
    }
    bool string(std::string &o) {
        if (i_ >= s_.size() || s_[i_] != '"')
            return false;
        ++i_;
        while (i_ < s_.size()) {
            const char c = s_[i_++];
            if (c == '"')
                return true;
            if ((unsigned char)c < 0x20)
                return false;
            if (c != '\\') {
                o += c;
                continue;
            }
            if (i_ >= s_.size())
                return false;
            const char e = s_[i_++];
            switch (e) {
            case '"': o += '"'; break;
            case '\\': o += '\\'; break;
            case '/': o += '/'; break;
            case 'b': o += '\b'; break;
            case 'f': o += '\f'; break;
            case 'n': o += '\n'; break;
            case 'r': o += '\r'; break;
            case 't': o += '\t'; break;
            case 'u': {
                uint32_t cp;
                if (!hex4(s_, i_, cp))
                    return false;
                i_ += 4;
                if (cp >= 0xD800 && cp < 0xDC00) {   // surrogate pair
                    uint32_t lo;
                    if (i_ + 6 > s_.size() || s_[i_] != '\\' || s_[i_ + 1] != 'u' || !hex4(s_, i_ + 2, lo) ||
                        lo < 0xDC00 || lo >= 0xE000)
                        return false;
                    i_ += 6;
                    cp = 0x10000 + ((cp - 0xD800) << 10) + (lo - 0xDC00);
                }
                utf8(o, cp);
                break;
            }
            default: return false;
            }
        }
        return false;
    }
    bool number(double &d) {
        const size_t b = i_;
        if (i_ < s_.size() && s_[i_] == '-')
            ++i_;
        if (i_ >= s_.size() || !(s_[i_] >= '0' && s_[i_] <= '9'))
            return false;
        while (i_ < s_.size() && ((s_[i_] >= '0' && s_[i_] <= '9') || s_[i_] == '.' || s_[i_] == 'e' ||
                                  s_[i_] == 'E' || s_[i_] == '+' || s_[i_] == '-'))
            ++i_;
        const std::string tok = s_.substr(b, i_ - b);
        char *end = nullptr;
        errno = 0;
        d = std::strtod(tok.c_str(), &end);
        return end && *end == '\0' && errno == 0 && std::isfinite(d);
    }
    bool value(JVal &v, int depth) {
        if (depth > kMaxDepth)
            return false;
        ws();
        if (i_ >= s_.size())
            return false;
        const char c = s_[i_];
        if (c == '{') {
            ++i_;
            v.kind = JVal::Obj;
            ws();
            if (i_ < s_.size() && s_[i_] == '}') {
                ++i_;
                return true;
            }
            while (true) {
                ws();
                std::string key;
                if (!string(key))
                    return false;
                ws();
                if (i_ >= s_.size() || s_[i_] != ':')
                    return false;
                ++i_;
                JVal child;
                if (!value(child, depth + 1))
                    return false;
                v.obj.emplace_back(std::move(key), std::move(child));
                ws();
                if (i_ < s_.size() && s_[i_] == ',') {
                    ++i_;
                    continue;
                }
                if (i_ < s_.size() && s_[i_] == '}') {
                    ++i_;
                    return true;
                }
                return false;
            }
        }
        if (c == '[') {
            ++i_;
            v.kind = JVal::Arr;
            ws();
            if (i_ < s_.size() && s_[i_] == ']') {
                ++i_;
                return true;
            }
            while (true) {
                JVal child;
                if (!value(child, depth + 1))
                    return false;
                v.arr.push_back(std::move(child));
                ws();
                if (i_ < s_.size() && s_[i_] == ',') {
                    ++i_;
                    continue;
                }
                if (i_ < s_.size() && s_[i_] == ']') {
                    ++i_;
                    return true;
                }
                return false;
            }
        }
        if (c == '"') {
            v.kind = JVal::Str;
            return string(v.str);
        }
        if (lit("true")) {
            v.kind = JVal::Bool;
            v.b = true;
            return true;
        }
        if (lit("false")) {
            v.kind = JVal::Bool;
            return true;
        }
        if (lit("null"))
            return true;
        v.kind = JVal::Num;
        return number(v.num);
    }
};

struct TuneEntry {
    uint32_t kind;
    uint32_t W;
    uint32_t log2_cap;
    lhs_config cfg;
};

std::mutex g_mu;
std::vector<TuneEntry> g_entries;

bool read_file(const char *path, std::string &out) {
    FILE *f = std::fopen(path, "rb");
    if (!f)
        return false;
    char buf[65536];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) {
        out.append(buf, n);
        if (out.size() > (64u << 20)) {
            std::fclose(f);
            return false;
        }
    }
    const bool ok = !std::ferror(f);
    std::fclose(f);
    return ok;
}

bool as_u32(const JVal *v, uint32_t &out) {
    if (!v || v->kind != JVal::Num || v->num < 0 || v->num > 4294967295.0 || v->num != std::floor(v->num))
        return false;
    out = (uint32_t)v->num;
    return true;
}

// Arch name of the current device without feature suffixes ("gfx950").
bool current_arch(std::string &out) {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    out = p.gcnArchName;
    const size_t colon = out.find(':');
    if (colon != std::string::npos)
        out.resize(colon);
    return true;
}

bool parse_entry(const JVal &e, TuneEntry &t) {
    if (e.kind != JVal::Obj)
        return false;
    const JVal *kind = e.get("kind"), *probe = e.get("probe");
    if (!kind || kind->kind != JVal::Str || !probe || probe->kind != JVal::Str)
        return false;
    if (kind->str == "table")
        t.kind = LHS_TUNE_TABLE;
    else if (kind->str == "batch")
        t.kind = LHS_TUNE_BATCH;
    else
        return false;
    if (probe->str == "double")
        t.cfg.probe = LHS_PROBE_DOUBLE;
    else if (probe->str == "linear")
        t.cfg.probe = LHS_PROBE_LINEAR;
    else if (probe->str == "quadratic")
        t.cfg.probe = LHS_PROBE_QUADRATIC;
    else
        return false;
    if (!as_u32(e.get("W"), t.W) || !as_u32(e.get("log2_capacity"), t.log2_cap) ||
        !as_u32(e.get("line_slots"), t.cfg.line_slots) || !as_u32(e.get("tps_find_or_put"), t.cfg.tps_find_or_put) ||
        !as_u32(e.get("tps_expand"), t.cfg.tps_expand))
        return false;
    return t.W >= 1 && t.W <= 32 && t.log2_cap >= 4 && t.log2_cap <= 32 &&
           lhs::valid_line_slots(t.cfg.line_slots) && lhs::valid_tps(t.cfg.tps_find_or_put) &&
           lhs::valid_tps(t.cfg.tps_expand);
}

uint32_t log2_floor(uint64_t x) {
    uint32_t r = 0;
    while (x > 1) {
        x >>= 1;
        ++r;
    }
    return r;
}

bool lookup_locked(uint32_t kind, uint32_t W, uint64_t capacity, lhs_config &out) {
    // smallest tuned W >= W, else the largest tuned W
    uint32_t best_w = 0, max_w = 0;
    for (const auto &e : g_entries) {
        if (e.kind != kind)
            continue;
        max_w = std::max(max_w, e.W);
        if (e.W >= W && (best_w == 0 || e.W < best_w))
            best_w = e.W;
    }
    if (max_w == 0)
        return false;
    if (best_w == 0)
        best_w = max_w;
    const int lc = (int)log2_floor(capacity ? capacity : 1);
    const TuneEntry *pick = nullptr;
    for (const auto &e : g_entries) {
        if (e.kind != kind || e.W != best_w)
            continue;
        if (!pick) {
            pick = &e;
            continue;
        }
        const int d = std::abs((int)e.log2_cap - lc), dp = std::abs((int)pick->log2_cap - lc);
        if (d < dp || (d == dp && e.log2_cap > pick->log2_cap))
            pick = &e;
    }
    out = pick->cfg;
    return true;
}

}  // namespace

namespace lhs {

lhs_config tuned_config(uint32_t kind, uint32_t W, uint64_t capacity) {
    lhs_config c{16, LHS_PROBE_DOUBLE, 0, 0};
    std::lock_guard<std::mutex> lk(g_mu);
    lookup_locked(kind, W, capacity, c);
    return c;
}

}  // namespace lhs

extern "C" {

static lhs_status lhs_tune_load_impl(const char *path, const char *device, uint32_t *n_loaded) {
    if (!path)
        return LHS_EINVAL;
    std::string arch;
    if (device)
        arch = device;
    else if (!current_arch(arch))
        return LHS_EDEVICE;
    std::string text;
    if (!read_file(path, text))
        return LHS_EINVAL;
    JVal root;
    if (!JParser(text).parse(root) || root.kind != JVal::Obj)
        return LHS_EINVAL;
    const JVal *fmt = root.get("format"), *dev = root.get("device"), *entries = root.get("entries");
    if (!fmt || fmt->kind != JVal::Str || fmt->str != "lhs-tune-1" || !dev || dev->kind != JVal::Str ||
        !entries || entries->kind != JVal::Arr)
        return LHS_EINVAL;
    std::vector<TuneEntry> parsed;
    for (const JVal &e : entries->arr) {
        TuneEntry t{};
        if (!parse_entry(e, t))
            return LHS_EINVAL;
        parsed.push_back(t);
    }
    if (dev->str != arch)
        parsed.clear();
    std::lock_guard<std::mutex> lk(g_mu);
    g_entries.swap(parsed);
    if (n_loaded)
        *n_loaded = (uint32_t)g_entries.size();
    return LHS_OK;
}

lhs_status lhs_tune_load(const char *path, const char *device, uint32_t *n_loaded) {
    return lhs::guard([&] { return lhs_tune_load_impl(path, device, n_loaded); });
}

lhs_status lhs_tune_clear(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_entries.clear();
    return LHS_OK;
}

lhs_status lhs_tune_lookup(uint32_t kind, uint32_t state_words, uint64_t capacity, lhs_config *out,
                           int32_t *found) {
    if (!out || kind > LHS_TUNE_BATCH || state_words < 1 || state_words > 32)
        return LHS_EINVAL;
    lhs_config c{16, LHS_PROBE_DOUBLE, 0, 0};
    bool f;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        f = lookup_locked(kind, state_words, capacity, c);
    }
    *out = c;
    if (found)
        *found = f ? 1 : 0;
    return LHS_OK;
}

}  // extern "C"
