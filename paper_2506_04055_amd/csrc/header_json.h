// Reader of the model header: the flat top-level JSON object passed to
// mlp_model_create.  Host-only C++ (no HIP), so that it can also be built
// and exercised on its own under AddressSanitizer / UndefinedBehaviorSanitizer.
#pragma once
#include <cctype>
#include <cstdlib>
#include <map>
#include <string>
#include <vector>

namespace mlp_json {
// Values: numbers and strings are kept; nested objects/arrays are skipped.
struct JsonTop {
    std::map<std::string, std::string> kv;
    bool ok = false;
};

inline void skip_ws(const char *&p) {
    while (*p && std::isspace((unsigned char)*p)) p++;
}

inline bool read_string(const char *&p, std::string &out) {
    if (*p != '"') return false;
    p++;
    out.clear();
    while (*p && *p != '"') {
        if (*p == '\\' && p[1]) p++;
        out.push_back(*p++);
    }
    if (*p != '"') return false;
    p++;
    return true;
}

inline bool skip_value(const char *&p, std::string *scalar) {
    skip_ws(p);
    if (*p == '"') {
        std::string s;
        if (!read_string(p, s)) return false;
        if (scalar) *scalar = s;
        return true;
    }
    if (*p == '{' || *p == '[') {
        const char *b0 = p;
        int depth = 0;
        bool in_str = false;
        do {
            char c = *p;
            if (!c) return false;
            if (in_str) {
                if (c == '\\' && p[1]) p++;
                else if (c == '"') in_str = false;
            } else if (c == '"') {
                in_str = true;
            } else if (c == '{' || c == '[') {
                depth++;
            } else if (c == '}' || c == ']') {
                depth--;
            }
            p++;
        } while (depth > 0);
        if (scalar) scalar->assign(b0, p);   // the raw text of the nested value
        return true;
    }
    const char *b = p;
    while (*p && *p != ',' && *p != '}' && !std::isspace((unsigned char)*p)) p++;
    if (scalar) scalar->assign(b, p);
    return p > b;
}

inline JsonTop parse_top(const char *s) {
    JsonTop r;
    const char *p = s;
    skip_ws(p);
    if (*p != '{') return r;
    p++;
    for (;;) {
        skip_ws(p);
        if (*p == '}') {
            r.ok = true;
            return r;
        }
        std::string key, val;
        if (!read_string(p, key)) return r;
        skip_ws(p);
        if (*p != ':') return r;
        p++;
        if (!skip_value(p, &val)) return r;
        r.kv[key] = val;
        skip_ws(p);
        if (*p == ',') {
            p++;
            continue;
        }
        if (*p == '}') {
            r.ok = true;
            return r;
        }
        return r;
    }
}

inline bool get_int(const JsonTop &j, const char *k, long *out) {
    auto it = j.kv.find(k);
    if (it == j.kv.end()) return false;
    char *end = nullptr;
    long v = std::strtol(it->second.c_str(), &end, 10);
    if (end == it->second.c_str() || *end) return false;
    *out = v;
    return true;
}

inline bool get_num(const JsonTop &j, const char *k, double *out) {
    auto it = j.kv.find(k);
    if (it == j.kv.end()) return false;
    char *end = nullptr;
    double v = std::strtod(it->second.c_str(), &end);
    if (end == it->second.c_str() || *end) return false;
    *out = v;
    return true;
}

// A flat list of integers, "[8, 16, 32]"; false unless every element is an
// integer and the list is non-empty.
inline bool get_int_list(const JsonTop &j, const char *k, std::vector<long> *out) {
    auto it = j.kv.find(k);
    if (it == j.kv.end()) return false;
    const std::string &v = it->second;
    if (v.size() < 2 || v.front() != '[' || v.back() != ']') return false;
    out->clear();
    const char *p = v.c_str() + 1;
    for (;;) {
        skip_ws(p);
        char *end = nullptr;
        long x = std::strtol(p, &end, 10);
        if (end == p) return false;
        out->push_back(x);
        p = end;
        skip_ws(p);
        if (*p == ',') {
            p++;
            continue;
        }
        return *p == ']' && p[1] == '\0' && !out->empty();
    }
}
}  // namespace mlp_json
