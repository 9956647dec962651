// Host-only driver of the model-header reader (paper_2506_04055_amd/csrc/
// header_json.h), built with AddressSanitizer and UndefinedBehaviorSanitizer
// by tests/test_sanitizers.py.  It parses valid headers, then many
// truncated, mutated and random strings, and checks the parsed fields of
// the valid ones; any out-of-bounds read or undefined behaviour aborts.
#include "../../paper_2506_04055_amd/csrc/header_json.h"

#include <cstdio>
#include <cstdint>
#include <string>
#include <vector>

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static uint64_t next_u64() {  // splitmix64
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

int main() {
    const std::vector<std::string> valid = {
        "{\"model\":\"painn\",\"F\":128,\"K\":20,\"T\":3,\"n_species\":2,\"r_c\":5.0,\"eps\":1e-8,"
        "\"basis\":\"bessel_sin_over_r\",\"envelope\":\"cosine\",\"units\":{\"length\":\"A\",\"energy\":\"eV\"},"
        "\"graph\":[\"csr\",\"full\"]}",
        "  { \"F\" : 32 , \"K\":8, \"T\" :2,\"n_species\":1,\"r_c\":5,\"eps\":1e-8, \"note\":\"a \\\"quoted\\\" }{\" } ",
        "{}",
    };
    int bad = 0;
    for (const std::string &v : valid) {
        mlp_json::JsonTop j = mlp_json::parse_top(v.c_str());
        if (!j.ok) { std::printf("valid header rejected: %s\n", v.c_str()); bad++; }
    }
    {
        mlp_json::JsonTop j = mlp_json::parse_top(valid[0].c_str());
        long F = 0, T = 0;
        double rc = 0;
        if (!mlp_json::get_int(j, "F", &F) || F != 128 || !mlp_json::get_int(j, "T", &T) || T != 3 ||
            !mlp_json::get_num(j, "r_c", &rc) || rc != 5.0 || j.kv["model"] != "painn" ||
            j.kv.count("units") != 1) {
            std::printf("fields of the valid header misread\n");
            bad++;
        }
        if (mlp_json::get_int(j, "r_c", &F)) { std::printf("5.0 read as an integer\n"); bad++; }
        std::vector<long> lv;
        mlp_json::JsonTop j2 = mlp_json::parse_top("{\"mlp_2b\": [8, 16 ,32,64], \"bad\": [1, x], \"e\": []}");
        if (!mlp_json::get_int_list(j2, "mlp_2b", &lv) || lv.size() != 4 || lv[3] != 64 ||
            mlp_json::get_int_list(j2, "bad", &lv) || mlp_json::get_int_list(j2, "e", &lv)) {
            std::printf("integer lists misread\n");
            bad++;
        }
    }
    const char alphabet[] = "{}[]\":,\\ \t\nabcFKT0123456789.eE-+";
    long n_ok = 0;
    for (int it = 0; it < 200000; it++) {
        std::string s;
        const int mode = (int)(next_u64() % 3);
        if (mode == 0) {  // truncation of a valid header
            const std::string &v = valid[next_u64() % valid.size()];
            s = v.substr(0, next_u64() % (v.size() + 1));
        } else if (mode == 1) {  // point mutations of a valid header
            s = valid[next_u64() % valid.size()];
            const int k = 1 + (int)(next_u64() % 4);
            for (int q = 0; q < k && !s.empty(); q++)
                s[next_u64() % s.size()] = alphabet[next_u64() % (sizeof(alphabet) - 1)];
        } else {  // random strings over the JSON alphabet
            const int len = (int)(next_u64() % 64);
            for (int q = 0; q < len; q++) s.push_back(alphabet[next_u64() % (sizeof(alphabet) - 1)]);
        }
        // exact-size heap copy, so a read past the terminator is caught
        std::vector<char> buf(s.begin(), s.end());
        buf.push_back('\0');
        mlp_json::JsonTop j = mlp_json::parse_top(buf.data());
        long iv;
        double dv;
        if (j.ok) {
            n_ok++;
            for (const char *k : {"F", "K", "T", "n_species"}) (void)mlp_json::get_int(j, k, &iv);
            for (const char *k : {"r_c", "eps"}) (void)mlp_json::get_num(j, k, &dv);
            std::vector<long> lv;
            for (const char *k : {"graph", "units", "F"}) (void)mlp_json::get_int_list(j, k, &lv);
        }
    }
    std::printf("json_fuzz: %d failures, %ld of 200000 inputs parsed as objects\n", bad, n_ok);
    return bad ? 1 : 0;
}
