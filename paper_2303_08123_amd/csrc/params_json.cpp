// gga_params_from_json: the model constants from a flat JSON object whose
// values are numbers or arrays of numbers (the format of the package's
// data/model_default.json).  Every field of gga_params must be present except
// repair_half_time (default 0), oer_max (default 1, no oxygen effect), oer_k
// (default 0.05) and mitotic_death (default 0); keys the struct does not have
// are ignored.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/gga.h"

namespace gga {
int check_params_host(const gga_params* p);   // the validation every simulation call applies
}

namespace {

struct Reader {
    const char* p;
    const char* end;
    void skip() {
        while (p < end && (*p == ' ' || *p == '\t' || *p == '\n' || *p == '\r')) ++p;
    }
    bool eat(char c) {
        skip();
        if (p < end && *p == c) {
            ++p;
            return true;
        }
        return false;
    }
    bool string(std::string* out) {
        skip();
        if (p >= end || *p != '"') return false;
        ++p;
        const char* s = p;
        while (p < end && *p != '"') {
            if (*p == '\\') return false;          // escapes never occur in key names here
            ++p;
        }
        if (p >= end) return false;
        out->assign(s, p - s);
        ++p;
        return true;
    }
    bool number(double* out) {
        skip();
        if (p >= end) return false;
        char buf[64];
        size_t n = 0;
        while (p + n < end && n < sizeof(buf) - 1 && std::strchr("+-0123456789.eE", p[n])) {
            buf[n] = p[n];
            ++n;
        }
        if (n == 0) return false;
        buf[n] = '\0';
        char* stop = nullptr;
        const double v = std::strtod(buf, &stop);
        if (stop != buf + n) return false;
        p += n;
        *out = v;
        return true;
    }
    // value: a number or an array of numbers
    bool value(std::vector<double>* out) {
        out->clear();
        double v;
        if (eat('[')) {
            if (eat(']')) return true;
            do {
                if (!number(&v)) return false;
                out->push_back(v);
            } while (eat(','));
            return eat(']');
        }
        if (!number(&v)) return false;
        out->push_back(v);
        return true;
    }
};

bool parse(const std::string& text, std::map<std::string, std::vector<double>>* kv) {
    Reader r{text.data(), text.data() + text.size()};
    if (!r.eat('{')) return false;
    if (r.eat('}')) return r.skip(), r.p == r.end;
    do {
        std::string key;
        std::vector<double> val;
        if (!r.string(&key) || !r.eat(':') || !r.value(&val)) return false;
        (*kv)[key] = val;
    } while (r.eat(','));
    if (!r.eat('}')) return false;
    r.skip();
    return r.p == r.end;
}

}  // namespace

extern "C" int gga_params_from_json(const char* path, gga_params* out) {
    if (!out) return GGA_E_ARG;
    if (out->struct_size != sizeof(gga_params)) return GGA_E_ABI;
    if (!path) return GGA_E_ARG;
    FILE* f = std::fopen(path, "rb");
    if (!f) return GGA_E_ARG;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
    const bool read_ok = !std::ferror(f);
    std::fclose(f);
    std::map<std::string, std::vector<double>> kv;
    if (!read_ok || !parse(text, &kv)) return GGA_E_ARG;

    gga_params p;
    std::memset(&p, 0, sizeof(p));
    p.struct_size = sizeof(gga_params);
    bool ok = true;
    auto floats = [&](const char* key, float* dst, size_t count) {
        auto it = kv.find(key);
        if (it == kv.end() || it->second.size() != count) return void(ok = false);
        for (size_t i = 0; i < count; ++i) dst[i] = (float)it->second[i];
    };
    auto doubles = [&](const char* key, double* dst, size_t count) {
        auto it = kv.find(key);
        if (it == kv.end() || it->second.size() != count) return void(ok = false);
        for (size_t i = 0; i < count; ++i) dst[i] = it->second[i];
    };
    auto ints = [&](const char* key, int32_t* dst, size_t count) {
        auto it = kv.find(key);
        if (it == kv.end() || it->second.size() != count) return void(ok = false);
        for (size_t i = 0; i < count; ++i) {
            const double v = it->second[i];
            if (!(std::fabs(v) < 2147483648.0) || v != std::floor(v)) return void(ok = false);
            dst[i] = (int32_t)v;
        }
    };
    floats("lambda", p.lambda, 3);
    floats("kappa", p.kappa, 3);
    floats("ghost", p.ghost, 3);
    floats("init_fields", p.init, 3);
    floats("activity", p.activity, 4);
    floats("theta_O_quiesce", &p.theta_O_quiesce, 1);
    floats("theta_G_quiesce", &p.theta_G_quiesce, 1);
    floats("theta_O_death", &p.theta_O_death, 1);
    floats("theta_G_death", &p.theta_G_death, 1);
    floats("theta_H_death", &p.theta_H_death, 1);
    ints("T_min", &p.T_min, 1);
    ints("T_lys", &p.T_lys, 1);
    ints("A0", &p.A0, 1);
    ints("seed_radius", &p.seed_radius, 1);
    ints("class_age", p.class_age, 2);
    doubles("P_div", &p.P_div, 1);
    doubles("alpha", &p.alpha, 1);
    doubles("beta", &p.beta, 1);
    doubles("m", p.m, 4);
    if (kv.count("repair_half_time")) doubles("repair_half_time", &p.repair_half_time, 1);   // optional, default 0
    p.oer_max = 1.0;                                  // optional: no oxygen effect
    p.oer_k = 0.05;
    if (kv.count("oer_max")) doubles("oer_max", &p.oer_max, 1);
    if (kv.count("oer_k")) doubles("oer_k", &p.oer_k, 1);
    if (kv.count("mitotic_death")) ints("mitotic_death", &p.mitotic_death, 1);   // optional, default 0
    if (!ok) return GGA_E_PARAM;
    const int rc = gga::check_params_host(&p);
    if (rc != GGA_OK) return rc;
    *out = p;
    return GGA_OK;
}
