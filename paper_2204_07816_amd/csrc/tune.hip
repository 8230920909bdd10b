// tune.hip -- the autotuner: which form of the exchanged-configuration pass
// (full recompute with a given tile variant, or the incremental receptive
// cone) is fastest for a configuration, measured on the device and kept in a
// JSON cache file shared by every context of the same configuration.
//
// Cache file: NQS_TUNE_CACHE if set, else $HOME/.cache/nqs/tune.json.  It is
// one JSON object whose members are configurations:
//   { "gfx950 L=36 K=8 C=32 bf16 J2": {"mode": "incremental", "full_nw": 8,
//     "full_maxt": 11, "cone_items": 6, "cone_waves": 4, "ms_full": 1234.5,
//     "ms_incremental": 83.0}, ... }
// cone_items / cone_waves: the shape of the incremental cone kernel (items
// per workgroup and waves; 1 / 0 for the one-configuration kernel); entries
// without them keep the default shape.
// A missing, unreadable or malformed file counts as empty (defaults apply);
// writing replaces the file through a temporary and a rename.
#include <hip/hip_runtime.h>

#include <cctype>
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <sys/stat.h>
#include <unistd.h>

#include "nqs_internal.h"

namespace nqs {
namespace {

struct Entry {
    std::string mode;          // "full" | "incremental"
    int full_nw = 0, full_maxt = 0;
    int cone_items = -1, cone_waves = -1;   // -1: not tuned
    double ms_full = -1.0, ms_incremental = -1.0;
};

// --- a small reader for exactly the cache's shape (object of objects whose
// members are strings or numbers) ---
struct Reader {
    const char *p, *end;
    void ws()
    {
        while (p < end && std::isspace((unsigned char)*p)) ++p;
    }
    bool lit(char ch)
    {
        ws();
        if (p < end && *p == ch) {
            ++p;
            return true;
        }
        return false;
    }
    bool str(std::string *out)
    {
        ws();
        if (p >= end || *p != '"') return false;
        ++p;
        out->clear();
        while (p < end && *p != '"') {
            if (*p == '\\') return false;   // the cache never holds escapes
            out->push_back(*p++);
        }
        if (p >= end) return false;
        ++p;
        return true;
    }
    bool num(double *out)
    {
        ws();
        char *e = nullptr;
        errno = 0;
        const double v = std::strtod(p, &e);
        if (e == p || e > end || errno != 0) return false;
        p = e;
        *out = v;
        return true;
    }
};

bool parse_entry(Reader &r, Entry *e)
{
    if (!r.lit('{')) return false;
    if (r.lit('}')) return true;
    do {
        std::string k;
        if (!r.str(&k) || !r.lit(':')) return false;
        if (k == "mode") {
            if (!r.str(&e->mode)) return false;
        } else {
            double v;
            if (!r.num(&v)) return false;
            if (k == "full_nw") e->full_nw = (int)v;
            else if (k == "full_maxt") e->full_maxt = (int)v;
            else if (k == "cone_items") e->cone_items = (int)v;
            else if (k == "cone_waves") e->cone_waves = (int)v;
            else if (k == "ms_full") e->ms_full = v;
            else if (k == "ms_incremental") e->ms_incremental = v;
        }
    } while (r.lit(','));
    return r.lit('}');
}

bool read_cache(const std::string &path, std::map<std::string, Entry> *out)
{
    out->clear();
    FILE *f = std::fopen(path.c_str(), "rb");
    if (!f) return false;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
    std::fclose(f);
    Reader r{text.data(), text.data() + text.size()};
    std::map<std::string, Entry> m;
    if (!r.lit('{')) return false;
    if (!r.lit('}')) {
        do {
            std::string key;
            Entry e;
            if (!r.str(&key) || !r.lit(':') || !parse_entry(r, &e)) return false;
            if (e.mode != "full" && e.mode != "incremental") return false;
            m[key] = e;
        } while (r.lit(','));
        if (!r.lit('}')) return false;
    }
    r.ws();
    if (r.p != r.end) return false;
    *out = std::move(m);
    return true;
}

bool write_cache(const std::string &path, const std::map<std::string, Entry> &m)
{
    // make the directory chain of the file
    for (size_t i = 1; i < path.size(); ++i)
        if (path[i] == '/') {
            const std::string d = path.substr(0, i);
            if (mkdir(d.c_str(), 0755) != 0 && errno != EEXIST) return false;
        }
    const std::string tmp = path + ".tmp." + std::to_string((long)getpid());
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return false;
    std::fprintf(f, "{\n");
    size_t i = 0;
    for (const auto &kv : m) {
        const Entry &e = kv.second;
        std::fprintf(f,
                     "  \"%s\": {\"mode\": \"%s\", \"full_nw\": %d, \"full_maxt\": %d, "
                     "\"cone_items\": %d, \"cone_waves\": %d, "
                     "\"ms_full\": %.6g, \"ms_incremental\": %.6g}%s\n",
                     kv.first.c_str(), e.mode.c_str(), e.full_nw, e.full_maxt, e.cone_items,
                     e.cone_waves, e.ms_full, e.ms_incremental, ++i < m.size() ? "," : "");
    }
    std::fprintf(f, "}\n");
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), path.c_str()) != 0) {
        std::remove(tmp.c_str());
        return false;
    }
    return true;
}

std::string key_of(int L, int K, int C, nqs_dtype dt, double J2)
{
    const char *d = dt == NQS_BF16X3 ? "bf16x3"
                    : dt == NQS_BF16 ? "bf16" : (dt == NQS_FP32 ? "fp32" : "fp64");
    char buf[96];
    std::snprintf(buf, sizeof buf, "gfx950 L=%d K=%d C=%d %s %s", L, K, C, d,
                  J2 != 0.0 ? "J2" : "J1only");
    return buf;
}

}  // namespace

std::string tune_cache_path()
{
    const char *env = std::getenv("NQS_TUNE_CACHE");
    if (env && *env) return env;
    const char *home = std::getenv("HOME");
    return std::string(home && *home ? home : "/tmp") + "/.cache/nqs/tune.json";
}

std::string tune_key(const nqs_ctx *c) { return key_of(c->L, c->K, c->C, c->dtype, c->J2); }

bool tune_lookup(const std::string &path, const std::string &key, nqs_mode *mode, int *nw,
                 int *maxt, int *cone_items, int *cone_waves)
{
    std::map<std::string, Entry> m;
    if (!read_cache(path, &m)) return false;
    auto it = m.find(key);
    if (it == m.end()) return false;
    *mode = it->second.mode == "incremental" ? NQS_INCREMENTAL : NQS_FULL;
    *nw = it->second.full_nw;
    *maxt = it->second.full_maxt;
    if (cone_items) *cone_items = it->second.cone_items;
    if (cone_waves) *cone_waves = it->second.cone_waves;
    return true;
}

bool tune_store(const std::string &path, const std::string &key, nqs_mode mode, int nw, int maxt,
                int cone_items, int cone_waves, double ms_full, double ms_inc)
{
    std::map<std::string, Entry> m;
    read_cache(path, &m);   // a malformed cache is replaced
    Entry e;
    e.mode = mode == NQS_INCREMENTAL ? "incremental" : "full";
    e.full_nw = nw;
    e.full_maxt = maxt;
    e.cone_items = cone_items;
    e.cone_waves = cone_waves;
    e.ms_full = ms_full;
    e.ms_incremental = ms_inc;
    m[key] = e;
    return write_cache(path, m);
}

}  // namespace nqs

extern "C" nqs_status nqs_tune_key(int32_t L, int32_t K, int32_t C, nqs_dtype dtype, double J2,
                                   char *buf, int64_t len)
{
    if (!buf || len <= 0) return NQS_E_ARG;
    const std::string k = nqs::key_of(L, K, C, dtype, J2);
    if ((int64_t)k.size() + 1 > len) return NQS_E_ARG;
    std::memcpy(buf, k.c_str(), k.size() + 1);
    return NQS_OK;
}

extern "C" nqs_status nqs_tune_lookup(const char *path, const char *key, nqs_mode *mode,
                                      int32_t *full_nw, int32_t *full_maxt, int32_t *cone_items,
                                      int32_t *cone_waves)
{
    if (!path || !key || !mode || !full_nw || !full_maxt) return NQS_E_ARG;
    nqs_mode m;
    int nw, mt, ci = -1, cw = -1;
    if (!nqs::tune_lookup(path, key, &m, &nw, &mt, &ci, &cw)) return NQS_E_ARG;
    *mode = m;
    *full_nw = nw;
    *full_maxt = mt;
    if (cone_items) *cone_items = ci;
    if (cone_waves) *cone_waves = cw;
    return NQS_OK;
}
