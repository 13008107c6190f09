// tune.cpp -- reader of the autotuner's JSON cache (see tune.h).
#include "tune.h"

#include <dlfcn.h>
#include <mutex>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <string>
#include <vector>

namespace aesctr {

namespace {

std::once_flag g_once;
std::vector<TuneEntry> g_entries;

std::string cache_path()
{
    const char *env = getenv("AESCTR_TUNE_CACHE");
    if (env && *env)
        return env;
    Dl_info info{};
    if (dladdr(reinterpret_cast<void *>(&tune_lookup), &info) && info.dli_fname) {
        std::string p(info.dli_fname);
        size_t slash = p.rfind('/');
        if (slash != std::string::npos)
            return p.substr(0, slash + 1) + "tune_cache.json";
    }
    return "tune_cache.json";
}

// Reads every {...} object after "entries" as flat "name": integer pairs.
void parse(const std::string &text)
{
    size_t pos = text.find("\"entries\"");
    if (pos == std::string::npos)
        return;
    while ((pos = text.find('{', pos)) != std::string::npos) {
        size_t end = text.find('}', pos);
        if (end == std::string::npos)
            break;
        TuneEntry e;
        size_t q = pos;
        while ((q = text.find('"', q)) != std::string::npos && q < end) {
            size_t q2 = text.find('"', q + 1);
            if (q2 == std::string::npos || q2 > end)
                break;
            std::string name = text.substr(q + 1, q2 - q - 1);
            size_t colon = text.find(':', q2);
            if (colon == std::string::npos || colon > end)
                break;
            long v = strtol(text.c_str() + colon + 1, nullptr, 10);
            if (name == "variant") e.variant = static_cast<int>(v);
            else if (name == "key_bits") e.key_bits = static_cast<int>(v);
            else if (name == "size_log2") e.size_log2 = static_cast<int>(v);
            else if (name == "bpl") e.bpl = static_cast<int>(v);
            else if (name == "wg") e.wg = static_cast<int>(v);
            else if (name == "grid_per_cu") e.grid_per_cu = static_cast<int>(v);
            else if (name == "copies") e.copies = static_cast<int>(v);
            else if (name == "tables") e.tables = static_cast<int>(v);
            else if (name == "first") e.first = static_cast<int>(v);
            else if (name == "tiles_per_cu") e.tiles_per_cu = static_cast<int>(v);
            else if (name == "max_tile_bytes") e.max_tile_bytes = static_cast<int>(v);
            q = colon + 1;
        }
        bool ok = e.bpl > 0 && e.wg >= 64 && e.wg <= 1024 && e.wg % 64 == 0 && e.grid_per_cu > 0;
        if (ok)
            g_entries.push_back(e);
        pos = end + 1;
    }
}

void load()
{
    std::string path = cache_path();
    FILE *f = fopen(path.c_str(), "rb");
    if (!f)
        return;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof(buf), f)) > 0)
        text.append(buf, n);
    fclose(f);
    parse(text);
}

int floor_log2(uint64_t v)
{
    int r = 0;
    while (v >>= 1)
        ++r;
    return r;
}

}  // namespace

bool tune_lookup(int variant, int key_bits, uint64_t len, TuneEntry *out)
{
    std::call_once(g_once, load);
    const int want = floor_log2(len ? len : 1);
    for (const TuneEntry &e : g_entries) {
        if (e.variant != variant || e.key_bits != key_bits || e.size_log2 != want)
            continue;
        if (e.variant == 1 && ((e.copies != 32 && e.copies != 64) || (e.tables != 0 && e.tables != 2 && e.tables != 4) ||
                               (e.copies == 64 && e.tables == 4)))
            continue;
        *out = e;
        return true;
    }
    return false;
}

bool tune_lookup_batch(TuneEntry *out)
{
    std::call_once(g_once, load);
    for (const TuneEntry &e : g_entries) {
        if (e.variant == 10) {
            *out = e;
            return true;
        }
    }
    return false;
}

}  // namespace aesctr
