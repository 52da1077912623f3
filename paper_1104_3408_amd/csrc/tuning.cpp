// Tile-shape table of the autotuner (host only).
//
// paper_1104_3408_amd/tune.py times every candidate tile shape of each
// contraction on the GPU and writes the fastest per shell size into a text
// table, one line per (N_r, N_theta, n_fields, precision):
//
//   # n_r n_theta n_fields precision dr_rows th_rows dph_rows ana_rows syn_rows filt_waves dph_par th_plane fuse
//   #   dph_mfma
//   49 48 50 0 9 3 13 11 8 4 0 1 0 1
//
// (the last four columns may be left out: defaults)
//
// shell_grid_create reads the table on every call: from the path in the
// environment variable SG_TUNING_FILE if set, else tuning.txt beside the
// loaded libshellspec.so.  A shell size without an entry, a missing file or
// an entry outside the kernels' ranges gets the defaults of sg::Tune.
#include <dlfcn.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "internal.h"

namespace sg {

namespace {

std::string table_path() {
    const char* env = std::getenv("SG_TUNING_FILE");
    if (env && *env) return env;
    Dl_info info;
    if (dladdr(reinterpret_cast<void*>(&lookup_tuning), &info) && info.dli_fname) {
        std::string so = info.dli_fname;
        const size_t slash = so.rfind('/');
        return (slash == std::string::npos ? std::string(".") : so.substr(0, slash)) + "/tuning.txt";
    }
    return "tuning.txt";
}

bool valid(const Tune& t) {
    for (int r : {t.dr_rows, t.th_rows, t.dph_rows, t.ana_rows, t.syn_rows})
        if (r < 1 || r > kMaxRows) return false;
    return (t.filt_waves == 4 || t.filt_waves == 8 || t.filt_waves == 16) && t.dph_par >= -1 && t.dph_par <= 1 &&
           (t.th_plane == 0 || t.th_plane == 1) && (t.fuse == 0 || t.fuse == 1) && (t.dph_mfma == 0 || t.dph_mfma == 1);
}

}  // namespace

Tune lookup_tuning(int n_r, int n_theta, int n_fields, int precision, std::string* source) {
    Tune def;
    if (source) *source = "defaults";
    const std::string path = table_path();
    FILE* f = std::fopen(path.c_str(), "r");
    if (!f) return def;
    char line[512];
    Tune found = def;
    bool hit = false;
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#') continue;
        int a, b, c, d;
        Tune t;
        const int n = std::sscanf(line, "%d %d %d %d %d %d %d %d %d %d %d %d %d %d", &a, &b, &c, &d, &t.dr_rows,
                                  &t.th_rows, &t.dph_rows, &t.ana_rows, &t.syn_rows, &t.filt_waves, &t.dph_par,
                                  &t.th_plane, &t.fuse, &t.dph_mfma);
        if (n < 10) continue;
        if (a == n_r && b == n_theta && c == n_fields && d == precision && valid(t)) {
            found = t;
            hit = true;
        }
    }
    std::fclose(f);
    if (hit && source) *source = path;
    return found;
}

}  // namespace sg
