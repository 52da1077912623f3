// Host-only check of the tuning-table parser (tuning.cpp) for the sanitizer
// test: a table with comments, blank, short, out-of-range, overlong and
// garbage lines, read through SG_TUNING_FILE.
#include "internal.h"
#include <cstdio>
#include <cstdlib>
#include <string>
int main(int argc, char** argv) {
    if (argc < 2) return 2;
    const char* path = argv[1];
    FILE* f = std::fopen(path, "w");
    std::fprintf(f, "# header\n\n49 48 50 0 8 3 13 6 8 8 0 0 0 1\n33 32 50 0 9 4\n17 16 50 0 3 3 4 3 3 8 0 0 0 0 99 99 99\n");
    std::fprintf(f, "25 24 50 0 99 4 8 8 8 8\nxx yy\n");
    for (int i = 0; i < 2000; ++i) std::fputc('7', f);
    std::fprintf(f, "\n65 64 58 0 9 4 16 3 6 8 0 0 1\n");
    std::fclose(f);
    setenv("SG_TUNING_FILE", path, 1);
    std::string src;
    sg::Tune t = sg::lookup_tuning(49, 48, 50, 0, &src);
    std::printf("49: %d %d %d dph_par %d plane %d fuse %d mfma %d src %s\n", t.dr_rows, t.th_rows, t.dph_rows, t.dph_par, t.th_plane, t.fuse, t.dph_mfma, src.c_str());
    t = sg::lookup_tuning(33, 32, 50, 0, &src);
    std::printf("33 (short line): %d %s\n", t.dr_rows, src.c_str());
    t = sg::lookup_tuning(25, 24, 50, 0, &src);
    std::printf("25 (out of range): %d %s\n", t.dr_rows, src.c_str());
    t = sg::lookup_tuning(17, 16, 50, 0, &src);
    std::printf("17 (long line): %d fuse %d %s\n", t.dr_rows, t.fuse, src.c_str());
    t = sg::lookup_tuning(65, 64, 58, 0, &src);
    std::printf("65: %d fuse %d %s\n", t.dph_rows, t.fuse, src.c_str());
    // expected: the full line, defaults for the short and out-of-range lines,
    // extra columns ignored, the line after a 2000-character one still read
    sg::Tune d;
    const bool ok = sg::lookup_tuning(49, 48, 50, 0, nullptr).dph_mfma == 1 &&
                    sg::lookup_tuning(33, 32, 50, 0, nullptr).dr_rows == d.dr_rows &&
                    sg::lookup_tuning(25, 24, 50, 0, nullptr).dr_rows == d.dr_rows &&
                    sg::lookup_tuning(17, 16, 50, 0, nullptr).dr_rows == 3 &&
                    sg::lookup_tuning(65, 64, 58, 0, nullptr).dph_rows == 16;
    std::printf(ok ? "ok\n" : "mismatch\n");
    return ok ? 0 : 1;
}
