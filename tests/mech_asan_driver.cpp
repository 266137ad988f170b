// Drives the library's host-side mechanism parser and packer
// (paper_2112_05834_amd/csrc/mech.cpp) under AddressSanitizer and
// UndefinedBehaviorSanitizer. TEST INFRASTRUCTURE ONLY.
//
// Usage: mech_asan_driver <file>... ; prints one line per file, "ok ns nr
// lds_bytes" or "error <message>". A sanitizer report stops it with a
// non-zero exit status; a file the parser rejects is not an error here.
#include <cstdio>
#include <string>

#include "mech.hpp"

int main(int argc, char** argv) {
  for (int i = 1; i < argc; ++i) {
    chem::MechHost m;
    std::string err;
    if (!chem::parse_mechanism(argv[i], m, err)) {
      std::printf("error %s\n", err.c_str());
      continue;
    }
    chem::Packed P = chem::pack(m);
    chem::Work w = chem::count_work(m);
    std::printf("ok %d %d %d %.0f\n", m.ns, m.nr, P.lds_bytes, w.f_rhs);
  }
  return 0;
}
