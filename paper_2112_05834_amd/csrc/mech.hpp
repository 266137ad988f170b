// Host-side mechanism: parser, validation, and the packed images the kernels
// read (an LDS image staged by every block, plus global thermo tables).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace chem {

constexpr int kMaxSide = 3;        // distinct species per reaction side on the device
constexpr int kMaxSpecies = 255;   // species index fits in a byte of the reaction word
constexpr int kMaxReactions = 4095;

struct Rxn {
  int type = 0;   // 0 elementary, 1 third body, 2 Troe falloff
  int rev = 1;
  std::vector<std::pair<int, int>> reac, prod;   // (species, order), distinct species
  double A = 0, b = 0, Ea = 0;
  std::vector<std::pair<int, double>> eff;        // (species, alpha)
  double A0 = 0, b0 = 0, Ea0 = 0, ta = 0, T3 = 1, T1 = 1, T2 = 0;
  bool has_T2 = false;
};

struct MechHost {
  int ns = 0, nr = 0, ne = 0;
  std::vector<int> elem;                 // [ns][ne] atoms of each element per molecule
  std::vector<double> W;                 // kg/mol
  std::vector<double> tmid;              // NASA range boundary per species
  std::vector<double> lo, hi;            // [ns][7]
  std::vector<Rxn> rx;
};

// Parse the text format; on failure returns false with a message.
bool parse_mechanism(const std::string& path, MechHost& m, std::string& err);

// Algorithmic work per right-hand side and per Jacobian (beyond its RHS).
struct Work { double f_rhs, f_jac, t_rhs, t_jac; };
Work count_work(const MechHost& m);

// Packed image. The LDS blob is a byte array whose sections start at the
// offsets below (all 16-byte aligned); the kernel copies it into LDS verbatim.
struct Packed {
  std::vector<uint8_t> blob;
  int off_lnA, off_b, off_EaR, off_rint, off_troe, off_eff_sp, off_eff_am1, off_sp_off, off_sp_ent,
      off_rW;
  int lds_bytes;    // leading part of blob staged in LDS
  int ntroe, neff, nent;
  std::vector<double> nasa;   // [ns][16]: lo a1..a7, tmid, hi a1..a7, 0
  std::vector<double> W, rW;  // [ns]
};
Packed pack(const MechHost& m);

}  // namespace chem
