// Mechanism parser and packer for the GPU library (independent of any other
// parser of the same file format).
#include "mech.hpp"

#include <algorithm>
#include <cerrno>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>

namespace chem {

namespace {

struct Tok {
  std::vector<std::string> t;
  size_t i = 0;
  bool next(std::string& s) {
    if (i >= t.size()) return false;
    s = t[i++];
    return true;
  }
  bool integer(int& v) {
    std::string s;
    if (!next(s)) return false;
    char* e = nullptr;
    errno = 0;
    long x = std::strtol(s.c_str(), &e, 10);
    if (*e || errno == ERANGE || x < INT_MIN || x > INT_MAX) return false;
    v = static_cast<int>(x);
    return true;
  }
  bool real(double& v) {
    std::string s;
    if (!next(s)) return false;
    char* e = nullptr;
    v = std::strtod(s.c_str(), &e);
    return *e == 0 && std::isfinite(v);
  }
  bool word(const char* w) {
    std::string s;
    return next(s) && s == w;
  }
};

// merge repeated species of one side into orders
bool side(Tok& tk, int ns, std::vector<std::pair<int, int>>& out) {
  int k;
  if (!tk.integer(k) || k < 1 || k > 8) return false;
  std::map<int, int> acc;
  std::vector<int> order;
  for (int j = 0; j < k; ++j) {
    int s, o;
    // an order above 3 is rejected here, so that merged orders stay small
    if (!tk.integer(s) || !tk.integer(o) || s < 0 || s >= ns || o < 1 || o > 3) return false;
    if (!acc.count(s)) order.push_back(s);
    acc[s] += o;
  }
  out.clear();
  for (int s : order) out.emplace_back(s, acc[s]);
  return true;
}

}  // namespace

bool parse_mechanism(const std::string& path, MechHost& m, std::string& err) {
  std::ifstream f(path);
  if (!f) {
    err = "cannot open mechanism file '" + path + "'";
    return false;
  }
  Tok tk;
  std::string line;
  while (std::getline(f, line)) {
    auto h = line.find('#');
    if (h != std::string::npos) line.resize(h);
    std::istringstream ss(line);
    std::string w;
    while (ss >> w) tk.t.push_back(w);
  }
  auto fail = [&](const std::string& what) {
    err = "mechanism '" + path + "': " + what + " near token " + std::to_string(tk.i);
    return false;
  };
  int ver, ne;
  if (!tk.word("chemmech") || !tk.integer(ver) || ver != 1) return fail("bad header");
  if (!tk.word("elements") || !tk.integer(ne) || ne < 1) return fail("bad elements count");
  for (int e = 0; e < ne; ++e) {
    std::string name;
    double w;
    if (!tk.next(name) || !tk.real(w)) return fail("bad element line");
  }
  if (!tk.word("species") || !tk.integer(m.ns) || m.ns < 1) return fail("bad species count");
  if (m.ns > kMaxSpecies) return fail("more than 255 species");
  m.ne = ne;
  m.elem.assign(static_cast<size_t>(m.ns) * ne, 0);
  m.W.resize(m.ns);
  m.tmid.resize(m.ns);
  m.lo.resize(7 * m.ns);
  m.hi.resize(7 * m.ns);
  for (int i = 0; i < m.ns; ++i) {
    std::string name;
    double tl, th;
    int c;
    if (!tk.next(name) || !tk.real(m.W[i]) || !tk.real(tl) || !tk.real(m.tmid[i]) || !tk.real(th))
      return fail("bad species line");
    if (!(m.W[i] > 0)) return fail("non-positive molecular weight");
    for (int e = 0; e < ne; ++e) {
      if (!tk.integer(c) || c < 0) return fail("bad element count");
      m.elem[static_cast<size_t>(i) * ne + e] = c;
    }
    for (int k = 0; k < 7; ++k)
      if (!tk.real(m.lo[7 * i + k])) return fail("bad NASA coefficient");
    for (int k = 0; k < 7; ++k)
      if (!tk.real(m.hi[7 * i + k])) return fail("bad NASA coefficient");
  }
  if (!tk.word("reactions") || !tk.integer(m.nr) || m.nr < 0) return fail("bad reactions count");
  if (m.nr > kMaxReactions) return fail("more than 4095 reactions");
  m.rx.resize(m.nr);
  for (int r = 0; r < m.nr; ++r) {
    Rxn& x = m.rx[r];
    if (!tk.word("reaction") || !tk.integer(x.type) || !tk.integer(x.rev)) return fail("bad reaction");
    if (x.type < 0 || x.type > 2) return fail("bad reaction type");
    if (!side(tk, m.ns, x.reac) || !side(tk, m.ns, x.prod)) return fail("bad reaction side");
    if (x.reac.size() > kMaxSide || x.prod.size() > kMaxSide)
      return fail("more than 3 distinct species on a reaction side");
    for (auto& p : x.reac) if (p.second > 3) return fail("reaction order of a species above 3 is not supported");
    for (auto& p : x.prod) if (p.second > 3) return fail("reaction order of a species above 3 is not supported");
    if (!tk.real(x.A) || !tk.real(x.b) || !tk.real(x.Ea)) return fail("bad Arrhenius parameters");
    if (!(x.A > 0)) return fail("non-positive pre-exponential factor");
    if (x.type >= 1) {
      int k;
      if (!tk.word("eff") || !tk.integer(k) || k < 0 || k > m.ns) return fail("bad efficiency list");
      std::map<int, double> seen;
      for (int j = 0; j < k; ++j) {
        int s;
        double a;
        if (!tk.integer(s) || !tk.real(a) || s < 0 || s >= m.ns) return fail("bad efficiency entry");
        seen[s] = a;   // a later entry for the same species wins
      }
      for (auto& p : seen) x.eff.emplace_back(p.first, p.second);
    }
    if (x.type == 2) {
      double h2;
      if (!tk.word("troe") || !tk.real(x.A0) || !tk.real(x.b0) || !tk.real(x.Ea0) || !tk.real(x.ta) ||
          !tk.real(x.T3) || !tk.real(x.T1) || !tk.real(x.T2) || !tk.real(h2))
        return fail("bad Troe parameters");
      x.has_T2 = h2 != 0.0;
      if (!(x.A0 > 0) || !(x.T3 > 0) || !(x.T1 > 0)) return fail("bad Troe values");
    }
  }
  if (!tk.word("end")) return fail("missing 'end'");
  return true;
}

Work count_work(const MechHost& m) {
  // Counted: each +, -, *, / and each half of an fma; transcendentals apart.
  const double ns = m.ns, n = m.ns + 1;
  double f = 0, t = 0, fj = 0, tj = 0;
  // mixture state and thermo (per species: cp 8, h 11, s 9, g 1) + sums
  f += 7 * ns + 6 + 29 * ns;
  t += 1;   // ln T
  size_t entries = 0;
  for (const Rxn& x : m.rx) {
    f += 5;  t += 1;                          // kf
    int part = 0, ord = 0;
    for (auto& p : x.reac) { part++; ord += p.second; }
    for (auto& p : x.prod) { part++; ord += p.second; }
    if (x.rev) { f += 2 * part + 4; t += 1; }  // sum nu g, kr
    f += ord + 3;                             // mass action products, q0
    if (x.type >= 1) f += 2 * x.eff.size() + 2;
    if (x.type == 2) { f += 32; t += 6; }
    entries += part;
    // Jacobian extras: dln k/dT, dq/dT, dtheta
    fj += 10 + 2 * part;
    if (x.type == 2) fj += 40;
    // per (row species, reaction): derivative of each participant + efficiencies
    fj += part * (part * 5 + (x.type >= 1 ? 2 * x.eff.size() + 2 : 0));
  }
  f += 2 * entries;        // omega gather
  f += 4 * ns + 5;         // f_Y, Q, f_T
  fj += 6 * ns;            // dcp, sums
  fj += 2 * ns * ns;       // s_i = sum_k D_ik C_k
  fj += 4 * ns * ns;       // species rows of J
  fj += 3 * ns * ns;       // column sums for the T row
  fj += 8 * n + 10;        // T row / column
  Work w{f, fj, t, tj};
  return w;
}

Packed pack(const MechHost& m) {
  Packed P;
  const int ns = m.ns, nr = m.nr;
  auto align16 = [](size_t x) { return (x + 15) & ~size_t(15); };
  std::vector<double> lnA(nr), bb(nr), EaR(nr);
  std::vector<uint32_t> rint(4 * nr, 0);
  std::vector<double> troe;
  std::vector<uint16_t> eff_sp;
  std::vector<double> eff_am1;
  const double R = 8.314462618;
  // Reactions are stored grouped by type (elementary, third body, Troe) so
  // that the lanes of one batch take the same branch; species sums keep the
  // original reaction order.
  std::vector<int> order(nr), newpos(nr);
  for (int r = 0; r < nr; ++r) order[r] = r;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return m.rx[a].type < m.rx[b].type; });
  for (int q = 0; q < nr; ++q) newpos[order[q]] = q;
  for (int q = 0; q < nr; ++q) {
    const int r = q;                 // slot in the packed arrays
    const Rxn& x = m.rx[order[q]];
    lnA[r] = std::log(x.A);
    bb[r] = x.b;
    EaR[r] = x.Ea / R;
    uint32_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;
    int dnu = 0;
    for (size_t j = 0; j < kMaxSide; ++j) {
      uint32_t s = j < x.reac.size() ? x.reac[j].first : 255u;
      uint32_t o = j < x.reac.size() ? x.reac[j].second : 0u;
      w0 |= s << (8 * j);
      w2 |= o << (4 * j);
      if (j < x.reac.size()) dnu -= x.reac[j].second;
    }
    for (size_t j = 0; j < kMaxSide; ++j) {
      uint32_t s = j < x.prod.size() ? x.prod[j].first : 255u;
      uint32_t o = j < x.prod.size() ? x.prod[j].second : 0u;
      w1 |= s << (8 * j);
      w2 |= o << (12 + 4 * j);
      if (j < x.prod.size()) dnu += x.prod[j].second;
    }
    // bit 31: a species on both sides (catalytic); its Jacobian updates then
    // cannot be issued as one batch of distinct columns
    bool overlap = false;
    for (auto& a : x.reac)
      for (auto& b : x.prod)
        if (a.first == b.first) overlap = true;
    w0 |= uint32_t(x.reac.size()) << 24 | uint32_t(x.type) << 28 | uint32_t(x.rev ? 1 : 0) << 30 |
          uint32_t(overlap ? 1 : 0) << 31;
    w1 |= uint32_t(x.prod.size()) << 24;
    w2 |= uint32_t((dnu + 64) & 0x7f) << 24;
    uint32_t troe_slot = 0;
    if (x.type == 2) {
      troe_slot = static_cast<uint32_t>(troe.size() / 8);
      troe.push_back(std::log(x.A0));
      troe.push_back(x.b0);
      troe.push_back(x.Ea0 / R);
      troe.push_back(x.ta);
      troe.push_back(1.0 / x.T3);
      troe.push_back(1.0 / x.T1);
      troe.push_back(x.T2);
      troe.push_back(x.has_T2 ? 1.0 : 0.0);
    }
    uint32_t eoff = static_cast<uint32_t>(eff_sp.size());
    for (auto& e : x.eff) {
      if (e.second == 1.0) continue;
      eff_sp.push_back(static_cast<uint16_t>(e.first));
      eff_am1.push_back(e.second - 1.0);
    }
    uint32_t neff = static_cast<uint32_t>(eff_sp.size()) - eoff;
    w3 = (eoff & 0xffff) | (neff & 0xff) << 16 | (troe_slot & 0xff) << 24;
    rint[4 * r + 0] = w0;
    rint[4 * r + 1] = w1;
    rint[4 * r + 2] = w2;
    rint[4 * r + 3] = w3;
  }
  // species -> (reaction, net stoichiometric coefficient) lists
  std::vector<std::vector<std::pair<int, int>>> per(ns);
  for (int r = 0; r < nr; ++r) {
    std::map<int, int> nu;
    for (auto& p : m.rx[r].reac) nu[p.first] -= p.second;
    for (auto& p : m.rx[r].prod) nu[p.first] += p.second;
    for (auto& q : nu)
      if (q.second != 0) per[q.first].emplace_back(newpos[r], q.second);
  }
  std::vector<uint16_t> sp_off(ns + 1, 0), sp_ent;
  for (int s = 0; s < ns; ++s) {
    sp_off[s] = static_cast<uint16_t>(sp_ent.size());
    for (auto& e : per[s]) sp_ent.push_back(static_cast<uint16_t>(e.first | ((e.second + 8) & 0xf) << 12));
  }
  sp_off[ns] = static_cast<uint16_t>(sp_ent.size());

  // Sections read at random by the species pass are staged in LDS (the
  // prefix of lds_bytes); the Arrhenius and Troe parameters, read once per
  // reaction by consecutive lanes, stay in global memory after it.
  size_t off = 0;
  auto place = [&](size_t bytes) { size_t o = off; off = align16(off + bytes); return static_cast<int>(o); };
  P.off_rint = place(16 * nr);
  P.off_eff_am1 = place(8 * eff_am1.size());
  P.off_eff_sp = place(2 * eff_sp.size());
  P.off_sp_off = place(2 * sp_off.size());
  P.off_sp_ent = place(2 * sp_ent.size());
  // rW is zero-padded to 64 entries, so that loops over the columns of a
  // padded state size may read it without a bound check
  P.off_rW = place(8 * std::max(ns, 64));
  P.lds_bytes = static_cast<int>(align16(off));
  P.off_lnA = place(8 * nr);
  P.off_b = place(8 * nr);
  P.off_EaR = place(8 * nr);
  P.off_troe = place(8 * troe.size());
  P.blob.assign(align16(off), 0);
  auto put = [&](int o, const void* src, size_t bytes) { if (bytes) std::memcpy(P.blob.data() + o, src, bytes); };
  put(P.off_lnA, lnA.data(), 8 * nr);
  put(P.off_b, bb.data(), 8 * nr);
  put(P.off_EaR, EaR.data(), 8 * nr);
  put(P.off_rint, rint.data(), 16 * nr);
  put(P.off_troe, troe.data(), 8 * troe.size());
  put(P.off_eff_am1, eff_am1.data(), 8 * eff_am1.size());
  put(P.off_eff_sp, eff_sp.data(), 2 * eff_sp.size());
  put(P.off_sp_off, sp_off.data(), 2 * sp_off.size());
  put(P.off_sp_ent, sp_ent.data(), 2 * sp_ent.size());
  std::vector<double> rW(ns);
  for (int s = 0; s < ns; ++s) rW[s] = 1.0 / m.W[s];
  put(P.off_rW, rW.data(), 8 * ns);
  P.ntroe = static_cast<int>(troe.size() / 8);
  P.neff = static_cast<int>(eff_sp.size());
  P.nent = static_cast<int>(sp_ent.size());
  P.nasa.assign(16 * ns, 0.0);
  P.W.resize(ns);
  P.rW.resize(ns);
  for (int s = 0; s < ns; ++s) {
    for (int k = 0; k < 7; ++k) {
      P.nasa[16 * s + k] = m.lo[7 * s + k];
      P.nasa[16 * s + 8 + k] = m.hi[7 * s + k];
    }
    P.nasa[16 * s + 7] = m.tmid[s];
    P.W[s] = m.W[s];
    P.rW[s] = 1.0 / m.W[s];
  }
  return P;
}

}  // namespace chem
