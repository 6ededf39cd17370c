// Autotuner cache of the batched kernels' tile choices (JSON file optional).
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>

#include "internal.h"

namespace rb {

const TuneConfig* Tuner::find(const std::string& key) const {
  for (const auto& kv : table)
    if (kv.first == key) return &kv.second;
  return nullptr;
}

void Tuner::put(const std::string& key, const TuneConfig& c) {
  for (auto& kv : table)
    if (kv.first == key) {
      kv.second = c;
      return;
    }
  table.push_back({key, c});
}

// File format: one JSON object,
// {"key": [qpb_a, qpb_b, qpb_gs, proj_target, kind_a, kind_b, kind_gs, kind_pro, zn_a,
// zn_b, np_gs, nb_b, nb_a], ...} (the last nine optional)
void Tuner::load() {
  if (loaded) return;
  loaded = true;
  const char* p = std::getenv("RB_AUTOTUNE_CACHE");
  if (!p || !*p) return;
  path = p;
  std::ifstream f(path);
  if (!f) return;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string t = ss.str();
  size_t i = 0;
  while (true) {
    const size_t a = t.find('"', i);
    if (a == std::string::npos) break;
    const size_t b = t.find('"', a + 1);
    const size_t l = t.find('[', b);
    const size_t r = t.find(']', l);
    if (b == std::string::npos || l == std::string::npos || r == std::string::npos) break;
    TuneConfig c;
    const int got =
        std::sscanf(t.c_str() + l + 1,
                    "%d , %d , %d , %d , %d , %d , %d , %d , %d , %d , %d , %d , %d",
                    &c.qpb_a, &c.qpb_b, &c.qpb_gs, &c.proj_target, &c.kind_a, &c.kind_b,
                    &c.kind_gs, &c.kind_pro, &c.zn_a, &c.zn_b, &c.np_gs, &c.nb_b, &c.nb_a);
    if (got == 4 || got == 6 || got == 7 || got == 8 || got == 10 || got == 11 || got == 12 ||
        got == 13)
      put(t.substr(a + 1, b - a - 1), c);
    i = r + 1;
  }
}

void Tuner::save() const {
  if (path.empty()) return;
  std::ofstream f(path);
  if (!f) return;
  f << "{\n";
  for (size_t i = 0; i < table.size(); ++i) {
    const TuneConfig& c = table[i].second;
    f << "  \"" << table[i].first << "\": [" << c.qpb_a << ", " << c.qpb_b << ", " << c.qpb_gs
      << ", " << c.proj_target << ", " << c.kind_a << ", " << c.kind_b << ", " << c.kind_gs
      << ", " << c.kind_pro << ", " << c.zn_a << ", " << c.zn_b << ", " << c.np_gs << ", "
      << c.nb_b << ", " << c.nb_a << "]"
      << (i + 1 < table.size() ? "," : "") << "\n";
  }
  f << "}\n";
}

}  // namespace rb
