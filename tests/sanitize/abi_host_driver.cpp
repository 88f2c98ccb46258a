// Host-side checks of libhybrid_raster built with AddressSanitizer and
// UndefinedBehaviorSanitizer: workspace planning, argument validation, loss
// sizes, autotune keys and the autotune cache file, all of which run without
// a GPU. Device pointers are never dereferenced by these paths, so aligned
// stand-in addresses are passed for them. Exits non-zero on the first failed
// expectation; the sanitizers abort on the first memory or UB error.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "hr.h"

namespace {

int g_checks = 0;

#define EXPECT(cond)                                                        \
  do {                                                                      \
    ++g_checks;                                                             \
    if (!(cond)) {                                                          \
      std::fprintf(stderr, "FAILED %s:%d: %s (last error: %s)\n", __FILE__, \
                   __LINE__, #cond, hr_last_error());                       \
      std::exit(1);                                                         \
    }                                                                       \
  } while (0)

template <class T>
const T* fake(uintptr_t a = 4096) { return reinterpret_cast<const T*>(a); }
template <class T>
T* fake_mut(uintptr_t a = 4096) { return reinterpret_cast<T*>(a); }

hr_gaussians gaussians(int32_t n, int32_t deg = 0) {
  hr_gaussians g;
  std::memset(&g, 0, sizeof g);
  g.n = n;
  g.sh_degree = deg;
  g.means = fake<float>();
  g.log_scales = fake<float>();
  g.quats = fake<float>();
  g.opacity_logits = fake<float>();
  g.sh = fake<float>();
  return g;
}

hr_mesh mesh(int32_t faces) {
  hr_mesh m;
  std::memset(&m, 0, sizeof m);
  if (faces) {
    m.n_verts = 4;
    m.n_faces = faces;
    m.n_tex = 1;
    m.tex_h = 8;
    m.tex_w = 8;
    m.verts = fake<float>();
    m.faces = fake<int32_t>();
    m.uvs = fake<float>();
    m.face_tex = fake<int32_t>();
    m.tex = fake<float>();
  }
  return m;
}

hr_camera camera(int32_t w, int32_t h, double f) {
  hr_camera c;
  std::memset(&c, 0, sizeof c);
  c.width = w;
  c.height = h;
  c.fx = c.fy = f;
  c.cx = w / 2.0;
  c.cy = h / 2.0;
  c.R[0] = c.R[4] = c.R[8] = 1.0;
  return c;
}

void workspace_planning() {
  hr_settings s = hr_default_settings();
  std::vector<hr_camera> cams = {camera(64, 48, 50.0)};
  size_t prev = 0;
  const int32_t ns[] = {0, 1, 10, 1000, 100000};
  for (int32_t n : ns) {
    hr_gaussians g = gaussians(n, 3);
    hr_mesh m = mesh(2);
    size_t b = hr_query_workspace(&g, &m, cams.data(), 1, &s, 1000);
    EXPECT(b > 0 && b >= prev);
    prev = b;
  }
  // uneven cameras, every flag combination the planner looks at
  std::vector<hr_camera> many;
  for (int i = 0; i < 16; ++i) many.push_back(camera(17 + 37 * i, 9 + 23 * i, 100.0 + i));
  for (uint32_t flags = 0; flags < 256; ++flags) {
    s = hr_default_settings();
    s.flags = flags;
    hr_gaussians g = gaussians(5000, flags & 3);
    hr_mesh m = mesh(flags & 1 ? 0 : 12);
    size_t b = hr_query_workspace(&g, &m, many.data(), 16, &s, 1 << 20);
    (void)b;  // some flag combinations are rejected; the planner must not misbehave
  }
  s = hr_default_settings();
  const int32_t batches[] = {32, 64, 128, 256};
  for (int32_t bt : batches)
    for (int32_t v = 0; v < 16; ++v) {
      s.batch = bt;
      s.variant = v;
      s.batch_bwd = bt;
      hr_gaussians g = gaussians(777, 1);
      hr_mesh m = mesh(0);
      (void)hr_query_workspace(&g, &m, many.data(), 16, &s, 12345);
    }
}

void invalid_arguments() {
  hr_settings s = hr_default_settings();
  hr_camera c = camera(64, 48, 50.0);
  hr_mesh m = mesh(0);
  hr_outputs out;
  std::memset(&out, 0, sizeof out);
  out.image = fake_mut<float>();
  struct Case {
    const char* what;
    void (*mutate)(hr_gaussians&, hr_mesh&, hr_settings&, hr_camera&);
  };
  const Case cases[] = {
      {"negative n", [](hr_gaussians& g, hr_mesh&, hr_settings&, hr_camera&) { g.n = -1; }},
      {"null means", [](hr_gaussians& g, hr_mesh&, hr_settings&, hr_camera&) { g.means = nullptr; }},
      {"misaligned quats",
       [](hr_gaussians& g, hr_mesh&, hr_settings&, hr_camera&) { g.quats = fake<float>(4100); }},
      {"sh degree", [](hr_gaussians& g, hr_mesh&, hr_settings&, hr_camera&) { g.sh_degree = 4; }},
      {"alpha_min", [](hr_gaussians&, hr_mesh&, hr_settings& s, hr_camera&) { s.alpha_min = 0.995f; }},
      {"t_min", [](hr_gaussians&, hr_mesh&, hr_settings& s, hr_camera&) { s.t_min = 0.0f; }},
      {"batch", [](hr_gaussians&, hr_mesh&, hr_settings& s, hr_camera&) { s.batch = 48; }},
      {"width", [](hr_gaussians&, hr_mesh&, hr_settings&, hr_camera& c) { c.width = 0; }},
      {"focal", [](hr_gaussians&, hr_mesh&, hr_settings&, hr_camera& c) { c.fx = -1.0; }},
      {"tiles",
       [](hr_gaussians&, hr_mesh&, hr_settings&, hr_camera& c) { c.width = c.height = 8000; }},
      {"mesh without texture",
       [](hr_gaussians&, hr_mesh& m, hr_settings&, hr_camera&) {
         m = mesh(2);
         m.tex = nullptr;
       }},
      {"negative faces", [](hr_gaussians&, hr_mesh& m, hr_settings&, hr_camera&) { m.n_faces = -3; }},
  };
  for (const Case& k : cases) {
    hr_gaussians g = gaussians(100);
    hr_mesh mm = m;
    hr_settings ss = s;
    hr_camera cc = c;
    k.mutate(g, mm, ss, cc);
    EXPECT(hr_query_workspace(&g, &mm, &cc, 1, &ss, 1000) == 0);
    EXPECT(std::strlen(hr_last_error()) > 0);
    hr_status rc = hr_render_hybrid(&g, &mm, &cc, 1, &ss, 1000, fake_mut<void>(), size_t(1) << 30,
                                    &out, nullptr);
    EXPECT(rc == HR_ERR_INVALID_ARGUMENT || rc == HR_ERR_UNSUPPORTED);
  }
  hr_gaussians g = gaussians(10);
  EXPECT(hr_query_workspace(&g, &m, &c, 1, &s, int64_t(1) << 32) == 0);
  EXPECT(hr_query_workspace(&g, &m, &c, 0, &s, 10) == 0);
  EXPECT(hr_query_workspace(nullptr, &m, &c, 1, &s, 10) == 0);
  EXPECT(hr_query_workspace(&g, &m, nullptr, 1, &s, 10) == 0);
  // a workspace smaller than the plan is refused before any launch
  size_t need = hr_query_workspace(&g, &m, &c, 1, &s, 1000);
  EXPECT(need > 0);
  EXPECT(hr_render_hybrid(&g, &m, &c, 1, &s, 1000, fake_mut<void>(), need - 1, &out, nullptr) ==
         HR_ERR_INVALID_ARGUMENT);
}

void loss_sizes() {
  const int32_t sz[] = {37, 29, 64, 48};
  size_t nb = hr_loss_scratch_bytes(sz, 2);
  EXPECT(nb > 0);
  EXPECT(hr_full_loss_scratch_bytes(sz, 2) > 0);
  const int32_t zero[] = {0, 5};
  EXPECT(hr_loss_scratch_bytes(zero, 1) == 0);
  EXPECT(hr_loss_scratch_bytes(sz, 0) == 0);
  EXPECT(hr_loss_scratch_bytes(nullptr, 1) == 0);
  EXPECT(hr_full_loss_scratch_bytes(zero, 1) == 0);
  const int32_t huge[] = {1 << 30, 1 << 30};
  EXPECT(hr_loss_scratch_bytes(huge, 1) == 0);
  std::vector<int32_t> many(2 * 300);
  for (size_t i = 0; i < many.size(); ++i) many[i] = 1 + int32_t(i % 97);
  EXPECT(hr_loss_scratch_bytes(many.data(), 300) > 0);
  const int32_t neg[] = {5, -1};
  float* d = fake_mut<float>();
  EXPECT(hr_hybrid_loss(d, d, d, fake<int32_t>(), d, neg, 1, 0.1f, 20.f, 0, d, d, d, d,
                        fake_mut<void>(), nullptr) == HR_ERR_INVALID_ARGUMENT);
  EXPECT(hr_hybrid_loss(d, nullptr, d, fake<int32_t>(), d, sz, 2, 0.1f, 20.f, 0, d, d, d, d,
                        fake_mut<void>(), nullptr) == HR_ERR_INVALID_ARGUMENT);
  // more images than the static scratch holds
  EXPECT(hr_hybrid_loss_noalloc(d, d, d, fake<int32_t>(), d, many.data(), 300, 0.1f, 20.f, 0, d,
                                d, d, d, nullptr) == HR_ERR_INVALID_ARGUMENT);
  EXPECT(hr_batch_status(nullptr, nullptr, nullptr) == HR_ERR_INVALID_ARGUMENT);
  {  // the timed backward checks its arguments before any launch
    hr_settings s = hr_default_settings();
    hr_camera c = camera(64, 48, 50.0);
    hr_gaussians g = gaussians(10);
    hr_mesh m = mesh(0);
    hr_grads gr;
    std::memset(&gr, 0, sizeof gr);
    float st[HR_N_BWD_STAGES];
    EXPECT(hr_render_hybrid_backward_timed(&g, &m, &c, 1, &s, 100, fake_mut<void>(), 1 << 20, d,
                                           nullptr, nullptr, &gr, nullptr, 1,
                                           nullptr) == HR_ERR_INVALID_ARGUMENT);
    EXPECT(hr_render_hybrid_backward_timed(&g, &m, &c, 1, &s, 100, fake_mut<void>(), 16, d,
                                           nullptr, nullptr, &gr, nullptr, 1,
                                           st) == HR_ERR_INVALID_ARGUMENT);
  }
}

void autotune_keys() {
  hr_settings s = hr_default_settings();
  hr_camera c = camera(1920, 1080, 1000.0);
  hr_gaussians g = gaussians(600000, 3);
  hr_mesh m = mesh(2);
  size_t need = hr_autotune_key("gfx950", 256, &g, &m, &c, 1, &s, 0, nullptr, 0);
  EXPECT(need > 1);
  std::vector<char> buf(need);
  EXPECT(hr_autotune_key("gfx950", 256, &g, &m, &c, 1, &s, 0, buf.data(), need) == need);
  EXPECT(std::string(buf.data()).rfind("fwd|gfx950|", 0) == 0);
  for (size_t cap = 1; cap < need; ++cap) {  // every truncation stays inside the buffer
    std::vector<char> small(cap, 'x');
    EXPECT(hr_autotune_key("gfx950", 256, &g, &m, &c, 1, &s, 1, small.data(), cap) > cap);
    EXPECT(std::strlen(small.data()) == cap - 1);
  }
  // an over-long architecture name gives a truncated key, not an overrun
  std::string long_arch(5000, 'a');
  const size_t nl = hr_autotune_key(long_arch.c_str(), 1 << 30, &g, &m, &c, 1, &s, 0, nullptr, 0);
  EXPECT(nl > 1 && nl <= 256);
  EXPECT(hr_autotune_key(nullptr, 256, &g, &m, &c, 1, &s, 0, nullptr, 0) == 0);
}

void write_file(const std::string& path, const std::string& text) {
  FILE* f = std::fopen(path.c_str(), "wb");
  EXPECT(f != nullptr);
  std::fwrite(text.data(), 1, text.size(), f);
  std::fclose(f);
}

void autotune_cache(const std::string& dir) {
  const std::string path = dir + "/tune.json";
  int32_t b = 0, v = 0;
  std::remove(path.c_str());
  EXPECT(hr_autotune_cache_lookup(path.c_str(), "fwd|x", &b, &v) == 0);
  EXPECT(hr_autotune_cache_store(path.c_str(), "fwd|gfx950|a", 256, 0) == HR_OK);
  EXPECT(hr_autotune_cache_store(path.c_str(), "bwd|gfx950|a", 128, 8) == HR_OK);
  EXPECT(hr_autotune_cache_store(path.c_str(), "fwd|gfx950|a", 128, 1) == HR_OK);
  EXPECT(hr_autotune_cache_lookup(path.c_str(), "fwd|gfx950|a", &b, &v) == 1);
  EXPECT(b == 128 && v == 1);
  for (int i = 0; i < 200; ++i) {
    std::string key = "fwd|k" + std::to_string(i) + std::string(size_t(i) * 7, 'z');
    EXPECT(hr_autotune_cache_store(path.c_str(), key.c_str(), 32 << (i % 4), i % 16) == HR_OK);
  }
  EXPECT(hr_autotune_cache_lookup(path.c_str(), "bwd|gfx950|a", &b, &v) == 1);
  EXPECT(b == 128 && v == 8);
  EXPECT(hr_autotune_cache_store(path.c_str(), "other|x", 1, 1) == HR_ERR_INVALID_ARGUMENT);
  EXPECT(hr_autotune_cache_store(path.c_str(), "fwd|\"x", 1, 1) == HR_ERR_INVALID_ARGUMENT);
  EXPECT(hr_autotune_cache_store(nullptr, "fwd|x", 1, 1) == HR_ERR_INVALID_ARGUMENT);
  EXPECT(hr_autotune_cache_store((dir + "/no_such_dir/t.json").c_str(), "fwd|x", 1, 1) ==
         HR_ERR_INTERNAL);
  // damaged or foreign files: the lookup reports a miss and never reads past the text
  const char* bad[] = {
      "",
      "{",
      "{\"hr_autotune_cache\": 1, \"entries\": {\"fwd|a\": [",
      "{\"hr_autotune_cache\": 1, \"entries\": {\"fwd|a\": [64",
      "{\"hr_autotune_cache\": 1, \"entries\": {\"fwd|a\": [64, ]}}",
      "{\"hr_autotune_cache\": 1, \"entries\": {\"fwd|a\": [99999999999999999999, 1]}}",
      "\"fwd|a\": [64, 1]\n\"fwd|a\"",
      "{\"entries\": {\"fwd|a\": \"text\"}}",
      "\n\n\n\"\n\"\"\n[[[[",
  };
  for (const char* text : bad) {
    write_file(path, text);
    b = v = -7;
    int32_t hit = hr_autotune_cache_lookup(path.c_str(), "fwd|b", &b, &v);
    EXPECT(hit == 0);
    (void)hr_autotune_cache_lookup(path.c_str(), "fwd|a", &b, &v);
    // a store over a damaged file rewrites it whole
    EXPECT(hr_autotune_cache_store(path.c_str(), "fwd|b", 64, 2) == HR_OK);
    EXPECT(hr_autotune_cache_lookup(path.c_str(), "fwd|b", &b, &v) == 1);
    EXPECT(b == 64 && v == 2);
  }
  std::remove(path.c_str());
}

void status_strings() {
  const hr_status all[] = {HR_OK, HR_ERR_INVALID_ARGUMENT, HR_ERR_CAPACITY, HR_ERR_HIP,
                           HR_ERR_UNSUPPORTED, HR_ERR_INTERNAL};
  for (hr_status s : all) EXPECT(hr_status_string(s) != nullptr && *hr_status_string(s));
  EXPECT(hr_abi_version() == HR_ABI_VERSION);
}

}  // namespace

int main(int argc, char** argv) {
  const std::string dir = argc > 1 ? argv[1] : ".";
  workspace_planning();
  invalid_arguments();
  loss_sizes();
  autotune_keys();
  autotune_cache(dir);
  status_strings();
  std::printf("abi host driver: %d checks passed\n", g_checks);
  return 0;
}
