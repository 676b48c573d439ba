// Host execution of the library's calibration-gradient code (the per-hit,
// per-track and per-track-partials functions of tpcca_calib.hip, run on the
// CPU with exact-size buffers).  Used by tests/test_calib_host_exec.py; reads
// raw little-endian arrays from a directory and writes the per-sector
// gradient [36][66] followed by chi2 (float64).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <string>
#include <vector>

#include "../../paper_1712_09434_amd/csrc/tpcca_calib.hip"

using namespace tpcca;

template <class T> static std::vector<T> rd(const std::string& d, const char* name) {
  std::ifstream f(d + "/" + name, std::ios::binary | std::ios::ate);
  const size_t n = (size_t)f.tellg();
  f.seekg(0);
  std::vector<T> v(n / sizeof(T));
  f.read((char*)v.data(), (std::streamsize)n);
  return v;
}

int main(int argc, char** argv) {
  if (argc < 3) return 2;
  const std::string d = argv[1];
  const int K = std::atoi(argv[2]);
  auto hoff = rd<int32_t>(d, "hit_off");
  auto hid = rd<uint32_t>(d, "hit_id");
  auto kp = rd<float>(d, "k0");
  auto ext = rd<float>(d, "ext");
  auto uv = rd<uint8_t>(d, "uv");
  auto cx = rd<float>(d, "x");
  auto cy = rd<float>(d, "y");
  auto cz = rd<float>(d, "z");
  auto cs = rd<uint8_t>(d, "sec");
  auto th = rd<float>(d, "theta");
  auto rx = rd<float>(d, "row_x");
  CalWs c{};
  c.S = 36; c.R = (int)rx.size();
  c.geo = CalGeo{36, 250.0f, rx[0], rx[c.R - 1] - rx[0], (float)std::tan(10.0 * M_PI / 180.0)};
  c.m.kfac = -((float)2.99792458e-3) * 0.5f;
  c.m.sin_max = 0.99f; c.m.vy = 0.1f * 0.1f; c.m.vz = 0.15f * 0.15f;
  c.sv2 = 0.01f * 0.01f; c.st2 = 1e-3f * 1e-3f;
  c.K = K; c.nck = (c.R - 1 + K - 1) / K + 1; c.nseg = 2 * K + kTail;
  c.T = (int64_t)hoff.size() - 1; c.H = (int64_t)hid.size(); c.NC = (int64_t)cx.size();
  c.hit_off = hoff.data(); c.hit_id = hid.data(); c.k_prior = kp.data(); c.ext_tgl = ext.data();
  c.use_vertex = uv.data(); c.cx = cx.data(); c.cy = cy.data(); c.cz = cz.data(); c.csec = cs.data();
  c.dl = th.data(); c.tau = th.data() + 36; c.map = th.data() + 72;
  std::vector<float> hx(c.H), hy(c.H), hz(c.H), gx(c.H), gy(c.H), gz(c.H), gpt(c.H), dzt(c.H);
  std::vector<float4> bva(c.H), bvb(c.H);
  std::vector<int32_t> bsp(c.H);
  std::vector<float> part(c.T * kPart), ck(c.T * c.nck * 20), sg(c.T * c.nseg * 20);
  std::vector<int32_t> tf(c.T), tn(c.T);
  uint32_t err = 0;
  unsigned long long ndf = 0;
  c.hx = hx.data(); c.hy = hy.data(); c.hz = hz.data(); c.gx = gx.data(); c.gy = gy.data();
  c.gz = gz.data(); c.gpt = gpt.data(); c.part = part.data(); c.tflag = tf.data(); c.tndf = tn.data();
  c.bva = bva.data(); c.bvb = bvb.data(); c.bsp = bsp.data(); c.dzt = dzt.data();
  c.ckpt = ck.data(); c.seg = sg.data(); c.err = &err; c.ndf_sum = &ndf;
  for (int64_t j = 0; j < c.H; ++j) calib_hit(c, j);
  for (int64_t t = 0; t < c.T; ++t) adjoint_track(c, t);
  for (int64_t t = 0; t < c.T; ++t)
    for (int l = 0; l < 64; ++l) partials_lane(c, t, l);
  std::vector<double> g(36 * 66 + 1, 0.0);
  for (int64_t t = 0; t < c.T; ++t) {
    if (tf[t] <= 0) continue;
    const int s = cs[hid[hoff[t]]];
    for (int q = 0; q < 66; ++q) g[s * 66 + q] += part[t * kPart + q];
    g[36 * 66] += part[t * kPart + 66];
  }
  std::ofstream o(d + "/out_grad", std::ios::binary);
  o.write((const char*)g.data(), (std::streamsize)(g.size() * 8));
  std::printf("err %u\n", err);
  return err ? 1 : 0;
}
