// Split-CTMRG on the GPU: left move (Sec. II B, Eqs. splitCTMRG_C1/C4/Tket/
// Tbra), projectors (Fig. proj_plots_green, App. A), the other moves by
// lattice symmetry, the nearest-neighbour energy, reverse-mode gradient with
// checkpointed sweeps, and the C ABI of include/splitctm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/splitctm.h"
#include "adj_kernels.hpp"
#include "engine.hpp"

using namespace sctm;

namespace {

enum { C1, C2, C3, C4, T1k, T1b, T2k, T2b, T3b, T3k, T4b, T4k, NT };

struct Site {
  Ten t[NT];
};

struct Env {
  int Lx = 0, Ly = 0;
  std::vector<Site> s;
  Site& at(int x, int y) { return s[(size_t)(((x % Lx) + Lx) % Lx) * Ly + (((y % Ly) + Ly) % Ly)]; }
  const Site& at(int x, int y) const {
    return s[(size_t)(((x % Lx) + Lx) % Lx) * Ly + (((y % Ly) + Ly) % Ly)];
  }
};

struct Peps {
  int Lx = 0, Ly = 0;
  std::vector<Ten> a;
  const Ten& at(int x, int y) const { return a[(size_t)(((x % Lx) + Lx) % Lx) * Ly + (((y % Ly) + Ly) % Ly)]; }
};

}  // namespace

struct ctm_ctx {
  ctm_config cfg{};
  Engine E;
  int chiE = 0, chiI = 0, D = 0, p = 0, Lx = 0, Ly = 0;
  Ten A64;                 // FP64 master copy [Lx Ly p D D D D]
  Ten Aflat;               // contraction-dtype copy, same layout
  Ten cur_blk, start_blk;  // environments in the packed layout (contraction dtype)
  Ten spec_prev;           // FP64 corner spectra [Lx Ly 4][chiE]
  Ten h64;                 // FP64 [p^2][p^2], horizontal bonds
  Ten h64v;                // FP64 [p^2][p^2], vertical bonds
  size_t transient_mark = 0;
  int host_flags[256];
  bool spec_current = false;   // spec_prev holds the spectra of the current environment
  double last_flops = 0, last_sweeps = 0;
  bool timing = false;     // HIP-event timing of the GEMM and Jacobi launches
  KernelTimer timer;
  int static_device = -1;  // >= 0: the workspace is that device's static scratch array
};

// ---------------------------------------------------------------------------
// Static device scratch for callers that cannot allocate (ctm_init_static).
// Each GPU the library runs on holds its own copy for the life of the process.
// In host code `scratch` is only a handle: its device address is looked up
// once per device with hipGetSymbolAddress and kept in static_ptr.
// ---------------------------------------------------------------------------
static constexpr size_t kStaticScratchBytes = CTM_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex static_mu;
void* static_ptr[kMaxDevices] = {};
bool static_busy[kMaxDevices] = {};
}  // namespace

namespace {

// ---------------------------------------------------------------------------
// layout helpers
// ---------------------------------------------------------------------------
void site_shapes(const ctm_ctx& c, long shp[NT][3], int rk[NT]) {
  for (int i = C1; i <= C4; ++i) {
    rk[i] = 2;
    shp[i][0] = c.chiE;
    shp[i][1] = c.chiE;
  }
  const int first[4] = {T1k, T2k, T3b, T4b}, second[4] = {T1b, T2b, T3k, T4k};
  for (int i = 0; i < 4; ++i) {
    rk[first[i]] = rk[second[i]] = 3;
    shp[first[i]][0] = c.chiE;
    shp[first[i]][1] = c.D;
    shp[first[i]][2] = c.chiI;
    shp[second[i]][0] = c.chiI;
    shp[second[i]][1] = c.D;
    shp[second[i]][2] = c.chiE;
  }
}

long site_elems(const ctm_ctx& c) {
  long shp[NT][3];
  int rk[NT];
  site_shapes(c, shp, rk);
  long n = 0;
  for (int i = 0; i < NT; ++i) {
    long k = 1;
    for (int j = 0; j < rk[i]; ++j) k *= shp[i][j];
    n += k;
  }
  return n;
}

// Views of a packed environment block as per-site tensors (no copies).
Env view_env(ctm_ctx& c, const Ten& blk) {
  Env e;
  e.Lx = c.Lx;
  e.Ly = c.Ly;
  e.s.resize((size_t)c.Lx * c.Ly);
  long shp[NT][3];
  int rk[NT];
  site_shapes(c, shp, rk);
  size_t off = 0;
  for (int x = 0; x < c.Lx; ++x)
    for (int y = 0; y < c.Ly; ++y)
      for (int i = 0; i < NT; ++i) {
        Ten t;
        t.dt = blk.dt;
        t.r = rk[i];
        for (int j = 0; j < rk[i]; ++j) t.d[j] = shp[i][j];
        t.p = (char*)blk.p + off * blk.esize();
        t.id = c.E.next_id++;
        off += t.n();
        e.at(x, y).t[i] = t;
      }
  return e;
}

// Copy tensors of an environment into a packed block (untaped).
void store_env(ctm_ctx& c, const Env& src, const Ten& blk) {
  Env dst = view_env(c, blk);
  Engine& E = c.E;
  if (E.dry || !E.ok()) return;
  for (size_t k = 0; k < src.s.size(); ++k)
    for (int i = 0; i < NT; ++i)
      E.check(hipMemcpyAsync(dst.s[k].t[i].p, src.s[k].t[i].p, src.s[k].t[i].bytes(), hipMemcpyDeviceToDevice, E.s));
}

// Fresh arena copies of a packed block, registered as inputs needing grads.
Env load_env(ctm_ctx& c, const Ten& blk, bool as_input) {
  Env v = view_env(c, blk);
  Env e = v;
  Engine& E = c.E;
  for (auto& st : e.s)
    for (int i = 0; i < NT; ++i) {
      Ten src = st.t[i];
      Ten t = E.alloc_like(src);
      if (!E.dry && E.ok()) E.check(hipMemcpyAsync(t.p, src.p, src.bytes(), hipMemcpyDeviceToDevice, E.s));
      st.t[i] = t;
      if (as_input) E.mark_input(t);
    }
  return e;
}

Peps peps_view(ctm_ctx& c, const Ten& flat) {
  Peps P;
  P.Lx = c.Lx;
  P.Ly = c.Ly;
  long per = (long)c.p * c.D * c.D * c.D * c.D;
  for (int x = 0; x < c.Lx; ++x)
    for (int y = 0; y < c.Ly; ++y) {
      Ten t;
      t.dt = flat.dt;
      t.r = 5;
      t.d[0] = c.p;
      t.d[1] = t.d[2] = t.d[3] = t.d[4] = c.D;
      t.p = (char*)flat.p + (size_t)(x * c.Ly + y) * per * flat.esize();
      t.id = c.E.next_id++;
      P.a.push_back(t);
    }
  return P;
}

// ---------------------------------------------------------------------------
// lattice symmetries (all moves are left moves in a transformed frame)
// ---------------------------------------------------------------------------
// Reflection through the C1-C3 diagonal: rows <-> columns, u <-> l, d <-> r;
// the ring runs backwards, so every tensor's leg order is reversed.
void frame_transpose(Engine& E, const Env& in, const Peps& A, Env& out, Peps& Aout) {
  out.Lx = in.Ly;
  out.Ly = in.Lx;
  out.s.assign(in.s.size(), Site());
  Aout.Lx = A.Ly;
  Aout.Ly = A.Lx;
  Aout.a.assign(A.a.size(), Ten());
  for (int x = 0; x < in.Lx; ++x)
    for (int y = 0; y < in.Ly; ++y) {
      const Site& e = in.at(x, y);
      Site& o = out.at(y, x);
      auto tr = [&](const Ten& t) { return E.permute(t, "ab->ba"); };
      auto rv = [&](const Ten& t) { return E.permute(t, "abc->cba"); };
      o.t[C1] = tr(e.t[C1]);
      o.t[C2] = tr(e.t[C4]);
      o.t[C3] = tr(e.t[C3]);
      o.t[C4] = tr(e.t[C2]);
      o.t[T1k] = rv(e.t[T4k]);
      o.t[T1b] = rv(e.t[T4b]);
      o.t[T4k] = rv(e.t[T1k]);
      o.t[T4b] = rv(e.t[T1b]);
      o.t[T2k] = rv(e.t[T3k]);
      o.t[T2b] = rv(e.t[T3b]);
      o.t[T3k] = rv(e.t[T2k]);
      o.t[T3b] = rv(e.t[T2b]);
      Aout.a[(size_t)y * Aout.Ly + x] = E.permute(A.at(x, y), "pabcd->pbadc");
    }
}

// Rotation by 180 degrees: a relabelling of the tensors (no data movement);
// the bra layer becomes the first layer along every edge.
void frame_rotate(Engine& E, const Env& in, const Peps& A, Env& out, Peps& Aout) {
  out.Lx = in.Lx;
  out.Ly = in.Ly;
  out.s.assign(in.s.size(), Site());
  Aout.Lx = A.Lx;
  Aout.Ly = A.Ly;
  Aout.a.assign(A.a.size(), Ten());
  for (int x = 0; x < in.Lx; ++x)
    for (int y = 0; y < in.Ly; ++y) {
      const Site& e = in.at(x, y);
      Site& o = out.at(-x, -y);
      o.t[C1] = e.t[C3];
      o.t[C2] = e.t[C4];
      o.t[C3] = e.t[C1];
      o.t[C4] = e.t[C2];
      o.t[T1k] = e.t[T3b];
      o.t[T1b] = e.t[T3k];
      o.t[T2k] = e.t[T4b];
      o.t[T2b] = e.t[T4k];
      o.t[T3b] = e.t[T1k];
      o.t[T3k] = e.t[T1b];
      o.t[T4b] = e.t[T2k];
      o.t[T4k] = e.t[T2b];
      int xo = ((-x) % A.Lx + A.Lx) % A.Lx, yo = ((-y) % A.Ly + A.Ly) % A.Ly;
      Aout.a[(size_t)xo * Aout.Ly + yo] = E.permute(A.at(x, y), "pabcd->pcdab");
    }
}

void to_frame(Engine& E, int dir, const Env& in, const Peps& A, Env& out, Peps& Aout) {
  if (dir == 0) {
    out = in;
    Aout = A;
  } else if (dir == 1) {
    frame_transpose(E, in, A, out, Aout);
  } else if (dir == 2) {
    frame_rotate(E, in, A, out, Aout);
  } else {
    Env t;
    Peps ta;
    frame_transpose(E, in, A, t, ta);
    frame_rotate(E, t, ta, out, Aout);
  }
}

// Inverse maps for the environment only (the site tensors are not needed back).
void from_frame(Engine& E, int dir, const Env& in, Env& out) {
  Peps dummyA, dA2;
  auto env_only_transpose = [&](const Env& a, Env& b) {
    b.Lx = a.Ly;
    b.Ly = a.Lx;
    b.s.assign(a.s.size(), Site());
    for (int x = 0; x < a.Lx; ++x)
      for (int y = 0; y < a.Ly; ++y) {
        const Site& e = a.at(x, y);
        Site& o = b.at(y, x);
        auto tr = [&](const Ten& t) { return E.permute(t, "ab->ba"); };
        auto rv = [&](const Ten& t) { return E.permute(t, "abc->cba"); };
        o.t[C1] = tr(e.t[C1]);
        o.t[C2] = tr(e.t[C4]);
        o.t[C3] = tr(e.t[C3]);
        o.t[C4] = tr(e.t[C2]);
        o.t[T1k] = rv(e.t[T4k]);
        o.t[T1b] = rv(e.t[T4b]);
        o.t[T4k] = rv(e.t[T1k]);
        o.t[T4b] = rv(e.t[T1b]);
        o.t[T2k] = rv(e.t[T3k]);
        o.t[T2b] = rv(e.t[T3b]);
        o.t[T3k] = rv(e.t[T2k]);
        o.t[T3b] = rv(e.t[T2b]);
      }
  };
  auto env_only_rotate = [&](const Env& a, Env& b) {
    b.Lx = a.Lx;
    b.Ly = a.Ly;
    b.s.assign(a.s.size(), Site());
    for (int x = 0; x < a.Lx; ++x)
      for (int y = 0; y < a.Ly; ++y) {
        const Site& e = a.at(x, y);
        Site& o = b.at(-x, -y);
        o.t[C1] = e.t[C3];
        o.t[C2] = e.t[C4];
        o.t[C3] = e.t[C1];
        o.t[C4] = e.t[C2];
        o.t[T1k] = e.t[T3b];
        o.t[T1b] = e.t[T3k];
        o.t[T2k] = e.t[T4b];
        o.t[T2b] = e.t[T4k];
        o.t[T3b] = e.t[T1k];
        o.t[T3k] = e.t[T1b];
        o.t[T4b] = e.t[T2k];
        o.t[T4k] = e.t[T2b];
      }
  };
  if (dir == 0) {
    out = in;
  } else if (dir == 1) {
    env_only_transpose(in, out);
  } else if (dir == 2) {
    env_only_rotate(in, out);
  } else {
    Env t;
    env_only_rotate(in, t);
    env_only_transpose(t, out);
  }
}

// ---------------------------------------------------------------------------
// half networks of one site (left frame); bra = ket (real states)
// ---------------------------------------------------------------------------
Ten rho_green_top(Engine& E, const Site& e, const Ten& a) {
  // open legs: E = T4b.d, K = ket.d | B = bra.d, F = T2b.d   (Fig. proj_plots_green (a))
  return E.ncon("ab,bce,efg,gh,hij,jkF,xya,Ewx,zcyKi,zfwBk->EKBF",
                {e.t[C1], e.t[T1k], e.t[T1b], e.t[C2], e.t[T2k], e.t[T2b], e.t[T4k], e.t[T4b], a, a});
}
Ten rho_green_bottom(Engine& E, const Site& e, const Ten& a) {
  // open legs: E = T4k.u, K = ket.u | B = bra.u, F = T2k.u
  return E.ncon("xyE,vwx,tv,qrt,noq,mn,jkm,Fij,zKyri,zBwok->EKBF",
                {e.t[T4k], e.t[T4b], e.t[C4], e.t[T3k], e.t[T3b], e.t[C3], e.t[T2b], e.t[T2k], a, a});
}
Ten rho_yellow_top(Engine& E, const Site& e, const Ten& a) {
  // ket sub-row + top edge: I = T4k.d, K = ket.d | P = ket phys, W = T1b.s, J = T2k.d
  return E.ncon("ab,bce,eWg,gh,hiJ,Iya,PcyKi->IKPWJ",
                {e.t[C1], e.t[T1k], e.t[T1b], e.t[C2], e.t[T2k], e.t[T4k], a});
}
Ten rho_yellow_bottom(Engine& E, const Site& e, const Ten& a) {
  // bra sub-row + bottom edge: I = T4b.u, K = T3k.s | P = bra phys, W = bra.u, J = T2b.u
  return E.ncon("vwI,tv,qKt,noq,mn,Jkm,PWwok->IKPWJ",
                {e.t[T4b], e.t[C4], e.t[T3k], e.t[T3b], e.t[C3], e.t[T2b], a});
}

struct Column {
  std::vector<std::vector<Ten>> G, Y, TH, R;   // per row: {P_T, P_B}
  std::vector<std::vector<double>> sG, sY, sTH, sR;
};

// One column of a left move (Sec. II B, App. A).  Writes the new C1, T4k,
// T4b, C4 of column y+1 into `env` unless `want_row` >= 0, in which case only
// the projectors of that row / cut are kept in `col` (env untouched).
void left_column(ctm_ctx& c, Env& env, const Peps& A, int y, Column* col, int want_row, int dir) {
  Engine& E = c.E;
  const int Lx = env.Lx, Ly = env.Ly, ce = c.chiE, ci = c.chiI;
  const int yn = (y + 1) % Ly;
  const bool spectra = col != nullptr;
  // App. B alternative: yellow (yellow') also cuts the ket (bra) physical
  // leg, which then rides on T4bt (T2kt) until the other layer is absorbed,
  // and red truncates (chi_I, D) only
  const bool alt = (c.cfg.projector_variant & CTM_PROJ_ALT_YR) != 0;
  // App. B teal half projectors: the teal networks are the left column of
  // the patch (left environment after the ket half-step, bra of column y),
  // their legs towards the right (T1b / T3b environment bond, ket and bra
  // right legs) left open
  const bool half = (c.cfg.projector_variant & CTM_PROJ_HALF_TEAL) != 0;
  const int ny = alt ? 3 : 2;
  std::vector<Ten> gT(Lx), gB(Lx), yT(Lx), yB(Lx), gT2, gB2, yT2, yB2;
  for (int x = 0; x < Lx; ++x) {
    gT[x] = rho_green_top(E, env.at(x, y), A.at(x, y));
    gB[x] = rho_green_bottom(E, env.at(x, y), A.at(x, y));
    yT[x] = rho_yellow_top(E, env.at(x, y), A.at(x, y));
    yB[x] = rho_yellow_bottom(E, env.at(x, y), A.at(x, y));
  }
  if (yn == y) {
    gT2 = gT;
    gB2 = gB;
    yT2 = yT;
    yB2 = yB;
  } else {
    gT2.resize(Lx);
    gB2.resize(Lx);
    yT2.resize(Lx);
    yB2.resize(Lx);
    for (int x = 0; x < Lx; ++x) {
      gT2[x] = rho_green_top(E, env.at(x, yn), A.at(x, yn));
      gB2[x] = rho_green_bottom(E, env.at(x, yn), A.at(x, yn));
      yT2[x] = rho_yellow_top(E, env.at(x, yn), A.at(x, yn));
      yB2[x] = rho_yellow_bottom(E, env.at(x, yn), A.at(x, yn));
    }
  }
  // first projectors: green (cut x|x+1) and yellow (row x) of column y; the
  // mirrored pair of column y+1 for the right environment (bra layer first).
  // All of them go through one batched SVD per matrix size.
  std::vector<std::vector<Ten>> G(Lx), Y(Lx), Gr(Lx), Yr(Lx);
  std::vector<std::vector<double>> sG(Lx), sY(Lx);
  {
    std::vector<ProjReq> rq;
    for (int x = 0; x < Lx; ++x) {
      const int xp = (x + 1) % Lx;
      rq.push_back({gT[x], gB[xp], 2, true, ce, spectra ? &sG[x] : nullptr});
      rq.push_back({gT2[x], gB2[xp], 2, false, ce, nullptr});
      rq.push_back({yT[x], yB[x], ny, true, ci, spectra ? &sY[x] : nullptr});
      rq.push_back({yT2[x], yB2[x], ny, false, ci, nullptr});
    }
    auto out = E.projectors_batch(rq);
    for (int x = 0; x < Lx; ++x) {
      G[x] = out[4 * x];
      Gr[x] = out[4 * x + 1];
      Y[x] = out[4 * x + 2];
      Yr[x] = out[4 * x + 3];
    }
  }
  // ket half-step of the left environment (first projection)
  std::vector<Ten> C1t(Lx), T4kt(Lx), T4bt(Lx), C4t(Lx);
  for (int x = 0; x < Lx; ++x) {
    const Site& e = env.at(x, y);
    const Ten& a = A.at(x, y);
    const int xu = (x - 1 + Lx) % Lx;
    C1t[x] = E.ncon("ab,bce,acg->ge", {e.t[C1], e.t[T1k], G[xu][0]});
    if (alt) {
      T4kt[x] = E.ncon("xya,PcykS,acg,xkPY->gSY", {e.t[T4k], a, G[xu][1], Y[x][0]});
      T4bt[x] = E.ncon("vwx,xkPY,vkg->YwgP", {e.t[T4b], Y[x][1], G[x][0]});
    } else {
      T4kt[x] = E.ncon("xya,PcykS,acg,xkY->gSYP", {e.t[T4k], a, G[xu][1], Y[x][0]});
      T4bt[x] = E.ncon("vwx,xkY,vkg->Ywg", {e.t[T4b], Y[x][1], G[x][0]});
    }
    C4t[x] = E.ncon("tv,qrt,vrg->gq", {e.t[C4], e.t[T3k], G[x][1]});
  }
  // bra half-step of the right environment of column y+1 (mirror image)
  std::vector<Ten> C2t(Lx), T2kt(Lx), T2bt(Lx), C3t(Lx);
  for (int x = 0; x < Lx; ++x) {
    const Site& e = env.at(x, yn);
    const Ten& a = A.at(x, yn);
    const int xu = (x - 1 + Lx) % Lx;
    C2t[x] = E.ncon("gF,eBg,BFk->ek", {e.t[C2], e.t[T1b], Gr[xu][0]});
    if (alt) {
      T2kt[x] = E.ncon("FSJ,WFk,PWJi->kSiP", {e.t[T2k], Gr[xu][1], Yr[x][0]});
      T2bt[x] = E.ncon("JkF,PWwBk,PWJi,BFg->iwg", {e.t[T2b], a, Yr[x][1], Gr[x][0]});
    } else {
      T2kt[x] = E.ncon("FSJ,WFk,WJi->kSi", {e.t[T2k], Gr[xu][1], Yr[x][0]});
      T2bt[x] = E.ncon("JkF,PWwBk,WJi,BFg->iwgP", {e.t[T2b], a, Yr[x][1], Gr[x][0]});
    }
    C3t[x] = E.ncon("Fq,qBi,BFk->ki", {e.t[C3], e.t[T3b], Gr[x][1]});
  }
  // second projectors from the 2-column patch
  //   [left env after ket step][bra of column y][ket of column y+1][right env after bra step]
  std::vector<std::vector<Ten>> TH(Lx), R(Lx);
  std::vector<std::vector<double>> sTH(Lx), sR(Lx);
  {
    std::vector<ProjReq> rq;
    for (int x = 0; x < Lx; ++x) {
      const int xp = (x + 1) % Lx;
      const Site &m = env.at(x, y), &mp = env.at(xp, y), &n = env.at(x, yn), &np_ = env.at(xp, yn);
      const Ten &b = A.at(x, y), &bp = A.at(xp, y), &k = A.at(x, yn), &kp = A.at(xp, yn);
      Ten rT, rB, sX, sZ, sT, sB;
      // the red upper half network factors through the (environment, D) bond
      // (h, S): rho_T = X^T Z, so M_red has rank <= chi_E D
      if (alt) {
        rT = E.ncon("ae,efh,hci,ij,aSY,YwGP,PfwBk,QcSKr,jrZQ,ZkF->GBKF",
                    {C1t[x], m.t[T1b], n.t[T1k], C2t[x], T4kt[x], T4bt[x], b, k, T2kt[x], T2bt[x]});
        rB = E.ncon("GSY,YwvP,vq,hoq,iXh,ni,PBwok,QKSXr,FrZQ,Zkn->GBKF",
                    {T4kt[xp], T4bt[xp], C4t[xp], mp.t[T3b], np_.t[T3k], C3t[xp], bp, kp, T2kt[xp], T2bt[xp]});
        sX = E.ncon("ae,eWh,aSY->YWhS", {C1t[x], m.t[T1b], T4kt[x]});
        sZ = E.ncon("hci,ij,QcSKr,jrJQ->hSKJ", {n.t[T1k], C2t[x], k, T2kt[x]});
        sT = E.contract("YWhS,hSKJ->YWKJ", sX, sZ);
        sB = E.ncon("YwvP,vq,hoq,iKh,ni,PWwok,Jkn->YWKJ", {T4bt[x], C4t[x], m.t[T3b], n.t[T3k], C3t[x], b, T2bt[x]});
      } else {
        rT = E.ncon("ae,efh,hci,ij,aSYP,YwG,PfwBk,QcSKr,jrZ,ZkFQ->GBKF",
                    {C1t[x], m.t[T1b], n.t[T1k], C2t[x], T4kt[x], T4bt[x], b, k, T2kt[x], T2bt[x]});
        rB = E.ncon("GSYP,Ywv,vq,hoq,iXh,ni,PBwok,QKSXr,FrZ,ZknQ->GBKF",
                    {T4kt[xp], T4bt[xp], C4t[xp], mp.t[T3b], np_.t[T3k], C3t[xp], bp, kp, T2kt[xp], T2bt[xp]});
        sX = E.ncon("ae,eWh,aSYP->YPWhS", {C1t[x], m.t[T1b], T4kt[x]});
        sZ = E.ncon("hci,ij,QcSKr,jrJ->hSKQJ", {n.t[T1k], C2t[x], k, T2kt[x]});
        sT = E.contract("YPWhS,hSKQJ->YPWKQJ", sX, sZ);
        sB = E.ncon("Ywv,vq,hoq,iKh,ni,PWwok,JknQ->YPWKQJ", {T4bt[x], C4t[x], m.t[T3b], n.t[T3k], C3t[x], b, T2bt[x]});
      }
      if (half) {
        if (alt) {
          rT = E.ncon("ae,efh,aSY,YwGP,PfwBk->GBhSk", {C1t[x], m.t[T1b], T4kt[x], T4bt[x], b});
          rB = E.ncon("GSY,YwvP,vq,hoq,PBwok->GBhSk", {T4kt[xp], T4bt[xp], C4t[xp], mp.t[T3b], bp});
        } else {
          rT = E.ncon("ae,efh,aSYP,YwG,PfwBk->GBhSk", {C1t[x], m.t[T1b], T4kt[x], T4bt[x], b});
          rB = E.ncon("GSYP,Ywv,vq,hoq,PBwok->GBhSk", {T4kt[xp], T4bt[xp], C4t[xp], mp.t[T3b], bp});
        }
      }
      rq.push_back({rT, rB, 2, true, ce, spectra ? &sTH[x] : nullptr});
      rq.push_back({sT, sB, alt ? 2 : 3, true, ci, spectra ? &sR[x] : nullptr, sX, sZ});
    }
    auto out = E.projectors_batch(rq);
    for (int x = 0; x < Lx; ++x) {
      TH[x] = out[2 * x];
      R[x] = out[2 * x + 1];
    }
  }
  if (col) {
    col->G = G;
    col->Y = Y;
    col->TH = TH;
    col->R = R;
    col->sG = sG;
    col->sY = sY;
    col->sTH = sTH;
    col->sR = sR;
  }
  if (want_row >= 0) return;
  // bra half-step (second projection) -> new left environment of column y+1
  std::vector<Site> nw(Lx);
  for (int x = 0; x < Lx; ++x) {
    const Site& e = env.at(x, y);
    const Ten& a = A.at(x, y);
    const int xu = (x - 1 + Lx) % Lx;
    nw[x].t[C1] = E.normalize(E.ncon("ge,efR,gfD->DR", {C1t[x], e.t[T1b], TH[xu][0]}));
    if (alt) {
      nw[x].t[T4k] = E.normalize(E.ncon("gSY,gWU,YWD->DSU", {T4kt[x], TH[xu][1], R[x][0]}));
      nw[x].t[T4b] = E.normalize(E.ncon("YwgP,PWwBs,YWU,gBD->DsU", {T4bt[x], a, R[x][1], TH[x][0]}));
    } else {
      nw[x].t[T4k] = E.normalize(E.ncon("gSYP,gWU,YPWD->DSU", {T4kt[x], TH[xu][1], R[x][0]}));
      nw[x].t[T4b] = E.normalize(E.ncon("Ywg,PWwBs,YPWU,gBD->DsU", {T4bt[x], a, R[x][1], TH[x][0]}));
    }
    nw[x].t[C4] = E.normalize(E.ncon("gq,Roq,goU->RU", {C4t[x], e.t[T3b], TH[x][1]}));
  }
  for (int x = 0; x < Lx; ++x) {
    Site& d = env.at(x, yn);
    d.t[C1] = nw[x].t[C1];
    d.t[T4k] = nw[x].t[T4k];
    d.t[T4b] = nw[x].t[T4b];
    d.t[C4] = nw[x].t[C4];
  }
}

// One move in direction dir (0 left, 1 top, 2 right, 3 bottom) -> new env.
Env do_move(ctm_ctx& c, const Env& env, const Peps& A, int dir) {
  Engine& E = c.E;
  Env fe;
  Peps fa;
  to_frame(E, dir, env, A, fe, fa);
  for (int y = 0; y < fe.Ly && E.ok(); ++y) left_column(c, fe, fa, y, nullptr, -1, dir);
  Env out;
  from_frame(E, dir, fe, out);
  return out;
}

// ---------------------------------------------------------------------------
// energy
// ---------------------------------------------------------------------------
Ten vertical_rho(Engine& E, const Env& env, const Peps& A, int x, int y) {
  const Site& e = env.at(x, y);
  const Site& f = env.at(x + 1, y);
  const Ten& a = A.at(x, y);
  const Ten& b = A.at(x + 1, y);
  Ten top = E.ncon("ab,bce,efg,gh,hij,jkF,xya,Ewx,PcyKi,RfwBk->EKBFPR",
                   {e.t[C1], e.t[T1k], e.t[T1b], e.t[C2], e.t[T2k], e.t[T2b], e.t[T4k], e.t[T4b], a, a});
  Ten bot = E.ncon("xyE,vwx,tv,qrt,noq,mn,jkm,Fij,QKyri,SBwok->EKBFQS",
                   {f.t[T4k], f.t[T4b], f.t[C4], f.t[T3k], f.t[T3b], f.t[C3], f.t[T2b], f.t[T2k], b, b});
  return E.contract("EKBFPR,EKBFQS->PQRS", top, bot);
}

// Returns per-site [e_h, e_v] device scalars (FP64 [2] each: value, norm)
void energies(ctm_ctx& c, const Env& env, const Peps& A, std::vector<Ten>& eh, std::vector<Ten>& ev) {
  Engine& E = c.E;
  eh.assign((size_t)c.Lx * c.Ly, Ten());
  ev.assign((size_t)c.Lx * c.Ly, Ten());
  for (int x = 0; x < c.Lx; ++x)
    for (int y = 0; y < c.Ly; ++y) ev[(size_t)x * c.Ly + y] = E.bond_energy(vertical_rho(E, env, A, x, y), c.h64v, c.p);
  Env te;
  Peps ta;
  frame_transpose(E, env, A, te, ta);
  for (int x = 0; x < c.Lx; ++x)
    for (int y = 0; y < c.Ly; ++y) eh[(size_t)x * c.Ly + y] = E.bond_energy(vertical_rho(E, te, ta, y, x), c.h64, c.p);
}

// Energy per site on the device: the bond energies (value slot of each
// [value, norm] pair) are gathered into one buffer, averaged over the sites by
// site_energy, and returned to the host with one copy.  bonds (optional, host,
// 2 Lx Ly entries) receives e_h, e_v of each site in site order.
double site_energy_dev(ctm_ctx& c, const std::vector<Ten>& eh, const std::vector<Ten>& ev, double* bonds) {
  Engine& E = c.E;
  const int nb = (int)(eh.size() + ev.size());
  Ten buf = E.alloc(F64, {(long)nb + 1});
  std::vector<double> hv((size_t)nb + 1, 0.0);
  if (!E.dry && E.ok()) {
    for (size_t i = 0; i < eh.size(); ++i) {
      E.check(hipMemcpyAsync(buf.f64() + 2 * i, eh[i].p, sizeof(double), hipMemcpyDeviceToDevice, E.s));
      E.check(hipMemcpyAsync(buf.f64() + 2 * i + 1, ev[i].p, sizeof(double), hipMemcpyDeviceToDevice, E.s));
    }
    E.check(site_energy(E.s, nb, buf.f64(), 1.0 / ((double)c.Lx * c.Ly), buf.f64() + nb));
    E.check(hipMemcpyAsync(hv.data(), buf.p, hv.size() * sizeof(double), hipMemcpyDeviceToHost, E.s));
    E.check(hipStreamSynchronize(E.s));
  }
  if (bonds) std::copy(hv.begin(), hv.begin() + nb, bonds);
  return hv[nb];
}

int status_from_engine(const Engine& E) {
  if (E.err != hipSuccess) return CTM_EDEVICE;
  if (E.ar.overflow) return CTM_EINVAL;
  if (E.status == 1) return CTM_EINVAL;
  if (E.status == 2) return CTM_EINVAL;
  if (E.status) return E.status;
  return CTM_OK;
}

bool finite_all(const double* v, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

void begin(ctm_ctx* c) {
  c->E.flops_gemm = 0;
  c->E.svd_sweeps_total = 0;
  c->E.status = 0;
  c->E.ar.overflow = false;
  c->E.ar.release(c->transient_mark);
  c->E.clear_tape();
  c->E.svdc_reset();
  kernel_timer() = c->timing ? &c->timer : nullptr;
}

ctm_status finish(ctm_ctx* c, ctm_status st) {
  c->last_flops = (double)c->E.flops_gemm;
  c->last_sweeps = (double)c->E.svd_sweeps_total;
  c->E.ar.release(c->transient_mark);
  c->E.clear_tape();
  if (c->timing) {
    if (hipStreamSynchronize(c->E.s) == hipSuccess) c->timer.collect();
    kernel_timer() = nullptr;
  }
  return st;
}

ctm_status validate(const ctm_config* cfg) {
  if (!cfg) return CTM_EINVAL;
  if (cfg->Lx < 1 || cfg->Ly < 1 || cfg->Lx > 8 || cfg->Ly > 8) return CTM_EINVAL;
  if (cfg->p < 1 || cfg->D < 1 || cfg->chi_E < 1 || cfg->chi_I < 1) return CTM_EINVAL;
  if (cfg->contract_prec < CTM_FP64 || cfg->contract_prec > CTM_BF16X6) return CTM_EINVAL;
  if (cfg->init != CTM_INIT_IDENTITY && cfg->init != CTM_INIT_PRODUCT) return CTM_EINVAL;
  if (cfg->init == CTM_INIT_IDENTITY && cfg->chi_I < cfg->D) return CTM_EINVAL;
  if (cfg->projector_variant < 0 || cfg->projector_variant > (CTM_PROJ_ALT_YR | CTM_PROJ_HALF_TEAL)) return CTM_EINVAL;
  // every projector matrix M (n_b x n_b, rank <= r0 when r0 < n_b) must fit
  // the SVD: the Jacobi takes n <= 4096, the rank-limited route's
  // Householder QR n_b <= 8192 rows
  const long ce = cfg->chi_E, ci = cfg->chi_I, D = cfg->D, p = cfg->p;
  const bool alt = (cfg->projector_variant & CTM_PROJ_ALT_YR) != 0;
  const bool half = (cfg->projector_variant & CTM_PROJ_HALF_TEAL) != 0;
  auto fits = [](long nb, long r0) { return nb <= 4096 || (r0 > 0 && r0 < nb && r0 <= 4096 && nb <= 8192); };
  if (!fits(ce * D, 0)) return CTM_EINVAL;                                        // green, green'
  if (!fits(half ? ce * D * D : ce * D, half ? ce * D : 0)) return CTM_EINVAL;    // teal
  if (!fits(alt ? ci * D : ci * p * D, alt ? 0 : ci * D)) return CTM_EINVAL;      // yellow, yellow'
  if (!fits(alt ? ci * D : ci * p * D, ce * D)) return CTM_EINVAL;                // red
  return CTM_OK;
}

void setup_ctx(ctm_ctx* c, const ctm_config* cfg, void* ws, size_t bytes, hipStream_t stream, bool dry) {
  c->cfg = *cfg;
  c->chiE = cfg->chi_E;
  c->chiI = cfg->chi_I;
  c->D = cfg->D;
  c->p = cfg->p;
  c->Lx = cfg->Lx;
  c->Ly = cfg->Ly;
  Engine& E = c->E;
  E.s = stream;
  E.dry = dry;
  E.ar.dry = dry;
  E.ar.base = (char*)ws;
  E.ar.cap = bytes;
  E.prec = (Prec)cfg->contract_prec;
  E.cdt = cfg->contract_prec == CTM_FP64 ? F64 : F32;
  E.cutoff = cfg->svd_rel_cutoff > 0 ? cfg->svd_rel_cutoff : 1e-12;
  E.adj_eps = cfg->svd_adj_eps > 0 ? cfg->svd_adj_eps : 1e-12;
  // Jacobi stopping level: working accuracy (sqrt(n) 1.2e-16 relative
  // off-orthogonality) for FP64 contractions; 1e-10 when the contractions
  // carry FP32-level rounding (1e-7 of |M| already in M itself).  Either way
  // the factors leave the SVD orthonormal to rounding (the reverse pass needs
  // that), so the stopping level only sets how close U S V^T is to M.
  E.svd_tol = cfg->contract_prec == CTM_FP64 ? 0.0 : 1e-10;
  E.host_flags = c->host_flags;
  E.host_flags_n = 256;
}

// Persistent buffers + initial environment.
void init_persistent(ctm_ctx* c, const double* A_dev, const double* bvec) {
  Engine& E = c->E;
  const long per = (long)c->p * c->D * c->D * c->D * c->D;
  c->A64 = E.alloc(F64, {(long)c->Lx * c->Ly * per});
  c->Aflat = (E.cdt == F64) ? c->A64 : E.alloc(F32, {(long)c->Lx * c->Ly * per});
  const long env_n = site_elems(*c) * c->Lx * c->Ly;
  c->cur_blk = E.alloc(E.cdt, {env_n});
  c->start_blk = E.alloc(E.cdt, {env_n});
  c->spec_prev = E.alloc(F64, {(long)c->Lx * c->Ly * 4 * c->chiE});
  c->h64 = E.alloc(F64, {(long)c->p * c->p * c->p * c->p});
  c->h64v = E.alloc(F64, {(long)c->p * c->p * c->p * c->p});
  Ten part = E.alloc(F64, {(long)reduce_partials()});
  E.partial = part.f64();
  if (!E.dry && E.ok()) {
    E.check(hipMemcpyAsync(c->A64.p, A_dev, c->A64.bytes(), hipMemcpyDeviceToDevice, E.s));
    if (E.cdt == F32) E.check(cast_f64_to_f32(E.s, c->A64.f64(), c->Aflat.f32(), c->A64.n()));
    // boundary environment, built on the host in FP64 then cast
    std::vector<double> h(env_n, 0.0);
    long shp[NT][3];
    int rk[NT];
    site_shapes(*c, shp, rk);
    size_t off = 0;
    for (int s = 0; s < c->Lx * c->Ly; ++s)
      for (int i = 0; i < NT; ++i) {
        long n = 1;
        for (int j = 0; j < rk[i]; ++j) n *= shp[i][j];
        if (i <= C4) {
          h[off] = 1.0;   // [0][0]
        } else {
          const bool first = (i == T1k || i == T2k || i == T3b || i == T4b);
          const long d1 = shp[i][1], d2 = shp[i][2];
          for (int sIdx = 0; sIdx < c->D; ++sIdx) {
            double v;
            long idx;
            if (c->cfg.init == CTM_INIT_IDENTITY) {
              v = 1.0;
              idx = first ? ((long)sIdx * d2 + sIdx)                 // [0][s][s]
                          : (((long)sIdx * d1 + sIdx) * d2);         // [s][s][0]
            } else {
              v = bvec[sIdx];
              idx = (long)sIdx * d2;                                 // [0][s][0]
            }
            h[off + idx] = v;
          }
        }
        off += n;
      }
    if (E.cdt == F64) {
      E.check(hipMemcpyAsync(c->cur_blk.p, h.data(), sizeof(double) * env_n, hipMemcpyHostToDevice, E.s));
    } else {
      std::vector<float> hf(h.begin(), h.end());
      E.check(hipMemcpyAsync(c->cur_blk.p, hf.data(), sizeof(float) * env_n, hipMemcpyHostToDevice, E.s));
      E.check(hipStreamSynchronize(E.s));
    }
    E.check(hipMemcpyAsync(c->start_blk.p, c->cur_blk.p, c->cur_blk.bytes(), hipMemcpyDeviceToDevice, E.s));
    E.check(hipStreamSynchronize(E.s));
  }
  c->transient_mark = E.ar.mark();
}

// Corner spectra of the current environment -> spec_prev.  Returns the
// largest 2-norm change of any corner's spectrum against the spectra held
// before (Sec. II B: the iteration stops at a fixed point of the corners), or
// INFINITY when those were not the spectra of the environment this one was
// computed from.
double corner_delta(ctm_ctx* c) {
  Engine& E = c->E;
  const int nc = c->Lx * c->Ly * 4, ch = c->chiE;
  size_t mk = E.ar.mark();
  Ten Cs = E.alloc(F64, {(long)nc, (long)ch, (long)ch});
  Ten U = E.alloc(F64, {(long)nc, (long)ch, (long)ch});
  Ten V = E.alloc(F64, {(long)nc, (long)ch, (long)ch});
  Ten S = E.alloc(F64, {(long)nc, (long)ch});
  Ten d = E.alloc(F64, {1});
  void* work = E.ar.alloc(svd_work_bytes(ch, nc));
  double delta = 0.0;
  if (!E.dry && E.ok()) {
    Env v = view_env(*c, c->cur_blk);
    for (int s = 0; s < c->Lx * c->Ly; ++s)
      for (int k = 0; k < 4; ++k) {
        const Ten& t = v.s[s].t[C1 + k];
        double* dst = Cs.f64() + (long)(s * 4 + k) * ch * ch;
        if (t.dt == F64)
          E.check(hipMemcpyAsync(dst, t.p, t.bytes(), hipMemcpyDeviceToDevice, E.s));
        else
          E.check(cast_f32_to_f64(E.s, t.f32(), dst, t.n()));
      }
    int sw = 0;
    E.check(svd_f64(E.s, ch, nc, Cs.f64(), U.f64(), S.f64(), V.f64(), work, E.svd_max_sweeps, E.svd_tol,
                    c->host_flags, &sw));
    E.check(spectra_delta(E.s, nc, ch, S.f64(), c->spec_prev.f64(), d.f64(), c->spec_current ? 1 : 0));
    E.check(hipMemcpyAsync(&delta, d.p, sizeof(double), hipMemcpyDeviceToHost, E.s));
    E.check(hipStreamSynchronize(E.s));
    if (!c->spec_current) delta = INFINITY;
    c->spec_current = true;
  }
  E.ar.release(mk);
  return delta;
}

// ---------------------------------------------------------------------------
// gradient: forward with checkpoints, then reverse move by move
// ---------------------------------------------------------------------------
// SPLITCTM_PHASES (diagnostics): the stream is synchronised at the phase
// boundaries of energy_grad and the host time of each phase is printed
// (forward sweeps, energy with its reverse, taped recompute of the moves,
// reverse of the moves).
struct PhaseClock {
  bool on = getenv("SPLITCTM_PHASES") != nullptr;
  double acc[4] = {0, 0, 0, 0};
  std::chrono::steady_clock::time_point t0;
  void start(Engine& E) {
    if (!on || E.dry) return;
    E.check(hipStreamSynchronize(E.s));
    t0 = std::chrono::steady_clock::now();
  }
  void stop(Engine& E, int k) {
    if (!on || E.dry) return;
    E.check(hipStreamSynchronize(E.s));
    acc[k] += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  void report(bool dry) const {
    if (on && !dry)
      fprintf(stderr, "[phases] forward %.3f s, energy %.3f s, taped recompute %.3f s, reverse %.3f s\n", acc[0],
              acc[1], acc[2], acc[3]);
  }
};

ctm_status energy_grad_impl(ctm_ctx* c, const double* h_host, const double* hv_host, int n_sweeps, int ckpt,
                            double* e_site, double* dA_dev) {
  Engine& E = c->E;
  if (n_sweeps < 0 || ckpt < 1) return CTM_EINVAL;
  const int nblk = (n_sweeps + ckpt - 1) / ckpt;
  const long env_n = c->cur_blk.n();
  // persistent (for this call): checkpoints, block move snapshots, cotangents
  std::vector<Ten> ck(nblk + 1);
  for (int b = 0; b <= nblk; ++b) ck[b] = E.alloc(E.cdt, {env_n});
  std::vector<Ten> mv((size_t)4 * ckpt);
  for (auto& t : mv) t = E.alloc(E.cdt, {env_n});
  Ten genv = E.alloc(E.cdt, {env_n});
  Ten gA = E.alloc(F64, {c->A64.n()});
  // SVD record / replay store: one slot per move of a checkpoint block, each
  // bounded by the decompositions of every site of the cell.  A matrix of
  // size n decomposed in full keeps U, S, V (2 n^2 + n); one of size nb
  // decomposed through its rank-r core keeps the core's U, S, V and the two
  // Q^T factors (2 r^2 + r + 2 r nb).
  {
    const bool alt = (c->cfg.projector_variant & CTM_PROJ_ALT_YR) != 0;
    const bool half = (c->cfg.projector_variant & CTM_PROJ_HALF_TEAL) != 0;
    const long ce = c->chiE, ci = c->chiI, D = c->D, p = c->p;
    auto full = [](long n) { return 2 * n * n + n; };
    auto fact = [](long nb, long r) { return 2 * r * r + r + 2 * r * nb; };
    const long green = full(ce * D);
    const long teal = half ? fact(ce * D * D, ce * D) : full(ce * D);
    const long yellow = alt ? full(ci * D) : fact(ci * p * D, ci * D);
    const long red = alt ? full(ci * D) : std::max(full(ci * p * D), fact(ci * p * D, std::min(ce * D, ci * p * D)));
    const long per_site = 2 * green + teal + 2 * yellow + red;
    const long per_slot = (long)c->Lx * c->Ly * per_site + 32L * 8 * (c->Lx + c->Ly) * 4;
    Ten buf = E.alloc(F64, {4L * ckpt, per_slot});
    E.svdc_setup(buf, 4 * ckpt, per_slot);
  }
  const int s_last = (nblk - 1) * ckpt;   // first sweep of the last block
  Ten ebuf = E.alloc(F64, {(long)c->Lx * c->Ly * 4});
  E.zero(gA);
  if (!E.dry && E.ok()) {
    E.check(hipMemcpyAsync(c->h64.p, h_host, c->h64.bytes(), hipMemcpyHostToDevice, E.s));
    E.check(hipMemcpyAsync(c->h64v.p, hv_host, c->h64v.bytes(), hipMemcpyHostToDevice, E.s));
    E.check(hipMemcpyAsync(ck[0].p, c->start_blk.p, c->start_blk.bytes(), hipMemcpyDeviceToDevice, E.s));
  }
  const Peps A = peps_view(*c, c->Aflat);
  PhaseClock pc;
  pc.start(E);
  // ---- forward: store the environment at the start of every block ----
  for (int s = 0; s < n_sweeps && E.ok(); ++s) {
    if (s % ckpt == 0 && s > 0) {
      // ck[s / ckpt] already written at the end of the previous sweep
    }
    const Ten& src = (s == 0) ? ck[0] : c->cur_blk;
    if (s == 0 && !E.dry && E.ok())
      E.check(hipMemcpyAsync(c->cur_blk.p, src.p, src.bytes(), hipMemcpyDeviceToDevice, E.s));
    for (int dir = 0; dir < 4 && E.ok(); ++dir) {
      // the inputs of the moves of the last block are kept as they go by: its
      // reverse pass needs no regeneration
      if (s >= s_last && !E.dry && E.ok())
        E.check(hipMemcpyAsync(mv[(s - s_last) * 4 + dir].p, c->cur_blk.p, c->cur_blk.bytes(), hipMemcpyDeviceToDevice,
                               E.s));
      size_t mk = E.ar.mark();
      E.svdc_select(s >= s_last ? (s - s_last) * 4 + dir : -1, 1);
      Env env = view_env(*c, c->cur_blk);
      Env out = do_move(*c, env, A, dir);
      store_env(*c, out, c->cur_blk);
      E.ar.release(mk);
    }
    E.svdc_select(-1, 0);
    if ((s + 1) % ckpt == 0 && (s + 1) / ckpt < nblk && !E.dry && E.ok())
      E.check(hipMemcpyAsync(ck[(s + 1) / ckpt].p, c->cur_blk.p, c->cur_blk.bytes(), hipMemcpyDeviceToDevice, E.s));
    if (E.dry) break;   // the workspace peak repeats every sweep
  }
  if (n_sweeps == 0 && !E.dry && E.ok())
    E.check(hipMemcpyAsync(c->cur_blk.p, ck[0].p, ck[0].bytes(), hipMemcpyDeviceToDevice, E.s));
  // the state after the n_sweeps sweeps (the last block may be shorter than
  // ckpt sweeps), restored into the current environment at the end
  if (nblk > 0 && !E.dry && E.ok())
    E.check(hipMemcpyAsync(ck[nblk].p, c->cur_blk.p, c->cur_blk.bytes(), hipMemcpyDeviceToDevice, E.s));
  pc.stop(E, 0);
  pc.start(E);
  // ---- energy (taped) and its reverse pass -> cotangent of the final env ----
  double esum = 0.0;
  {
    size_t mk = E.ar.mark();
    E.clear_tape();
    E.taping = true;
    Env env = load_env(*c, c->cur_blk, true);
    Peps Ai = A;
    for (auto& t : Ai.a) {
      t.id = E.next_id++;
      E.mark_input(t);
    }
    std::vector<Ten> eh, ev;
    energies(*c, env, Ai, eh, ev);
    E.taping = false;
    const double w = 1.0 / (c->Lx * c->Ly);
    esum = site_energy_dev(*c, eh, ev, nullptr);
    for (size_t i = 0; i < eh.size(); ++i) {
      Ten g1 = E.grad(eh[i]), g2 = E.grad(ev[i]);
      if (!E.dry && E.ok()) {
        E.check(fill_f64(E.s, g1.f64(), w, 1));
        E.check(fill_f64(E.s, g2.f64(), w, 1));
      }
    }
    E.backward();
    // env cotangent -> genv (packed), A cotangent -> gA
    Env gv = view_env(*c, genv);
    for (size_t s = 0; s < env.s.size(); ++s)
      for (int i = 0; i < NT; ++i) {
        Ten g = E.grad(env.s[s].t[i]);
        if (!E.dry && E.ok())
          E.check(hipMemcpyAsync(gv.s[s].t[i].p, g.p, g.bytes(), hipMemcpyDeviceToDevice, E.s));
      }
    for (size_t i = 0; i < Ai.a.size(); ++i) {
      Ten g = E.grad(Ai.a[i]);
      if (!E.dry && E.ok()) E.check(add_cast(E.s, g.p, g.dt == F64, gA.f64() + (long)i * Ai.a[i].n(), true, g.n()));
    }
    E.clear_tape();
    E.ar.release(mk);
  }
  pc.stop(E, 1);
  if (e_site) *e_site = esum;
  if (!std::isfinite(esum) && !E.dry) return CTM_ENUMERIC;
  // ---- reverse over blocks and moves ----
  for (int b = nblk - 1; b >= 0 && E.ok(); --b) {
    const int s0 = b * ckpt, s1 = std::min(n_sweeps, s0 + ckpt);
    // regenerate the environments at every move of the block (untaped; the
    // last block kept them during the forward pass)
    if (!E.dry && E.ok())
      E.check(hipMemcpyAsync(c->cur_blk.p, ck[b].p, ck[b].bytes(), hipMemcpyDeviceToDevice, E.s));
    if (b != nblk - 1)   // the slots hold a later block: re-record (the block's last move recomputes)
      for (auto& sl : E.svdc_slots) sl.valid = false;
    int nm = 0;
    if (b == nblk - 1) nm = (s1 - s0) * 4;   // inputs kept by the forward pass
    for (int s = s0; s < s1 && E.ok() && b != nblk - 1; ++s)
      for (int dir = 0; dir < 4 && E.ok(); ++dir) {
        if (!E.dry && E.ok())
          E.check(hipMemcpyAsync(mv[nm].p, c->cur_blk.p, c->cur_blk.bytes(), hipMemcpyDeviceToDevice, E.s));
        ++nm;
        if (s == s1 - 1 && dir == 3) break;   // the last move's input is enough
        size_t mk = E.ar.mark();
        E.svdc_select((s - s0) * 4 + dir, b == nblk - 1 ? 2 : 1);
        Env env = view_env(*c, c->cur_blk);
        Env out = do_move(*c, env, A, dir);
        store_env(*c, out, c->cur_blk);
        E.ar.release(mk);
        if (E.dry) break;
      }
    E.svdc_select(-1, 0);
    // reverse the moves of the block
    for (int m = nm - 1; m >= 0 && E.ok(); --m) {
      const int dir = m % 4;
      size_t mk = E.ar.mark();
      E.clear_tape();
      E.taping = true;
      Env env = load_env(*c, mv[m], true);
      Peps Ai = A;
      for (auto& t : Ai.a) {
        t.id = E.next_id++;
        E.mark_input(t);
      }
      pc.start(E);
      E.svdc_select(m, 2);
      Env out = do_move(*c, env, Ai, dir);
      E.svdc_select(-1, 0);
      E.taping = false;
      pc.stop(E, 2);
      pc.start(E);
      // seed with the cotangent of the move's output
      Env gv = view_env(*c, genv);
      for (size_t s = 0; s < out.s.size(); ++s)
        for (int i = 0; i < NT; ++i) {
          Ten g = E.grad(out.s[s].t[i]);
          E.add_into(gv.s[s].t[i], g);
        }
      E.backward();
      for (size_t s = 0; s < env.s.size(); ++s)
        for (int i = 0; i < NT; ++i) {
          Ten g = E.grad(env.s[s].t[i]);
          if (!E.dry && E.ok())
            E.check(hipMemcpyAsync(gv.s[s].t[i].p, g.p, g.bytes(), hipMemcpyDeviceToDevice, E.s));
        }
      for (size_t i = 0; i < Ai.a.size(); ++i) {
        Ten g = E.grad(Ai.a[i]);
        if (!E.dry && E.ok())
          E.check(add_cast(E.s, g.p, g.dt == F64, gA.f64() + (long)i * Ai.a[i].n(), true, g.n()));
      }
      E.clear_tape();
      E.ar.release(mk);
      pc.stop(E, 3);
      if (E.dry) break;
    }
    if (E.dry) break;
  }
  pc.report(E.dry);
  // leave the current environment at the state after n_sweeps
  if (!E.dry && E.ok() && nblk > 0)
    E.check(hipMemcpyAsync(c->cur_blk.p, ck[nblk].p, ck[nblk].bytes(), hipMemcpyDeviceToDevice, E.s));
  if (dA_dev && !E.dry && E.ok())
    E.check(hipMemcpyAsync(dA_dev, gA.p, gA.bytes(), hipMemcpyDeviceToDevice, E.s));
  if (!E.dry && E.ok()) E.check(hipStreamSynchronize(E.s));
  return (ctm_status)status_from_engine(E);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* ctm_strerror(ctm_status s) {
  switch (s) {
    case CTM_OK: return "ok";
    case CTM_EINVAL: return "invalid argument or workspace too small";
    case CTM_ENOMEM: return "out of memory";
    case CTM_EDEVICE: return "HIP runtime error";
    case CTM_ENOTCONV: return "not converged within the sweep budget";
    case CTM_ENUMERIC: return "non-finite value or rank-zero projector";
  }
  return "unknown status";
}

size_t ctm_env_elems(const ctm_config* cfg) {
  if (validate(cfg) != CTM_OK) return 0;
  ctm_ctx c;
  c.chiE = cfg->chi_E;
  c.chiI = cfg->chi_I;
  c.D = cfg->D;
  return (size_t)site_elems(c) * cfg->Lx * cfg->Ly;
}

size_t ctm_projectors_elems(const ctm_config* cfg) {
  if (validate(cfg) != CTM_OK) return 0;
  const size_t ce = cfg->chi_E, ci = cfg->chi_I, D = cfg->D, p = cfg->p;
  return 2 * (ce * D * ce) * 2 + 2 * (ci * D * ci) + 2 * (ci * p * D * ci);
}

ctm_status ctm_workspace_size(const ctm_config* cfg, int with_grad, int n_sweeps, int ckpt_every, size_t* bytes) {
  ctm_status st = validate(cfg);
  if (st != CTM_OK || !bytes) return CTM_EINVAL;
  if (with_grad && (n_sweeps < 0 || ckpt_every < 1)) return CTM_EINVAL;
  ctm_ctx* c = new (std::nothrow) ctm_ctx();
  if (!c) return CTM_ENOMEM;
  setup_ctx(c, cfg, nullptr, 0, nullptr, true);
  std::vector<double> bvec(cfg->D, 1.0);
  init_persistent(c, nullptr, bvec.data());
  size_t peak = c->E.ar.peak;
  const Peps A = peps_view(*c, c->Aflat);
  // one sweep (each move) and the corner spectra
  for (int dir = 0; dir < 4; ++dir) {
    size_t mk = c->E.ar.mark();
    Env env = view_env(*c, c->cur_blk);
    Env out = do_move(*c, env, A, dir);
    c->E.ar.release(mk);
  }
  corner_delta(c);
  // energy
  {
    size_t mk = c->E.ar.mark();
    Env env = view_env(*c, c->cur_blk);
    std::vector<Ten> eh, ev;
    energies(*c, env, A, eh, ev);
    c->E.ar.release(mk);
  }
  // projectors
  {
    size_t mk = c->E.ar.mark();
    Env env = view_env(*c, c->cur_blk);
    Column col;
    left_column(*c, env, A, 0, &col, 0, -1);
    c->E.ar.release(mk);
  }
  if (with_grad) energy_grad_impl(c, nullptr, nullptr, n_sweeps, ckpt_every, nullptr, nullptr);
  peak = std::max(peak, c->E.ar.peak);
  const int planning = c->E.status;
  delete c;
  if (planning) return CTM_EINVAL;
  *bytes = peak + peak / 16 + (size_t(64) << 20);
  return CTM_OK;
}

namespace {
// aux_stream: also create the second stream and its events (contexts on the
// static array skip them: that entry point creates no runtime objects)
ctm_status init_ctx(const ctm_config* cfg, const double* A_dev, const double* bvec, void* ws, size_t ws_bytes,
                    void* stream, ctm_ctx** out, bool aux_stream) {
  if (!out) return CTM_EINVAL;
  *out = nullptr;
  ctm_status st = validate(cfg);
  if (st != CTM_OK || !A_dev || !ws) return CTM_EINVAL;
  if (cfg->init == CTM_INIT_PRODUCT && !bvec) return CTM_EINVAL;
  size_t need = 0;
  // persistent part only must fit; the transient part is checked per call
  ctm_ctx* c = new (std::nothrow) ctm_ctx();
  if (!c) return CTM_ENOMEM;
  setup_ctx(c, cfg, ws, ws_bytes, (hipStream_t)stream, false);
  if (aux_stream) {
    Engine& E = c->E;
    E.check(hipStreamCreateWithFlags(&E.aux, hipStreamNonBlocking));
    for (auto& ev : E.aux_ev)
      if (E.ok()) E.check(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  }
  init_persistent(c, A_dev, bvec);
  (void)need;
  st = (ctm_status)status_from_engine(c->E);
  if (st != CTM_OK) {
    ctm_destroy(c);
    return st;
  }
  *out = c;
  return CTM_OK;
}
}  // namespace

ctm_status ctm_init(const ctm_config* cfg, const double* A_dev, const double* bvec, void* ws, size_t ws_bytes,
                    void* stream, ctm_ctx** out) {
  return init_ctx(cfg, A_dev, bvec, ws, ws_bytes, stream, out, true);
}

ctm_status ctm_init_static(const ctm_config* cfg, const double* A_dev, const double* bvec, void* stream,
                           ctm_ctx** out) {
  if (!out) return CTM_EINVAL;
  *out = nullptr;
  ctm_status st = validate(cfg);
  if (st != CTM_OK || !A_dev) return CTM_EINVAL;
  if (cfg->init == CTM_INIT_PRODUCT && !bvec) return CTM_EINVAL;
  // the configuration's workspace (dry run, no device memory) must fit the array
  size_t need = 0;
  st = ctm_workspace_size(cfg, 0, 0, 1, &need);
  if (st != CTM_OK) return st;
  if (need > kStaticScratchBytes) return CTM_EINVAL;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return CTM_EDEVICE;
  std::lock_guard<std::mutex> lock(static_mu);
  if (static_busy[dev]) return CTM_EINVAL;   // the device's array belongs to a live context
  if (!static_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CTM_EDEVICE;
    static_ptr[dev] = p;
  }
  st = init_ctx(cfg, A_dev, bvec, static_ptr[dev], kStaticScratchBytes, stream, out, false);
  if (st != CTM_OK) return st;
  (*out)->static_device = dev;
  static_busy[dev] = true;
  return CTM_OK;
}

void ctm_destroy(ctm_ctx* c) {
  if (c && c->static_device >= 0) {
    std::lock_guard<std::mutex> lock(static_mu);
    static_busy[c->static_device] = false;
  }
  if (c) {
    for (auto& ev : c->E.aux_ev)
      if (ev) (void)hipEventDestroy(ev);
    if (c->E.aux) {
      (void)hipStreamSynchronize(c->E.aux);
      (void)hipStreamDestroy(c->E.aux);
    }
  }
  delete c;
}

ctm_status ctm_sweep(ctm_ctx* c, int max_sweeps, double tol, int* sweeps_done, double* delta) {
  if (!c || max_sweeps < 0) return CTM_EINVAL;
  Engine& E = c->E;
  begin(c);
  const Peps A = peps_view(*c, c->Aflat);
  int done = 0;
  double d = INFINITY;
  bool conv = false;
  for (int s = 0; s < max_sweeps && E.ok(); ++s) {
    // a measured sweep compares with the spectra of its own start environment
    const bool measure = tol > 0 || (delta && s == max_sweeps - 1);
    if (measure && !c->spec_current) corner_delta(c);
    for (int dir = 0; dir < 4 && E.ok(); ++dir) {
      size_t mk = E.ar.mark();
      Env env = view_env(*c, c->cur_blk);
      Env out = do_move(*c, env, A, dir);
      store_env(*c, out, c->cur_blk);
      E.ar.release(mk);
    }
    ++done;
    if (!measure) c->spec_current = false;   // spec_prev no longer belongs to the current environment
    if (measure) {
      d = corner_delta(c);
      if (!(d == d)) {
        if (sweeps_done) *sweeps_done = done;
        if (delta) *delta = d;
        return finish(c, CTM_ENUMERIC);
      }
      if (tol > 0 && d < tol) {
        conv = true;
        break;
      }
    }
  }
  if (E.ok()) E.check(hipStreamSynchronize(E.s));
  if (sweeps_done) *sweeps_done = done;
  if (delta) *delta = d;
  ctm_status st = (ctm_status)status_from_engine(E);
  if (st == CTM_OK && tol > 0 && !conv) st = CTM_ENOTCONV;
  return finish(c, st);
}

ctm_status ctm_energy(ctm_ctx* c, const double* h_host, double* e_site, double* e_bonds) {
  return ctm_energy_hv(c, h_host, h_host, e_site, e_bonds);
}

ctm_status ctm_energy_hv(ctm_ctx* c, const double* h_host, const double* hv_host, double* e_site, double* e_bonds) {
  if (!c || !h_host || !hv_host) return CTM_EINVAL;
  Engine& E = c->E;
  begin(c);
  if (E.ok()) E.check(hipMemcpyAsync(c->h64.p, h_host, c->h64.bytes(), hipMemcpyHostToDevice, E.s));
  if (E.ok()) E.check(hipMemcpyAsync(c->h64v.p, hv_host, c->h64v.bytes(), hipMemcpyHostToDevice, E.s));
  const Peps A = peps_view(*c, c->Aflat);
  Env env = view_env(*c, c->cur_blk);
  std::vector<Ten> eh, ev;
  energies(*c, env, A, eh, ev);
  const double tot = site_energy_dev(*c, eh, ev, e_bonds);
  if (e_site) *e_site = tot;
  ctm_status st = (ctm_status)status_from_engine(E);
  if (st == CTM_OK && !std::isfinite(tot)) st = CTM_ENUMERIC;
  return finish(c, st);
}

ctm_status ctm_projectors(ctm_ctx* c, int direction, int x, int y, double* out_dev, double* trunc_err) {
  if (!c || direction < 0 || direction > 3 || !out_dev) return CTM_EINVAL;
  if (x < 0 || y < 0 || x >= c->Lx || y >= c->Ly) return CTM_EINVAL;
  Engine& E = c->E;
  begin(c);
  const Peps A = peps_view(*c, c->Aflat);
  Env env = view_env(*c, c->cur_blk);
  Env fe;
  Peps fa;
  to_frame(E, direction, env, A, fe, fa);
  int fx = x, fy = y;
  if (direction == 1) {
    fx = y;
    fy = x;
  } else if (direction == 2) {
    fx = (c->Lx - x) % c->Lx;
    fy = (c->Ly - y) % c->Ly;
  } else if (direction == 3) {
    fx = (fe.Lx - y) % fe.Lx;
    fy = (fe.Ly - x) % fe.Ly;
  }
  Column col;
  left_column(*c, fe, fa, fy, &col, fx, -1);
  const std::vector<Ten> pr[4] = {col.G[fx], col.TH[fx], col.Y[fx], col.R[fx]};
  const std::vector<double>* sp[4] = {&col.sG[fx], &col.sTH[fx], &col.sY[fx], &col.sR[fx]};
  const int chis[4] = {c->chiE, c->chiE, c->chiI, c->chiI};
  size_t off = 0;
  for (int k = 0; k < 4 && E.ok(); ++k) {
    for (int j = 0; j < 2; ++j) {
      const Ten& t = pr[k][j];
      if (t.dt == F64)
        E.check(hipMemcpyAsync(out_dev + off, t.p, t.bytes(), hipMemcpyDeviceToDevice, E.s));
      else
        E.check(cast_f32_to_f64(E.s, t.f32(), out_dev + off, t.n()));
      off += t.n();
    }
    if (trunc_err) {
      const std::vector<double>& S = *sp[k];
      double tot = 0, kept = 0;
      int cnt = 0;
      for (size_t i = 0; i < S.size(); ++i) {
        tot += S[i] * S[i];
        if (S[0] > 0 && S[i] > E.cutoff * S[0] && cnt < chis[k]) {
          kept += S[i] * S[i];
          ++cnt;
        }
      }
      trunc_err[k] = tot > 0 ? (tot - kept) / tot : 0.0;
    }
  }
  if (E.ok()) E.check(hipStreamSynchronize(E.s));
  return finish(c, (ctm_status)status_from_engine(E));
}

ctm_status ctm_move_column(ctm_ctx* c, int direction, int y) {
  if (!c || direction < 0 || direction > 3) return CTM_EINVAL;
  const int ny = (direction == 1 || direction == 3) ? c->Lx : c->Ly;   // columns in the move's frame
  if (y < 0 || y >= ny) return CTM_EINVAL;
  Engine& E = c->E;
  begin(c);
  const Peps A = peps_view(*c, c->Aflat);
  {
    size_t mk = E.ar.mark();
    Env env = view_env(*c, c->cur_blk);
    Env fe;
    Peps fa;
    to_frame(E, direction, env, A, fe, fa);
    // frame column y holds the sites that direction's move absorbs y-th
    left_column(*c, fe, fa, y, nullptr, -1, direction);
    Env out;
    from_frame(E, direction, fe, out);
    store_env(*c, out, c->cur_blk);
    E.ar.release(mk);
  }
  c->spec_current = false;
  if (E.ok()) E.check(hipStreamSynchronize(E.s));
  return finish(c, (ctm_status)status_from_engine(E));
}

ctm_status ctm_energy_grad(ctm_ctx* c, const double* h_host, int n_sweeps, int ckpt_every, double* e_site,
                           double* dA_dev) {
  return ctm_energy_grad_hv(c, h_host, h_host, n_sweeps, ckpt_every, e_site, dA_dev);
}

ctm_status ctm_energy_grad_hv(ctm_ctx* c, const double* h_host, const double* hv_host, int n_sweeps, int ckpt_every,
                              double* e_site, double* dA_dev) {
  if (!c || !h_host || !hv_host || !dA_dev || n_sweeps < 0 || ckpt_every < 1) return CTM_EINVAL;
  begin(c);
  c->spec_current = false;
  ctm_status st = energy_grad_impl(c, h_host, hv_host, n_sweeps, ckpt_every, e_site, dA_dev);
  return finish(c, st);
}

ctm_status ctm_env_export(ctm_ctx* c, double* env_dev) {
  if (!c || !env_dev) return CTM_EINVAL;
  Engine& E = c->E;
  if (c->cur_blk.dt == F64)
    E.check(hipMemcpyAsync(env_dev, c->cur_blk.p, c->cur_blk.bytes(), hipMemcpyDeviceToDevice, E.s));
  else
    E.check(cast_f32_to_f64(E.s, c->cur_blk.f32(), env_dev, c->cur_blk.n()));
  E.check(hipStreamSynchronize(E.s));
  return (ctm_status)status_from_engine(E);
}

ctm_status ctm_env_import(ctm_ctx* c, const double* env_dev) {
  if (!c || !env_dev) return CTM_EINVAL;
  Engine& E = c->E;
  if (c->cur_blk.dt == F64)
    E.check(hipMemcpyAsync(c->cur_blk.p, env_dev, c->cur_blk.bytes(), hipMemcpyDeviceToDevice, E.s));
  else
    E.check(cast_f64_to_f32(E.s, env_dev, c->cur_blk.f32(), c->cur_blk.n()));
  E.check(hipMemcpyAsync(c->start_blk.p, c->cur_blk.p, c->cur_blk.bytes(), hipMemcpyDeviceToDevice, E.s));
  E.check(hipStreamSynchronize(E.s));
  c->spec_current = false;
  return (ctm_status)status_from_engine(E);
}

size_t ctm_debug_gemm_work_bytes(int prec, int M, int N, int K) {
  if (prec == CTM_BF16X3 && M > 0 && N > 0 && K > 0) {
    const size_t bb = bf16x3_big_scratch_bytes(M, N, K);
    if (bb) return bb;
  }
  return (size_t)splitk_scratch_elems(M, N, K) * (prec == CTM_FP64 ? 8 : 4);
}

ctm_status ctm_debug_gemm(int prec, int transA, int transB, int M, int N, int K, const void* A, const void* B,
                          void* C, void* work, void* stream) {
  if (M < 0 || N < 0 || K < 1 || !A || !B || !C || prec < 0 || prec > 3) return CTM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const long lda = transA ? M : K, ldb = transB ? K : N;
  const bool split = work && splitk_scratch_elems(M, N, K) > 0;
  hipError_t e;
  if (prec == CTM_BF16X3 && work && M > 0 && N > 0 && bf16x3_big_scratch_bytes(M, N, K) > 0) {
    e = gemm_bf16x3_big(s, transA, transB, M, N, K, 1.f, (const float*)A, lda, (const float*)B, ldb, 0.f, (float*)C,
                        N, work);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? CTM_OK : CTM_EDEVICE;
  }
  if (prec == CTM_FP64)
    e = split ? gemm_f64_splitk(s, transA, transB, M, N, K, 1.0, (const double*)A, lda, (const double*)B, ldb, 0.0,
                                (double*)C, N, (double*)work)
              : gemm_f64(s, transA, transB, M, N, K, 1.0, (const double*)A, lda, 0, (const double*)B, ldb, 0, 0.0,
                         (double*)C, N, 0, 1);
  else {
    const Prec md = (Prec)prec;
    e = split ? gemm_f32_splitk(s, md, transA, transB, M, N, K, 1.f, (const float*)A, lda, (const float*)B, ldb, 0.f,
                                (float*)C, N, (float*)work)
              : gemm_f32(s, md, transA, transB, M, N, K, 1.f, (const float*)A, lda, 0, (const float*)B, ldb, 0, 0.f,
                         (float*)C, N, 0, 1);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? CTM_OK : CTM_EDEVICE;
}

size_t ctm_debug_svd_work_bytes(int n, int batch) { return svd_precond_work_bytes(n, batch); }

size_t ctm_debug_qr_work_bytes(int m, int k, int batch) {
  return (m >= k && k >= 1 && batch >= 1) ? qr_work_bytes(m, k, batch) : 0;
}

ctm_status ctm_debug_qr(int m, int k, int batch, double* Xt, double* R, double* Qt, void* work, void* stream) {
  if (m < k || k < 1 || batch < 1 || m > 8192 || !Xt || !work) return CTM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = qr_f64(s, m, k, batch, Xt, R, Qt, work);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? CTM_OK : CTM_EDEVICE;
}

ctm_status ctm_debug_svd(int n, int batch, const double* M, double* U, double* S, double* V, void* work,
                         int* sweeps, void* stream) {
  if (n < 1 || n > 4096 || batch < 1 || batch > 256 || !M || !U || !S || !V || !work) return CTM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  int flags[256];
  const int max_sweeps = (sweeps && *sweeps > 0) ? *sweeps : 60;
  hipError_t e = svd_precond_f64(s, n, batch, M, U, S, V, work, max_sweeps, 0.0, flags, sweeps);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? CTM_OK : CTM_EDEVICE;
}

ctm_status ctm_kernel_timing_enable(ctm_ctx* c, int on) {
  if (!c || on < 0) return CTM_EINVAL;
  c->timing = on != 0;
  c->timer.reset();
  c->timer.stride = on > 0 ? on : 1;
  return CTM_OK;
}

ctm_status ctm_kernel_timing(ctm_ctx* c, int kernel_class, double* ms, double* launches, double* flops,
                             double* bytes) {
  if (!c || kernel_class < 0 || kernel_class >= KC_COUNT) return CTM_EINVAL;
  if (ms) *ms = c->timer.ms(kernel_class);
  if (launches) *launches = c->timer.launches[kernel_class];
  if (flops) *flops = c->timer.flops[kernel_class];
  if (bytes) *bytes = c->timer.bytes[kernel_class];
  return CTM_OK;
}

ctm_status ctm_last_stats(ctm_ctx* c, double* gemm_flops, double* svd_sweeps) {
  if (!c) return CTM_EINVAL;
  if (gemm_flops) *gemm_flops = c->last_flops;
  if (svd_sweeps) *svd_sweeps = c->last_sweeps;
  return CTM_OK;
}

}  // extern "C"
