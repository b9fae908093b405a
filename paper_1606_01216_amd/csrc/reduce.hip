// AIRGA's outer iteration as one library call (Algorithm 1, with the SPAI
// preconditioned solves of Algorithm 3 and the updated chains of
// Algorithm 5).  Host orchestration only: every vector operation runs in the
// library's kernels through its own entry points (batched SPAI builds and
// updates, batched PCG, the moment-sequence block operations, the
// projection), and the small decisions run on the host (poles, next
// expansion points, H2 distances).
//
// Readings of the steps the paper leaves to Bonin et al.:
//   A1  the moment error at s_i is ||X after|| / ||X before|| of the newest
//       moment block orthogonalised against V_1..V_j; sigma_{j+1} is the
//       point with the largest (first index on a tie), sigma_1 = s_1.
//   A2  points are told apart by index.
//   A3  the final basis has J <= floor(r_max / m) blocks.
//   A4  next points: -Re(lambda) per conjugate pair, -lambda per real pole,
//       the l smallest |lambda|, ascending (airga_next_shifts); the i-th new
//       point's preconditioner is the update of the i-th old one.
//   A5  both loops stop on the relative H2 change of the reduced model.
#include <cmath>
#include <cstring>
#include <limits>
#include <vector>

#include "internal.hpp"

namespace airga {
namespace {

constexpr int kOrthChunk = 16;  // basis blocks per airga_global_orth call

// Host copy of a small device matrix (synchronises the context stream).
airga_status host_copy(airga_ctx ctx, const double* d, size_t count, std::vector<double>* h) {
  h->resize(count);
  if (count == 0) return AIRGA_OK;
  AIRGA_HIP(hipMemcpyAsync(h->data(), d, sizeof(double) * count, hipMemcpyDeviceToHost,
                           ctx->stream));
  AIRGA_HIP(hipStreamSynchronize(ctx->stream));
  return AIRGA_OK;
}

// A reduced model held on the host (column-major).
struct Reduced {
  int r = 0, m = 0, p = 0;
  bool has_cv = false;
  std::vector<double> mh, kh, fh, cph, cvh;
  airga_reduced_model view() const {
    airga_reduced_model v;
    v.r = r;
    v.m = m;
    v.p = p;
    v.mhat = mh.data();
    v.khat = kh.data();
    v.fhat = fh.data();
    v.cphat = cph.data();
    v.cvhat = has_cv ? cvh.data() : nullptr;
    return v;
  }
};

struct Problem {
  airga_ctx ctx;
  int64_t n;
  int32_t m, p;
  const double* F;
  int64_t ldf;
  const double* Cp;
  const double* Cv;
  int64_t ldc;
  double* G;  // device scratch for W^T F and W^T C (64 x max(m, p) doubles)
};

// Galerkin projection of eq. (1.4) onto the k orthonormal columns of W:
// Mh = W^T M W, Kh = W^T K W, Fh = W^T F, Cph = C_p W, Cvh = C_v W.
airga_status project_model(const Problem& P, int k, const double* W, int64_t ldw, Reduced* out) {
  out->r = k;
  out->m = P.m;
  out->p = P.p;
  out->has_cv = P.Cv != nullptr;
  out->mh.resize((size_t)k * k);
  out->kh.resize((size_t)k * k);
  AIRGA_TRY(airga_project(P.ctx, k, W, ldw, out->mh.data(), out->kh.data()));
  std::vector<double> g;
  AIRGA_TRY(airga_gram(P.ctx, k, W, ldw, P.m, P.F, P.ldf, P.G));
  AIRGA_TRY(host_copy(P.ctx, P.G, (size_t)k * P.m, &out->fh));
  for (int pass = 0; pass < (P.Cv ? 2 : 1); ++pass) {
    AIRGA_TRY(airga_gram(P.ctx, k, W, ldw, P.p, pass ? P.Cv : P.Cp, P.ldc, P.G));
    AIRGA_TRY(host_copy(P.ctx, P.G, (size_t)k * P.p, &g));
    // G = W^T C^T is k x p; the model keeps C W, p x k
    std::vector<double>& c = pass ? out->cvh : out->cph;
    c.resize((size_t)P.p * k);
    for (int i = 0; i < k; ++i)
      for (int q = 0; q < P.p; ++q) c[q + (size_t)i * P.p] = g[i + (size_t)q * k];
  }
  return AIRGA_OK;
}

// Relative H2 change ||H_new - H_old|| / ||H_new|| (reading A5); NaN when
// the norm is not a positive finite number (then no test can pass).
airga_status relative_change(const Reduced& a, const Reduced& b, double alpha, double beta,
                             double* out) {
  const airga_reduced_model va = a.view(), vb = b.view();
  double d = 0, nrm = 0;
  AIRGA_TRY(airga_h2_distance(&va, &vb, alpha, beta, &d));
  AIRGA_TRY(airga_h2_distance(&va, nullptr, alpha, beta, &nrm));
  *out = (std::isfinite(nrm) && nrm > 0) ? d / nrm : std::numeric_limits<double>::quiet_NaN();
  return AIRGA_OK;
}

// X_x (nx blocks of m columns at X) orthogonalised against the nb blocks at
// V in the trace inner product, in the order of the loop over t, in chunks
// the block kernel takes; fro = the blocks' Frobenius norms afterwards.
airga_status orth_chunks(const Problem& P, int nb, const double* V, int64_t ldv, int nx, double* X,
                         std::vector<double>* fro) {
  fro->assign(nx, 0.0);
  std::vector<double> gam((size_t)nx * kOrthChunk);
  if (nb == 0) return airga_global_orth(P.ctx, P.m, 0, nullptr, P.n, nx, X, P.n, 0, nullptr,
                                        fro->data());
  for (int t0 = 0; t0 < nb; t0 += kOrthChunk) {
    const int cnt = nb - t0 < kOrthChunk ? nb - t0 : kOrthChunk;
    AIRGA_TRY(airga_global_orth(P.ctx, P.m, cnt, V + (int64_t)t0 * P.m * ldv, ldv, nx, X, P.n, 0,
                                gam.data(), fro->data()));
  }
  return AIRGA_OK;
}

int first_max(const std::vector<double>& e) {
  int q = 0;
  for (int i = 1; i < (int)e.size(); ++i)
    if (e[i] > e[q]) q = i;
  return q;
}

}  // namespace
}  // namespace airga

using namespace airga;

extern "C" {

void airga_reduce_opts_default(airga_reduce_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->r_max = 24;
  o->tol_inner = 1e-6;
  o->tol_outer = 1e-6;
  o->max_outer = 10;
  o->update_from = 0;
  airga_spai_opts_default(&o->spai);
  airga_pcg_opts_default(&o->pcg);
}

airga_status airga_reduce(airga_ctx ctx, int32_t m, const double* F, int64_t ldf, int32_t p,
                          const double* Cp, const double* Cv, int64_t ldc, int32_t l,
                          const double* shifts0, const airga_reduce_opts* opts, double* V,
                          int64_t ldv, airga_reduce_result* res, double* shift_hist,
                          int32_t* sigma_hist, airga_reduce_iter* iter_hist) {
  AIRGA_TRY(check_pencil(ctx));
  DeviceGuard dg(ctx->device);
  airga_reduce_opts o;
  if (opts) o = *opts;
  else airga_reduce_opts_default(&o);
  const int64_t n = ctx->pen.n;
  if (m <= 0 || p <= 0 || l <= 0) return fail(AIRGA_EINVAL, "reduce: m, p and l must be positive");
  if (!F || !Cp || !shifts0 || !V || !res) return fail(AIRGA_EINVAL, "reduce: null argument");
  if (ldf < n || ldc < n || ldv < n) return fail(AIRGA_EINVAL, "reduce: leading dimension < n");
  const int jmax = o.r_max / m;
  if (jmax < 1) return fail(AIRGA_EINVAL, "reduce: r_max below the input count");
  if (o.max_outer < 1) return fail(AIRGA_EINVAL, "reduce: max_outer must be positive");
  if (!(o.tol_inner >= 0) || !(o.tol_outer >= 0))
    return fail(AIRGA_EINVAL, "reduce: tolerances must be non-negative");
  if (o.update_from != 0 && o.update_from < 2)
    return fail(AIRGA_EINVAL, "reduce: update_from must be 0 or at least 2");
  if (jmax * m > 64 || l * m > 64 || m > 16 || p > 256)
    return fail(AIRGA_EUNSUPPORTED,
                "reduce: at most 64 basis columns, l m <= 64, m <= 16 and p <= 256");
  for (int i = 0; i < l; ++i)
    if (!(shifts0[i] > 0) || !std::isfinite(shifts0[i]))
      return fail(AIRGA_EINVAL, "reduce: expansion points must be positive and finite");
  const double alpha = ctx->pen.alpha, beta = ctx->pen.beta;
  const int lm = l * m;

  // device work areas: the l state blocks, their normalised copy W, the
  // right-hand side of a moment solve, and W^T F / W^T C
  DevBuf area;
  const size_t blk = (size_t)n * lm;
  AIRGA_TRY(area.reserve(sizeof(double) * (2 * blk + (size_t)n * m + 64 * 256)));
  double* xs = area.as<double>();
  double* W = xs + blk;
  double* rhs = W + blk;
  const Problem P{ctx, n, m, p, F, ldf, Cp, Cv, ldc, rhs + (size_t)n * m};

  std::vector<double> shifts(shifts0, shifts0 + l);
  std::vector<airga_prec> precs(l, nullptr), old(l, nullptr);
  auto release_all = [&](std::vector<airga_prec>& v) {
    for (auto& q : v) {
      airga_prec_release(q);
      q = nullptr;
    }
  };
  std::vector<airga_sys_stats> st((size_t)lm);
  Reduced final_prev, final_cur;
  bool have_prev = false;
  // the caller's output pointers stay; the scalar results start cleared
  res->iterations = 0;
  res->converged = 0;
  res->r = 0;
  res->change = std::numeric_limits<double>::quiet_NaN();
  airga_status status = AIRGA_OK;
  int z = 0;
  for (; z < o.max_outer; ++z) {
    airga_reduce_iter it;
    std::memset(&it, 0, sizeof it);
    it.change = std::numeric_limits<double>::quiet_NaN();
    it.last_inner_change = std::numeric_limits<double>::quiet_NaN();
    it.all_converged = 1;
    // preconditioners at this iteration's points: new builds, or (from
    // iteration update_from on) the updates of the previous ones
    const bool upd = o.update_from > 0 && z + 1 >= o.update_from && old[0] != nullptr;
    if (upd)
      status = airga_spai_update_many(ctx, l, old.data(), shifts.data(), &o.spai, precs.data());
    else
      status = airga_spai_build_many(ctx, l, shifts.data(), &o.spai, precs.data());
    if (status != AIRGA_OK) break;
    it.updated = upd ? 1 : 0;
    for (int i = 0; i < l; ++i) {
      airga_prec_info pi;
      if ((status = airga_get_prec_info(precs[i], &pi)) != AIRGA_OK) break;
      if (pi.chain_len > it.chain_len_max) it.chain_len_max = pi.chain_len;
    }
    if (status != AIRGA_OK) break;
    auto note = [&](const airga_sys_stats* s, int count) {
      for (int i = 0; i < count; ++i) {
        if (s[i].status != AIRGA_SYS_CONVERGED) it.all_converged = 0;
        if (s[i].iters > it.max_iters) it.max_iters = s[i].iters;
      }
    };
    // X(s_i) = K(s_i)^{-1} F at every point, each replaced by its thin QR
    airga_pcg_opts po = o.pcg;
    po.x0_given = 0;
    if ((status = airga_pcg_solve(ctx, l, shifts.data(), precs.data(), m, F, ldf, xs, n, &po,
                                  st.data())) != AIRGA_OK)
      break;
    note(st.data(), lm);
    std::vector<double> rr((size_t)m * m);
    for (int i = 0; i < l && status == AIRGA_OK; ++i)
      status = airga_block_qr(ctx, m, xs + (size_t)i * m * n, n, rr.data());
    if (status != AIRGA_OK) break;

    // the moment loop
    std::vector<int> sigmas;
    std::vector<double> errors, before, after;
    bool have_errors = false;
    Reduced inner_prev, inner_cur;
    bool have_inner = false;
    auto take_block = [&]() -> airga_status {
      const int q = have_errors ? first_max(errors) : 0;
      sigmas.push_back(q);
      double* vj = V + (int64_t)(sigmas.size() - 1) * m * ldv;
      for (int c = 0; c < m; ++c)
        AIRGA_HIP(hipMemcpyAsync(vj + (int64_t)c * ldv, xs + ((size_t)q * m + c) * n,
                                 sizeof(double) * n, hipMemcpyDeviceToDevice, ctx->stream));
      std::vector<double> fro(1);
      return airga_global_orth(ctx, m, 0, nullptr, ldv, 1, vj, ldv, 1, nullptr, fro.data());
    };
    while ((int)sigmas.size() + 1 < jmax) {
      if ((status = take_block()) != AIRGA_OK) break;
      const int q = sigmas.back();
      const int j = (int)sigmas.size();
      const double* vj = V + (int64_t)(j - 1) * m * ldv;
      // the next moment at sigma: -K(sigma)^{-1} M V_j, into the state block
      if ((status = airga_pencil_apply(ctx, -1.0, 0.0, m, vj, ldv, rhs, n)) != AIRGA_OK) break;
      if ((status = airga_pcg_solve(ctx, 1, &shifts[q], &precs[q], m, rhs, n,
                                    xs + (size_t)q * m * n, n, &po, st.data())) != AIRGA_OK)
        break;
      note(st.data(), m);
      // moment errors: the part of each block outside V_1..V_j (A1)
      if ((status = orth_chunks(P, 0, nullptr, ldv, l, xs, &before)) != AIRGA_OK) break;
      if ((status = orth_chunks(P, j, V, ldv, l, xs, &after)) != AIRGA_OK) break;
      errors.resize(l);
      for (int i = 0; i < l; ++i) errors[i] = before[i] > 0 ? after[i] / before[i] : 0.0;
      have_errors = true;
      // the intermediate model on the normalised blocks
      AIRGA_HIP(hipMemcpyAsync(W, xs, sizeof(double) * blk, hipMemcpyDeviceToDevice, ctx->stream));
      std::vector<double> fro(l);
      if ((status = airga_global_orth(ctx, m, 0, nullptr, n, l, W, n, 1, nullptr, fro.data())) !=
          AIRGA_OK)
        break;
      std::vector<double> rw((size_t)lm * lm);
      if ((status = airga_block_qr(ctx, lm, W, n, rw.data())) != AIRGA_OK) break;
      if ((status = project_model(P, lm, W, n, &inner_cur)) != AIRGA_OK) break;
      it.moment_steps += 1;
      if (have_inner) {
        double ch = 0;
        if ((status = relative_change(inner_cur, inner_prev, alpha, beta, &ch)) != AIRGA_OK) break;
        it.last_inner_change = ch;
        if (ch < o.tol_inner) break;
      }
      inner_prev = inner_cur;
      have_inner = true;
    }
    if (status != AIRGA_OK) break;
    if ((status = take_block()) != AIRGA_OK) break;
    const int J = (int)sigmas.size();
    const int r = J * m;
    std::vector<double> rv((size_t)r * r);
    if ((status = airga_block_qr(ctx, r, V, ldv, rv.data())) != AIRGA_OK) break;
    if ((status = project_model(P, r, V, ldv, &final_cur)) != AIRGA_OK) break;
    it.blocks = J;
    if (have_prev &&
        (status = relative_change(final_cur, final_prev, alpha, beta, &it.change)) != AIRGA_OK)
      break;
    if (shift_hist)
      for (int i = 0; i < l; ++i) shift_hist[(size_t)z * l + i] = shifts[i];
    if (sigma_hist)
      for (int t = 0; t < jmax; ++t) sigma_hist[(size_t)z * jmax + t] = t < J ? sigmas[t] : -1;
    if (iter_hist) iter_hist[z] = it;
    res->iterations = z + 1;
    res->r = r;
    res->change = it.change;
    final_prev = final_cur;
    have_prev = true;
    release_all(old);
    old.swap(precs);
    if (it.change < o.tol_outer) {
      res->converged = 1;
      break;
    }
    // the next expansion points from the poles of the reduced model (A4)
    std::vector<double> re((size_t)2 * r), im((size_t)2 * r), nxt(l);
    if ((status = airga_qep_poles(r, final_cur.mh.data(), final_cur.kh.data(), alpha, beta,
                                  re.data(), im.data())) != AIRGA_OK)
      break;
    if ((status = airga_next_shifts(2 * r, re.data(), im.data(), l, nxt.data())) != AIRGA_OK)
      break;
    for (int i = 0; i < l; ++i) {
      if (!(nxt[i] > 0)) {
        status = fail(AIRGA_EUNSUPPORTED, "reduce: a new expansion point is not positive (%g)",
                      nxt[i]);
        break;
      }
      shifts[i] = nxt[i];
    }
    if (status != AIRGA_OK) break;
  }
  release_all(precs);
  release_all(old);
  if (status != AIRGA_OK) return status;
  // the last final model, for the caller
  const Reduced& fm = final_prev;
  const int r = fm.r;
  if (res->mhat) std::memcpy(res->mhat, fm.mh.data(), sizeof(double) * r * r);
  if (res->khat) std::memcpy(res->khat, fm.kh.data(), sizeof(double) * r * r);
  if (res->fhat) std::memcpy(res->fhat, fm.fh.data(), sizeof(double) * r * m);
  if (res->cphat) std::memcpy(res->cphat, fm.cph.data(), sizeof(double) * p * r);
  if (res->cvhat && Cv) std::memcpy(res->cvhat, fm.cvh.data(), sizeof(double) * p * r);
  if (res->next_shifts) std::memcpy(res->next_shifts, shifts.data(), sizeof(double) * l);
  return AIRGA_OK;
}

}  // extern "C"
