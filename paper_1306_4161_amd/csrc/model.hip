// Communication-cost model of the distributed algorithm (Sec. IV) and the
// choice of the number of groups G.  Host code only: the paper's analysis
// of the P x Q grid's broadcasts under Hockney's model, which the one-GPU
// library uses to say which G a distributed run would take.
//
// Every broadcast is T(m, q) = L(q) alpha + m W(q) beta (eq. (1)); binomial
// tree L = W = log2 q, Van de Geijn L = log2 q + q - 1, W = 2 (q - 1) / q.
// An inner step (block b) broadcasts A's pivot block of n b / P elements per
// process along a process row inside its group (Q / J processes) and B's
// block of n b / Q elements along a process column (P / I processes); an
// outer step (block B) does the same between groups, over J and I groups.
// There are ceil(n / b) inner and ceil(n / B) outer steps; the paper's
// closed forms take n / b and n / B, which is what is evaluated here.
#include <climits>
#include <cmath>
#include <set>
#include <utility>
#include <vector>

#include "internal.h"

namespace {

int model_invalid(const char* msg) {
  hs::set_error(msg);
  return HSUMMA_ERR_INVALID;
}

bool algo_ok(int32_t algo) {
  return algo == HSUMMA_BCAST_BINOMIAL || algo == HSUMMA_BCAST_VAN_DE_GEIJN;
}

// latency factor L(q) and bandwidth factor W(q) of one broadcast among q
void factors(int32_t algo, double q, double* L, double* W) {
  const double lg = std::log2(q);
  if (algo == HSUMMA_BCAST_BINOMIAL) {
    *L = lg;
    *W = lg;
  } else {
    *L = lg + q - 1.0;
    *W = 2.0 * (q - 1.0) / q;
  }
}

bool platform_ok(const hsumma_platform* pf) {
  return pf && pf->alpha >= 0.0 && pf->beta >= 0.0 && pf->gamma >= 0.0 &&
         std::isfinite(pf->alpha) && std::isfinite(pf->beta) && std::isfinite(pf->gamma);
}

// cost with the groups arranged I x J (validated by the caller)
void cost_of(int32_t algo, const hsumma_platform& pf, double n, int P, int Q, int I, int J,
             double b, double B, hsumma_cost* c) {
  double L, W;
  c->latency_inner = c->latency_outer = c->bandwidth_inner = c->bandwidth_outer = 0.0;
  // inside groups: n / b steps, row broadcast among Q / J, column among P / I
  const double in_steps = n / b;
  factors(algo, (double)Q / J, &L, &W);
  c->latency_inner += in_steps * L * pf.alpha;
  c->bandwidth_inner += in_steps * (n * b / P) * W * pf.beta;
  factors(algo, (double)P / I, &L, &W);
  c->latency_inner += in_steps * L * pf.alpha;
  c->bandwidth_inner += in_steps * (n * b / Q) * W * pf.beta;
  // between groups: n / B steps, row broadcast among J groups, column among I
  const double out_steps = n / B;
  factors(algo, (double)J, &L, &W);
  c->latency_outer += out_steps * L * pf.alpha;
  c->bandwidth_outer += out_steps * (n * B / P) * W * pf.beta;
  factors(algo, (double)I, &L, &W);
  c->latency_outer += out_steps * L * pf.alpha;
  c->bandwidth_outer += out_steps * (n * B / Q) * W * pf.beta;
  c->comm = c->latency_inner + c->latency_outer + c->bandwidth_inner + c->bandwidth_outer;
  c->comp = 2.0 * n * n * n / ((double)P * Q) * pf.gamma;
  c->total = c->comp + c->comm;
}

int check_shape(int64_t n, int32_t P, int32_t Q, int64_t b, int64_t B) {
  if (n < 1 || P < 1 || Q < 1 || b < 1 || B < 1) return model_invalid("sizes must be positive");
  if (b > B) return model_invalid("inner block b must not exceed the outer block B");
  return HSUMMA_OK;
}

}  // namespace

extern "C" {

int hsumma_model_bcast(int32_t algo, const hsumma_platform* pf, double m, double q,
                       double* seconds) {
  if (!seconds || !platform_ok(pf)) return model_invalid("null or invalid argument");
  if (!algo_ok(algo)) return model_invalid("unknown broadcast algorithm");
  if (!(q >= 1.0) || !(m >= 0.0)) return model_invalid("need q >= 1 and m >= 0");
  double L, W;
  factors(algo, q, &L, &W);
  *seconds = L * pf->alpha + m * W * pf->beta;
  return HSUMMA_OK;
}

int hsumma_model_cost(int32_t algo, const hsumma_platform* pf, int64_t n, int32_t P, int32_t Q,
                      int32_t G, int64_t b, int64_t B, hsumma_cost* out) {
  if (!out || !platform_ok(pf)) return model_invalid("null or invalid argument");
  if (!algo_ok(algo)) return model_invalid("unknown broadcast algorithm");
  int rc = check_shape(n, P, Q, b, B);
  if (rc) return rc;
  int I = 0, J = 0;
  if (G < 1 || !hs::factor_groups(P, Q, G, &I, &J))
    return model_invalid("G cannot be arranged as I x J groups with I | P and J | Q");
  cost_of(algo, *pf, (double)n, P, Q, I, J, (double)b, (double)B, out);
  return HSUMMA_OK;
}

int hsumma_model_dcomm_dgroups(const hsumma_platform* pf, int64_t n, double p, double G,
                               int64_t b, double* derivative) {
  if (!derivative || !platform_ok(pf)) return model_invalid("null or invalid argument");
  if (n < 1 || b < 1 || !(p >= 1.0) || !(G >= 1.0) || G > p)
    return model_invalid("need n, b >= 1 and 1 <= G <= p");
  // d/dG of the Van de Geijn cost with b = B on a sqrt(p) x sqrt(p) grid
  const double nd = (double)n;
  *derivative = (G - std::sqrt(p)) / (G * std::sqrt(G)) *
                (nd * pf->alpha / (double)b - 2.0 * nd * nd / p * pf->beta);
  return HSUMMA_OK;
}

int hsumma_model_cost_levels(int32_t algo, const hsumma_platform* pf, int64_t n, int32_t P,
                             int32_t Q, int32_t nlevels, const int32_t* I, const int32_t* J,
                             const int64_t* blocks, hsumma_cost* out, double* per_level) {
  if (!out || !I || !J || !blocks || !platform_ok(pf)) return model_invalid("null or invalid argument");
  if (!algo_ok(algo)) return model_invalid("unknown broadcast algorithm");
  if (n < 1 || P < 1 || Q < 1) return model_invalid("sizes must be positive");
  if (nlevels < 1 || nlevels > 16) return model_invalid("need 1 <= nlevels <= 16");
  int64_t pi = 1, pj = 1;
  for (int l = 0; l < nlevels; ++l) {
    if (I[l] < 1 || J[l] < 1 || blocks[l] < 1) return model_invalid("level sizes must be positive");
    if (l > 0 && blocks[l] > blocks[l - 1])
      return model_invalid("blocks must not grow from the outer to the inner levels");
    pi *= I[l];
    pj *= J[l];
    if (pi > P || pj > Q) break;
  }
  if (pi != P || pj != Q) return model_invalid("the levels' arrangements must multiply to P x Q");
  *out = hsumma_cost{};
  const double nd = (double)n;
  for (int l = 0; l < nlevels; ++l) {
    const double steps = nd / (double)blocks[l];
    double L, W, lat = 0.0, band = 0.0;
    factors(algo, (double)J[l], &L, &W);      // A's block along a row
    lat += steps * L * pf->alpha;
    band += steps * (nd * blocks[l] / P) * W * pf->beta;
    factors(algo, (double)I[l], &L, &W);      // B's block along a column
    lat += steps * L * pf->alpha;
    band += steps * (nd * blocks[l] / Q) * W * pf->beta;
    if (l == nlevels - 1) {
      out->latency_inner = lat;
      out->bandwidth_inner = band;
    } else {
      out->latency_outer += lat;
      out->bandwidth_outer += band;
    }
    if (per_level) per_level[l] = lat + band;
  }
  out->comm = out->latency_inner + out->latency_outer + out->bandwidth_inner + out->bandwidth_outer;
  out->comp = 2.0 * nd * nd * nd / ((double)P * Q) * pf->gamma;
  out->total = out->comp + out->comm;
  return HSUMMA_OK;
}

int hsumma_model_select_groups(int32_t algo, const hsumma_platform* pf, int64_t n, int32_t P,
                               int32_t Q, int64_t b, int64_t B, int32_t* G_best,
                               hsumma_cost* best, hsumma_cost* summa) {
  if (!platform_ok(pf)) return model_invalid("null or invalid argument");
  if (!algo_ok(algo)) return model_invalid("unknown broadcast algorithm");
  int rc = check_shape(n, P, Q, b, B);
  if (rc) return rc;
  // every arrangeable G = I x J (I | P, J | Q), each in the plan's arrangement
  std::set<int64_t> counts;
  for (int32_t I = 1; I <= P; ++I)
    if (P % I == 0)
      for (int32_t J = 1; J <= Q; ++J)
        if (Q % J == 0) counts.insert((int64_t)I * J);
  std::vector<std::pair<int32_t, hsumma_cost>> all;
  double cmin = 0.0;
  for (int64_t G : counts) {
    int I = 0, J = 0;
    if (G > INT32_MAX || !hs::factor_groups(P, Q, (int)G, &I, &J)) continue;
    hsumma_cost c{};
    cost_of(algo, *pf, (double)n, P, Q, I, J, (double)b, (double)B, &c);
    if (all.empty() || c.comm < cmin) cmin = c.comm;
    all.push_back({(int32_t)G, c});
  }
  // costs equal up to rounding (e.g. binomial broadcasts with b = B, where
  // every G costs the same) go to the smaller G
  int32_t gbest = 0;
  hsumma_cost cbest{};
  for (auto& gc : all)
    if (gc.second.comm <= cmin * (1.0 + 1e-12)) {
      gbest = gc.first;
      cbest = gc.second;
      break;
    }
  if (G_best) *G_best = gbest;
  if (best) *best = cbest;
  if (summa) cost_of(algo, *pf, (double)n, P, Q, 1, 1, (double)b, (double)b, summa);
  return HSUMMA_OK;
}

}  // extern "C"
