// Scalar part of one step of the stop and branch logic (Alg. 2; Alg. 4
// with a schedule; the McWeeny stop of sec. 3), shared by the finalize
// kernel of the launch-per-step driver and the persistent batch kernel. It
// runs on one thread of the workgroup that finished the step's partial
// sums, so that both drivers take the same decisions from the same values.
#pragma once

#include <math.h>

#include "sp2_device.h"

namespace sp2 {

// C of Alg. 2: the smallest constant with r_k >= 2 in exact arithmetic over
// two alternating SP2 steps, (71 + 17 sqrt 17) / 32.
__device__ __forceinline__ double c_sp2() {
  return (71.0 + 17.0 * sqrt(17.0)) / 32.0;
}
// q~ of sec. 2.
constexpr double kQTilde = 1.8;
// sec. 3: C_2 of the McWeeny and McW-ACC expansions.
constexpr double kCMcWeeny = 4.0;

__device__ __forceinline__ void publish(DevState* st, int32_t* ndone,
                                        int count, HostMirror* m, int status,
                                        int n) {
  st->status = status;
  st->n = n;
  st->done = 1;
  __threadfence();
  const int before = atomicAdd(ndone, 1);
  if (before == count - 1 && m)
    __hip_atomic_store(&m->all_done, 1, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_SYSTEM);
}

// Applies step `iter` of the scalar logic to instance `in` from the sums of
// its partial triples (a = sum (x - s)^2, b = Tr, c = sum x^2; mk, mk_steps:
// the mixed norm and its Lanczos steps):
//   iter == 0: Tr X~_0, Tr X~_0^2; divergence check; choose p_1 (an
//     instance with n_occ = 0 or n stops here with n = 0).
//   iter >= 1: v_{iter-1} from the square of X~_{iter-1}; Tr/Tr^2 of X~_iter;
//     stop test at k = iter - 1 (from k = 2, or from n_min with a schedule;
//     a schedule also ends at k = n_max); divergence; max_iter; choose
//     p_{iter+1}, its stretch and its epilogue coefficients.
// Returns true when the instance's outcome was published (it stopped).
__device__ inline bool finalize_scalar(const Instance& in, int iter, double a,
                                       double b, double c, double mk,
                                       int mk_steps, int32_t* ndone, int count,
                                       HostMirror* mirror) {
  DevState* st = in.st;
  const StopParams& prm = in.prm;
  const bool sched = prm.n_max > 0;
  const bool mw = (prm.method == 1);
  const double t1 = b, t2 = c;
  st->t1[iter] = t1;
  st->t2[iter] = t2;
  if (iter == 0) {
    if (prm.n_occ == 0.0 || prm.n_occ == prm.n) {
      publish(st, ndone, count, mirror, /*OK*/ 0, 0);
      return true;
    }
    if (!isfinite(t1) || !isfinite(t2)) {
      publish(st, ndone, count, mirror, /*DIVERGED*/ 5, 0);
      return true;
    }
  } else {
    const int k = iter - 1;
    const double vk = sqrt(a);
    st->v[k] = vk;
    if (prm.norm == 1) {   // the spectral kernel writes m[k] itself
      st->m[k] = mk;
      st->krylov[k] = mk_steps;
    }
    st->squares = iter;
    // the error the stop test reads: Frobenius, mixed or spectral (sec. 2)
    const double* e = (prm.norm != 0) ? st->m : st->v;
    const double ek = e[k];
    double r = NAN;
    if (mw) {
      // McWeeny: one polynomial per step, C = 4 (sec. 3)
      if (k >= 1) {
        const double ekm1 = e[k - 1];
        if (ekm1 > 0.0 && ekm1 < 1.0 && ek > 0.0)
          r = log(ek / kCMcWeeny) / log(ekm1);
      }
    } else if (k >= 2) {
      const double ekm2 = e[k - 2];
      if (ekm2 > 0.0 && ekm2 < 1.0 && ek > 0.0)
        r = log(ek / c_sp2()) / log(ekm2);   // observed order (sec. 2)
    }
    st->r[k] = r;
    if (!isfinite(vk)) {
      publish(st, ndone, count, mirror, 5, k);
      return true;
    }
    if (vk == 0.0) {                          // exactly idempotent
      publish(st, ndone, count, mirror, 0, k);
      return true;
    }
    if (mw) {
      if (k >= prm.mw_first && !isnan(r) && r < kQTilde) {
        publish(st, ndone, count, mirror, 0, k);   // McWeeny stop (sec. 3)
        return true;
      }
    } else {
      const int kmin = sched ? prm.n_min : 2;
      if (k >= kmin && st->p[k] != st->p[k - 1] && !isnan(r) && r < kQTilde) {
        publish(st, ndone, count, mirror, 0, k);   // Alg. 2 / Alg. 4 stop
        return true;
      }
    }
    if (sched && k >= prm.n_max) {               // the schedule has ended
      publish(st, ndone, count, mirror, 0, k);
      return true;
    }
    if (!isfinite(t1) || !isfinite(t2) || t2 > t1 + prm.n) {
      publish(st, ndone, count, mirror, 5, iter);
      return true;
    }
    if (iter >= prm.max_iter) {
      publish(st, ndone, count, mirror, /*NOT_CONVERGED*/ 4, iter);
      return true;
    }
  }
  // Polynomial of the next step: from the schedule (Alg. 4), or from the
  // traces of X~_iter (Alg. 2 branch). Past the schedule's end one more
  // square is needed for v_{n_max}; the iterate it yields is not used.
  // McWeeny: one polynomial; the stretch of McW-ACC from the host's table
  // (computed from the beta recursion at set-up, switched off once
  // beta < 0.01 with the Frobenius or the mixed norm).
  int pn;
  double an = 1.0;
  if (mw) {
    const int i = iter + 1;
    pn = 1;
    if (i <= prm.mw_len) an = in.sched_alpha[i];
  } else if (sched) {
    const int i = iter + 1;
    if (i <= prm.n_max) {
      pn = in.sched_p[i];
      an = in.sched_alpha[i];
    } else {
      pn = 1 - st->p[iter];
    }
  } else if (prm.branch == 1) {
    pn = (t1 > prm.n_occ) ? 1 : 0;
  } else {
    pn = (fabs(t2 - prm.n_occ) < fabs(2.0 * t1 - t2 - prm.n_occ)) ? 1 : 0;
  }
  st->p[iter + 1] = static_cast<int8_t>(pn);
  st->alpha[iter + 1] = an;
  // epilogue coefficients of step iter + 1: the error of X~_iter from the
  // stored matrix of that step and its square, and the map of the matrix
  // it stores for step iter + 2
  const OpMap nxt = step_map(in, iter + 2);
  const StepCoef e = step_coef(op_map(prm.method, pn, an), nxt);
  st->ecoef[0] = e.ey;
  st->ecoef[1] = e.es;
  st->ecoef[2] = e.ei;
  st->ecoef[3] = e.an;
  st->ecoef[4] = e.cn;
  st->stretch = (nxt.a != 1.0 || nxt.c != 0.0) ? 1 : 0;
  return false;
}

}  // namespace sp2
