// Admission policy of the serving scheduler, kept free of HIP so that the
// same code runs in the library and, over a simulated pool, in host tests.
//
// A queued job goes to an idle worker when that worker's workspace, each
// buffer grown to the job's need, fits beside what the other workers hold
// (busy ones: the larger of their reservation and their real size; idle
// ones: their workspace).  When it does not fit, every idle workspace is
// released and the test is repeated.  Jobs may pass a job at the head of the
// queue that does not fit, until the head has waited too long; from then on
// only the head is considered.
#pragma once

#include <cstddef>

namespace gbem {

// One scheduling pass; returns true when a job was dispatched.  Pool:
//   size_t queue_size()                 jobs waiting, in submission order
//   int first_idle()                    an idle worker, or -1
//   size_t others(int w)                bytes the workers other than w may hold
//   size_t grown(int w, size_t qi)      w's workspace after growing to job qi's need
//   bool release_idle(size_t qi)        free the idle workspaces; false when job qi
//                                       is no longer at position qi (rescan)
//   void dispatch(size_t qi, int w, size_t mine, size_t total)
template <class Pool>
bool admit_one(Pool &pool, size_t budget, bool head_starving)
{
    for (size_t qi = 0; qi < pool.queue_size(); ++qi) {
        if (qi > 0 && head_starving) return false;
        const int w = pool.first_idle();
        if (w < 0) return false;
        size_t others = pool.others(w);
        size_t mine = pool.grown(w, qi);
        if (others + mine > budget) {
            if (!pool.release_idle(qi)) return false;
            others = pool.others(w);
            mine = pool.grown(w, qi);
        }
        if (others + mine <= budget) {
            pool.dispatch(qi, w, mine, others + mine);
            return true;
        }
    }
    return false;
}

}  // namespace gbem
