// Host side of the packed solver (library-internal; used by usbs.hip and the
// request loop in server.hip).  A packed launch runs one workgroup per handle;
// between launches the host moves each handle's counters in and out of the
// PackState table and retires or admits instances.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/usbs.h"
#include "packed.h"

namespace usbs_pack {

// usbs_create; with cold = false the cold start is left to the first packed launch
int create(const usbs_problem *prob, const usbs_params *prm, usbs_handle **out, bool cold);
// usbs_warm_start; with eval_f = false the closing eigen-solve for f(y0) is left to the
// first packed launch
int warm_prepare(usbs_handle *h, const usbs_problem *grown, bool eval_f);

// descriptor and state tables of the launches on one stream (pinned host copies and
// device copies, grown on demand and released by the destructor).  On a non-null stream a
// launch is the replay of a captured graph (table uploads, packed kernel, state download),
// captured again when the number of instances, the iterations per launch or the tables
// change; on the null stream the steps are issued directly.
struct Runner {
    hipStream_t stream = nullptr;
    usbs::PackDesc *desc_dev = nullptr, *desc_host = nullptr;
    usbs::PackState *state_dev = nullptr, *state_host = nullptr;
    int cap = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int graph_count = 0, graph_iters = 0;
    bool graph_failed = false;   // capture not available: issue the steps directly
    int graph_replays = 0;
    explicit Runner(hipStream_t s) : stream(s) {}
    ~Runner();
    Runner(const Runner &) = delete;
    Runner &operator=(const Runner &) = delete;
};

// counters of a new solve on h; 'init' (usbs::PackInit) is what its first launch does first
usbs::PackState begin(const usbs_handle *h, int init);
// one packed launch over the handles whose state is still running (hs[q], st[q], q < count):
// each runs its init step and up to 'iters' iterations; states and handles are updated.
// Returns USBS_OK or a negative USBS_E_* code (message in *err).
int launch(Runner &R, usbs_handle *const *hs, usbs::PackState *st, int count, int iters, std::string *err);
// status and results of a finished packed solve (secs: its wall time)
int finish(usbs_handle *h, const usbs::PackState &st, usbs_result *res, double secs);

}  // namespace usbs_pack
