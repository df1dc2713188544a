// Launch knobs: built-in defaults, explicit caller overrides, and the autotuner cache.
#include "bc_internal.h"

#include <cstdlib>

namespace bcmi {

bool tuning_enabled() {
    const char* e = std::getenv("BCMI_TUNE");
    return !(e && std::string(e) == "off");
}

Knobs default_knobs(const Graph& g) {
    Knobs k;
    k.wg_size = 256;
    k.team = 1;
    k.teams = 0;
    k.hub = 64;
    k.lds_max_n = 4096;
    k.use_graph = true;
    (void)g;
    return k;
}

Knobs resolve_knobs(Graph& g, const bc_tuning* t) {
    Knobs k = default_knobs(g);
    if (!t) return k;
    if (t->wg_size) {
        BC_REQUIRE(t->wg_size >= 64 && t->wg_size <= 1024 && t->wg_size % 64 == 0, BC_E_INVAL,
                   "wg_size must be a multiple of 64 in [64, 1024]");
        k.wg_size = t->wg_size;
    }
    if (t->wgs_per_source) {
        BC_REQUIRE(t->wgs_per_source == 1, BC_E_INVAL, "wgs_per_source must be 1");
        k.team = 1;
    }
    if (t->sources_per_launch) {
        BC_REQUIRE(t->sources_per_launch > 0, BC_E_INVAL, "sources_per_launch must be > 0");
        k.teams = t->sources_per_launch;
    }
    if (t->hub_threshold) k.hub = t->hub_threshold;
    if (t->lds_max_n) k.lds_max_n = t->lds_max_n;
    if (t->use_graph) k.use_graph = t->use_graph > 0;
    if (t->batched) k.batched = t->batched;
    if (t->batch_wg_size) {
        BC_REQUIRE(t->batch_wg_size == 256 || t->batch_wg_size == 512 || t->batch_wg_size == 1024, BC_E_INVAL,
                   "batch_wg_size must be 256, 512 or 1024");
        k.batch_wg = t->batch_wg_size;
    }
    return k;
}

}  // namespace bcmi

namespace bcmi {
Knobs tune_graph(Graph& g) { return default_knobs(g); }
}  // namespace bcmi
