// Serving loop (continuous batching): placeholder until the server lands.
#include "runtime_internal.hpp"

namespace epi {
struct Server {};
void server_shutdown_all(Ctx *c) { c->servers.clear(); }
}  // namespace epi

using namespace epi;
extern "C" {
int epi_server_start(epi_ctx *, const epi_server_config *, int32_t *) { return fail(EPI_EUNSUPPORTED, "server not built"); }
int epi_server_submit(epi_ctx *, int32_t, int32_t, int32_t, int32_t, int32_t *) { return fail(EPI_EUNSUPPORTED, "server not built"); }
int epi_server_poll(epi_ctx *, int32_t, int32_t, int32_t *) { return fail(EPI_EUNSUPPORTED, "server not built"); }
int epi_server_results(epi_ctx *, int32_t, int32_t, int32_t, int32_t *, float *, uint32_t *, int32_t *, double *) { return fail(EPI_EUNSUPPORTED, "server not built"); }
int epi_server_stats(epi_ctx *, int32_t, uint64_t *) { return fail(EPI_EUNSUPPORTED, "server not built"); }
int epi_server_stop(epi_ctx *, int32_t) { return fail(EPI_EUNSUPPORTED, "server not built"); }
}
