/*
 * mg_clients.h -- C ABI of the serving client driver (libmg_clients.so, host
 * code only, linked against libmg.so): replays a recorded arrival trace against
 * an mg_server from many client threads at once, the way many independent
 * clients would use the serving loop of mg.h (the parallel environments of
 * Sec. II served to several users).  Used to measure served latency under
 * concurrent submission.
 */
#ifndef MG_CLIENTS_H
#define MG_CLIENTS_H

#include "mg.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Replays n requests from n_clients threads.  Thread c submits, in order, the
 * requests i with client[i] == c, each at t0_ns + at_ns[i] on the mg_clock_ns()
 * clock (it sleeps until 200 us before, then spins), with reqs[i].arrival_ns
 * overwritten by that scheduled time so latency counts from the schedule; a
 * submit answered MG_ERR_BUSY (queue full) is retried.  After its last
 * submission the thread waits for each of its tickets.
 *   client      host int32 [n], each in [0, n_clients); at_ns: host [n],
 *               non-decreasing within a client
 *   reqs        host [n] requests as for mg_server_submit (caller-owned; every
 *               buffer they name must stay valid until this call returns)
 *   status      host int32 [n] (written): the submit status if it failed, else
 *               the wait status
 *   latency_s   host [n] (written): arrival -> result in out, or -1
 *   lag_ns      host int64 [n] (written): submission time - scheduled arrival
 * Returns 0 once every thread has finished, -1 for a NULL or out-of-range
 * argument (nothing submitted).  Blocks the calling thread throughout. */
int mgc_replay(mg_server* srv, int32_t n_clients, int64_t n, const int32_t* client,
               const uint64_t* at_ns, mg_request* reqs, uint64_t t0_ns, int32_t* status,
               double* latency_s, int64_t* lag_ns);

#ifdef __cplusplus
}
#endif
#endif /* MG_CLIENTS_H */
