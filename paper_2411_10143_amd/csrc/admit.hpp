// Admission scan of the request loop: requests wait in arrival order in one
// queue, but belong to one of two paths (0: batched slots, 1: worker
// streams).  A request that waits only for its path's slot or worker stops
// later requests of the same path (each path stays first-come first-served)
// and lets the other path go on; a request that waits for memory stops the
// scan, so no later request can take the memory it waits for.  A request
// that can never be admitted (it does not fit the budget even with nothing
// else resident) is completed with an error and leaves the queue (REJECTED).
#pragma once

#include <utility>

namespace ck {

enum Admit { ADMITTED, WAIT_CLASS, WAIT_MEMORY, REJECTED };

// step(request, blocked) returns {path, outcome}; it must not admit a
// request whose path is already blocked (it returns WAIT_CLASS then).
// Admitted and rejected requests are erased from `pending`.
template <typename Queue, typename Step>
void admit_scan(Queue &pending, Step step) {
    bool blocked[2] = {false, false};
    for (auto it = pending.begin(); it != pending.end() && !(blocked[0] && blocked[1]);) {
        const std::pair<int, Admit> r = step(*it, (const bool *)blocked);
        if (r.second == ADMITTED || r.second == REJECTED)
            it = pending.erase(it);
        else if (r.second == WAIT_MEMORY)
            break;
        else {
            blocked[r.first] = true;
            ++it;
        }
    }
}

}  // namespace ck
