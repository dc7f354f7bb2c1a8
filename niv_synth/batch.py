"""G-buffers of several rooms, built concurrently.

Ray casting is vectorised numpy, which releases the interpreter lock inside
its array operations, so a thread pool overlaps the frames without forking
the (possibly GPU-initialised) process."""
from concurrent.futures import ThreadPoolExecutor

from .gbuffer import make_room_gbuffer


def make_room_gbuffers(seeds, sizes, workers=8):
    """[(room, gbuffer)] for each (seed, (width, height)), in order."""
    assert len(seeds) == len(sizes)
    with ThreadPoolExecutor(max_workers=max(1, min(workers, len(seeds)))) as ex:
        futs = [ex.submit(make_room_gbuffer, s, w, h) for s, (w, h) in zip(seeds, sizes)]
        return [f.result() for f in futs]
