"""Host driver of one transport problem on a world: inject histories in chunks as bank slots
free up and step until every history has ended (paper section "Transport Algorithm").
Every step runs in the library's kernels; this loop only decides how many births to inject."""
from __future__ import annotations

from . import binding


def run_problem(world: binding.World, problem, n_hist: int, seed: int, sampler: int,
                model: binding.Model | None = None, K: int = 16, chunk: int | None = None,
                stream=None, integrator: str = "euler", source_model=None, source_K: int = 16,
                streaming: int | None = None) -> dict:
    """Runs histories [0, n_hist) of `problem` to completion.  Returns the tallies summed over
    histories (divide by n_hist for per-source-particle values) and step statistics:
    `transmissions` counts cell transmissions (with the first-flight split also those streamed
    inside steps, see World.set_streaming), `steps` the transport steps."""
    world.set_integrator(integrator)
    world.set_source_model(source_model, source_K)
    if streaming is not None:
        world.set_streaming(streaming)
    t0 = world.transmissions()
    pid = world.add_problem(problem, seed, stream)
    chunk = world.capacity // 2 if chunk is None else chunk
    injected, steps = 0, 0
    alive = 0
    while injected < n_hist or alive > 0:
        free = world.capacity - alive
        if injected < n_hist and free >= min(chunk, n_hist - injected):
            cnt = min(chunk, n_hist - injected, free)
            alive = world.inject(pid, injected, cnt, stream)
            injected += cnt
        if alive > 0:
            alive = world.step(sampler, model, K, stream)
            steps += 1
    out = world.tally(pid, stream)
    world.remove(pid)
    out.update(steps=steps, transmissions=world.transmissions() - t0)
    return out
