"""Autotuner for the launch shape of a Solver.

Knobs (all exposed by the C interface): steps per history pass (temporal
blocking), nodes per lane of the history kernel, the age-chunk split of each
channel's window (set through a common target chunk length so that tiles of
uneven channels have similar work), plain vs persistent history pass, and
the hipGraph replay length.  Each candidate is timed with HIP events on the
solver's stream for a few blocks of steps; the solver's state is saved before
and restored after, and the fastest candidate is applied.
"""
from __future__ import annotations

import itertools
import math
import time
from typing import Dict, Iterable, List, Optional

LANES_FOR_BLOCK = {1: (1, 2, 4), 2: (1, 2), 4: (1, 2), 8: (1,), 16: (1,), 32: (1,)}


def chunks_for(solver, ch: int, chunk_len: int) -> int:
    n_hist = int(solver.channels[ch].n_hist)
    return max(1, min(solver.max_chunks(ch), math.ceil(n_hist / chunk_len)))


def apply(solver, cfg: Dict) -> None:
    solver.set_graph(0)
    solver.set_block(cfg["block"])
    for ch in range(len(solver.channels)):
        solver.set_tiling(ch, chunks_for(solver, ch, cfg["chunk_len"]), cfg["vec"])
    solver.set_persistent(cfg["persistent"])
    solver.set_graph(cfg["graph"])


def candidates(solver, blocks: Iterable[int] = (1, 4, 8, 16),
               chunk_lens: Iterable[int] = (256, 1024, 4096, 1 << 30),
               persistent: Iterable[bool] = (False, True),
               graphs: Iterable[int] = (0,)) -> List[Dict]:
    out = []
    for M, L, P, G in itertools.product(blocks, chunk_lens, persistent, graphs):
        for V in LANES_FOR_BLOCK[M]:
            if G and G % M:
                continue
            out.append(dict(block=M, vec=V, chunk_len=L, persistent=P, graph=G))
    return out


def time_config(solver, cfg: Dict, steps: int) -> float:
    """Milliseconds per step of `steps` steps under cfg (after one warm block)."""
    import torch
    apply(solver, cfg)
    solver.step(cfg["block"] + (cfg["graph"] or 0))
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    stream = solver.stream
    e0.record(stream)
    solver.step(steps)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / steps


def tune(solver, cands: Optional[List[Dict]] = None, min_steps: int = 32,
         time_budget_s: float = 60.0, verbose: bool = False, refine_top: int = 3) -> Dict:
    """Try the candidates on the solver's current state, re-time the
    `refine_top` fastest over four times as many steps (short trials are
    noisy at the few-percent level that separates the best shapes), restore
    the state, apply and return the fastest configuration (with its ms/step
    and the table of all timings)."""
    cands = candidates(solver) if cands is None else cands
    solver.set_graph(0)
    solver.set_block(1)             # save at a block boundary
    saved = solver.save_state()
    results = []
    t_start = time.perf_counter()
    for cfg in cands:
        steps = max(min_steps, 2 * cfg["block"], cfg["graph"] or 0)
        steps = int(math.ceil(steps / cfg["block"]) * cfg["block"])
        ms = time_config(solver, cfg, steps)
        results.append(dict(cfg, ms_per_step=ms))
        if verbose:
            print(f"tune: {cfg} -> {ms:.4f} ms/step", flush=True)
        if time.perf_counter() - t_start > time_budget_s:
            break
    if refine_top > 1:
        for r in sorted(results, key=lambda r: r["ms_per_step"])[:refine_top]:
            cfg = {k: r[k] for k in ("block", "vec", "chunk_len", "persistent", "graph")}
            steps = 4 * max(min_steps, 2 * cfg["block"], cfg["graph"] or 0)
            steps = int(math.ceil(steps / cfg["block"]) * cfg["block"])
            r["ms_per_step_refined"] = time_config(solver, cfg, steps)
            if verbose:
                print(f"tune: refine {cfg} -> {r['ms_per_step_refined']:.4f} ms/step", flush=True)
        refined = [r for r in results if "ms_per_step_refined" in r]
        best = min(refined, key=lambda r: r["ms_per_step_refined"])
        best = dict(best, ms_per_step=best["ms_per_step_refined"])
    else:
        best = min(results, key=lambda r: r["ms_per_step"])
    solver.set_graph(0)
    solver.set_block(1)
    solver.load_state(saved)
    del saved
    cfg = {k: best[k] for k in ("block", "vec", "chunk_len", "persistent", "graph")}
    apply(solver, cfg)
    return dict(cfg, ms_per_step=best["ms_per_step"], table=results)
