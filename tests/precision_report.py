"""Precision report for the 256^3, K=2 SDF fit with FP32, BF16 and FP16 coefficient storage.

Each form trains the same seeded initial grid (N(0, 0.05) coefficients) for a number of Adam
steps on 2^22-query batches of the sphere/torus scene (L1 + 0.1 eikonal, lr 1e-2), then
evaluates 2^16 held-out points (scene batch seed 1) and reports, as max and RMS:
  * deployment error: the 16-bit-storage grid's value vs an FP32 grid holding the same FP32
    master coefficients (both evaluated by the library: the error that storage rounding adds);
  * fit error: GPU value vs the analytic scene SDF (context: how well the grid fits).
The arithmetic error of the kernels against the FP64 oracle is the parity tests' subject
(tests/test_gpu_precision.py, on inputs that do not come from the GPU).
Run on a GPU:  python tests/precision_report.py [--steps 100]
Prints one JSON document.
"""
import argparse
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--res", type=int, default=256)
    ap.add_argument("--nq", type=int, default=1 << 22)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--batches", type=int, default=4)
    ap.add_argument("--heldout", type=int, default=1 << 16)
    args = ap.parse_args()

    import torch

    from paper_2402_14415_amd import synth
    from paper_2402_14415_amd.grid import TaylorGrid, sdf_loss

    dev = torch.device("cuda", 0)
    res, nq = args.res, args.nq
    scene = synth.Scene(0)
    print(f"generating {args.batches} batches of {nq} queries", file=sys.stderr, flush=True)
    batches = []
    for b in range(args.batches):
        q, d = synth.scene_batch(scene, nq, seed=0, step=b)
        batches.append((torch.tensor(q, dtype=torch.float32, device=dev), torch.tensor(d, dtype=torch.float32, device=dev)))
    qh, dh = synth.scene_batch(scene, args.heldout, seed=1, step=0)
    qh_t = torch.tensor(qh, dtype=torch.float32, device=dev)
    rng = np.random.default_rng(0)
    C0 = torch.from_numpy(rng.standard_normal(size=(res, res, res, 10), dtype=np.float32) * np.float32(0.05))

    def stats(x):
        x = np.abs(np.asarray(x, dtype=np.float64))
        return {"max": float(x.max()), "rms": float(np.sqrt(np.mean(x ** 2)))}

    report = {"grid": f"{res}^3", "order": 2, "queries_per_step": nq, "steps": args.steps, "heldout": args.heldout,
              "forms": {}}
    for storage in ("f32", "bf16", "f16"):
        grid = TaylorGrid(3, (res,) * 3, 2, (-1.0,) * 3, (1.0,) * 3, storage=storage, coeffs=C0, device=dev)
        ws = grid.workspace(nq)
        f = torch.empty(nq, device=dev)
        g = torch.empty((nq, 3), device=dev)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        loss = None
        for it in range(args.steps):
            if it == 5:
                ev[0].record()
            q, d = batches[it % len(batches)]
            grid.sort(q, ws)
            grid.forward(q, ws, out=(f, g))
            loss, gf, gg = sdf_loss(f, g, d, 0.1, ws)
            grid.backward(q, ws, gf, gg)
            grid.adam_step(ws, lr=1e-2)
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / max(1, args.steps - 5)
        wsh = grid.workspace(qh_t.shape[0])
        grid.sort(qh_t, wsh)
        fh, _ = grid.forward(qh_t, wsh)
        torch.cuda.synchronize()
        f_gpu = fh.double().cpu().numpy()
        ref = TaylorGrid(3, (res,) * 3, 2, (-1.0,) * 3, (1.0,) * 3, coeffs=grid.master, device=dev, optimizer=False)
        wsr = ref.workspace(qh_t.shape[0])
        ref.sort(qh_t, wsr)
        fm, _ = ref.forward(qh_t, wsr)
        torch.cuda.synchronize()
        f_master = fm.double().cpu().numpy()
        report["forms"][storage] = {
            "ms_per_step": ms, "final_loss": float(loss[0]),
            "deployment_error": stats(f_gpu - f_master),
            "fit_error_vs_scene": stats(f_gpu - dh),
        }
        print(f"{storage}: {report['forms'][storage]}", file=sys.stderr, flush=True)
        del ref, wsr
        del grid, ws, wsh
        torch.cuda.empty_cache()
    print(json.dumps(report, indent=1))


if __name__ == "__main__":
    main()
