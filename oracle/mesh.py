"""Element geometry and face connectivity (oracle, FP64).

Appendix A partitions the domain into non-overlapping elements (Eq. 9) and
couples neighbours only through the numerical flux on shared faces, with the
outward unit normal of each element (Eq. 10).  For straight-sided
tetrahedra the map from the reference element is affine:

    x(r,s,t) = lam0 v0 + lam1 v1 + lam2 v2 + lam3 v3,

so every geometric factor is constant per element.  Normals and areas are
taken from cross products of physical face edges; faces are matched by the
sorted triple of topological vertex ids, and face nodes by their barycentric
coordinates on the shared vertices (exact, no coordinate tolerance, and
periodic images match automatically).
"""
import numpy as np

from .nodes import barycentric

FACE_VERTS = ((0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3))


class MeshError(ValueError):
    pass


class Mesh:
    """Geometry + connectivity of a tetrahedral mesh for a RefElement."""

    def __init__(self, ref, xyz, EToV, bc):
        xyz = np.array(xyz, dtype=np.float64)
        EToV = np.array(EToV, dtype=np.int64)
        bc = np.array(bc, dtype=np.int64)
        K = xyz.shape[0]
        self.K = K
        self.ref = ref

        # orientation: make every element positively oriented by swapping
        # local vertices 1 and 2 (faces f1 and f3 trade places).
        e = xyz[:, 1:4] - xyz[:, 0:1]
        det6 = np.einsum("kd,kd->k", np.cross(e[:, 0], e[:, 1]), e[:, 2])
        scale = np.max(np.abs(e), axis=(1, 2)) ** 3
        if np.any(np.abs(det6) <= 1e-12 * scale):
            raise MeshError("degenerate element")
        neg = det6 < 0
        xyz[neg] = xyz[neg][:, [0, 2, 1, 3]]
        EToV[neg] = EToV[neg][:, [0, 2, 1, 3]]
        bc[neg] = bc[neg][:, [0, 3, 2, 1]]
        self.xyz, self.EToV, self.bc = xyz, EToV, bc
        self.flipped = neg

        # Jacobian matrix of the affine map and its inverse
        Jm = 0.5 * np.stack([xyz[:, 1] - xyz[:, 0], xyz[:, 2] - xyz[:, 0],
                             xyz[:, 3] - xyz[:, 0]], axis=2)       # [K, x, rst]
        self.J = np.linalg.det(Jm)
        self.drst_dx = np.linalg.inv(Jm)                            # [K, rst, x]

        lam = barycentric(ref.rst)                                  # [Np, 4]
        self.x = np.einsum("iv,kvd->kid", lam, xyz)                 # [K, Np, 3]

        vol = np.abs(det6) / 6.0
        self.normals = np.zeros((K, 4, 3))
        self.area = np.zeros((K, 4))
        for f, (a, b, c) in enumerate(FACE_VERTS):
            d = ({0, 1, 2, 3} - {a, b, c}).pop()
            n = np.cross(xyz[:, b] - xyz[:, a], xyz[:, c] - xyz[:, a])
            inward = np.einsum("kd,kd->k", n, xyz[:, d] - xyz[:, a]) > 0
            n[inward] *= -1
            nn = np.linalg.norm(n, axis=1)
            self.area[:, f] = 0.5 * nn
            self.normals[:, f] = n / nn[:, None]
        self.Fscale = (2.0 / 3.0) * self.area / vol[:, None]       # = sJ / J

        self._connect(lam)

    def _connect(self, lam):
        ref, K = self.ref, self.K
        faces = {}
        for k in range(K):
            for f, vs in enumerate(FACE_VERTS):
                key = tuple(sorted(int(self.EToV[k, v]) for v in vs))
                faces.setdefault(key, []).append((k, f))
        self.EToE = np.full((K, 4), -1, dtype=np.int64)
        self.EToF = np.full((K, 4), -1, dtype=np.int64)
        for key, lst in faces.items():
            if len(lst) > 2:
                raise MeshError("face shared by more than two elements")
            if len(lst) == 1:
                k, f = lst[0]
                if self.bc[k, f] == 0:
                    raise MeshError("unmatched face tagged interior")
                continue
            (k1, f1), (k2, f2) = lst
            t1, t2 = self.bc[k1, f1], self.bc[k2, f2]
            if t1 == 0 and t2 == 0:
                self.EToE[k1, f1], self.EToF[k1, f1] = k2, f2
                self.EToE[k2, f2], self.EToF[k2, f2] = k1, f1
            elif t1 == 0 or t2 == 0:
                raise MeshError("shared face tagged interior on one side only")
            # both tagged: a zero-thickness boundary seen from both sides

        # face-node matching: mapP[k, f, i] = k'*Np + j' for the neighbour node
        # at the same point.  Node i of face f has barycentric coordinates on
        # the face's three global vertex ids; it matches the neighbour node
        # with the same coordinates on the same ids.  The match depends only
        # on (f, f', how the neighbour orders the shared ids), so it is
        # computed once per such class and reused.
        Np, Nfp = ref.Np, ref.Nfp
        self.mapP = np.full((K, 4, Nfp), -1, dtype=np.int64)
        cache = {}
        for k in range(K):
            for f in range(4):
                k2, f2 = self.EToE[k, f], self.EToF[k, f]
                if k2 < 0:
                    continue
                mine = [int(self.EToV[k, v]) for v in FACE_VERTS[f]]
                theirs = [int(self.EToV[k2, v]) for v in FACE_VERTS[f2]]
                cls = (f, int(f2), tuple(theirs.index(g) for g in mine))
                if cls not in cache:
                    cache[cls] = self._match(f, mine, int(f2), theirs, lam)
                self.mapP[k, f] = k2 * Np + ref.Fmask[f2][cache[cls]]

    def _match(self, f, mine, f2, theirs, lam):
        ref = self.ref
        perm = np.full(ref.Nfp, -1, dtype=np.int64)
        for i, node in enumerate(ref.Fmask[f]):
            bi = {g: lam[node, v] for g, v in zip(mine, FACE_VERTS[f])}
            for j, node2 in enumerate(ref.Fmask[f2]):
                bj = {g: lam[node2, v] for g, v in zip(theirs, FACE_VERTS[f2])}
                if all(abs(bi[g] - bj[g]) < 1e-9 for g in bi):
                    perm[i] = j
                    break
            if perm[i] < 0:
                raise MeshError("face nodes do not match")
        return perm
