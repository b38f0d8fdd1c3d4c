"""Index-tree bookkeeping of the oracle (test infrastructure, never product code).

Follows the paper's definitions:
  * Def. 3 (index tree): the children of a node are disjoint and contained in it;
    modes of a node in none of its children are its free modes (below).
  * Def. 4 / Def. 5 (dummy nodes): a childless node above the deepest level is a leaf;
    dummies carry identity DRMs and projectors and are never materialised.
  * Fig. 1 labels: nodes are numbered level by level, left to right by smallest mode,
    root = 0.
  * Sec. 5 (STTNN ordering) and Fig. 5: node t reuses the contractions of the set
    S_t = preceding siblings of t together with the preceding siblings of every
    ancestor of t (the reading that reproduces all nine panels of Fig. 5).  The paper
    takes the lexicographic order (level by level, left to right) and notes that the
    order is a free choice; `visit` gives another one: the children of each node are
    visited in a chosen order instead of left to right, and "preceding" refers to it.
    Every such S_t is a set of earlier contractions disjoint from I_t, so each
    projection keeps the form of the general sequential projection of Sec. 5.

Tree specs are nested Python tuples of 1-based modes: an int is a one-mode leaf,
a frozenset of ints a multi-mode leaf, a tuple an internal node whose children are
listed left to right.  A visiting order is given as a second spec over the same nodes
with the children of each node listed in the order they are visited (each node's free
modes may stand anywhere among them).  A negative int -m inside a tuple is a free mode m of that node
(Def. 3 allows a node to contain more than the union of its children): it is no node
of its own; in the sketches and the cores it behaves as a child whose maps, projector
and core are identities, the convention the paper takes for dummy nodes, so its index
appears in the node's transfer tensor at its mode position with size n_m.  The
tensor-train tree of Fig. 4 is (((1, -2), -3), ..., -d).  Every node must cover a
contiguous interval of modes, its children and free modes listed in mode order.
"""

from dataclasses import dataclass, field


class TreeError(ValueError):
    pass


@dataclass
class Node:
    id: int
    modes: tuple          # 1-based modes, ascending, contiguous
    level: int
    parent: int           # -1 for the root
    children: list = field(default_factory=list)
    visit: list = field(default_factory=list)    # children in the STTNN visiting order
    rank: int = 0         # r_t (unused at the root)
    over: int = 0         # p_t (unused at the root)
    free: tuple = ()      # free modes (1-based, ascending): in I_t, in no child

    @property
    def first(self):
        return self.modes[0]

    @property
    def last(self):
        return self.modes[-1]

    @property
    def is_leaf(self):
        return not self.children

    @property
    def k(self):
        """Column count of the left DRM, r_t + p_t (eq. "sketch" of Sec. 4)."""
        return self.rank + self.over


def _modes_of(spec):
    if isinstance(spec, int):
        return (abs(spec),)
    if isinstance(spec, frozenset):
        return tuple(sorted(spec))
    if isinstance(spec, tuple):
        out = ()
        for c in spec:
            out += _modes_of(c)
        return out
    raise TreeError(f"bad tree spec element {spec!r}")


def _visit_lists(spec):
    """{modes of an internal node: [modes of its children in the listed order]}."""
    out = {}

    def walk(s):
        if not isinstance(s, tuple):
            return
        kids = [c for c in s if not (isinstance(c, int) and c < 0)]
        key = tuple(sorted(_modes_of(s)))
        if key in out:
            raise TreeError(f"node {key} listed twice in the visiting order")
        out[key] = [tuple(sorted(_modes_of(c))) for c in kids]
        for c in kids:
            walk(c)

    walk(spec)
    return out


class Tree:
    """A validated index tree with level-order numbering.

    rank / over may be ints (same for every non-root node) or dicts keyed by the
    tuple of modes of a node.  visit: None (lexicographic, the paper's order) or a spec
    of the same tree listing each node's children in the order STTNN visits them.
    """

    def __init__(self, spec, dims, rank, over, visit=None):
        self.dims = tuple(int(n) for n in dims)
        self.d = len(self.dims)
        if self.d < 2:
            raise TreeError("order must be at least 2")
        if not isinstance(spec, tuple):
            raise TreeError("root must be an internal node")
        root_modes = _modes_of(spec)
        if sorted(root_modes) != list(range(1, self.d + 1)):
            raise TreeError("root must cover every mode exactly once")

        # breadth-first traversal with children left to right gives level order
        self.nodes = []
        queue = [(spec, -1, 0)]
        while queue:
            nxt = []
            for s, par, lev in queue:
                modes = _modes_of(s)
                if list(modes) != list(range(modes[0], modes[-1] + 1)):
                    raise TreeError(f"node {modes} is not a contiguous interval in order")
                if isinstance(s, int) and s < 0:
                    raise TreeError("a free mode must sit inside an internal node")
                nid = len(self.nodes)
                node = Node(nid, modes, lev, par)
                self.nodes.append(node)
                if par >= 0:
                    self.nodes[par].children.append(nid)
                if isinstance(s, tuple):
                    kids = [c for c in s if not (isinstance(c, int) and c < 0)]
                    node.free = tuple(sorted(-c for c in s if isinstance(c, int) and c < 0))
                    if not kids:
                        raise TreeError("internal node without children (a node of free modes only is a leaf)")
                    if len(s) == 1 and lev > 0:
                        raise TreeError("internal node with a single child equal to itself")
                    firsts = [_modes_of(c)[0] for c in s]
                    if firsts != sorted(firsts):
                        raise TreeError(f"children and free modes of {modes} are not in mode order")
                    for c in kids:
                        nxt.append((c, nid, lev + 1))
            queue = nxt
        # within a level, order is by smallest mode: true by construction, check anyway
        for a, b in zip(self.nodes, self.nodes[1:]):
            if a.level == b.level and a.first >= b.first:
                raise TreeError("level order violated")
        self.depth = max(n.level for n in self.nodes)

        # visiting order of each node's children (default: left to right)
        for n in self.nodes:
            n.visit = list(n.children)
        if visit is not None:
            order = _visit_lists(visit)
            for n in self.nodes:
                if n.is_leaf:
                    continue
                want = order.get(n.modes)
                if want is None or sorted(want) != sorted(self.nodes[c].modes for c in n.children):
                    raise TreeError(f"the visiting order does not list the children of {n.modes}")
                n.visit = [self.by_modes(m) for m in want]
            if len(order) != sum(1 for n in self.nodes if not n.is_leaf):
                raise TreeError("the visiting order has nodes the tree does not have")

        for n in self.nodes[1:]:
            key = n.modes
            n.rank = int(rank[key] if isinstance(rank, dict) else rank)
            n.over = int(over[key] if isinstance(over, dict) else over)
            if n.rank < 1 or n.over < 0:
                raise TreeError("ranks must be >= 1 and oversamples >= 0")

    # ------------------------------------------------------------------ helpers
    def __len__(self):
        return len(self.nodes)

    def __getitem__(self, i):
        return self.nodes[i]

    def n_of(self, node_id):
        """n_{I_t}: product of the mode sizes of node t."""
        p = 1
        for m in self.nodes[node_id].modes:
            p *= self.dims[m - 1]
        return p

    def by_modes(self, modes):
        for n in self.nodes:
            if n.modes == tuple(modes):
                return n.id
        raise KeyError(modes)

    def ancestors(self, t):
        out = []
        p = self.nodes[t].parent
        while p >= 0:
            out.append(p)
            p = self.nodes[p].parent
        return out

    def positions(self, t):
        """Row positions of node t's sketches and core, in mode order: ("c", child id)
        for a child, ("f", mode) for a free mode."""
        n = self.nodes[t]
        items = [(self.nodes[c].first, ("c", c)) for c in n.children] + [(m, ("f", m)) for m in n.free]
        return [it for _, it in sorted(items)]

    @property
    def has_free_modes(self):
        return any(n.free for n in self.nodes)

    def preceding_siblings(self, t):
        """Siblings of t visited before t (left of t in the lexicographic order)."""
        p = self.nodes[t].parent
        if p < 0:
            return []
        sib = self.nodes[p].visit
        return sib[: sib.index(t)]

    def S(self, t):
        """STTNN set S_t (Sec. 5, Fig. 5), ordered left to right by smallest mode."""
        if t == 0:
            return []
        out = list(self.preceding_siblings(t))
        for a in self.ancestors(t):
            out += self.preceding_siblings(a)
        return sorted(out, key=lambda s: self.nodes[s].first)

    def x_rows_ttnn(self, t):
        """Rows of X_t in TTNN: n_{D \\ I_t} (eq. "sketch" of Sec. 4)."""
        p = 1
        for m in range(1, self.d + 1):
            if m not in self.nodes[t].modes:
                p *= self.dims[m - 1]
        return p

    def x_shape_sttnn(self, t):
        """Index sizes of the rows of X_t in STTNN, first index fastest.

        The contracted tensor keeps every contracted group in place as a single
        index of size r_s + p_s; the row index of X_t runs over all indices of that
        tensor except those of I_t, in positional order.
        """
        node = self.nodes[t]
        items = []
        covered = set()
        for s in self.S(t):
            items.append((self.nodes[s].first, self.nodes[s].k))
            covered.update(self.nodes[s].modes)
        for m in range(1, self.d + 1):
            if m in node.modes or m in covered:
                continue
            items.append((m, self.dims[m - 1]))
        return [size for _, size in sorted(items)]

    def x_rows(self, t, variant):
        if variant == "ttnn":
            return self.x_rows_ttnn(t)
        p = 1
        for s in self.x_shape_sttnn(t):
            p *= s
        return p


# Trees used by the paper and by the workloads --------------------------------
TOY = (((1, 2), 3), 4, (5, 6))          # Fig. 1
T4 = ((1, 2), (3, 4))                   # balanced binary tree on four modes
T5 = (((1, 2), 3), (4, 5))              # order-5 tree of the streaming workload
